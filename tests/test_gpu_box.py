"""Parity of the uniform-filter blur (sift3d_box_blur) with the FP64 oracle.

Tolerance, from the arithmetic: a pass sums w = 2h+1 float32 values of
magnitude at most M (every pass is a mean, so M = max |input| bounds all
of them) in index order, with error at most (w - 1) u w M, u = 2^-24, then
multiplies by the rounded 1/w (two more roundings of the mean): at most
(w + 1) u M per pass. A mean does not amplify earlier errors, so 3 m
passes give at most 3 m (w + 1) u M, the bound the tests use.

Cases: ragged shapes spanning several 64-wide tiles on every axis, axes
shorter than the filter's reach, a single voxel, h = 0, the largest reach
(passes * h = 28); and 512x512x384 (the launch configuration the benchmark
times) on sampled voxels, each against the oracle on the voxel's cropped
neighbourhood (exact: the reach of m passes is m h).
"""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def _tol(h, m, vol):
    return 3 * m * (2 * h + 2) * U * float(np.abs(vol).max())


def _gpu(vol, h, m):
    import torch

    import paper_2112_10258_amd as S
    d = torch.from_numpy(np.ascontiguousarray(vol, dtype=np.float32)).cuda()
    out = S.box_blur(d, h, m)
    torch.cuda.synchronize()
    return out.cpu().numpy()


CASES = [
    ((67, 130, 150), 3, 3),   # sigma 3.09 with three passes
    ((67, 130, 150), 1, 3),   # sigma 1.6
    ((40, 70, 129), 7, 4),    # reach 28
    ((3, 5, 200), 8, 3),      # y and z shorter than the reach
    ((130, 2, 1), 2, 2),
    ((1, 1, 1), 5, 4),
    ((33, 65, 64), 0, 2),     # identity
]


@pytest.mark.parametrize("shape,h,m", CASES)
def test_box_blur_matches_oracle(shape, h, m):
    print(f"[box] shape={shape} h={h} passes={m}", flush=True)
    vol = np.random.default_rng(hash(shape) % 1000 + h).standard_normal(shape).astype(np.float32)
    got = _gpu(vol, h, m)
    ref = O.box_blur(vol, h, m)
    err = float(np.abs(got.astype(np.float64) - ref).max())
    assert err <= _tol(h, m, vol), (err, _tol(h, m, vol))
    if h == 0:
        assert np.array_equal(got, vol)


def test_box_blur_full_size_sampled():
    import torch

    import paper_2112_10258_amd as S
    nx, ny, nz = 512, 512, 384
    h, m = S.box_half_width(3.09, 3), 3
    print(f"[box] full size {nx}x{ny}x{nz} h={h} passes={m}", flush=True)
    vol = np.random.default_rng(384).standard_normal((nz, ny, nx), dtype=np.float32)
    d = torch.from_numpy(vol).cuda()
    got = S.box_blur(d, h, m)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    pts = [(x, y, z) for x in (0, nx - 1) for y in (0, ny - 1) for z in (0, nz - 1)]
    pts += [(1, ny // 2, nz - 3), (nx // 2, 4, nz // 2), (nx - 5, ny - 2, 2)]
    pts += [(int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))) for _ in range(40)]
    reach = m * h
    tol = _tol(h, m, vol)
    g = got.cpu().numpy()
    for x, y, z in pts:
        z0, y0, x0 = max(0, z - reach), max(0, y - reach), max(0, x - reach)
        blk = vol[z0:z + reach + 1, y0:y + reach + 1, x0:x + reach + 1]
        ref = O.box_blur(blk, h, m)[z - z0, y - y0, x - x0]
        assert abs(float(g[z, y, x]) - ref) <= tol, (x, y, z)


def test_box_blur_binding_checks_buffers():
    """Wrong-sized, wrong-typed or aliased out/tmp buffers are refused on the
    host, before any launch."""
    import torch

    import paper_2112_10258_amd as S
    vol = torch.zeros(8, 9, 10, device="cuda")
    with pytest.raises(ValueError):
        S.box_blur(vol, 1, 3, out=torch.empty(8, 9, 9, device="cuda"))
    with pytest.raises(ValueError):
        S.box_blur(vol, 1, 3, tmp=torch.empty(8, 9, 10, device="cuda", dtype=torch.float64))
    with pytest.raises(ValueError):
        S.box_blur(vol, 1, 3, out=vol)
    o = torch.empty_like(vol)
    with pytest.raises(ValueError):
        S.box_blur(vol, 1, 3, out=o, tmp=o)
