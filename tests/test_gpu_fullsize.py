"""Parity at full workload sizes, in the launch configuration the benchmark
times, on outputs the oracle can compute one by one.

512x512x384 (fused streaming passes and xy + z launches on octaves 0 and 1,
compact passes below):
  - G_i at sampled voxels (volume corners, faces and random interior) equals
    the oracle's blur of the GPU's own G_{i-1} (the input for G_0 of octave
    0) evaluated at that voxel, within 1e-5 of the level's max;
  - G_0 of octave o > 0 at sampled voxels equals the mean of the GPU's
    2x2x2 block of G_S of octave o-1;
  - every D_i equals G_i - G_{i+1} rounded to float32, bit for bit;
  - the oracle's detection on the GPU's D levels gives the same keypoints;
  - descriptors of a sample of keypoints match the oracle on the GPU's G
    levels under the near-tie margins.
The 32-volume batch (each axis U{96..192}) gives every volume the plain
path's results bit for bit.
"""
import numpy as np
import pytest

import oracle as O
from gen import phantoms as P
from tests.helpers import LEVEL_RTOL, MARGIN, kp_keys, oracle_params, rank_mismatch_excused, unpack_bits

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[fullsize] {msg}", flush=True)


def _points(dims, n_random, rng):
    nx, ny, nz = dims
    pts = {(x, y, z) for x in (0, nx - 1) for y in (0, ny - 1) for z in (0, nz - 1)}
    pts |= {(nx // 2, ny // 2, 0), (0, ny // 2, nz // 2), (nx // 2, 0, nz // 2), (nx - 1, ny // 3, nz - 2)}
    for _ in range(n_random):
        pts.add((int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))))
    return sorted(pts)


def _blur_at(src, sigma, trunc, pts):
    """Oracle blur of src evaluated at each point, from its clamped (2r+1)^3
    neighbourhood (the x, y and z passes of the centre voxel read nothing else)."""
    r = int(np.ceil(trunc * sigma))
    nz, ny, nx = src.shape
    out = []
    for x, y, z in pts:
        zi = np.clip(np.arange(z - r, z + r + 1), 0, nz - 1)
        yi = np.clip(np.arange(y - r, y + r + 1), 0, ny - 1)
        xi = np.clip(np.arange(x - r, x + r + 1), 0, nx - 1)
        blk = src[np.ix_(zi, yi, xi)].astype(np.float64)
        out.append(O.blur(blk, sigma, trunc)[r, r, r])
    return np.array(out)


def test_config4_sampled_parity():
    import torch

    import paper_2112_10258_amd as S
    vol = P.config4()
    nz, ny, nx = vol.shape
    _say(f"case=config4 shape={vol.shape} (bench launch configuration, pyramid_mode 0)")
    gp = S.default_params()
    ctx = S.Context(gp, P.pair_draws())
    cap = 1 << 17
    plan = S.Plan(ctx, (nx, ny, nz), cap)
    buf = S.Buffers(plan)
    passes = plan.pyramid_passes()
    assert any(p[5] == 1 for p in passes if p[0] == 0), "octave 0 is expected on the fused pass"
    dvol = torch.from_numpy(vol).cuda()
    S.run_extract(plan, dvol, buf)
    torch.cuda.synchronize()
    res = S.fetch_results(plan, buf)
    _say(f"{plan.n_octaves} octaves, {res['count']} keypoints")
    assert 0 < res["count"] <= cap
    p = oracle_params(gp)
    sig0, incs = O.level_increments(p)
    rng = np.random.default_rng(44)
    Sn = gp.scales
    G_keep = []
    D_all = []
    for o in range(plan.n_octaves):
        dims = plan.octave_dims(o)
        pts = _points(dims, 40, rng)
        idx = tuple(np.array(pts).T[::-1])   # (z, y, x) index arrays
        G = [plan.level(buf.ws, o, 0, i).cpu().numpy() for i in range(Sn + 3)]
        if o == 0:
            ref = _blur_at(vol, sig0, p.trunc, pts)
        else:
            prev = G_keep[o - 1][Sn]
            ref = np.array([prev[2 * z:2 * z + 2, 2 * y:2 * y + 2, 2 * x:2 * x + 2].astype(np.float64).mean()
                            for x, y, z in pts])
        err = np.abs(G[0][idx] - ref).max() / np.abs(G[0]).max()
        assert err <= LEVEL_RTOL, (o, 0, err)
        worst = err
        for i in range(1, Sn + 3):
            ref = _blur_at(G[i - 1], incs[i - 1], p.trunc, pts)
            err = np.abs(G[i][idx].astype(np.float64) - ref).max() / np.abs(G[i]).max()
            assert err <= LEVEL_RTOL, (o, i, err)
            worst = max(worst, err)
        D = [plan.level(buf.ws, o, 1, i).cpu().numpy() for i in range(Sn + 2)]
        for i in range(Sn + 2):
            assert np.array_equal(D[i], G[i] - G[i + 1]), (o, i)
        _say(f"octave {o} dims {dims}: {len(pts)} points per level, worst rel err {worst:.2e}; D exact")
        # keep what the descriptors (G_1..G_S) and the next octave's G_0 check (G_S) need
        G_keep.append([G[s] if 1 <= s <= Sn else None for s in range(Sn + 3)])
        D_all.append(D)
        del G
    want = O.detect(D_all, p)
    got = res["keypoints"]
    assert res["count"] == len(want)
    assert kp_keys(got) == kp_keys(want)
    assert np.array_equal(got["polarity"], want["polarity"])
    assert np.array_equal(got["dog"], want["dog"].astype(np.float32))
    _say(f"detection on the GPU's D levels: {len(got)} keypoints identical")
    del D_all
    sel = np.unique(np.linspace(0, len(got) - 1, min(len(got), 240)).astype(int))
    ks = got[sel]
    G64 = [[None if g is None else g.astype(np.float64) for g in Gs] for Gs in G_keep]
    d = O.describe(G64, ks, P.pair_draws(), p)
    for j, i in enumerate(sel):
        h = d["hist"][j]
        assert rank_mismatch_excused(h, res["siftrank"][i], d["siftrank"][j], MARGIN * max(h.max(), 1e-300)), i
        assert rank_mismatch_excused(d["diff"][j], res["rrief"][i], d["rrief"][j], MARGIN), i
    gb = unpack_bits(res["brief"][sel], p.brief_n)
    ob = unpack_bits(d["brief"], p.brief_n)
    assert np.all(np.abs(d["diff"][gb != ob]) < MARGIN)
    _say(f"descriptors of {len(sel)} sampled keypoints match; brief bits differing {int((gb != ob).sum())}")


def test_config3_batch_equals_plain_at_full_size():
    import torch

    import paper_2112_10258_amd as S
    vols = P.config3()
    shapes = [(v.shape[2], v.shape[1], v.shape[0]) for v in vols]
    _say(f"case=config3 batch of {len(vols)} volumes")
    cap = 1 << 14
    ctx = S.Context(S.default_params(), P.pair_draws())
    bplan = S.Plan(ctx, shapes, cap, batch=True)
    bbuf = S.Buffers(bplan)
    S.run_extract(bplan, bplan.pack_volumes(vols), bbuf)
    torch.cuda.synchronize()
    total = 0
    for v, (vol, sh) in enumerate(zip(vols, shapes)):
        plan = S.Plan(ctx, sh, cap)
        buf = S.Buffers(plan)
        S.run_extract(plan, torch.from_numpy(vol).cuda(), buf)
        torch.cuda.synchronize()
        a, b = S.fetch_results(bplan, bbuf, v), S.fetch_results(plan, buf)
        assert a["count"] == b["count"] and a["count"] <= cap, v
        assert a["keypoints"].tobytes() == b["keypoints"].tobytes(), v
        for f in ("siftrank", "brief", "rrief"):
            assert np.array_equal(a[f], b[f]), (v, f)
        total += a["count"]
        del plan, buf
    _say(f"all {len(vols)} volumes identical to the plain path ({total} keypoints)")
