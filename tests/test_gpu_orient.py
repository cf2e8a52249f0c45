"""Dominant orientations and oriented SIFT-Rank on the GPU (sift3d_orient)
against the FP64 oracle run on the GPU's own Gaussian levels and keypoints.

Contract (stage-wise): for every keypoint whose oracle decision margin
(nearest-direction choices, peak thresholds and comparisons, peak order,
signs of rotated offsets and gradients) is at least 1e-9, the frame count is
equal, every frame equals the oracle's within 1e-6 (float32 output of an
FP64 computation) and the ranks are equal except between histogram bins
within 1e-6 of the largest bin. Keypoints under the margin are counted and
must stay rare. The GPU sums are fixed-point integers, so repeated runs are
bit-identical and a batch plan gives each volume the plain plan's result.
"""
import numpy as np
import pytest

import oracle as O
from gen import phantoms as P
from tests.helpers import MARGIN, gpu_extract, oracle_params, rank_mismatch_excused

pytestmark = pytest.mark.gpu

FRAME_TOL = 1e-6
DECISION_MARGIN = 1e-9


def _say(msg):
    print(f"[orient] {msg}", flush=True)


def _gpu_orient(g, peak_ratio=0.8):
    """Run sift3d_orient on a gpu_extract result; host copies."""
    import torch

    import paper_2112_10258_amd as S
    ctx, plan, buf, dvol = g["_keep"]
    n = plan.n_volumes * max(plan.capacity, 1)
    K = S.MAX_ORIENTATIONS
    nf = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    fr = torch.full((n, K, 9), 7.0, dtype=torch.float32, device="cuda")
    sr = torch.full((n, K, 64), 255, dtype=torch.uint8, device="cuda")
    plan.orient(buf.ws, buf.kp, buf.count, nf, fr, sr, peak_ratio)
    torch.cuda.synchronize()
    k = min(g["count"], plan.capacity)
    return nf[:k].cpu().numpy(), fr[:k].cpu().numpy().reshape(k, K, 3, 3), sr[:k].cpu().numpy()


def _compare(g, label, peak_ratio=0.8):
    p = oracle_params(g["params"])
    nf, fr, sr = _gpu_orient(g, peak_ratio)
    G64 = [[x.astype(np.float64) for x in Gs] for Gs in g["G"]]
    ref = O.orientations(G64, g["keypoints"], p, tau=peak_ratio, kmax=4)
    K = len(nf)
    excused = 0
    for i in range(K):
        if ref["margin"][i] < DECISION_MARGIN:
            excused += 1
            continue
        assert nf[i] == ref["nframes"][i], (label, i, nf[i], ref["nframes"][i])
        for f in range(nf[i]):
            np.testing.assert_allclose(fr[i, f], ref["frames"][i, f], atol=FRAME_TOL, err_msg=f"{label} kp {i} frame {f}")
            h = ref["hist"][i, f]
            assert rank_mismatch_excused(h, sr[i, f], ref["rank"][i, f], MARGIN * max(h.max(), 1e-300)), (label, i, f)
        for f in range(nf[i], 4):
            assert not fr[i, f].any() and not sr[i, f].any(), (label, i, f)
    hist = np.bincount(nf, minlength=5)
    _say(f"{label}: {K} keypoints, frames per keypoint {hist.tolist()}, {excused} under the decision margin")
    assert excused <= max(2, K // 50), (label, excused, K)
    return nf, fr, sr


@pytest.mark.parametrize("case", ["config1", "ragged", "config2"])
def test_orientations_match_oracle(case):
    if case == "config1":
        g = gpu_extract(P.config1(), n_octaves=2)
    elif case == "ragged":
        g = gpu_extract(P.noise_blob_volume((45, 38, 53), 77))
    else:
        g = gpu_extract(P.config2())
    assert g["count"] > 0
    _compare(g, case)


def test_orientation_peak_ratio_and_repeatability():
    g = gpu_extract(P.config1(), n_octaves=2)
    a = _gpu_orient(g)
    b = _gpu_orient(g)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    # a lower peak ratio keeps at least as many frames
    lo = _compare(g, "config1, peak ratio 0.6", peak_ratio=0.6)[0]
    assert np.all(lo >= np.minimum(a[0], 4)) or lo.sum() >= a[0].sum()


def test_orientation_batch_equals_plain():
    import torch

    import paper_2112_10258_amd as S
    vols = [P.noise_blob_volume(s, 400 + i) for i, s in enumerate([(64, 64, 64), (41, 37, 33)])]
    shapes = [(v.shape[2], v.shape[1], v.shape[0]) for v in vols]
    ctx = S.Context(S.default_params(), P.pair_draws())
    cap = 1 << 12
    bplan = S.Plan(ctx, shapes, cap, batch=True)
    bbuf = S.Buffers(bplan)
    S.run_extract(bplan, bplan.pack_volumes(vols), bbuf)
    n = len(vols) * cap
    bnf = torch.zeros(n, dtype=torch.int32, device="cuda")
    bfr = torch.zeros(n, 4, 9, dtype=torch.float32, device="cuda")
    bsr = torch.zeros(n, 4, 64, dtype=torch.uint8, device="cuda")
    bplan.orient(bbuf.ws, bbuf.kp, bbuf.count, bnf, bfr, bsr)
    torch.cuda.synchronize()
    for v, (vol, sh) in enumerate(zip(vols, shapes)):
        g = gpu_extract(vol, cap=cap)
        nf, fr, sr = _gpu_orient(g)
        k = len(nf)
        assert k == int(bbuf.count[v].item()) and k > 0
        assert np.array_equal(bnf[v * cap:v * cap + k].cpu().numpy(), nf)
        assert np.array_equal(bfr[v * cap:v * cap + k].cpu().numpy().reshape(k, 4, 3, 3), fr)
        assert np.array_equal(bsr[v * cap:v * cap + k].cpu().numpy(), sr)
    _say("batch plan: every volume's frames and descriptors equal the plain plan's")


def test_orient_rejects_bad_arguments():
    import torch

    import paper_2112_10258_amd as S
    g = gpu_extract(P.config1(), n_octaves=2)
    ctx, plan, buf, dvol = g["_keep"]
    n = max(plan.capacity, 1)
    nf = torch.zeros(n, dtype=torch.int32, device="cuda")
    fr = torch.zeros(n, 4, 9, dtype=torch.float32, device="cuda")
    sr = torch.zeros(n, 4, 64, dtype=torch.uint8, device="cuda")
    for bad in (0.0, -0.5, 1.5):
        with pytest.raises(S.Sift3dError):
            plan.orient(buf.ws, buf.kp, buf.count, nf, fr, sr, bad)
