"""The matching stage on the GPU against the FP64 oracle: unit-length
normalisation (Section 3.1 e), matching units, and the 7-DoF similarity
Hough vote with its inliers (Section 3.3; reading R26).

Contract:
  - normalisation: float32 rounding of the oracle's double values, bit for
    bit (one correctly rounded square root and quotient on each side);
  - units: bit-exact copies of the GPU's own keypoints, frames and
    descriptors, in (keypoint, frame) order;
  - Hough: winning bin, its votes, fit-set size, inlier count and every
    inlier flag equal the oracle's on the same inputs when every valid
    match's decision margin (distance of a bin coordinate to a multiple of
    1/2, of an inlier test to its threshold) is at least 1e-9; the
    transform agrees within 1e-9 (both double, different closed forms:
    Horn's quaternion on the GPU, Umeyama's SVD in the oracle).
End to end, a brain-like phantom against a copy under a known similarity:
GPU extraction, orientation, units, matching and Hough recover the
transform and the inliers are true correspondences.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle.hough import _inliers as oracle_inliers
from gen import phantoms as P
from tests.helpers import gpu_extract

pytestmark = pytest.mark.gpu

DECISION_MARGIN = 1e-9
TRANSFORM_TOL = 1e-9


def _say(msg):
    print(f"[hough] {msg}", flush=True)


def _oracle_hp(hp):
    return O.HoughParams(scale_bin=hp.scale_bin, angle_bin=hp.angle_bin, trans_bin=hp.trans_bin,
                         centre=tuple(hp.centre), inlier_sigmas=hp.inlier_sigmas, inlier_log2s=hp.inlier_log2s,
                         iterations=hp.iterations)


def _gpu_hough(ga, gb, m, hp, ws=None):
    import torch

    import paper_2112_10258_amd as S
    dga = torch.from_numpy(np.ascontiguousarray(ga, dtype=np.float32)).cuda()
    dgb = torch.from_numpy(np.ascontiguousarray(gb, dtype=np.float32)).cuda()
    dm = torch.from_numpy(np.ascontiguousarray(m, dtype=np.int32)).cuda()
    res, inl = S.hough(dga, dgb, dm, hp, ws=ws)
    torch.cuda.synchronize()
    return res, inl.cpu().numpy().astype(bool)


def _compare(ga, gb, m, hp, label):
    res, inl = _gpu_hough(ga, gb, m, hp)
    ref = O.hough(ga, gb, m, _oracle_hp(hp))
    valid = (m >= 0) & (m < len(gb))
    mg = ref["margin"][valid]
    small = int(np.sum(mg < DECISION_MARGIN))
    _say(f"{label}: {len(m)} matches, votes {res['votes']}, fit {res['n_fit']}, inliers {res['n_inliers']}, "
         f"status {res['status']}, smallest margin {mg.min() if len(mg) else float('inf'):.2e}")
    assert small == 0, (label, "decision within rounding of a bin or inlier threshold", small)
    assert res["status"] == ref["status"], label
    assert res["bin"] == ref["bin"] and res["votes"] == ref["votes"], label
    assert res["n_fit"] == ref["n_fit"] and res["n_inliers"] == ref["n_inliers"], label
    assert np.array_equal(inl, ref["inlier"]), label
    if ref["status"]:
        assert abs(res["scale"] - ref["scale"]) <= TRANSFORM_TOL * ref["scale"], label
        np.testing.assert_allclose(res["R"], ref["R"], atol=TRANSFORM_TOL, err_msg=label)
        np.testing.assert_allclose(res["t"], ref["t"], atol=TRANSFORM_TOL * 1e3, err_msg=label)
    else:
        assert res["scale"] == 0.0 and not res["R"].any()
    return res, inl, ref


# ------------------------------------------------------------ normalisation
@pytest.mark.parametrize("words,n", [(1, 1), (4, 1001), (3, 77)])
def test_normalize_brief_matches_oracle(words, n):
    import torch

    import paper_2112_10258_amd as S
    rng = np.random.default_rng(words * 1000 + n)
    w = rng.integers(0, 2 ** 62, size=(n, words), dtype=np.int64) * 4 + rng.integers(0, 4, size=(n, words))
    got = S.normalize(torch.from_numpy(w).cuda(), S.MATCH_BRIEF).cpu().numpy()
    ref = O.unit_normalize(w.view(np.uint64), 0).astype(np.float32)
    assert got.shape == ref.shape and np.array_equal(got, ref)


@pytest.mark.parametrize("m,n", [(64, 1), (64, 999), (256, 130), (192, 5)])
def test_normalize_ranks_matches_oracle(m, n):
    import torch

    import paper_2112_10258_amd as S
    rng = np.random.default_rng(m + n)
    r = np.stack([rng.permutation(m) for _ in range(n)]).astype(np.uint8)
    if n > 2:
        r[1] = 0            # an unused slot stays zero
        r[2] = rng.integers(0, 256, m)   # any row, not only permutations
    got = S.normalize(torch.from_numpy(r).cuda(), S.MATCH_RANKS).cpu().numpy()
    ref = O.unit_normalize(r, 1).astype(np.float32)
    assert np.array_equal(got, ref)


def test_normalize_empty():
    import torch

    import paper_2112_10258_amd as S
    out = S.normalize(torch.zeros((0, 64), dtype=torch.uint8, device="cuda"), S.MATCH_RANKS)
    assert out.shape == (0, 64)


# ------------------------------------------------------------ Hough, synthetic
@pytest.mark.parametrize("n_true,n_false,seed", [(150, 250, 21), (40, 3000, 22), (1, 0, 23), (2, 1, 24),
                                                 (600, 400, 25)])
def test_hough_matches_oracle_on_planted_scenes(n_true, n_false, seed):
    import paper_2112_10258_amd as S
    ga, gb, m, tr = P.hough_scene(n_true, n_false, seed=seed)
    hp = S.hough_default_params((145, 174, 145))
    res, inl, _ = _compare(ga, gb, m, hp, f"scene {n_true}+{n_false} seed {seed}")
    if n_true >= 40 and n_false <= 20 * n_true:
        assert res["status"] == 1 and inl[:n_true].all()
        assert abs(math.log2(res["scale"] / tr["s"])) < 0.01
    elif n_true >= 40:
        # 75 outliers per true match: a few outliers that agree by chance
        # pull the fit, so most (not all) true matches stay inliers
        assert res["status"] == 1 and inl[:n_true].mean() >= 0.9
        assert abs(math.log2(res["scale"] / tr["s"])) < 0.1


def test_hough_invalid_matches_and_scales():
    import paper_2112_10258_amd as S
    ga, gb, m, _ = P.hough_scene(80, 80, seed=26)
    m = m.copy()
    m[::17] = -1                 # no match
    m[5] = len(gb)               # out of range
    m[6] = 1 << 30
    ga = ga.copy()
    ga[7, 3] = 0.0               # scales that are not positive
    ga[8, 3] = -2.0
    ga[9, 3] = np.nan
    gb = gb.copy()
    gb[m[10], 3] = 0.0
    hp = S.hough_default_params((145, 174, 145))
    _compare(ga, gb, m, hp, "invalid rows")


def test_hough_parameters_and_rounds():
    import paper_2112_10258_amd as S
    ga, gb, m, _ = P.hough_scene(120, 200, seed=27)
    for it, sb, ab, tb in ((1, 1.0, math.pi / 6, 43.5), (4, 0.5, math.pi / 9, 20.0), (16, 2.0, math.pi / 4, 80.0)):
        hp = S.hough_default_params((145, 174, 145))
        hp.iterations, hp.scale_bin, hp.angle_bin, hp.trans_bin = it, sb, ab, tb
        _compare(ga, gb, m, hp, f"iterations {it}, widths {sb}/{ab:.3f}/{tb}")


def test_hough_empty_and_reused_workspace():
    import torch

    import paper_2112_10258_amd as S
    hp = S.hough_default_params((64, 64, 64))
    ga, gb, m, _ = P.hough_scene(0, 0, seed=28)
    res, inl = _gpu_hough(ga, gb, m, hp)
    assert res["status"] == 0 and res["bin"] == -1 and res["votes"] == 0 and len(inl) == 0
    # one workspace for a large call, then a small one: the table is cleared
    big = P.hough_scene(300, 2000, seed=29)
    small = P.hough_scene(30, 10, seed=30)
    ws = torch.empty(S.hough_workspace_bytes(len(big[0])), dtype=torch.uint8, device="cuda")
    r1 = _gpu_hough(*big[:3], hp, ws=ws)
    r2 = _gpu_hough(*small[:3], hp, ws=ws)
    r3 = _gpu_hough(*big[:3], hp, ws=ws)
    assert r1[0]["bin"] == r3[0]["bin"] and r1[0]["scale"] == r3[0]["scale"] and np.array_equal(r1[1], r3[1])
    ref = O.hough(*small[:3], _oracle_hp(hp))
    assert r2[0]["votes"] == ref["votes"] and np.array_equal(r2[1], ref["inlier"])


def test_hough_large_scene_matches_oracle_and_repeats():
    import paper_2112_10258_amd as S
    ga, gb, m, _ = P.hough_scene(3000, 30000, seed=31)
    hp = S.hough_default_params((145, 174, 145))
    res, inl, _ = _compare(ga, gb, m, hp, "33000 matches")
    again = _gpu_hough(ga, gb, m, hp)
    assert again[0]["bin"] == res["bin"] and again[0]["scale"] == res["scale"]
    assert np.array_equal(again[0]["R"], res["R"]) and np.array_equal(again[1], inl)



def test_hough_maximum_size_on_sampled_matches():
    """n_a = 2^21, the largest the entry point accepts: the planted
    similarity is recovered, and on 4000 sampled valid matches each inlier
    flag equals the oracle's inlier rule applied to the GPU's transform (a
    full oracle vote at this size would take minutes)."""
    import paper_2112_10258_amd as S
    from scipy.spatial.transform import Rotation
    n = 1 << 21
    n_true = 1 << 15
    ga, gb, m, truth = P.hough_scene(n_true, n - n_true, seed=37)
    hp = S.hough_default_params((145, 174, 145))
    _say(f"maximum size: {n} matches, workspace {S.hough_workspace_bytes(n) / 2**30:.2f} GiB")
    res, inl = _gpu_hough(ga, gb, m, hp)
    _say(f"maximum size: votes {res['votes']}, fit {res['n_fit']}, inliers {res['n_inliers']}, "
         f"scale {res['scale']:.5f}")
    assert res["status"] == 1
    assert abs(res["scale"] / truth["s"] - 1.0) < 0.01
    err = Rotation.from_matrix(res["R"] @ truth["R"].T).magnitude()
    assert np.degrees(err) < 0.5, np.degrees(err)
    assert int(inl.sum()) == res["n_inliers"]
    # the true pairs are the first n_true rows of A
    assert inl[:n_true].mean() >= 0.99
    # a random pair passes both inlier tests with probability about 1e-3
    assert res["n_inliers"] <= n_true + (n - n_true) // 200
    rng = np.random.default_rng(38)
    pick = np.sort(rng.choice(n, 4000, replace=False))
    pick = np.concatenate([np.arange(200), pick[pick >= 200]])
    valid = np.ones(len(pick), dtype=bool)
    ref, mg = oracle_inliers(ga[pick], gb, m[pick], valid, res["scale"], np.asarray(res["R"]), np.asarray(res["t"]),
                         _oracle_hp(hp))
    keep = mg >= DECISION_MARGIN
    assert keep.sum() >= 0.99 * len(pick)
    assert np.array_equal(inl[pick][keep], ref[keep])


# ------------------------------------------------------------ units
def _units_expected(kp, nf, fr, sr):
    unit, geo, desc = [], [], []
    for k in range(len(kp)):
        for f in range(nf[k]):
            unit.append(k * 4 + f)
            geo.append([kp["xf"][k], kp["yf"][k], kp["zf"][k], kp["sigma"][k]] + list(fr[k, f].reshape(9)))
            desc.append(sr[k, f])
    return (np.array(unit, dtype=np.int32), np.array(geo, dtype=np.float32).reshape(-1, 13),
            np.array(desc, dtype=np.uint8).reshape(-1, 64))


def _oriented(vol):
    """GPU extraction + orientation + units of one volume."""
    import torch

    import paper_2112_10258_amd as S
    g = gpu_extract(vol, levels=False)
    ctx, plan, buf, dvol = g["_keep"]
    cap = plan.capacity
    nf = torch.zeros(cap, dtype=torch.int32, device="cuda")
    fr = torch.zeros(cap, 4, 9, dtype=torch.float32, device="cuda")
    sr = torch.zeros(cap, 4, 64, dtype=torch.uint8, device="cuda")
    plan.orient(buf.ws, buf.kp, buf.count, nf, fr, sr)
    unit, geo, desc = S.units(buf.kp, buf.count, cap, nf, fr, sr)
    torch.cuda.synchronize()
    k = min(g["count"], cap)
    host = (g["keypoints"], nf[:k].cpu().numpy(), fr[:k].cpu().numpy().reshape(k, 4, 3, 3), sr[:k].cpu().numpy())
    return g, (unit, geo, desc), host, (buf, cap)


def test_units_oriented_and_upright():
    import torch

    import paper_2112_10258_amd as S
    g, (unit, geo, desc), (kp, nf, fr, sr), (buf, cap) = _oriented(P.config1())
    eu, eg, ed = _units_expected(kp, nf, fr, sr)
    assert np.array_equal(unit.cpu().numpy(), eu)
    assert np.array_equal(geo.cpu().numpy(), eg)
    assert np.array_equal(desc.cpu().numpy(), ed)
    # upright: one unit per keypoint, identity frame, descriptor row k
    up_u, up_g, up_d = S.units(buf.kp, buf.count, cap, desc=buf.siftrank)
    k = len(kp)
    assert np.array_equal(up_u.cpu().numpy(), np.arange(k, dtype=np.int32) * 4)
    G = up_g.cpu().numpy()
    assert np.array_equal(G[:, 3], kp["sigma"]) and np.array_equal(G[:, 0], kp["xf"])
    assert np.array_equal(G[:, 4:], np.tile(np.eye(3, dtype=np.float32).reshape(9), (k, 1)))
    assert np.array_equal(up_d.cpu().numpy(), buf.siftrank[:k].cpu().numpy())
    # no copy requested
    u2, g2, d2 = S.units(buf.kp, buf.count, cap)
    assert d2 is None and np.array_equal(g2.cpu().numpy(), G)
    # a count above the capacity is clamped; zero capacity gives no unit
    cnt = torch.tensor([cap + 5], dtype=torch.int32, device="cuda")
    u3, _, _ = S.units(buf.kp, cnt, cap)
    assert len(u3) == cap
    u4, _, _ = S.units(buf.kp, cnt, 0)
    assert len(u4) == 0
    _say(f"units: {k} keypoints -> {len(eu)} oriented units; upright and clamped cases exact")


# ------------------------------------------------------------ end to end
def test_phantom_pair_recovers_the_similarity():
    import torch

    import paper_2112_10258_amd as S
    from scipy.spatial.transform import Rotation
    A = P.config2()
    B, s, R, t = P.similarity_copy(A, scale=1.15, angle_deg=20.0)
    _, ua, _, _ = _oriented(A)
    _, ub, _, _ = _oriented(B)
    ga, gb = ua[1], ub[1]
    idx, d1, d2 = S.match(ua[2].reshape(len(ua[2]), 64), ub[2].reshape(len(ub[2]), 64), S.MATCH_RANKS)
    torch.cuda.synchronize()
    da, db = ua[2].cpu().numpy(), ub[2].cpu().numpy()
    ridx, _, _ = O.match_nn(da, db, 1)
    assert np.array_equal(idx.cpu().numpy(), ridx)
    nz, ny, nx = A.shape
    hp = S.hough_default_params((nx, ny, nz))
    res, inl, ref = _compare(ga.cpu().numpy(), gb.cpu().numpy(), idx.cpu().numpy(), hp, "phantom pair")
    # ground truth: the planted transform and the true correspondences
    assert res["status"] == 1
    assert abs(math.log2(res["scale"] / s)) < 0.01
    rot_err = math.degrees(np.linalg.norm(Rotation.from_matrix(res["R"] @ R.T).as_rotvec()))
    assert rot_err < 1.0
    c = np.asarray(hp.centre)
    assert np.linalg.norm(res["scale"] * res["R"] @ c + res["t"] - (s * R @ c + t)) < 1.0
    GA, GB, I = ga.cpu().numpy().astype(np.float64), gb.cpu().numpy().astype(np.float64), idx.cpu().numpy()
    true = np.linalg.norm(s * GA[:, :3] @ R.T + t - GB[I, :3], axis=1) <= 2.0 * GB[I, 3]
    prec = (true & inl).sum() / max(inl.sum(), 1)
    rec = (true & inl).sum() / max(true.sum(), 1)
    _say(f"phantom pair: {len(GA)}/{len(GB)} units, {res['n_inliers']} inliers, precision {prec:.3f}, "
         f"recall {rec:.3f}, rotation error {rot_err:.3f} deg, scale {res['scale']:.4f} (true {s})")
    assert res["n_inliers"] >= 100 and prec >= 0.95 and rec >= 0.9
