"""Pins of the matching oracle (unit-length normalisation, Section 3.1 e;
7-DoF Hough vote and inliers, Section 3.3, reading R26) against what the
mathematics fixes: closed forms, scipy's rotation routines, optimality of
the least-squares fit, brute-force vote counts written differently from the
oracle's, planted transforms with known correspondences and invariances."""
import itertools
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle as O
from gen import phantoms as P


def _rng(seed):
    return np.random.default_rng(seed)


# --------------------------------------------------------- normalisation
def test_unit_normalize_brief_is_scaled_signs():
    rng = _rng(1)
    w = rng.integers(0, 2 ** 63, size=(20, 4), dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, size=(20, 4)).astype(np.uint64)
    f = O.unit_normalize(w, 0)
    assert f.shape == (20, 256)
    np.testing.assert_allclose(np.linalg.norm(f, axis=1), 1.0, rtol=0, atol=1e-15)
    # entries are +-1/16 and the bit order is least significant first
    assert np.all(np.abs(np.abs(f) - 1.0 / 16.0) == 0.0)
    assert (f[0, 0] > 0) == bool(int(w[0, 0]) & 1)
    assert (f[0, 64 + 5] > 0) == bool((int(w[0, 1]) >> 5) & 1)
    # squared distance = 4 * Hamming / n, Hamming from the matcher's definition
    idx, d1, _ = O.match_nn(w[:10], w[10:], 0)
    for i in range(10):
        d2 = float(((f[i] - f[10 + idx[i]]) ** 2).sum())
        assert abs(d2 - 4.0 * d1[i] / 256.0) <= 1e-14


@pytest.mark.parametrize("m", [64, 256])
def test_unit_normalize_ranks_closed_form_and_dot_product_search(m):
    rng = _rng(m)
    A = np.stack([rng.permutation(m) for _ in range(30)]).astype(np.uint8)
    B = np.stack([rng.permutation(m) for _ in range(50)]).astype(np.uint8)
    fa, fb = O.unit_normalize(A, 1), O.unit_normalize(B, 1)
    # |r|^2 of a permutation of 0..m-1 is (m-1) m (2m-1) / 6
    nrm = math.sqrt((m - 1) * m * (2 * m - 1) / 6.0)
    np.testing.assert_allclose(fa, A / nrm, rtol=1e-15, atol=0)
    # the largest scalar product is the nearest neighbour (Section 3.1 e)
    idx, d1, d2 = O.match_nn(A, B, 1)
    dots = fa @ fb.T
    for i in range(len(A)):
        if d1[i] < d2[i]:
            assert int(np.argmax(dots[i])) == idx[i]
    # unused (all-zero) slots stay zero
    assert not O.unit_normalize(np.zeros((2, m), dtype=np.uint8), 1).any()


# -------------------------------------------------------- rotation vector
def test_rotation_vector_matches_scipy():
    rots = Rotation.random(200, random_state=np.random.Generator(np.random.PCG64(3)))
    for R, w in zip(rots.as_matrix(), rots.as_rotvec()):
        got, _ = O.rotation_vector(R)
        np.testing.assert_allclose(got, w, atol=1e-12)


@pytest.mark.parametrize("angle", [0.0, 1e-7, 1e-4, 0.5, 2.0, math.pi - 0.2, math.pi - 1e-3, math.pi - 1e-8])
def test_rotation_vector_small_and_near_pi(angle):
    for axis in ([0.0, 0.0, 1.0], [1.0, -2.0, 0.5], [-0.3, 0.1, -0.9]):
        a = np.array(axis) / np.linalg.norm(axis)
        R = Rotation.from_rotvec(a * angle).as_matrix()
        got, _ = O.rotation_vector(R)
        np.testing.assert_allclose(got, a * angle, atol=1e-7 if angle > 3.1 else 1e-12)


def test_rotation_vector_at_pi_up_to_sign():
    a = np.array([2.0, -1.0, 0.5])
    a /= np.linalg.norm(a)
    R = Rotation.from_rotvec(a * math.pi).as_matrix()
    got, _ = O.rotation_vector(R)
    assert np.allclose(got, a * math.pi, atol=1e-7) or np.allclose(got, -a * math.pi, atol=1e-7)


# ------------------------------------------------------------ similarity fit
def _random_similarity(seed):
    rng = _rng(seed)
    R = Rotation.random(random_state=np.random.Generator(np.random.PCG64(seed))).as_matrix()
    return float(2.0 ** rng.uniform(-1, 1)), R, rng.uniform(-50, 50, 3)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_similarity_fit_exact_recovery(seed):
    s, R, t = _random_similarity(seed)
    xa = _rng(seed + 10).uniform(0, 100, (25, 3))
    xb = s * xa @ R.T + t
    s2, R2, t2 = O.similarity_fit(xa, xb)
    assert abs(s2 - s) <= 1e-12 * s
    np.testing.assert_allclose(R2, R, atol=1e-12)
    np.testing.assert_allclose(t2, t, atol=1e-10)
    assert abs(np.linalg.det(R2) - 1.0) <= 1e-12


def test_similarity_fit_is_least_squares_optimal():
    s, R, t = _random_similarity(4)
    rng = _rng(5)
    xa = rng.uniform(0, 100, (40, 3))
    xb = s * xa @ R.T + t + rng.normal(0, 2.0, (40, 3))
    s2, R2, t2 = O.similarity_fit(xa, xb)

    def sse(s_, R_, t_):
        return float(((s_ * xa @ R_.T + t_ - xb) ** 2).sum())

    base = sse(s2, R2, t2)
    for k in range(200):
        d = rng.normal(0, 1e-3, 7)
        Rp = Rotation.from_rotvec(d[1:4]).as_matrix() @ R2
        assert sse(s2 * (1 + d[0]), Rp, t2 + 10 * d[4:]) >= base - 1e-9 * base


def test_similarity_fit_of_a_mirror_image_is_a_proper_rotation():
    xa = _rng(6).uniform(0, 50, (30, 3))
    xb = xa * np.array([-1.0, 1.0, 1.0])
    _, R2, _ = O.similarity_fit(xa, xb)
    assert abs(np.linalg.det(R2) - 1.0) <= 1e-12


def test_similarity_fit_permutation_invariant():
    s, R, t = _random_similarity(7)
    rng = _rng(8)
    xa = rng.uniform(0, 100, (30, 3))
    xb = s * xa @ R.T + t + rng.normal(0, 1.0, (30, 3))
    p = rng.permutation(30)
    a, b = O.similarity_fit(xa, xb), O.similarity_fit(xa[p], xb[p])
    assert abs(a[0] - b[0]) <= 1e-12 * a[0]
    np.testing.assert_allclose(a[1], b[1], atol=1e-12)
    np.testing.assert_allclose(a[2], b[2], atol=1e-9)


# ------------------------------------------------------------- hypothesis
def test_hypothesis_hand_computed_bins():
    hp = O.HoughParams(scale_bin=1.0, angle_bin=math.pi / 4, trans_bin=10.0, centre=(0.0, 0.0, 0.0))
    Rz = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    ga = O.geometry(np.array([[5.0, 5.0, 5.0, 2.0]]), np.eye(3)[None])[0]
    gb = O.geometry(np.array([[13.0, 2.0, 24.0, 4.0]]), Rz[None])[0]
    lo, s, R, _ = O.hypothesis(ga, gb, hp)
    # s = 2: log2 s = 1 -> bin 1, side -1 -> lo 0; rotation (0, 0, pi/2):
    # q = (0, 0, 2) -> lo (-1, -1, 1); p = x_b + 2 Rz (0 - x_a) = (23, -8, 14):
    # q = (2.3, -0.8, 1.4), bins (2, -1, 1), all on the lower side -> (1, -2, 0)
    assert s == 2.0 and np.array_equal(R, Rz)
    assert lo.tolist() == [0, -1, -1, 1, 1, -2, 0]
    r = O.hough(ga[None], gb[None], np.array([0]), hp)
    assert r["votes"] == 1 and r["bin"] == O.pack_key(lo) and r["status"] == 0


def test_pack_key_order_and_roundtrip():
    rng = _rng(9)
    for _ in range(100):
        c = rng.integers(-256, 256, 7)
        assert O.unpack_key(O.pack_key(c)) == c.tolist()
    assert O.pack_key([-256] * 7) == 0 and O.pack_key([255] * 7) == 2 ** 63 - 1


# ------------------------------------------------------------------ Hough
def _brute_votes(lo, voted):
    """Vote counts by testing, for every bin any match touches, which
    matches' 2^7 cubes contain it."""
    cands = set()
    for i in np.nonzero(voted)[0]:
        for corner in itertools.product((0, 1), repeat=7):
            cands.add(tuple(int(v) for v in lo[i] + np.array(corner)))
    counts = {}
    L = lo[voted]
    for b in cands:
        bb = np.array(b)
        counts[b] = int(np.sum(np.all((L <= bb) & (bb <= L + 1), axis=1)))
    return counts


def test_hough_recovers_planted_similarity_and_true_correspondences():
    ga, gb, m, tr = P.hough_scene(150, 250, seed=11)
    hp = O.hough_default_params((145, 174, 145))
    r = O.hough(ga, gb, m, hp)
    assert r["status"] == 1
    assert abs(math.log2(r["scale"] / tr["s"])) < 0.01
    ang = np.linalg.norm(Rotation.from_matrix(r["R"] @ tr["R"].T).as_rotvec())
    assert ang < math.radians(0.5)
    c = np.asarray(hp.centre)
    assert np.linalg.norm(r["scale"] * r["R"] @ c + r["t"] - (tr["s"] * tr["R"] @ c + tr["t"])) < 0.5
    # every true correspondence is an inlier; an accepted outlier must lie
    # within the inlier distance of the true mapping as well
    assert r["inlier"][:150].all()
    for i in np.nonzero(r["inlier"][150:])[0] + 150:
        xb = gb[m[i], :3]
        assert np.linalg.norm(tr["s"] * tr["R"] @ ga[i, :3] + tr["t"] - xb) <= 2.5 * gb[m[i], 3]
    assert r["n_inliers"] <= 155


def test_hough_votes_equal_brute_force_and_ties_take_the_smallest_key():
    ga, gb, m, _ = P.hough_scene(40, 60, seed=12, angle_deg=80.0)
    hp = O.hough_default_params((145, 174, 145))
    r = O.hough(ga, gb, m, hp)
    counts = _brute_votes(r["lo"], r["voted"])
    best = max(counts.values())
    assert r["votes"] == best
    assert r["bin"] == min(O.pack_key(b) for b, c in counts.items() if c == best)
    # with 2-bin voting a tight cluster fills several bins equally: a tie
    assert sum(1 for c in counts.values() if c == best) >= 2


def test_hough_invariant_to_match_order():
    ga, gb, m, _ = P.hough_scene(60, 90, seed=13)
    hp = O.hough_default_params((145, 174, 145))
    a = O.hough(ga, gb, m, hp)
    rng = _rng(14)
    pa, pb = rng.permutation(len(ga)), rng.permutation(len(gb))
    inv_b = np.argsort(pb)
    b = O.hough(ga[pa], gb[pb], inv_b[m[pa]], hp)
    assert (a["bin"], a["votes"], a["n_inliers"], a["n_fit"]) == (b["bin"], b["votes"], b["n_inliers"], b["n_fit"])
    assert np.array_equal(a["inlier"][pa], b["inlier"])
    assert abs(a["scale"] - b["scale"]) <= 1e-12 * a["scale"]
    np.testing.assert_allclose(a["R"], b["R"], atol=1e-12)


def test_hough_degenerate_inputs():
    hp = O.hough_default_params((64, 64, 64))
    ga, gb, m, _ = P.hough_scene(2, 0, seed=15)
    # fewer than three matches: votes but no transform
    r = O.hough(ga, gb, m, hp)
    assert r["votes"] == 2 and r["status"] == 0 and not r["inlier"].any()
    # no valid match (negative or out-of-range index): no vote at all
    r = O.hough(ga, gb, np.array([-1, 7]), hp)
    assert r["bin"] == -1 and r["votes"] == 0 and r["status"] == 0
    # an empty A
    r = O.hough(ga[:0], gb, m[:0], hp)
    assert r["bin"] == -1 and r["status"] == 0


def test_hough_out_of_range_coordinates_do_not_vote():
    ga, gb, m, _ = P.hough_scene(5, 0, seed=16)
    hp = O.hough_default_params((145, 174, 145))
    hp.trans_bin = 0.01   # predicted centres far beyond 256 bins
    r = O.hough(ga, gb, m, hp)
    assert not r["voted"].any() and r["bin"] == -1


def test_hough_inlier_rule_checks_the_scale_ratio():
    ga, gb, m, tr = P.hough_scene(60, 0, seed=17)
    hp = O.hough_default_params((145, 174, 145))
    # append matches whose B keypoint sits exactly where the true mapping
    # puts A's, with a scale ratio off by 2^1.5 (rejected) or 2^0.25 (kept)
    extra_a, extra_b = ga[:8].copy(), gb[m[:8]].copy()
    extra_b[:, :3] = (tr["s"] * extra_a[:, :3].astype(np.float64) @ tr["R"].T + tr["t"]).astype(np.float32)
    extra_b[:4, 3] = extra_a[:4, 3] * tr["s"] * 2.0 ** 1.5
    extra_b[4:, 3] = extra_a[4:, 3] * tr["s"] * 2.0 ** 0.25
    GA = np.concatenate([ga, extra_a])
    GB = np.concatenate([gb, extra_b])
    M = np.concatenate([m, len(gb) + np.arange(8)]).astype(np.int32)
    r = O.hough(GA, GB, M, hp)
    assert r["status"] == 1
    assert not r["inlier"][60:64].any()
    assert r["inlier"][64:68].all()


def test_hough_refits_on_the_inliers_of_the_previous_round():
    ga, gb, m, _ = P.hough_scene(80, 120, seed=18)
    hp = O.hough_default_params((145, 174, 145))
    hp.iterations = 1
    r1 = O.hough(ga, gb, m, hp)
    assert r1["status"] == 1 and r1["n_fit"] == r1["votes"]
    hp.iterations = 2
    r2 = O.hough(ga, gb, m, hp)
    assert r2["n_fit"] == r1["n_inliers"] and r2["votes"] == r1["votes"]
    idx = np.nonzero(r1["inlier"])[0]
    s, R, t = O.similarity_fit(ga[idx, :3], gb[m[idx], :3])
    assert abs(r2["scale"] - s) <= 1e-12 * s
    np.testing.assert_allclose(r2["R"], R, atol=1e-12)
    # the first round's fit set (the bin's voters) differs from its inliers
    assert r1["n_fit"] != r1["n_inliers"]


def test_similarity_copy_moves_a_blob_where_the_transform_says():
    # generator check: a blob centred at x in A is centred at s R x + t in B
    n = 48
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    c = np.array([30.0, 20.0, 26.0])
    A = np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) / (2 * 3.0 ** 2)).astype(np.float32)
    B, s, R, t = P.similarity_copy(A, scale=1.2, angle_deg=30.0)
    w = B.astype(np.float64)
    m = w > 0.5 * w.max()
    got = np.array([(x * w)[m].sum(), (y * w)[m].sum(), (z * w)[m].sum()]) / w[m].sum()
    assert np.linalg.norm(got - (s * R @ c + t)) < 0.2


def test_hough_ignores_rows_without_a_positive_scale():
    ga, gb, m, _ = P.hough_scene(30, 0, seed=19)
    hp = O.hough_default_params((145, 174, 145))
    ref = O.hough(ga, gb, m, hp)
    ga2 = np.concatenate([ga, ga[:3]])
    ga2[30:, 3] = [0.0, -1.0, np.nan]
    r = O.hough(ga2, gb, np.concatenate([m, m[:3]]), hp)
    assert not r["voted"][30:].any() and not r["inlier"][30:].any()
    assert (r["bin"], r["votes"], r["n_inliers"]) == (ref["bin"], ref["votes"], ref["n_inliers"])


def test_similarity_copy_warp_stays_within_its_amplitude():
    # generator check: with a smooth warp of up to w voxels a blob moves at
    # most about w from where the similarity alone puts it
    n = 48
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    c = np.array([24.0, 22.0, 25.0])
    A = np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) / (2 * 3.0 ** 2)).astype(np.float32)
    B0, s, R, t = P.similarity_copy(A, scale=1.1, angle_deg=10.0)
    Bw, _, _, _ = P.similarity_copy(A, scale=1.1, angle_deg=10.0, warp=2.0, warp_sigma=6.0)
    def centroid(V):
        w = V.astype(np.float64)
        m = w > 0.5 * w.max()
        return np.array([(x * w)[m].sum(), (y * w)[m].sum(), (z * w)[m].sum()]) / w[m].sum()
    assert np.linalg.norm(centroid(B0) - (s * R @ c + t)) < 0.2
    d = np.linalg.norm(centroid(Bw) - centroid(B0))
    assert 0.05 < d < 2.0 * 1.1 * np.sqrt(3)
