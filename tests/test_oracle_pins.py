"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed
form, a brute-force computation written differently, a library routine the
operation reduces to, an invariant, or a planted structure with a known
answer. The tests are chosen so that a plausible slip (a dropped term, a
wrong sign or index, a transposed axis, a wrong source level) fails one.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle as O
from gen import phantoms as P

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def rnd(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


# ------------------------------------------------------------------ P1 taps
@pytest.mark.parametrize("sigma", [0.95, 1.2263, 1.6, 1.9466, 3.09])
def test_taps_sum_symmetry_and_shape(sigma):
    w = O.gauss_taps(sigma, 3.0)
    r = (len(w) - 1) // 2
    assert r == math.ceil(3.0 * sigma)
    assert abs(w.sum() - 1.0) <= 1e-15
    assert np.array_equal(w, w[::-1])
    # ratio to the centre tap is the Gaussian density ratio
    t = np.arange(-r, r + 1)
    np.testing.assert_allclose(w / w[r], np.exp(-t * t / (2 * sigma * sigma)), rtol=1e-14)
    # variance of a +/-3 sigma truncated normal is 0.9733 sigma^2
    var = float((w * t * t).sum())
    assert 0.96 * sigma ** 2 < var < 1.0 * sigma ** 2


def test_zero_sigma_is_identity():
    assert np.array_equal(O.gauss_taps(0.0), np.array([1.0]))
    v = rnd((5, 6, 7), 1)
    assert np.array_equal(O.blur(v, 0.0), v)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_blur_axis_equals_scipy_correlate_nearest(axis):
    v = rnd((9, 11, 13), 2)
    w = O.gauss_taps(1.5)
    ref = ndi.correlate1d(v, w, axis=2 - axis, mode="nearest")
    np.testing.assert_allclose(O.blur_axis(v, w, axis), ref, rtol=0, atol=1e-13)


def test_impulse_response_is_outer_product():
    n = 31
    v = np.zeros((n, n, n))
    v[15, 15, 15] = 1.0
    sigma = 2.0
    w = O.gauss_taps(sigma)
    r = (len(w) - 1) // 2
    out = O.blur(v, sigma)
    ref = np.zeros_like(v)
    ref[15 - r:15 + r + 1, 15 - r:15 + r + 1, 15 - r:15 + r + 1] = w[:, None, None] * w[None, :, None] * w[None, None, :]
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-17)


def test_constant_volume_unchanged_everywhere():
    p = O.Params(n_octaves=3, min_dim=8)
    v = np.full((40, 36, 44), 0.37)
    octs = O.pyramid(v, p)
    assert len(octs) == 3
    for oc in octs:
        for g in oc.G:
            np.testing.assert_allclose(g, 0.37, rtol=0, atol=1e-15)
        for d in oc.D:
            assert np.abs(d).max() <= 1e-15
    assert len(O.detect([oc.D for oc in octs], p)) == 0


# ------------------------------------------------------------------ P2 brute force
def test_separable_equals_bruteforce_3d_convolution():
    v = rnd((16, 16, 16), 3)
    sigma = 1.2263
    w = O.gauss_taps(sigma)
    r = (len(w) - 1) // 2
    n = 16
    idx = np.arange(n)
    ref = np.zeros_like(v)
    for k in range(-r, r + 1):
        zk = np.clip(idx + k, 0, n - 1)
        for j in range(-r, r + 1):
            yj = np.clip(idx + j, 0, n - 1)
            for i in range(-r, r + 1):
                xi = np.clip(idx + i, 0, n - 1)
                ref += w[i + r] * w[j + r] * w[k + r] * v[np.ix_(zk, yj, xi)]
    np.testing.assert_allclose(O.blur(v, sigma), ref, rtol=0, atol=1e-12)


# ------------------------------------------------------------------ P3 sub-sampling
def test_subsample_ramp_constant_and_odd_dims():
    nz, ny, nx = 9, 8, 11
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ramp = 3.0 * x - 2.0 * y + 0.5 * z + 1.0
    out = O.subsample(ramp)
    assert out.shape == (4, 4, 5)
    Z, Y, X = np.meshgrid(np.arange(4), np.arange(4), np.arange(5), indexing="ij")
    np.testing.assert_array_equal(out, 3.0 * (2 * X + 0.5) - 2.0 * (2 * Y + 0.5) + 0.5 * (2 * Z + 0.5) + 1.0)
    np.testing.assert_array_equal(O.subsample(np.full((5, 5, 5), 2.5)), np.full((2, 2, 2), 2.5))
    v = rnd((8, 6, 10), 4)
    ref = v.reshape(4, 2, 3, 2, 5, 2).mean(axis=(1, 3, 5))
    np.testing.assert_allclose(O.subsample(v), ref, rtol=0, atol=1e-15)
    assert GOLD["subsample_inputs_per_output"]["value"] == 8


# ------------------------------------------------------------------ P4 sum of signs
def _brute_extremum(dm, d0, dp, x, y, z):
    v = d0[z, y, x]
    nb = np.concatenate([dm[z - 1:z + 2, y - 1:y + 2, x - 1:x + 2].ravel(),
                         np.delete(d0[z - 1:z + 2, y - 1:y + 2, x - 1:x + 2].ravel(), 13),
                         dp[z - 1:z + 2, y - 1:y + 2, x - 1:x + 2].ravel()])
    assert len(nb) == GOLD["neighbours_per_extremum_test"]["value"]
    return bool(np.all(v > nb)), bool(np.all(v < nb)), int(np.sign(v - nb).sum())


def test_sum_of_signs_matches_bruteforce_with_ties():
    rng = np.random.default_rng(5)
    for trial in range(6):
        # quantised values make ties common
        dm, d0, dp = (np.round(rng.standard_normal((6, 7, 8)) * (2 if trial % 2 else 50)) for _ in range(3))
        # plant one strict maximum and one tied maximum
        d0[2, 3, 3] = 1000.0
        d0[3, 3, 5] = 1000.0
        dm[3, 3, 5] = 1000.0  # tie with the neighbour below: not strict
        rows = O.detect_triple(dm, d0, dp, 0.0, 80)
        got = {(int(r[0]), int(r[1]), int(r[2])): int(r[3]) for r in rows}
        want = {}
        for z in range(1, 5):
            for y in range(1, 6):
                for x in range(1, 7):
                    mx, mn, f = _brute_extremum(dm, d0, dp, x, y, z)
                    assert O.sum_of_signs(dm, d0, dp, x, y, z) == f
                    assert (f == GOLD["peak_sum_of_signs"]["value"]) == mx
                    assert (f == GOLD["valley_sum_of_signs"]["value"]) == mn
                    if (mx or mn) and abs(d0[z, y, x]) > 0.0:
                        want[(x, y, z)] = 1 if mx else -1
        assert got == want
        assert got.get((3, 3, 2)) == 1
        assert (5, 3, 3) not in got


def test_relaxed_votes_and_threshold():
    rng = np.random.default_rng(6)
    dm, d0, dp = (rng.standard_normal((7, 7, 7)) for _ in range(3))
    for votes in (60, 78):
        rows = O.detect_triple(dm, d0, dp, 0.5, votes)
        got = {(int(r[0]), int(r[1]), int(r[2])) for r in rows}
        want = set()
        for z in range(1, 6):
            for y in range(1, 6):
                for x in range(1, 6):
                    _, _, f = _brute_extremum(dm, d0, dp, x, y, z)
                    if abs(d0[z, y, x]) > 0.5 and abs(f) >= votes:
                        want.add((x, y, z))
        assert got == want


# ------------------------------------------------------------------ schedule
def test_level_schedule_closed_form():
    p = O.Params()
    base, inc = O.level_increments(p)
    assert base == pytest.approx(1.6)
    assert len(inc) == p.scales + 2
    tot = base ** 2
    for i, s in enumerate(inc, start=1):
        tot += s * s
        assert math.sqrt(tot) == pytest.approx(1.6 * 2 ** (i / 3), rel=1e-14)
    # tap radii of the hot path: 5 for the base blur, then 4, 5, 6, 8, 10
    assert [math.ceil(3 * s) for s in [base] + inc] == [5, 4, 5, 6, 8, 10]
    assert [O.siftrank_radius(p, s) for s in (1, 2, 3)] == [5, 6, 7]


def test_octave_dims():
    p = O.Params()
    assert O.octave_dims((145, 174, 145), p) == [(145, 174, 145), (72, 87, 72), (36, 43, 36), (18, 21, 18)]
    assert O.octave_dims((64, 64, 64), O.Params(n_octaves=2)) == [(64, 64, 64), (32, 32, 32)]
    assert len(O.octave_dims((512, 512, 384), p)) == 5
    assert O.octave_dims((15, 40, 40), p) == []


# ------------------------------------------------------------------ P5 planted blobs
def _blob(n, c, s, a=1.0):
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return a * np.exp(-((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2) / (2 * s * s))


@pytest.mark.parametrize("sb,o,s", [(2.8, 0, 1), (3.5, 0, 2), (4.4, 0, 3), (5.5, 1, 1), (7.0, 1, 2), (8.8, 1, 3)])
@pytest.mark.parametrize("amp", [1.0, -0.5])
def test_planted_blob_recovered_at_centre_and_scale(sb, o, s, amp):
    # the continuous DoG maximiser of a Gaussian blob is sigma* = 0.7267 sigma_b
    # for kappa = 2^(1/3); sigma_b in the interior of a scale bin picks that bin.
    p = O.Params(n_octaves=2, min_dim=8)
    n = 96 if o == 1 else 64
    c = (n // 2) * 1.0 + (0.5 if o == 1 else 0.0)   # a voxel centre of octave o
    v = _blob(n, c, sb, amp)
    octs = O.pyramid(v, p)
    k = O.detect([oc.D for oc in octs], p)
    hit = k[(np.abs(k["xf"] - c) < 1) & (np.abs(k["yf"] - c) < 1) & (np.abs(k["zf"] - c) < 1)]
    assert len(hit) == 1
    h = hit[0]
    assert (int(h["octave"]), int(h["scale"])) == (o, s)
    assert int(h["polarity"]) == (1 if amp > 0 else -1)
    assert abs(float(h["dog"])) == pytest.approx(0.127 * abs(amp), rel=0.03)
    assert float(h["sigma"]) / sb == pytest.approx(0.7267, rel=0.2)


def test_blob_below_smallest_detectable_scale_not_found():
    p = O.Params(n_octaves=2, min_dim=8)
    octs = O.pyramid(_blob(64, 32.0, 2.0), p)
    k = O.detect([oc.D for oc in octs], p)
    assert not np.any((k["x"] == 32) & (k["y"] == 32) & (k["z"] == 32) & (k["octave"] == 0))


# ------------------------------------------------------------------ descriptors, closed forms
def _ramp(n, axis, a=1.0):
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return a * (x, y, z)[axis].astype(np.float64)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("a", [0.7, -1.3])
def test_siftrank_histogram_of_a_ramp(axis, a):
    R = 5
    G = _ramp(24, axis, a)
    hist, rk = O.siftrank(G, np.array([[12, 12, 12]]), R)
    bo = (1 << axis) if a > 0 else 0
    want = np.zeros(64)
    for bs in range(8):
        want[8 * bs + bo] = abs(a) * (R + 0.5) ** 3
    np.testing.assert_allclose(hist[0], want, rtol=1e-13, atol=1e-12)
    assert sorted(rk[0].tolist()) == list(range(64))


def test_siftrank_spatial_bins_of_abs_profile():
    # G = |x - 12|: gradient -1 on the left (bin 0), +1 on the right (bin 1),
    # 0 on the centre plane; left samples land in spatial bx = 0, right in bx = 1
    n, R = 24, 4
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    G = np.abs(x - 12.0)
    hist, _ = O.siftrank(G, np.array([[12, 12, 12]]), R)
    want = np.zeros(64)
    half = (R + 0.5) ** 2 * R  # R planes per side, (R+0.5)^2 weight per plane per (by, bz) half
    for by in range(2):
        for bz in range(2):
            want[8 * (0 + 2 * by + 4 * bz) + 0] = half
            want[8 * (1 + 2 * by + 4 * bz) + 1] = half
    np.testing.assert_allclose(hist[0], want, rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_brief_on_a_ramp_is_offset_difference(axis):
    # a Gaussian blur leaves a linear function unchanged away from the edges,
    # so d_i = B(p1) - B(p2) = a (o1 - o2) along the ramp axis
    G = _ramp(40, axis, 0.5)
    draws = P.pair_draws(1, 256)
    p = O.Params()
    off = O.pair_offsets(draws, p, 1)
    assert np.abs(off).max() <= 12
    wb = O.gauss_taps(0.95)
    d, bits, rk = O.brief_rrief(G, np.array([[20, 20, 20]]), off, wb)
    want = 0.5 * (off[:, 0, axis] - off[:, 1, axis]).astype(np.float64)
    np.testing.assert_allclose(d[0], want, rtol=0, atol=1e-12)
    for i in range(256):
        assert bool((int(bits[0, i // 64]) >> (i % 64)) & 1) == (want[i] > 0)
    assert sorted(rk[0].tolist()) == list(range(256))


def test_brief_special_cases():
    G = rnd((20, 20, 20), 7)
    off = np.zeros((64, 2, 3), dtype=np.int32)
    off[:, 0] = np.random.default_rng(8).integers(-4, 5, (64, 3))
    off[:, 1] = off[:, 0]
    d, bits, rk = O.brief_rrief(G, np.array([[10, 10, 10]]), off, O.gauss_taps(0.95))
    assert np.all(d == 0.0) and np.all(bits == 0)
    assert rk[0].tolist() == list(range(64))     # ties broken by index
    # sigma_b = 0: B(p) is the sample itself
    off2 = np.array([[[1, 0, 0], [0, -2, 3]]], dtype=np.int32)
    d2, _, _ = O.brief_rrief(G, np.array([[10, 10, 10]]), off2, np.array([1.0]))
    assert d2[0, 0] == G[10, 10, 11] - G[13, 8, 10]
    # sample points clamp at the volume edge
    d3, _, _ = O.brief_rrief(G, np.array([[0, 19, 1]]), np.array([[[-5, 4, 0], [0, 0, -9]]], dtype=np.int32),
                             np.array([1.0]))
    assert d3[0, 0] == G[1, 19, 0] - G[0, 19, 0]


def test_pair_offsets_follow_method_3():
    # p1 ~ N(0, sigma), p2 ~ N(p1, sigma): var(p1) = sigma^2, var(p2) = 2 sigma^2,
    # corr(p1, p2) = 1/sqrt(2); a method-2 slip (independent p2) gives corr 0
    p = O.Params(brief_n=60000)
    draws = P.pair_draws(99, 60000)
    off = O.pair_offsets(draws, p, 3).astype(np.float64)
    sig = O.scale_sigma(p, 3)
    assert sig == pytest.approx(3.2)
    a, b = off[:, 0].ravel(), off[:, 1].ravel()
    assert np.var(a) / sig ** 2 == pytest.approx(1.0 + 1.0 / (12 * sig ** 2), rel=0.03)
    assert np.var(b) / sig ** 2 == pytest.approx(2.0 + 1.0 / (12 * sig ** 2), rel=0.03)
    assert np.corrcoef(a, b)[0, 1] == pytest.approx(1 / math.sqrt(2), abs=0.01)
    assert abs(a.mean()) < 0.05 and abs(b.mean()) < 0.05
    assert np.all(off == np.floor(off))


def _pairs(method, n, seed=98):
    p = O.Params(brief_n=n, brief_method=method)
    return p, O.pair_points(P.pair_draws(seed, n), p, 3), O.scale_sigma(p, 3)


def test_pair_points_method_1_uniform_in_ball():
    # uniform in the ball of radius a = 2 sigma: (|p|/a)^3 ~ U(0,1), so its mean
    # is 1/2 and variance 1/12; E[x^2] = a^2/5 per axis; p1 and p2 independent
    p, pts, sig = _pairs(1, 60000)
    a = 2.0 * sig
    for w in (0, 1):
        q = pts[:, w]
        r = np.sqrt((q * q).sum(axis=1))
        assert r.max() <= a * (1 + 1e-12)
        u = (r / a) ** 3
        assert u.mean() == pytest.approx(0.5, abs=0.005)
        assert u.var() == pytest.approx(1.0 / 12.0, abs=0.003)
        assert (q[:, 2] ** 2).mean() / a ** 2 == pytest.approx(0.2, rel=0.03)
        assert np.abs(q.mean(axis=0)).max() < 0.03 * a
    assert abs(np.corrcoef(pts[:, 0, 0], pts[:, 1, 0])[0, 1]) < 0.02
    assert abs(np.corrcoef(np.abs(pts[:, 0]).sum(1), np.abs(pts[:, 1]).sum(1))[0, 1]) < 0.02


def test_pair_points_method_2_independent_normals():
    p, pts, sig = _pairs(2, 60000)
    a, b = pts[:, 0].ravel(), pts[:, 1].ravel()
    assert np.var(a) / sig ** 2 == pytest.approx(1.0, rel=0.03)
    assert np.var(b) / sig ** 2 == pytest.approx(1.0, rel=0.03)
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.02


def test_pair_points_method_4_centre_and_normal():
    p, pts, sig = _pairs(4, 60000)
    assert np.all(pts[:, 0] == 0.0)
    b = pts[:, 1].ravel()
    assert np.var(b) / sig ** 2 == pytest.approx(1.0, rel=0.03)
    assert abs(b.mean()) < 0.03 * sig


def test_pair_points_method_5_spherical_grid():
    # p1 at the centre; p2 on n/64 shells of radius 2 sigma (k+1)/(n/64), 64 points
    # per shell symmetric about the centre (zero mean), no two points equal
    for n in (64, 256):
        p, pts, sig = _pairs(5, n)
        assert np.all(pts[:, 0] == 0.0)
        q = pts[:, 1]
        r = np.sqrt((q * q).sum(axis=1))
        nr = n // 64
        for k in range(nr):
            shell = q[64 * k:64 * (k + 1)]
            assert np.allclose(r[64 * k:64 * (k + 1)], 2.0 * sig * (k + 1) / nr, rtol=1e-12)
            assert np.abs(shell.mean(axis=0)).max() < 1e-12 * sig
        assert len({tuple(np.round(v, 9)) for v in q}) == n


def test_pair_offsets_round_the_points():
    for m in range(1, 6):
        p = O.Params(brief_method=m)
        draws = P.pair_draws(4, 256)
        assert np.array_equal(O.pair_offsets(draws, p, 2), np.floor(O.pair_points(draws, p, 2) + 0.5))


def test_rank_is_stable_permutation():
    v = np.array([3.0, 1.0, 3.0, -2.0, 1.0])
    assert O.rank(v).tolist() == [3, 1, 4, 0, 2]
    assert GOLD["siftrank_length"]["value"] == 2 * 2 * 2 * GOLD["siftrank_orientation_bins"]["value"]
    assert 64 <= 2 ** GOLD["siftrank_bits_per_element"]["value"]


# ------------------------------------------------------------------ P6-P10 invariants
@pytest.fixture(scope="module")
def small_case():
    p = O.Params(n_octaves=2, min_dim=8)
    v = P.noise_blob_volume((48, 40, 44), 11, n_blobs=14, margin=8).astype(np.float64)
    draws = P.pair_draws(5, 256)
    octs, k, desc = O.extract(v, p, draws)
    assert len(k) > 10
    return p, v, draws, octs, k, desc


def _key(k):
    return [(int(r["octave"]), int(r["scale"]), int(r["z"]), int(r["y"]), int(r["x"])) for r in k]


def test_canonical_order_and_ranks_are_permutations(small_case):
    p, v, draws, octs, k, desc = small_case
    keys = _key(k)
    assert keys == sorted(keys)
    assert np.all(np.sort(desc["siftrank"], axis=1) == np.arange(64))
    assert np.all(np.sort(desc["rrief"].astype(int), axis=1) == np.arange(256))


def test_offset_invariance(small_case):
    p, v, draws, octs, k, desc = small_case
    _, k2, d2 = O.extract(v + 0.25, p, draws)
    assert _key(k2) == _key(k)
    assert np.array_equal(d2["siftrank"], desc["siftrank"])
    np.testing.assert_allclose(d2["diff"], desc["diff"], rtol=0, atol=1e-12)


def test_scaling_invariance(small_case):
    p, v, draws, octs, k, desc = small_case
    p2 = O.Params(**{**p.__dict__, "dog_threshold": 2 * p.dog_threshold})
    _, k2, d2 = O.extract(2.0 * v, p2, draws)
    assert _key(k2) == _key(k)
    for f in ("siftrank", "brief", "rrief"):
        assert np.array_equal(d2[f], desc[f])


def test_negation_swaps_peaks_and_valleys(small_case):
    p, v, draws, octs, k, desc = small_case
    _, k2, d2 = O.extract(-v, p, draws)
    assert _key(k2) == _key(k)
    assert np.array_equal(k2["polarity"], -k["polarity"])
    assert np.array_equal(d2["diff"], -desc["diff"])
    nz = desc["diff"] != 0
    for kk in range(len(k)):
        for i in range(256):
            b1 = (int(desc["brief"][kk, i // 64]) >> (i % 64)) & 1
            b2 = (int(d2["brief"][kk, i // 64]) >> (i % 64)) & 1
            if nz[kk, i]:
                assert b1 != b2
    dd = desc["diff"]
    untied = np.array([len(np.unique(row)) == len(row) for row in dd])
    assert np.array_equal(d2["rrief"][untied].astype(int), 255 - desc["rrief"][untied].astype(int))
    # SIFT-Rank: orientation bin bo -> 7 - bo for every non-zero gradient component
    perm = np.array([8 * (e // 8) + 7 - (e % 8) for e in range(64)])
    np.testing.assert_allclose(d2["hist"], desc["hist"][:, perm], rtol=1e-12, atol=1e-14)


def test_x_mirror(small_case):
    p, v, draws, octs, k, desc = small_case
    assert v.shape[2] % 4 == 0
    _, k2, d2 = O.extract(v[:, :, ::-1].copy(), p, draws)
    m = {}
    for i, r in enumerate(k2):
        nx_o = v.shape[2] >> int(r["octave"])
        m[(int(r["octave"]), int(r["scale"]), int(r["z"]), int(r["y"]), nx_o - 1 - int(r["x"]))] = i
    keys = _key(k)
    assert set(m) == set(keys)
    # spatial bx flips and orientation bit 0 flips
    perm = np.array([8 * ((e // 8) ^ 1) + ((e % 8) ^ 1) for e in range(64)])
    for i, key in enumerate(keys):
        np.testing.assert_allclose(d2["hist"][m[key]], desc["hist"][i][perm], rtol=1e-11, atol=1e-13)


# ------------------------------------------------------------------ matching (descriptor consumer)
def test_match_nn_hand_values():
    # Hamming on one word: A = 1011b against B = {0001b, 1111b, 1011b, 0011b}:
    # distances 2, 1, 0, 1 -> nearest 2 at 0, second-smallest 1
    A = np.array([[0b1011]], dtype=np.uint64)
    B = np.array([[0b0001], [0b1111], [0b1011], [0b0011]], dtype=np.uint64)
    idx, d1, d2 = O.match_nn(A, B, 0)
    assert (idx[0], d1[0], d2[0]) == (2, 0, 1)
    # squared distance of rank vectors: (0,1,2,3) vs (1,0,2,3) -> 2, vs (3,2,1,0) -> 20,
    # vs (0,1,2,3) -> 0 at index 2 and again at index 3 (the lower index wins, d2 = 0)
    A = np.array([[0, 1, 2, 3]], dtype=np.uint8)
    B = np.array([[1, 0, 2, 3], [3, 2, 1, 0], [0, 1, 2, 3], [0, 1, 2, 3]], dtype=np.uint8)
    idx, d1, d2 = O.match_nn(A, B, 1)
    assert (idx[0], d1[0], d2[0]) == (2, 0, 0)
    idx, d1, d2 = O.match_nn(A, B[:2], 1)
    assert (idx[0], d1[0], d2[0]) == (0, 2, 20)


def test_match_nn_edge_cases_and_self_match():
    big = 2 ** 31 - 1
    A = np.array([[5, 6, 7, 8]], dtype=np.uint8)
    idx, d1, d2 = O.match_nn(A, A[:0], 1)
    assert (idx[0], d1[0], d2[0]) == (-1, big, big)
    idx, d1, d2 = O.match_nn(A, A, 1)
    assert (idx[0], d1[0], d2[0]) == (0, 0, big)
    # distinct permutations matched against themselves: each finds itself at 0;
    # against a shuffled copy: the shuffle's inverse
    rng = np.random.default_rng(7)
    R = np.array([rng.permutation(64) for _ in range(40)], dtype=np.uint8)
    idx, d1, _ = O.match_nn(R, R, 1)
    assert np.array_equal(idx, np.arange(40)) and np.all(d1 == 0)
    perm = rng.permutation(40)
    idx, _, _ = O.match_nn(R, R[perm], 1)
    assert np.array_equal(perm[idx], np.arange(40))


# ------------------------------------------- uniform-filter approximation


def test_box_axis_hand_values():
    # [1, 2, 4] with h = 1, edges clamped: (1+1+2)/3, (1+2+4)/3, (2+4+4)/3
    v = np.array([1.0, 2.0, 4.0]).reshape(1, 1, 3)
    assert np.allclose(O.box_axis(v, 1, 0).ravel(), [4 / 3, 7 / 3, 10 / 3], rtol=0, atol=1e-15)
    # the same line along z and along y
    assert np.allclose(O.box_axis(v.reshape(3, 1, 1), 1, 2).ravel(), [4 / 3, 7 / 3, 10 / 3], rtol=0, atol=1e-15)
    assert np.allclose(O.box_axis(v.reshape(1, 3, 1), 1, 1).ravel(), [4 / 3, 7 / 3, 10 / 3], rtol=0, atol=1e-15)
    # h = 0 is the identity
    x = rnd((4, 5, 6), 1)
    assert np.array_equal(O.box_blur(x, 0, 3), x)


def test_box_blur_equals_scipy_uniform_filter():
    # scipy's uniform filter with mode 'nearest' is the clamp-to-edge mean;
    # ragged dims, one of them shorter than the filter
    x = rnd((5, 9, 13), 2)
    for h, m in ((1, 1), (2, 3), (4, 2), (3, 4)):
        ref = x.copy()
        for ax in (2, 1, 0):   # x, y, z of a [z,y,x] array
            for _ in range(m):
                ref = ndi.uniform_filter1d(ref, 2 * h + 1, axis=ax, mode="nearest")
        assert np.allclose(O.box_blur(x, h, m), ref, rtol=0, atol=1e-12), (h, m)


def test_box_impulse_response_and_moments():
    # an interior impulse gives the separable product of the m-fold
    # self-convolution of the uniform kernel, with mass 1 and per-axis
    # variance m h (h + 1) / 3 (the uniform law's variance (w^2 - 1)/12, m times)
    h, m, n = 2, 3, 41
    v = np.zeros((n, n, n))
    c = n // 2
    v[c, c, c] = 1.0
    out = O.box_blur(v, h, m)
    k = np.ones(2 * h + 1) / (2 * h + 1)
    p1 = np.array([1.0])
    for _ in range(m):
        p1 = np.convolve(p1, k)
    prof = np.zeros(n)
    prof[c - m * h:c + m * h + 1] = p1
    assert np.allclose(out, prof[:, None, None] * prof[None, :, None] * prof[None, None, :], rtol=0, atol=1e-15)
    assert abs(out.sum() - 1.0) < 1e-12
    idx = np.arange(n) - c
    for ax in range(3):
        marg = out.sum(axis=tuple(a for a in range(3) if a != ax))
        assert abs((marg * idx).sum()) < 1e-12
        assert abs((marg * idx * idx).sum() - m * h * (h + 1) / 3) < 1e-12


def test_box_half_width_values():
    # ideal width sqrt(12 sigma^2 / m + 1), h = round((width - 1) / 2)
    assert O.box_half_width(2.0, 1) == 3      # width 7 exactly: variance (49 - 1)/12 = 4
    assert O.box_half_width(1.6, 3) == 1      # sqrt(11.24) = 3.353 -> 1.18
    assert O.box_half_width(3.09, 3) == 3     # sqrt(39.19) = 6.260 -> 2.63
    assert O.box_half_width(0.0, 3) == 0
    # constants and linear ramps pass through the interior unchanged
    ramp = np.broadcast_to(np.arange(30.0)[None, None, :], (3, 4, 30)).copy()
    out = O.box_blur(ramp, 2, 3)
    assert np.allclose(out[:, :, 6:24], ramp[:, :, 6:24], rtol=0, atol=1e-12)
    assert np.allclose(O.box_blur(np.full((6, 7, 8), 2.5), 3, 2), 2.5, rtol=0, atol=1e-14)


# ------------------------------------------------------------------ describe() and detect() wiring
# The pins above call the descriptor primitives directly. These go through
# describe() and detect(), so that the choice of level (G_s of octave o),
# SIFT-Rank half-width (R_s) and pair table (scale s), the pre-blur taps and
# the input-space position are each fixed by a value a slip would change.

def _sigma_s(s):
    # keypoint scale of level s in its octave's voxels: sigma0 * 2^(s/S)
    return 1.6 * 2.0 ** (s / 3.0)


def _levels(n_oct, make):
    """G_levels[o][i] = make(o, i) for i = 0..S+2."""
    return [[make(o, i) for i in range(6)] for o in range(n_oct)]


def _kps(rows):
    k = np.zeros(len(rows), dtype=O.KEYPOINT_DTYPE)
    for j, (o, s, x, y, z) in enumerate(rows):
        k[j]["octave"], k[j]["scale"], k[j]["x"], k[j]["y"], k[j]["z"] = o, s, x, y, z
    return k


def test_describe_takes_level_radius_and_pair_scale_of_each_keypoint():
    # Every level G_i of octave o is a ramp along x with its own slope a(o, i).
    # On a ramp (away from the edges) SIFT-Rank puts |a| (R + 1/2)^3 into the
    # +x (or -x) orientation bin of each spatial bin, with R the half-width of
    # the keypoint's scale: 5, 6, 7 for s = 1, 2, 3 (ceil(2 sigma_s)). The
    # pre-blur leaves a ramp unchanged, so BRIEF gives d_i = a (o1 - o2)_x with
    # the offsets of the keypoint's own scale. A wrong level, octave, radius
    # or pair table changes one of these numbers.
    n = 80
    slope = {(o, i): (0.3 + 0.1 * i + 0.05 * o) * (-1.0) ** i for o in range(2) for i in range(6)}
    G = _levels(2, lambda o, i: _ramp(n, 0, slope[(o, i)]))
    rows = [(o, s, 40, 40, 40) for o in range(2) for s in (1, 2, 3)]
    kps = _kps(rows)
    draws = P.pair_draws(1, 256)
    p = O.Params()
    out = O.describe(G, kps, draws, p)
    z = draws.reshape(-1, 2, 3)
    for j, (o, s, _, _, _) in enumerate(rows):
        a = slope[(o, s)]
        R = {1: 5, 2: 6, 3: 7}[s]
        assert R == math.ceil(2.0 * _sigma_s(s))
        bo = 1 if a > 0 else 0
        want = np.zeros(64)
        for bs in range(8):
            want[8 * bs + bo] = abs(a) * (R + 0.5) ** 3
        np.testing.assert_allclose(out["hist"][j], want, rtol=1e-13, atol=1e-12)
        # method 3 at this scale: o1 = round(sigma_s z1), o2 = round(sigma_s (z1 + z2))
        o1 = np.floor(_sigma_s(s) * z[:, 0, 0] + 0.5)
        o2 = np.floor(_sigma_s(s) * (z[:, 0, 0] + z[:, 1, 0]) + 0.5)
        assert max(np.abs(o1).max(), np.abs(o2).max()) + 3 < 40
        np.testing.assert_allclose(out["diff"][j], a * (o1 - o2), rtol=0, atol=1e-12)


def _draws_for_offsets(o1, o2, s):
    """Method-3 draws (z1, z2) whose scale-s offsets are exactly o1 and o2."""
    sig = _sigma_s(s)
    z1 = np.asarray(o1, dtype=np.float64) / sig
    z2 = (np.asarray(o2, dtype=np.float64) - np.asarray(o1, dtype=np.float64)) / sig
    return np.stack([z1, z2], axis=1)


def test_describe_preblur_weights_from_an_impulse():
    # G_s holds one impulse of height A(o, s) at the keypoint. Pair i has p1 at
    # offset (a, b, c) from it, |a|, |b|, |c| <= 3 = ceil(3 * 0.95), and p2 far
    # away, so d_i = B(p1) = A(o, s) w_a w_b w_c with w the pre-blur taps of
    # sigma_b = 0.95 (exp(-t^2 / (2 sigma_b^2)) normalised over t = -3..3).
    # Unequal (a, b, c) catch a stencil that reuses one axis's index; a wrong
    # sigma_b, level or octave changes every d_i.
    n, c0 = 48, 24
    rng = np.random.default_rng(11)
    o1 = rng.integers(-3, 4, (64, 3))
    o1[:8] = [[1, 2, 3], [-3, 0, 2], [0, 0, 0], [3, 3, 3], [-1, -2, 0], [2, -3, 1], [0, 1, -2], [-3, -3, 3]]
    o2 = np.tile([[15, -15, 15]], (64, 1))
    amp = {(o, i): 1.0 + 0.25 * i + 2.0 * o for o in range(2) for i in range(6)}

    def impulse(o, i):
        g = np.zeros((n, n, n))
        g[c0, c0, c0] = amp[(o, i)]
        return g

    G = _levels(2, impulse)
    t = np.arange(-3, 4)
    w = np.exp(-t * t / (2 * 0.95 ** 2))
    w /= w.sum()
    p = O.Params(brief_n=64)
    for o in range(2):
        for s in (1, 2, 3):
            draws = _draws_for_offsets(o1, o2, s)
            np.testing.assert_array_equal(O.pair_offsets(draws, p, s)[:, 0], o1)
            out = O.describe(G, _kps([(o, s, c0, c0, c0)]), draws, p)
            want = amp[(o, s)] * w[3 - o1[:, 0]] * w[3 - o1[:, 1]] * w[3 - o1[:, 2]]
            np.testing.assert_allclose(out["diff"][0], want, rtol=1e-13, atol=0)
            assert np.all(out["diff"][0] > 0)


@pytest.mark.parametrize("sb,o,s", [(3.5, 0, 2), (5.5, 1, 1), (7.0, 1, 2)])
def test_detect_input_space_position_and_sigma_exact(sb, o, s):
    # A blob centred on a voxel centre of octave o is found at that voxel; its
    # input-space position is 2^o x + (2^o - 1)/2, the centre of the 2^o-wide
    # block of input voxels the octave voxel averages, which is the blob centre
    # itself. sigma = sigma0 2^(s/S) 2^o.
    p = O.Params(n_octaves=2, min_dim=8)
    n = 96 if o == 1 else 64
    c = (n // 2) * 1.0 + (0.5 if o == 1 else 0.0)
    octs = O.pyramid(_blob(n, c, sb), p)
    k = O.detect([oc.D for oc in octs], p)
    hit = k[(k["octave"] == o) & (k["scale"] == s) & (np.abs(k["xf"] - c) < 1.5)
            & (np.abs(k["yf"] - c) < 1.5) & (np.abs(k["zf"] - c) < 1.5)]
    assert len(hit) == 1
    h = hit[0]
    assert (float(h["xf"]), float(h["yf"]), float(h["zf"])) == (c, c, c)
    assert int(h["x"]) * 2 ** o + (2 ** o - 1) / 2 == c
    assert float(h["sigma"]) == pytest.approx(_sigma_s(s) * 2 ** o, rel=1e-7)


# ------------------------------------------------------------------ orientation (reading R25)
def _cube_rotations():
    """The 24 proper signed permutation matrices (rotations of the cube)."""
    import itertools
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            Q = np.zeros((3, 3))
            for i, j in enumerate(perm):
                Q[i, j] = signs[i]
            if round(np.linalg.det(Q)) == 1:
                out.append(Q)
    return out


def _rotate_volume(V, Q):
    """V'(Q x) = V(x) about the centre voxel of a cubic volume of odd side;
    volumes are [z, y, x], Q acts on (x, y, z)."""
    n = V.shape[0]
    c = (n - 1) // 2
    idx = np.indices((n, n, n)).reshape(3, -1)          # (z, y, x) of each output voxel
    xyz = idx[::-1] - c                                  # (x, y, z) relative to the centre
    src = (Q.T @ xyz).round().astype(int) + c            # x = Q^T x'
    return V[src[2], src[1], src[0]].reshape(V.shape)


def _smooth_cube(n, seed):
    v = ndi.gaussian_filter(rnd((n, n, n), seed), 2.0, mode="wrap")
    return v / np.abs(v).max()


def test_orientation_identity_frame_is_the_upright_descriptor():
    G = _smooth_cube(21, 40)
    kp = np.array([[10, 10, 10], [3, 17, 8], [0, 0, 20]])
    for R in (5, 6, 7):
        h0, r0 = O.siftrank(G, kp, R)
        h1, r1, _ = O.siftrank_frames(G, kp, R, np.repeat(np.eye(3)[None], len(kp), axis=0))
        assert np.array_equal(h0, h1) and np.array_equal(r0, r1), R


def test_orientation_covariant_under_the_24_cube_rotations():
    """Rotating the volume about the keypoint by a rotation of the cube
    rotates every frame by it and leaves every oriented descriptor
    unchanged (the 26 directions and their neighbour relation are closed
    under these rotations; sums differ only in rounding order)."""
    n, R = 25, 6
    c = (n - 1) // 2
    G = _smooth_cube(n, 41)
    kp = np.array([[c, c, c]])
    ref = O.orient(G, kp, R)
    assert ref["margin"][0] > 1e-9 and ref["nframes"][0] >= 1
    nf = ref["nframes"][0]
    for Q in _cube_rotations():
        got = O.orient(_rotate_volume(G, Q), kp, R)
        assert got["nframes"][0] == nf
        for f in range(nf):
            np.testing.assert_allclose(got["frames"][0, f], Q @ ref["frames"][0, f], atol=1e-12)
            assert np.array_equal(got["rank"][0, f], ref["rank"][0, f])
            np.testing.assert_allclose(got["hist"][0, f], ref["hist"][0, f], rtol=1e-12, atol=0)


def test_orientation_of_an_axis_aligned_anisotropic_blob():
    """A Gaussian blob whose axes are the grid axes, shortest along x and
    longest along z: the gradient histogram peaks at +-x (equal heights by
    symmetry), the secondary at +-y, so the four frames are (+-x, +-y)."""
    n = 31
    c = (n - 1) // 2
    z, y, x = np.indices((n, n, n)) - c
    G = np.exp(-(x ** 2 / (2 * 2.0 ** 2) + y ** 2 / (2 * 3.5 ** 2) + z ** 2 / (2 * 5.0 ** 2)))
    r = O.orient(G, np.array([[c, c, c]]), 7)
    assert r["nframes"][0] == 4
    e1 = sorted(tuple(np.round(r["frames"][0, f][:, 0], 9)) for f in range(4))
    e2 = sorted(tuple(np.round(r["frames"][0, f][:, 1], 9)) for f in range(4))
    assert e1 == sorted([(-1.0, 0.0, 0.0)] * 2 + [(1.0, 0.0, 0.0)] * 2)
    assert e2 == sorted([(0.0, -1.0, 0.0), (0.0, 1.0, 0.0)] * 2)
    for f in range(4):
        F = r["frames"][0, f]
        np.testing.assert_allclose(F.T @ F, np.eye(3), atol=1e-12)
        assert abs(np.linalg.det(F) - 1.0) < 1e-12


def test_orientation_of_a_rotated_anisotropic_blob():
    """A strongly anisotropic blob rotated by a generic rotation: the
    primary axis is its short axis (up to sign) and the secondary its middle
    axis, within the bin's averaging error."""
    n = 41
    c = (n - 1) // 2
    a, b, g = 0.4, 0.7, 1.1                                # Euler angles
    Rz = lambda t: np.array([[np.cos(t), -np.sin(t), 0], [np.sin(t), np.cos(t), 0], [0, 0, 1]])
    Ry = lambda t: np.array([[np.cos(t), 0, np.sin(t)], [0, 1, 0], [-np.sin(t), 0, np.cos(t)]])
    Q0 = Rz(a) @ Ry(b) @ Rz(g)
    z, y, x = np.indices((n, n, n)) - c
    X = np.stack([x, y, z]).reshape(3, -1).astype(float)
    U = Q0.T @ X                                           # coordinates along the blob's axes
    G = np.exp(-(U[0] ** 2 / (2 * 1.5 ** 2) + U[1] ** 2 / (2 * 4.0 ** 2) + U[2] ** 2 / (2 * 8.0 ** 2))).reshape(n, n, n)
    r = O.orient(G, np.array([[c, c, c]]), 7)
    assert r["nframes"][0] >= 1
    F = r["frames"][0, 0]
    assert abs(F[:, 0] @ Q0[:, 0]) > math.cos(math.radians(10))
    assert abs(F[:, 1] @ Q0[:, 1]) > math.cos(math.radians(20))


def test_orientation_offset_and_power_of_two_scaling_invariance():
    """Values on a 2^-20 grid: adding 1 and doubling are exact, so the
    gradients, decisions, frames and descriptors are identical."""
    G = np.round(_smooth_cube(21, 42) * 2 ** 20) / 2 ** 20
    kp = np.array([[10, 10, 10], [6, 12, 9]])
    ref = O.orient(G, kp, 6)
    for H in (G + 1.0, 2.0 * G):
        got = O.orient(H, kp, 6)
        assert np.array_equal(got["nframes"], ref["nframes"])
        assert np.array_equal(got["frames"], ref["frames"])
        assert np.array_equal(got["rank"], ref["rank"])


@pytest.mark.parametrize("ratio,primaries", [(0.95, 2), (0.85, 2), (0.75, 1), (0.6, 1)])
def test_orientation_peak_threshold_and_neighbours(ratio, primaries):
    """Gradient a along x below the keypoint's plane and b along y from it
    on (6 of the window's 11 planes against 5): H(+y) / H(+x) ~ ratio. +y is
    90 degrees from +x, so it is not a neighbour and is a second primary
    exactly when it reaches 0.8 of the maximum; each primary then takes the
    other direction as its secondary."""
    n, c = 21, 10
    z, y, x = np.indices((n, n, n)) - c
    G = np.where(z < 0, 1.0 * x, ratio * 5 / 6 * y).astype(float)
    r = O.orient(G, np.array([[c, c, c]]), 5)
    assert r["nframes"][0] == primaries
    got = {tuple(np.round(r["frames"][0, f][:, 0], 9)) for f in range(primaries)}
    want = {(1.0, 0.0, 0.0), (0.0, 1.0, 0.0)} if primaries == 2 else {(1.0, 0.0, 0.0)}
    assert got == want
    for f in range(primaries):
        e1, e2 = r["frames"][0, f][:, 0], r["frames"][0, f][:, 1]
        assert abs(e1 @ e2) < 1e-12 and set(np.round(np.abs(e1 + e2), 9)) == {0.0, 1.0}
