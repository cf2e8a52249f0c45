"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Stage-wise checks are binding: every G and D level within 1e-5 relative
max error; detection on the GPU's own D levels bit-identical; descriptors
on the GPU's own G levels identical up to the near-tie margins. The
end-to-end comparison (oracle all the way from the input) must agree except
for candidates whose oracle margin is below 1e-6.
"""
import numpy as np
import pytest

import oracle as O
from gen import phantoms as P
from tests.helpers import (LEVEL_RTOL, MARGIN, detection_margin, gpu_extract, kp_keys, level_rel_err,
                           oracle_params, rank_mismatch_excused, unpack_bits)

pytestmark = pytest.mark.gpu


def _vol(name):
    if name == "config1":
        return P.config1(), dict(n_octaves=2)
    if name == "config2":
        return P.config2(), {}
    if name == "ragged":
        # odd, non-tile-multiple dims, 3 octaves at min_dim 8
        return P.noise_blob_volume((45, 38, 53), 21, n_blobs=10, margin=6), dict(min_dim=8)
    if name == "flat":
        return P.noise_blob_volume((70, 33, 34), 22, n_blobs=6, margin=6), dict(min_dim=8)
    if name == "config1_fused":
        # the fused streaming pass on every octave
        return P.config1(), dict(n_octaves=2, pyramid_mode=1)
    if name == "ragged_fused":
        return P.noise_blob_volume((45, 38, 53), 21, n_blobs=10, margin=6), dict(min_dim=8, pyramid_mode=1)
    if name == "ragged_split":
        # the xy + z launches on every octave
        return P.noise_blob_volume((45, 38, 53), 21, n_blobs=10, margin=6), dict(min_dim=8, pyramid_mode=2)
    raise KeyError(name)


CASES = ["config1", "ragged", "flat", "config2", "config1_fused", "ragged_fused", "ragged_split"]
_cache = {}


def _run(name):
    if name not in _cache:
        vol, kw = _vol(name)
        print(f"[parity] case={name} shape={vol.shape} params={kw}", flush=True)
        g = gpu_extract(vol, **kw)
        p = oracle_params(g["params"])
        ref = O.pyramid(vol, p)
        _cache[name] = (vol, g, p, ref)
    return _cache[name]


@pytest.mark.parametrize("name", CASES)
def test_levels_match_oracle(name):
    vol, g, p, ref = _run(name)
    assert g["n_octaves"] == len(ref)
    errs = {}
    for o, oc in enumerate(ref):
        for i, lev in enumerate(oc.G):
            errs[f"G{o}.{i}"] = level_rel_err(g["G"][o][i], lev)
        for i, lev in enumerate(oc.D):
            errs[f"D{o}.{i}"] = level_rel_err(g["D"][o][i], lev)
    worst = max(errs, key=errs.get)
    print(f"[parity] {name}: worst level rel err {errs[worst]:.3e} at {worst}; "
          f"worst G {max(v for k, v in errs.items() if k[0] == 'G'):.3e}")
    bad = {k: v for k, v in errs.items() if v > LEVEL_RTOL}
    assert not bad, f"levels over {LEVEL_RTOL}: {bad}"


@pytest.mark.parametrize("name", CASES)
def test_preblur_levels_match_oracle(name):
    """B_s (the BRIEF pre-blur, Section 3.2.3) of every octave equals the
    oracle's blur of the GPU's own G_s by sigma_b, whichever kernel wrote it
    (on config 2: the octave-0 fused level passes G_2..G_4, which write
    B_1..B_3 alongside; the compact pass below)."""
    vol, g, p, ref = _run(name)
    errs = {}
    for o, Gs in enumerate(g["G"]):
        for s in range(1, p.scales + 1):
            want = O.blur(Gs[s].astype(np.float64), p.brief_blur, p.trunc)
            errs[f"B{o}.{s}"] = level_rel_err(g["B"][o][s - 1], want)
    worst = max(errs, key=errs.get)
    print(f"[parity] {name}: worst pre-blur rel err {errs[worst]:.3e} at {worst}")
    bad = {k: v for k, v in errs.items() if v > LEVEL_RTOL}
    assert not bad, f"pre-blurred levels over {LEVEL_RTOL}: {bad}"


@pytest.mark.parametrize("name", CASES)
def test_detection_stagewise_bit_identical(name):
    vol, g, p, ref = _run(name)
    want = O.detect([[d.astype(np.float64) for d in Ds] for Ds in g["D"]], p)
    got = g["keypoints"]
    assert g["count"] == len(want)
    assert kp_keys(got) == kp_keys(want)
    assert np.array_equal(got["polarity"], want["polarity"])
    assert np.array_equal(got["dog"], want["dog"].astype(np.float32))
    for f in ("xf", "yf", "zf", "sigma"):
        np.testing.assert_allclose(got[f], want[f], rtol=1e-6, atol=0)
    print(f"[parity] {name}: {len(got)} keypoints")


@pytest.mark.parametrize("name", CASES)
def test_descriptors_stagewise(name):
    vol, g, p, ref = _run(name)
    k = g["keypoints"]
    assert len(k) > 0
    d = O.describe([[x.astype(np.float64) for x in Gs] for Gs in g["G"]], k, P.pair_draws(), p)
    # SIFT-Rank: ranks identical except bins within 1e-6 of the largest bin
    bad_sr = 0
    for i in range(len(k)):
        h = d["hist"][i]
        ok = rank_mismatch_excused(h, g["siftrank"][i], d["siftrank"][i], MARGIN * max(h.max(), 1e-300))
        assert ok, f"SIFT-Rank mismatch at keypoint {i}"
        bad_sr += int(np.any(g["siftrank"][i] != d["siftrank"][i]))
    # BRIEF: bit-exact except |d| < 1e-6
    gb = unpack_bits(g["brief"], p.brief_n)
    ob = unpack_bits(d["brief"], p.brief_n)
    diff = gb != ob
    assert np.all(np.abs(d["diff"][diff]) < MARGIN), "BRIEF bit mismatch outside the margin"
    # RRIEF: identical except differences within 1e-6
    for i in range(len(k)):
        assert rank_mismatch_excused(d["diff"][i], g["rrief"][i], d["rrief"][i], MARGIN), f"RRIEF mismatch kp {i}"
    print(f"[parity] {name}: siftrank rows differing (excused) {bad_sr}, brief bits differing {int(diff.sum())}")


@pytest.mark.parametrize("name", ["config1", "ragged", "config2", "config1_fused"])
def test_end_to_end_keypoints(name):
    vol, g, p, ref = _run(name)
    want = O.detect([oc.D for oc in ref], p)
    a, b = set(kp_keys(g["keypoints"])), set(kp_keys(want))
    for key in a ^ b:
        o, s, z, y, x = key
        m = detection_margin(ref[o].D, s, x, y, z, p.dog_threshold)
        assert m < MARGIN, f"keypoint {key} differs with oracle margin {m:.3e}"
    common = sorted(a & b)
    assert len(common) >= 0.99 * max(len(b), 1)
    # descriptors of common keypoints, FP64 oracle all the way
    kref = want[[kp_keys(want).index(c) for c in common]]
    kgpu_idx = [kp_keys(g["keypoints"]).index(c) for c in common]
    d = O.describe([oc.G for oc in ref], kref, P.pair_draws(), p)
    # BRIEF/RRIEF: the GPU's d_i comes from its pre-blurred levels B, the
    # oracle's from blur(G_ref). B is a positive average (weights sum to 1), so
    # |B_gpu - B_ref| <= beta + delta with delta = max|G_gpu - G_ref| on that
    # level and beta = max|B_gpu - blur(G_gpu)|; hence |d_gpu - d_ref| <= 2
    # (beta + delta): a bit may flip only where |d_ref| is below that, and a
    # rank may move only past differences within twice that.
    bound = {}
    for o in range(len(ref)):
        for s_ in range(1, p.scales + 1):
            delta = float(np.abs(g["G"][o][s_].astype(np.float64) - ref[o].G[s_]).max())
            beta = float(np.abs(g["B"][o][s_ - 1] - O.blur(g["G"][o][s_].astype(np.float64), p.brief_blur,
                                                            p.trunc)).max())
            bound[(o, s_)] = 2.0 * (beta + delta) * (1 + 1e-6) + 1e-12
    gb = unpack_bits(g["brief"][kgpu_idx], p.brief_n)
    ob = unpack_bits(d["brief"], p.brief_n)
    flips = 0
    for j, c in enumerate(common):
        b_ = bound[(c[0], c[1])]
        fl = gb[j] != ob[j]
        assert np.all(np.abs(d["diff"][j][fl]) <= b_), (name, c)
        flips += int(fl.sum())
        assert rank_mismatch_excused(d["diff"][j], g["rrief"][kgpu_idx[j]], d["rrief"][j], 2 * b_), (name, c)
    # SIFT-Rank: a sample whose gradient component is within the level error
    # of zero moves its whole magnitude to the neighbouring octant bin, so no
    # margin bounds the histograms end to end; the share of rows that differ
    # at all is bounded instead (5%).
    sr_rows = int(np.sum(np.any(g["siftrank"][kgpu_idx] != d["siftrank"], axis=1)))
    print(f"[parity] {name} end-to-end: gpu {len(a)} oracle {len(b)} common {len(common)}; "
          f"siftrank rows differing {sr_rows}/{len(common)}; brief bits differing {flips} "
          f"(all within 2(beta+delta) <= {max(bound.values()):.2e})")
    assert sr_rows <= 0.05 * len(common), (name, sr_rows, len(common))


def test_determinism_bitwise():
    vol, kw = _vol("config1")
    a = gpu_extract(vol, **kw)
    b = gpu_extract(vol, **kw)
    for o in range(a["n_octaves"]):
        for i in range(len(a["G"][o])):
            assert np.array_equal(a["G"][o][i], b["G"][o][i])
        for i in range(len(a["D"][o])):
            assert np.array_equal(a["D"][o][i], b["D"][o][i])
    assert a["keypoints"].tobytes() == b["keypoints"].tobytes()
    for f in ("siftrank", "brief", "rrief"):
        assert np.array_equal(a[f], b[f])


def test_plan_rejects_oversized_planes():
    """Planes are addressed with 32-bit byte offsets: nx * ny above 2^28 is
    refused at plan time (no launch), 2^28 itself is accepted by the check."""
    import paper_2112_10258_amd as S
    ctx = S.Context(S.default_params(), P.pair_draws())
    with pytest.raises(S.Sift3dError) as ei:
        S.Plan(ctx, (1 << 15, 1 << 14, 16), 16)
    assert ei.value.code == -1


def test_capacity_overflow_keeps_canonical_prefix():
    vol, kw = _vol("config1")
    full = gpu_extract(vol, levels=False, **kw)
    n = full["count"]
    assert n > 20
    cap = n // 3
    part = gpu_extract(vol, cap=cap, levels=False, **kw)
    assert part["count"] == n
    assert part["keypoints"].tobytes() == full["keypoints"][:cap].tobytes()
    assert np.array_equal(part["siftrank"], full["siftrank"][:cap])
    assert np.array_equal(part["rrief"], full["rrief"][:cap])
    zero = gpu_extract(vol, cap=0, levels=False, **kw)
    assert zero["count"] == n and len(zero["keypoints"]) == 0


def test_describe_one_family_equals_both():
    """The descriptor launch splits its workgroups between SIFT-Rank and
    BRIEF / RRIEF according to what is asked for: each family alone, with a
    small and a large keypoint capacity (one workgroup per slot, and the
    3 : 1 split once the slots exceed the device), equals the call that
    writes both."""
    import torch

    import paper_2112_10258_amd as S
    vol, kw = _vol("config1")
    ctx = S.Context(S.default_params(**kw), P.pair_draws())
    nz, ny, nx = vol.shape
    for cap in (256, 1 << 14):
        plan = S.Plan(ctx, (nx, ny, nz), cap)
        buf = S.Buffers(plan)
        S.run_extract(plan, torch.from_numpy(vol).cuda(), buf)
        torch.cuda.synchronize()
        both = S.fetch_results(plan, buf)
        assert both["count"] > 0
        for f in ("siftrank", "brief", "rrief"):
            getattr(buf, f).zero_()
        plan.describe(buf.ws, buf.kp, buf.count, siftrank=buf.siftrank)
        plan.describe(buf.ws, buf.kp, buf.count, brief=buf.brief)
        plan.describe(buf.ws, buf.kp, buf.count, rrief=buf.rrief)
        torch.cuda.synchronize()
        alone = S.fetch_results(plan, buf)
        for f in ("siftrank", "brief", "rrief"):
            assert np.array_equal(alone[f], both[f]), (cap, f)


@pytest.mark.parametrize("method", [1, 2, 4, 5])
def test_brief_pair_methods(method):
    """BRIEF bits and RRIEF ranks with each of the other point-pair methods of
    Section 3.2.3 match the oracle on the GPU's own levels (bits exact except
    |d| < 1e-6, ranks exact except differences within 1e-6)."""
    vol, kw = _vol("config1")
    g = gpu_extract(vol, brief_method=method, **kw)
    p = oracle_params(g["params"])
    assert p.brief_method == method
    k = g["keypoints"]
    assert len(k) > 0
    d = O.describe([[x.astype(np.float64) for x in Gs] for Gs in g["G"]], k, P.pair_draws(), p)
    gb = unpack_bits(g["brief"], p.brief_n)
    ob = unpack_bits(d["brief"], p.brief_n)
    diff = gb != ob
    assert np.all(np.abs(d["diff"][diff]) < MARGIN), "BRIEF bit mismatch outside the margin"
    for i in range(len(k)):
        assert rank_mismatch_excused(d["diff"][i], g["rrief"][i], d["rrief"][i], MARGIN), i
    if method in (4, 5):
        # p1 at the centre: every pair compares the keypoint's own voxel
        assert np.all(O.pair_offsets(P.pair_draws(), p, 1)[:, 0] == 0)
    print(f"[parity] brief method {method}: {len(k)} keypoints, bits differing {int(diff.sum())}", flush=True)


def test_brief_wide_preblur():
    """The largest pre-blur of the paper's sigma_b sweep (3.05: tap radius 10)
    runs as its own level tasks; B_s and the descriptors match the oracle."""
    vol, kw = _vol("config1")
    g = gpu_extract(vol, brief_blur=3.05, **kw)
    p = oracle_params(g["params"])
    for o, Gs in enumerate(g["G"]):
        for s in range(1, p.scales + 1):
            want = O.blur(Gs[s].astype(np.float64), p.brief_blur, p.trunc)
            assert level_rel_err(g["B"][o][s - 1], want) <= LEVEL_RTOL, (o, s)
    k = g["keypoints"]
    d = O.describe([[x.astype(np.float64) for x in Gs] for Gs in g["G"]], k, P.pair_draws(), p)
    gb = unpack_bits(g["brief"], p.brief_n)
    ob = unpack_bits(d["brief"], p.brief_n)
    assert np.all(np.abs(d["diff"][gb != ob]) < MARGIN)
    for i in range(len(k)):
        assert rank_mismatch_excused(d["diff"][i], g["rrief"][i], d["rrief"][i], MARGIN), i


def test_constant_volume_has_no_keypoints():
    vol = np.full((40, 40, 40), 0.5, dtype=np.float32)
    g = gpu_extract(vol, min_dim=8)
    assert g["count"] == 0
    for o in range(g["n_octaves"]):
        # FP32 taps and FMA chains leave a few ulp of drift over ~50 1D passes
        for lev in g["G"][o]:
            assert np.abs(lev - 0.5).max() <= 0.5 * 1e-6
        for lev in g["D"][o]:
            assert np.abs(lev).max() <= 0.5 * 1e-6


def test_relaxed_votes_and_small_volume():
    vol = P.noise_blob_volume((20, 17, 18), 31, n_blobs=3, margin=5)
    g = gpu_extract(vol, min_dim=4, votes=70, dog_threshold=0.005)
    p = oracle_params(g["params"])
    assert g["n_octaves"] == len(O.octave_dims((20, 17, 18), p))
    want = O.detect([[d.astype(np.float64) for d in Ds] for Ds in g["D"]], p)
    assert kp_keys(g["keypoints"]) == kp_keys(want)
    assert len(want) > 0


def test_pair_offsets_equal_oracle_tables():
    import paper_2112_10258_amd as S
    gp = S.default_params()
    ctx = S.Context(gp, P.pair_draws())
    for s in (1, 2, 3):
        assert np.array_equal(ctx.pair_offsets(s), O.pair_offsets(P.pair_draws(), O.Params(), s))


def test_brief_n64_and_no_preblur():
    vol, kw = _vol("config1")
    g = gpu_extract(vol, brief_n=64, brief_blur=0.0, **kw)
    p = oracle_params(g["params"])
    d = O.describe([[x.astype(np.float64) for x in Gs] for Gs in g["G"]], g["keypoints"], P.pair_draws(), p)
    gb = unpack_bits(g["brief"], 64)
    ob = unpack_bits(d["brief"], 64)
    assert np.all(np.abs(d["diff"][gb != ob]) < MARGIN)
    for i in range(len(g["keypoints"])):
        assert rank_mismatch_excused(d["diff"][i], g["rrief"][i], d["rrief"][i], MARGIN)
