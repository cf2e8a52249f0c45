"""Shared helpers of the GPU tests: run the HIP path, fetch levels, and the
near-tie margins of the parity contract."""
from __future__ import annotations

import numpy as np

import oracle as O

# Parity contract
LEVEL_RTOL = 1e-5      # max|gpu - oracle| / max|oracle| per G and D level
MARGIN = 1e-6          # near-tie margin for keypoints, BRIEF bits and ranks


def oracle_params(gp) -> O.Params:
    """Oracle parameters equal to a binding Params struct."""
    return O.Params(n_octaves=gp.n_octaves, min_dim=gp.min_dim, scales=gp.scales, sigma0=gp.sigma0,
                    sigma_in=gp.sigma_in, trunc=gp.trunc, dog_threshold=float(np.float32(gp.dog_threshold)),
                    votes=gp.votes, brief_n=gp.brief_n, brief_blur=gp.brief_blur,
                    siftrank_factor=gp.siftrank_factor, brief_method=gp.brief_method)


def gpu_extract(vol: np.ndarray, cap: int = 1 << 15, draws=None, levels: bool = True, **params):
    """Run sift3d_extract on cuda:0; return host copies of everything."""
    import torch

    import paper_2112_10258_amd as S
    from gen import phantoms as P

    if draws is None:
        draws = P.pair_draws()
    gp = S.default_params(**params)
    ctx = S.Context(gp, draws)
    nz, ny, nx = vol.shape
    plan = S.Plan(ctx, (nx, ny, nz), cap)
    buf = S.Buffers(plan)
    dvol = torch.from_numpy(np.ascontiguousarray(vol, dtype=np.float32)).cuda()
    S.run_extract(plan, dvol, buf)
    torch.cuda.synchronize()
    res = S.fetch_results(plan, buf)
    res["params"] = gp
    res["n_octaves"] = plan.n_octaves
    if levels:
        res["G"] = [[plan.level(buf.ws, o, 0, i).cpu().numpy() for i in range(gp.scales + 3)]
                    for o in range(plan.n_octaves)]
        res["D"] = [[plan.level(buf.ws, o, 1, i).cpu().numpy() for i in range(gp.scales + 2)]
                    for o in range(plan.n_octaves)]
        if gp.brief_blur > 0 and gp.brief_n > 0:
            # B[o][s - 1] = pre-blurred G_s, s = 1..S
            res["B"] = [[plan.level(buf.ws, o, 2, s).cpu().numpy() for s in range(1, gp.scales + 1)]
                        for o in range(plan.n_octaves)]
    res["_keep"] = (ctx, plan, buf, dvol)
    return res


def level_rel_err(gpu: np.ndarray, ref: np.ndarray) -> float:
    den = float(np.abs(ref).max())
    num = float(np.abs(gpu.astype(np.float64) - ref).max())
    return num / den if den > 0 else num


def kp_keys(k):
    return [(int(r["octave"]), int(r["scale"]), int(r["z"]), int(r["y"]), int(r["x"])) for r in k]


def detection_margin(D, s, x, y, z, thr):
    """Distance of voxel (x,y,z) of D_s from flipping: min(| |D|-thr |, min |D - neighbour|)."""
    v = D[s][z, y, x]
    m = abs(abs(v) - thr)
    for l in (s - 1, s, s + 1):
        blk = D[l][z - 1:z + 2, y - 1:y + 2, x - 1:x + 2].ravel().astype(np.float64)
        if l == s:
            blk = np.delete(blk, 13)
        m = min(m, float(np.abs(v - blk).min()))
    return m


def rank_mismatch_excused(vals: np.ndarray, r_gpu: np.ndarray, r_ref: np.ndarray, margin: float) -> bool:
    """True if every rank difference is explained by values within `margin` of each other."""
    bad = np.nonzero(r_gpu.astype(np.int64) != r_ref.astype(np.int64))[0]
    if len(bad) == 0:
        return True
    for e in bad:
        # element e may only move past elements whose value is within the margin
        near = np.abs(vals - vals[e]) < margin
        lo = int(np.sum(vals < vals[e] - margin))
        hi = lo + int(np.sum(near)) - 1
        if not (lo <= int(r_gpu[e]) <= hi):
            return False
    return True


def unpack_bits(words: np.ndarray, n: int) -> np.ndarray:
    w = words.astype(np.uint64)
    out = np.zeros(w.shape[:-1] + (n,), dtype=bool)
    for i in range(n):
        out[..., i] = ((w[..., i // 64] >> np.uint64(i % 64)) & np.uint64(1)) == 1
    return out


def stagewise_check(g, p, label, ref=None, draws=None, say=print):
    """The binding stage-wise contract on one extraction `g` (gpu_extract
    output or the same keys): every G and D level against the oracle's
    pyramid `ref` (from the input; skipped if None), B_s against the oracle's
    blur of the GPU's own G_s, detection of the oracle on the GPU's D levels
    bit-identical, descriptors of the oracle on the GPU's G levels identical
    up to the near-tie margins. Returns the oracle keypoints."""
    from gen import phantoms as P
    if draws is None:
        draws = P.pair_draws()
    if ref is not None:
        assert g["n_octaves"] == len(ref), label
        worst = 0.0
        for o, oc in enumerate(ref):
            for i, lev in enumerate(oc.G):
                e = level_rel_err(g["G"][o][i], lev)
                assert e <= LEVEL_RTOL, (label, "G", o, i, e)
                worst = max(worst, e)
            for i, lev in enumerate(oc.D):
                e = level_rel_err(g["D"][o][i], lev)
                assert e <= LEVEL_RTOL, (label, "D", o, i, e)
                worst = max(worst, e)
        say(f"{label}: levels within {LEVEL_RTOL} (worst {worst:.2e})")
    if "B" in g:
        for o, Gs in enumerate(g["G"]):
            for s in range(1, p.scales + 1):
                e = level_rel_err(g["B"][o][s - 1], O.blur(Gs[s].astype(np.float64), p.brief_blur, p.trunc))
                assert e <= LEVEL_RTOL, (label, "B", o, s, e)
    want = O.detect([[d.astype(np.float64) for d in Ds] for Ds in g["D"]], p)
    got = g["keypoints"]
    assert g["count"] == len(want), label
    assert kp_keys(got) == kp_keys(want), label
    assert np.array_equal(got["polarity"], want["polarity"]), label
    assert np.array_equal(got["dog"], want["dog"].astype(np.float32)), label
    d = O.describe([[x.astype(np.float64) for x in Gs] for Gs in g["G"]], got, draws, p)
    for i in range(len(got)):
        h = d["hist"][i]
        assert rank_mismatch_excused(h, g["siftrank"][i], d["siftrank"][i], MARGIN * max(h.max(), 1e-300)), \
            (label, "siftrank", i)
        assert rank_mismatch_excused(d["diff"][i], g["rrief"][i], d["rrief"][i], MARGIN), (label, "rrief", i)
    gb = unpack_bits(g["brief"], p.brief_n)
    ob = unpack_bits(d["brief"], p.brief_n)
    assert np.all(np.abs(d["diff"][gb != ob]) < MARGIN), (label, "brief")
    sr_rows = int(np.sum(np.any(g["siftrank"] != d["siftrank"], axis=1)))
    say(f"{label}: {len(got)} keypoints identical; descriptors within the margins "
        f"(siftrank rows differing {sr_rows}, brief bits differing {int((gb != ob).sum())})")
    return want
