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
