"""A batch plan (several volumes of different sizes, one launch per stage)
gives every volume exactly the results of its own one-volume plan."""
import numpy as np
import pytest

from gen import phantoms as P

pytestmark = pytest.mark.gpu

SHAPES = [(64, 64, 64), (45, 38, 53), (70, 33, 34), (20, 17, 18), (33, 48, 40)]
PARAMS = dict(min_dim=8)


def _vols():
    return [P.noise_blob_volume(s, 40 + i, n_blobs=max(2, int(np.prod(s) / 12000)), margin=5)
            for i, s in enumerate(SHAPES)]


def _run_plain(vol, cap, **kw):
    import torch
    import paper_2112_10258_amd as S
    ctx = S.Context(S.default_params(**kw), P.pair_draws())
    nz, ny, nx = vol.shape
    plan = S.Plan(ctx, (nx, ny, nz), cap)
    buf = S.Buffers(plan)
    S.run_extract(plan, torch.from_numpy(vol).cuda(), buf)
    torch.cuda.synchronize()
    res = S.fetch_results(plan, buf)
    res["G"] = [[plan.level(buf.ws, o, 0, i).cpu().numpy() for i in range(6)] for o in range(plan.n_octaves)]
    res["D"] = [[plan.level(buf.ws, o, 1, i).cpu().numpy() for i in range(5)] for o in range(plan.n_octaves)]
    return res


@pytest.mark.parametrize("cap,mode", [(4096, 0), (7, 0), (4096, 1), (4096, 2)])
def test_batch_equals_plain(cap, mode):
    """mode 0 runs these small octaves on the compact pass, mode 1 on the
    fused pass (one fused launch per level covers all volumes: a job table
    with per-volume slabs), mode 2 as xy + z launches."""
    import torch
    import paper_2112_10258_amd as S
    vols = _vols()
    params = dict(PARAMS, pyramid_mode=mode)
    print(f"[batch] shapes={SHAPES} cap={cap} mode={mode}", flush=True)
    ctx = S.Context(S.default_params(**params), P.pair_draws())
    plan = S.Plan(ctx, [(v.shape[2], v.shape[1], v.shape[0]) for v in vols], cap, batch=True)
    assert plan.n_volumes == len(vols)
    buf = S.Buffers(plan)
    S.run_extract(plan, plan.pack_volumes(vols), buf)
    torch.cuda.synchronize()
    for v, vol in enumerate(vols):
        ref = _run_plain(vol, cap, **params)
        got = S.fetch_results(plan, buf, v)
        assert got["count"] == ref["count"], v
        assert got["keypoints"].tobytes() == ref["keypoints"].tobytes(), v
        for f in ("siftrank", "brief", "rrief"):
            assert np.array_equal(got[f], ref[f]), (v, f)
        for o in range(plan.volumes[v]["n_octaves"]):
            for i in range(6):
                assert np.array_equal(plan.level(buf.ws, o, 0, i, v).cpu().numpy(), ref["G"][o][i]), (v, o, i)
            for i in range(5):
                assert np.array_equal(plan.level(buf.ws, o, 1, i, v).cpu().numpy(), ref["D"][o][i]), (v, o, i)
        print(f"[batch] volume {v}: {got['count']} keypoints identical", flush=True)


def test_batch_plan_of_many_volumes_plans_quickly():
    """Planning scales linearly with the number of volumes (the scheduler
    resolves each task's dependency once): 4096 small volumes plan in well
    under a few seconds."""
    import time

    import paper_2112_10258_amd as S
    ctx = S.Context(S.default_params(**PARAMS), P.pair_draws())
    shapes = [(16 + (i % 5), 16 + (i % 3), 16 + (i % 7)) for i in range(4096)]
    t0 = time.perf_counter()
    plan = S.Plan(ctx, shapes, 4, batch=True)
    dt = time.perf_counter() - t0
    print(f"[batch] plan over {plan.n_volumes} volumes built in {dt:.2f} s", flush=True)
    assert plan.n_volumes == len(shapes)
    assert dt < 5.0
