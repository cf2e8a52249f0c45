"""Autotuned plans (sift3d_plan_tune): the tuner times tile-height and slab
candidates of every fused streaming launch and keeps the fastest. Tile
heights and slab splits do not change any voxel's arithmetic, so a tuned
plan must give the default plan's results bit for bit (every level,
keypoints, descriptors), for one volume and for a batch."""
import numpy as np
import pytest

from gen import phantoms as P

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[tune] {msg}", flush=True)


def _levels(plan, ws, nvol):
    out = []
    S = plan.ctx.params.scales
    for v in range(nvol):
        no = plan.volumes[v]["n_octaves"]
        for o in range(no):
            for kind, idxs in ((0, range(S + 3)), (1, range(S + 2)), (2, range(1, S + 1))):
                for i in idxs:
                    out.append(plan.level(ws, o, kind, i, v).cpu().numpy())
    return out


def _run(plan, vol_dev):
    import torch

    import paper_2112_10258_amd as S
    buf = S.Buffers(plan)
    S.run_extract(plan, vol_dev, buf)
    torch.cuda.synchronize()
    res = [S.fetch_results(plan, buf, v) for v in range(plan.n_volumes)]
    return res, _levels(plan, buf.ws, plan.n_volumes)


def _same(a, b, what):
    (ra, la), (rb, lb) = a, b
    assert len(la) == len(lb)
    for x, y in zip(la, lb):
        assert np.array_equal(x, y), what
    for x, y in zip(ra, rb):
        assert x["count"] == y["count"], what
        assert x["keypoints"].tobytes() == y["keypoints"].tobytes(), what
        for f in ("siftrank", "brief", "rrief"):
            assert np.array_equal(x[f], y[f]), (what, f)


def test_tuned_plan_is_bitwise_equal_to_default():
    import torch

    import paper_2112_10258_amd as S
    vol = P.config2()
    nz, ny, nx = vol.shape
    ctx = S.Context(S.default_params(), P.pair_draws())
    dvol = torch.from_numpy(vol).cuda()
    ref = _run(S.Plan(ctx, (nx, ny, nz), 1 << 14), dvol)
    plan = S.Plan(ctx, (nx, ny, nz), 1 << 14)
    ws = plan.alloc_workspace()
    recs = plan.tune(dvol, ws, reps=2)
    assert recs, "no fused launch was tuned"
    for r in recs:
        assert r["candidates"] >= 1 and r["tuned"]["ms"] <= r["default"]["ms"]
    _say("145x174x145: " + "; ".join(f"step {r['step']}: ty {r['default']['ty']}/{r['default']['slabs']} slabs "
                                      f"{r['default']['ms'] * 1e3:.1f} us -> ty {r['tuned']['ty']}/{r['tuned']['slabs']} "
                                      f"{r['tuned']['ms'] * 1e3:.1f} us" for r in recs))
    _same(_run(plan, dvol), ref, "tuned 145x174x145")
    # tuning again starts from the default rule and is as valid
    plan.tune(dvol, ws, reps=1)
    _same(_run(plan, dvol), ref, "re-tuned 145x174x145")


def test_tuned_batch_plan_is_bitwise_equal_to_default():
    import paper_2112_10258_amd as S
    vols = [P.noise_blob_volume(s, 500 + i) for i, s in enumerate([(96, 128, 112), (150, 100, 120), (64, 64, 64)])]
    shapes = [(v.shape[2], v.shape[1], v.shape[0]) for v in vols]
    ctx = S.Context(S.default_params(pyramid_mode=1), P.pair_draws())
    dplan = S.Plan(ctx, shapes, 1 << 12, batch=True)
    packed = dplan.pack_volumes(vols)
    ref = _run(dplan, packed)
    plan = S.Plan(ctx, shapes, 1 << 12, batch=True)
    recs = plan.tune(packed, plan.alloc_workspace(), reps=1)
    assert recs
    _same(_run(plan, packed), ref, "tuned batch")
    _say(f"batch of 3, all fused: {len(recs)} launches tuned, results identical")
