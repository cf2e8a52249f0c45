"""Stream and graph behaviour of the C ABI on the 145x174x145 volume (its
schedule mixes fused, split and compact launches). Checks, bit for bit
against the same volume run alone:
  - two extractions enqueued back to back on one stream and one workspace;
  - extractions of one plan on two caller streams at once (the server's
    pattern: a plan is shared by the groups of one shape);
  - a pyramid captured into a HIP graph and replayed, with eager work on
    the same workspace between the replays.
"""
import numpy as np
import pytest

from gen import phantoms as P

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[streams] {msg}", flush=True)


def _setup():
    import torch

    import paper_2112_10258_amd as S

    ctx = S.Context(S.default_params(), P.pair_draws())
    plan = S.Plan(ctx, (145, 174, 145), 1 << 14)
    vols = [torch.from_numpy(np.ascontiguousarray(P.config2(seed), dtype=np.float32)).cuda() for seed in (2, 5)]
    return S, ctx, plan, vols


def _alone(S, plan, vol):
    import torch

    buf = S.Buffers(plan)
    S.run_extract(plan, vol, buf)
    torch.cuda.synchronize()
    return S.fetch_results(plan, buf)


def _same(a, b):
    assert a["count"] == b["count"]
    assert a["keypoints"].tobytes() == b["keypoints"].tobytes()
    for f in ("siftrank", "brief", "rrief"):
        assert np.array_equal(a[f], b[f])


def test_back_to_back_extracts_on_one_workspace():
    import torch

    S, ctx, plan, vols = _setup()
    _say("two extractions back to back, one workspace, 145x174x145")
    ref = [_alone(S, plan, v) for v in vols]
    assert ref[0]["count"] > 0 and ref[1]["count"] > 0
    b0, b1 = S.Buffers(plan), S.Buffers(plan)
    b1.ws = b0.ws
    for _ in range(3):
        S.run_extract(plan, vols[0], b0)
        S.run_extract(plan, vols[1], b1)
    torch.cuda.synchronize()
    _same(S.fetch_results(plan, b0), ref[0])
    _same(S.fetch_results(plan, b1), ref[1])


def test_one_plan_on_two_streams():
    import torch

    S, ctx, plan, vols = _setup()
    _say("one plan, two caller streams at once, 145x174x145")
    ref = [_alone(S, plan, v) for v in vols]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    bufs = [S.Buffers(plan), S.Buffers(plan)]
    torch.cuda.synchronize()
    for _ in range(3):
        for i in range(2):
            S.run_extract(plan, vols[i], bufs[i], stream=streams[i])
    torch.cuda.synchronize()
    for i in range(2):
        _same(S.fetch_results(plan, bufs[i]), ref[i])


def test_pyramid_graph_replays_equal_eager():
    import torch

    S, ctx, plan, vols = _setup()
    _say("pyramid captured into a HIP graph, 145x174x145")
    ws_e, ws_g = plan.alloc_workspace(), plan.alloc_workspace()
    plan.build_pyramid(vols[0], ws_e)
    torch.cuda.synchronize()
    sc = ctx.params.scales
    levels = [(o, k, i) for o in range(plan.n_octaves) for k, n in ((0, sc + 3), (1, sc + 2)) for i in range(n)]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.build_pyramid(vols[0], ws_g, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        ws_g.zero_()
        g.replay()
        torch.cuda.synchronize()
        for o, k, i in levels:
            assert torch.equal(plan.level(ws_g, o, k, i), plan.level(ws_e, o, k, i)), (rep, o, k, i)
        # eager work on the same workspace between replays
        plan.build_pyramid(vols[1], ws_g)
        torch.cuda.synchronize()
