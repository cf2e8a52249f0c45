"""Request server (continuous batching): every request's result is the one
the plain path gives for its volume, alone and among others in flight;
admission respects the HBM budget; oversize and cancelled requests fail
cleanly."""
import numpy as np
import pytest

from gen import phantoms as P

pytestmark = pytest.mark.gpu

SHAPES = [(64, 64, 64), (45, 38, 53), (70, 33, 34), (20, 17, 18), (33, 48, 40), (64, 64, 64), (45, 38, 53)]
PARAMS = dict(min_dim=8)
CAP = 4096


def _vols():
    return [P.noise_blob_volume(s, 60 + i, n_blobs=max(2, int(np.prod(s) / 12000)), margin=5)
            for i, s in enumerate(SHAPES)]


def _ctx():
    import paper_2112_10258_amd as S
    return S.Context(S.default_params(**PARAMS), P.pair_draws())


def _plain(ctx, vol):
    import torch
    import paper_2112_10258_amd as S
    nz, ny, nx = vol.shape
    plan = S.Plan(ctx, (nx, ny, nz), CAP)
    buf = S.Buffers(plan)
    S.run_extract(plan, torch.from_numpy(vol).cuda(), buf)
    torch.cuda.synchronize()
    return S.fetch_results(plan, buf)


def _same(a, b, what):
    assert a["count"] == b["count"], what
    assert a["keypoints"].tobytes() == b["keypoints"].tobytes(), what
    for f in ("siftrank", "brief", "rrief"):
        assert np.array_equal(a[f], b[f]), (what, f)


def test_server_alone_and_in_the_mix_equal_plain():
    import torch
    import paper_2112_10258_amd as S
    ctx = _ctx()
    vols = _vols()
    dvols = [torch.from_numpy(v).cuda() for v in vols]
    torch.cuda.synchronize()
    refs = [_plain(ctx, v) for v in vols]
    srv = S.Server(ctx, hbm_budget=8 << 30, n_streams=4, max_inflight=6, max_batch=8, kp_capacity=CAP)
    try:
        # alone: one request at a time
        alone = []
        for i, dv in enumerate(dvols):
            t = srv.submit(dv)
            alone.append(srv.fetch(t))
            srv.release(t)
            _same(alone[-1], refs[i], f"alone {i}")
        print(f"[serve] alone: {[a['count'] for a in alone]} keypoints, identical to plain", flush=True)
        # in the mix: all submitted back to back, twice over, several in flight
        tickets = [srv.submit(dv) for dv in dvols + dvols]
        res = [srv.result(t) for t in tickets]
        assert all(r.status == 0 for r in res)
        assert len({r.stream for r in res}) > 1, "requests did not spread over streams"
        overlap = sum(1 for i in range(1, len(res)) if res[i].t_start < res[i - 1].t_done)
        for k, t in enumerate(tickets):
            _same(srv.fetch(t), refs[k % len(vols)], f"mix {k}")
            srv.release(t)
        st = srv.stats()
        print(f"[serve] mix: {len(tickets)} requests, {overlap} started before their predecessor finished, "
              f"stats {st}", flush=True)
        assert st["completed"] == len(vols) + len(tickets) and st["failed"] == 0
        assert st["in_flight"] == 0 and st["pending"] == 0
    finally:
        srv.close()


def test_server_admission_within_a_small_budget():
    import torch
    import paper_2112_10258_amd as S
    ctx = _ctx()
    vols = _vols()
    dvols = [torch.from_numpy(v).cuda() for v in vols]
    torch.cuda.synchronize()
    probe = S.Server(ctx, hbm_budget=1 << 40, n_streams=1, max_inflight=1, kp_capacity=CAP)
    fps = [probe.footprint((v.shape[2], v.shape[1], v.shape[0])) for v in vols]
    probe.close()
    # room for the largest slot plus a little: at most two small ones at a time
    budget = max(fps) + min(fps)
    srv = S.Server(ctx, hbm_budget=budget, n_streams=3, max_inflight=8, kp_capacity=CAP)
    try:
        refs = [_plain(ctx, v) for v in vols]
        tickets = [srv.submit(dv) for dv in dvols]
        for k, t in enumerate(tickets):
            _same(srv.fetch(t), refs[k], f"budget {k}")
            srv.release(t)
        st = srv.stats()
        print(f"[serve] budget {budget} B: stats {st}", flush=True)
        assert st["peak_allocated"] <= budget
        assert st["slot_evictions"] > 0
        assert st["completed"] == len(vols)
    finally:
        srv.close()


def test_server_rejects_oversize_and_cancels_on_close():
    import torch
    import paper_2112_10258_amd as S
    ctx = _ctx()
    vol = torch.from_numpy(_vols()[0]).cuda()
    torch.cuda.synchronize()
    probe = S.Server(ctx, hbm_budget=1 << 40, n_streams=1, max_inflight=1, kp_capacity=CAP)
    fp = probe.footprint((64, 64, 64))
    probe.close()
    small = S.Server(ctx, hbm_budget=fp - 256, n_streams=1, max_inflight=1, kp_capacity=CAP)
    with pytest.raises(S.Sift3dError) as ei:
        small.submit(vol)
    assert ei.value.code == -3
    small.close()
    # one slot of room: the first request holds it until released, so the
    # second waits; closing the server cancels the waiting one
    srv = S.Server(ctx, hbm_budget=fp, n_streams=2, max_inflight=4, kp_capacity=CAP)
    t1 = srv.submit(vol)
    t2 = srv.submit(vol)
    r1 = srv.result(t1)
    assert r1.status == 0
    assert srv.result(t2, wait=False) is None
    assert srv.stats()["pending"] == 1
    srv.close()
    print("[serve] oversize rejected; waiting request cancelled on close", flush=True)


def test_server_groups_waiting_requests_of_one_shape():
    """With one group in flight, requests that arrive meanwhile wait; the next
    admission takes the waiting requests of the head's shape as one batch
    extraction. Every result still equals the plain path's."""
    import torch
    import paper_2112_10258_amd as S
    ctx = _ctx()
    vols = _vols()
    order = [0, 0, 1, 0, 5, 0, 1, 0, 0, 2, 0, 1]        # indices into SHAPES (0 and 5 share a shape)
    dvols = [torch.from_numpy(v).cuda() for v in vols]
    torch.cuda.synchronize()
    refs = {i: _plain(ctx, vols[i]) for i in set(order)}
    srv = S.Server(ctx, hbm_budget=8 << 30, n_streams=2, max_inflight=1, max_batch=4, kp_capacity=CAP)
    try:
        tickets = [srv.submit(dvols[i]) for i in order]
        for t, i in zip(tickets, order):
            _same(srv.fetch(t), refs[i], f"grouped request of volume {i}")
        for t in tickets:
            srv.release(t)
        st = srv.stats()
        print(f"[serve] grouping: {len(order)} requests in {st['groups']} groups, stats {st}", flush=True)
        assert st["completed"] == len(order) and st["grouped_requests"] == len(order)
        assert st["groups"] < len(order), "no requests were grouped"
    finally:
        srv.close()


def test_admission_timeout_ends_requests_that_wait_too_long():
    """With one group on the device at a time and a 1 ms admission timeout,
    a burst of requests cannot all be admitted in time: the late ones end
    with SIFT3D_E_TIMEOUT (and can be released), the others equal the
    plain path. Without a timeout the same burst completes."""
    import torch
    import paper_2112_10258_amd as S
    ctx = _ctx()
    vol = _vols()[0]
    ref = _plain(ctx, vol)
    dv = torch.from_numpy(vol).cuda()
    torch.cuda.synchronize()
    for timeout in (1e-3, 0.0):
        srv = S.Server(ctx, hbm_budget=8 << 30, n_streams=1, max_inflight=1, max_batch=1, kp_capacity=CAP,
                       admit_timeout_s=timeout)
        try:
            tickets = [srv.submit(dv) for _ in range(40)]
            res = [srv.result(t) for t in tickets]
            ok = [t for t, r in zip(tickets, res) if r.status == 0]
            late = [r for r in res if r.status == S.E_TIMEOUT]
            assert len(ok) + len(late) == len(tickets)
            for t in ok:
                _same(srv.fetch(t), ref, f"timeout {timeout}")
            for r in late:
                assert r.t_done - r.t_submit >= timeout * 0.999
            for t in tickets:
                srv.release(t)
            st = srv.stats()
            print(f"[serve] admission timeout {timeout}: {len(ok)} admitted, {len(late)} timed out", flush=True)
            if timeout > 0:
                assert len(ok) >= 1 and len(late) >= 1
                assert st["failed"] == len(late)
            else:
                assert not late and st["failed"] == 0
        finally:
            srv.close()
