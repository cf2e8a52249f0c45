"""sift3d_detect_static (detection scratch in the library's static device
array, nothing allocated) against sift3d_detect (scratch in the workspace):
identical keypoint lists and counts, bit for bit, on two calls in a row
whose second input is smaller than the first (the array keeps the first
call's contents), then with a capacity below the count, on a batch plan,
and the size limit refused before any launch."""
import numpy as np
import pytest

from gen import phantoms as P

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[static-scratch] {msg}", flush=True)


def _both(plan, ws, nv, cap):
    """Keypoints and counts from sift3d_detect and sift3d_detect_static on
    the same built pyramid (the static call's buffers start as 0xAB bytes)."""
    import torch

    import paper_2112_10258_amd as S
    c = max(cap, 1)
    kp_a = torch.zeros(nv * c * S.KEYPOINT_BYTES, dtype=torch.uint8, device="cuda")
    kp_b = torch.full_like(kp_a, 0xAB)
    cnt_a = torch.zeros(nv, dtype=torch.int32, device="cuda")
    cnt_b = torch.full_like(cnt_a, -7)
    plan.detect(ws, kp_a, cnt_a)
    plan.detect_static(ws, kp_b, cnt_b)
    torch.cuda.synchronize()
    return kp_a.cpu().numpy(), cnt_a.cpu().numpy(), kp_b.cpu().numpy(), cnt_b.cpu().numpy()


def _check_same(plan, ws, nv, cap, what):
    import paper_2112_10258_amd as S
    kp_a, cnt_a, kp_b, cnt_b = _both(plan, ws, nv, cap)
    assert np.array_equal(cnt_a, cnt_b), (what, cnt_a, cnt_b)
    c = max(cap, 1)
    for v in range(nv):
        k = min(int(cnt_a[v]), cap) * S.KEYPOINT_BYTES
        base = v * c * S.KEYPOINT_BYTES
        assert kp_a[base:base + k].tobytes() == kp_b[base:base + k].tobytes(), (what, v)
    _say(f"{what}: counts {cnt_a.tolist()} identical, keypoint records identical")
    return cnt_a


def _plain(ctx, vol, cap):
    import torch

    import paper_2112_10258_amd as S
    nz, ny, nx = vol.shape
    plan = S.Plan(ctx, (nx, ny, nz), cap)
    ws = plan.alloc_workspace()
    plan.build_pyramid(torch.from_numpy(np.ascontiguousarray(vol)).cuda(), ws)
    return plan, ws


def test_static_scratch_detection_equals_workspace_detection():
    import paper_2112_10258_amd as S
    ctx = S.Context(S.default_params(), P.pair_draws())
    big = P.config2()
    small = P.noise_blob_volume((45, 38, 53), 77)
    _say(f"call 1: 145x174x145 phantom, call 2: 45x38x53 (smaller), cap 1<<14")
    plan1, ws1 = _plain(ctx, big, 1 << 14)
    assert plan1.detect_scratch_bytes() <= S.DETECT_STATIC_SCRATCH
    n1 = _check_same(plan1, ws1, 1, 1 << 14, "145x174x145")
    assert n1[0] > 0
    plan2, ws2 = _plain(ctx, small, 1 << 14)
    assert plan2.detect_scratch_bytes() < plan1.detect_scratch_bytes()
    n2 = _check_same(plan2, ws2, 1, 1 << 14, "45x38x53 after the larger call")
    assert n2[0] > 0
    # capacity below the count: the canonical prefix and the true count
    plan3 = S.Plan(ctx, (45, 38, 53), 3)
    assert int(n2[0]) > 3
    _check_same(plan3, ws2, 1, 3, "45x38x53, capacity 3")
    # the larger volume again, after the smaller one
    _check_same(plan1, ws1, 1, 1 << 14, "145x174x145 again")


def test_static_scratch_detection_on_a_batch_plan():
    import torch

    import paper_2112_10258_amd as S
    ctx = S.Context(S.default_params(), P.pair_draws())
    vols = [P.noise_blob_volume(s, 300 + i) for i, s in enumerate([(64, 64, 64), (33, 41, 29), (50, 36, 44)])]
    shapes = [(v.shape[2], v.shape[1], v.shape[0]) for v in vols]
    plan = S.Plan(ctx, shapes, 1 << 12, batch=True)
    ws = plan.alloc_workspace()
    plan.build_pyramid(plan.pack_volumes(vols), ws)
    torch.cuda.synchronize()
    counts = _check_same(plan, ws, len(vols), 1 << 12, "batch of 3 volumes")
    assert all(c > 0 for c in counts)


def test_static_scratch_refuses_plans_beyond_its_size():
    import torch

    import paper_2112_10258_amd as S
    ctx = S.Context(S.default_params(), P.pair_draws())
    plan = S.Plan(ctx, (1024, 1024, 512), 16)
    need = plan.detect_scratch_bytes()
    assert need > S.DETECT_STATIC_SCRATCH
    ws = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda")
    kp = torch.zeros(16 * S.KEYPOINT_BYTES, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(S.Sift3dError) as ei:
        plan.detect_static(ws, kp, cnt)
    assert ei.value.code == S.sift3d.E_SCRATCH
    _say(f"1024x1024x512 plan needs {need} B of detection scratch: refused with E_SCRATCH")
