#!/usr/bin/env python3
"""Benchmark of the 3D SIFT-Rank hot path on one MI355X.

A step is one whole extraction (Gaussian/DoG pyramid with sub-sampling,
4D extremum detection with ordered compaction, SIFT-Rank + BRIEF + RRIEF
descriptors) of one synthetic volume already resident in HBM. Prints one
JSON line on stdout; diagnostics go to stderr.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload config2]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "config1": ("64x64x64 smoothed noise + 24 blobs, 2 octaves", dict(n_octaves=2)),
    "config2": ("145x174x145 brain-like phantom, full pyramid to min dim 16", {}),
    "config4": ("512x512x384 smoothed noise + 4000 blobs, full pyramid to min dim 16", {}),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_volume(name):
    from gen import phantoms as P
    return {"config1": P.config1, "config2": P.config2, "config4": P.config4}[name]()


def time_calls(fn, reps, stream):
    """Average ms of fn() over reps calls, HIP events on the launch stream."""
    import torch
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record(stream)
    for _ in range(reps):
        fn()
    e.record(stream)
    e.synchronize()
    return s.elapsed_time(e) / reps


PMC_SUMMARY = os.path.join(ROOT, "profiles", "pyramid_pass_hbm_traffic.json")
COPY_BYTES = 1 << 30


def kernel_source_hash():
    """Hash of the pyramid kernel sources and their shared header."""
    h = hashlib.sha256()
    for f in ("pyramid.hip", "pyramid_tall.hip", "pyramid_kernel.h", "separable.hip", "sift3d_internal.h"):
        with open(os.path.join(ROOT, "paper_2112_10258_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(workload):
    """Measured bytes beyond L2 per octave-0 level pass from the committed
    counter summary, or None if absent or taken on a different kernel source."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    try:
        d = json.load(open(PMC_SUMMARY))
    except ValueError:
        return None
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    w = d.get("workloads", {}).get(workload)
    return None if w is None else w.get("hbm_bytes_per_launch")


def octave0_grids(shape_xyz):
    """Grid sizes (threads) of a solo octave-0 level pass: fused, xy, z."""
    nx, ny, nz = shape_xyz
    cdiv = lambda a, b: (a + b - 1) // b  # noqa: E731
    tiles = cdiv(nx, 64) * cdiv(ny, 16)
    planes = 4   # planes per xy block, as the plan picks them
    while planes > 1 and tiles * cdiv(nz, planes) < 1024:
        planes //= 2
    return {"xy": tiles * cdiv(nz, planes) * 256, "z": cdiv(nx, 32) * cdiv(ny, 8) * cdiv(nz, 16) * 256}


def summarize_pmc(fetch_dir, write_dir, workloads, out_path, reps):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of two rocprofv3 --pmc runs
    of this script (with --copy-calibration) -> bytes per octave-0 level pass
    G_1..G_5, scaled by what the same counters read for a 1 GiB device copy.

    Level i of octave 0 (default parameters: radii 4, 5, 6, 8, 10) runs on the
    fused pass when the octave has >= 24M voxels, or >= 2M voxels and radius
    <= 8 (the plan's rule); its dispatches are blur_level_kernel<R, true, *>
    at the largest grid of that instantiation. Otherwise it is the xy + z
    pair launched alone, at the octave-0 grids of those kernels. The counter
    runs use --pmc-passes reps, whose last dispatches are the octave-0 passes
    launched alone, reps times each."""
    import csv
    import glob
    import re

    def rows(d, counter):
        fs = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not fs:
            raise SystemExit(f"no counter_collection.csv under {d}")
        out = []
        for f in fs:
            for r in csv.DictReader(open(f)):
                if r.get("Counter_Name") == counter:
                    name = (r["Kernel_Name"].replace("void ", "").replace("s3d::(anonymous namespace)::", "")
                            .replace("s3d::fused::", ""))
                    out.append((name, int(r["Grid_Size"]), float(r["Counter_Value"])))
        return out

    fr, wr = rows(fetch_dir, "FETCH_SIZE"), rows(write_dir, "WRITE_SIZE")

    def copy_kib(rs):
        c = [v for k, g, v in rs if ("copy" in k.lower() or "elementwise" in k.lower()) and v * 1024 > COPY_BYTES / 2]
        if not c:
            raise SystemExit("copy calibration dispatch not found")
        return float(np.median(c))

    cf, cw = copy_kib(fr), copy_kib(wr)
    f_factor, w_factor = COPY_BYTES / (cf * 1024), COPY_BYTES / (cw * 1024)
    calib = {"bytes": COPY_BYTES, "fetch_kib": cf, "write_kib": cw,
             "fetch_factor": round(f_factor, 4), "write_factor": round(w_factor, 4)}
    out = {"what": "bytes beyond L2 (TCC FETCH_SIZE + WRITE_SIZE) per octave-0 level pass G_1..G_5, "
                   "scaled by the counters' reading on a plain 1 GiB device copy",
           "kernel_source_sha256_16": kernel_source_hash(), "workloads": {}}
    if os.path.exists(out_path):
        try:
            old = json.load(open(out_path))
            if old.get("kernel_source_sha256_16") == out["kernel_source_sha256_16"]:
                out["workloads"] = old.get("workloads", {})
        except ValueError:
            pass
    fused_re = re.compile(r"^blur_level_kernel<(\d+), (true|false)")

    def fused_sel(rs, R):
        # the --pmc-passes runs end with the octave-0 passes: the last reps
        # dispatches of this instantiation
        ds = [v for k, g, v in rs if (m := fused_re.match(k)) and int(m.group(1)) == R and m.group(2) == "true"]
        return ds[-reps:]

    for wl, shape in workloads.items():
        n = int(np.prod(shape))
        grids = octave0_grids(shape)
        levels = []
        for i, R in enumerate((4, 5, 6, 8, 10), start=1):
            fused = n >= (24 << 20) or (n >= (2 << 20) and R <= 8)
            if fused:
                f, w = fused_sel(fr, R), fused_sel(wr, R)
                kern = f"blur_level_kernel<{R}>"
            else:
                f = [sum(v) for v in zip(*[[v for k, g, v in fr if k.startswith(kn) and g == grids[key]][-reps:]
                                           for kn, key in (("blur_xy_kernel", "xy"), ("blur_z_kernel", "z"))])]
                w = [sum(v) for v in zip(*[[v for k, g, v in wr if k.startswith(kn) and g == grids[key]][-reps:]
                                           for kn, key in (("blur_xy_kernel", "xy"), ("blur_z_kernel", "z"))])]
                kern = "blur_xy_kernel + blur_z_kernel"
            if not f or not w:
                continue
            levels.append({"level": f"G_{i}", "radius": R, "kernel": kern, "dispatches": len(f),
                           "fetch_bytes": int(np.mean(f) * 1024 * f_factor),
                           "write_bytes": int(np.mean(w) * 1024 * w_factor)})
        if not levels:
            continue
        tot = float(np.mean([lv["fetch_bytes"] + lv["write_bytes"] for lv in levels]))
        out["workloads"][wl] = {"shape_xyz": list(shape), "levels": levels, "hbm_bytes_per_launch": int(tot),
                                "copy_calibration": calib, "fetch_dir": fetch_dir, "write_dir": write_dir}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out, indent=1))


def octave0_roofline(plan, passes, pass_ms, workload):
    """Roofline of the octave-0 level passes G_1..G_{S+2} (blur + DoG +
    sub-sample): algorithmic bytes per pass over its measured duration."""
    sel = [i for i, p in enumerate(passes) if p[0] == 0 and p[1] > 0]
    names = {1: "blur_level_kernel", 2: "blur_compact_kernel", 0: "blur_xy_kernel + blur_z_kernel"}
    kparts = []
    for path in (1, 2, 0):
        lv = [f"G_{passes[i][1]}" for i in sel if passes[i][5] == path]
        if lv:
            kparts.append(names[path] + " (" + ", ".join(lv) + ")")
    bytes_per_launch = sum(passes[i][4] for i in sel) / len(sel)
    dur_ms = sum(pass_ms[i] for i in sel) / len(sel)
    achieved = bytes_per_launch / (dur_ms * 1e-3) / 1e9
    return {
        "kernel": " + ".join(kparts) + ": octave-0 pyramid level passes (blur + DoG + sub-sample)",
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": read_traffic(workload),
        "bytes_per_launch": int(bytes_per_launch),
        "avg_launch_us": round(dur_ms * 1e3, 3),
    }


def match_throughput(stream, n=16384, reps=5):
    """Nearest-neighbour matching (sift3d_match) of n x n seeded synthetic
    descriptors: 64-element rank vectors (random permutations, as SIFT-Rank
    rows are) and 4-word BRIEF rows. Reported as pairs compared per second."""
    import torch

    import paper_2112_10258_amd as S
    rng = np.random.default_rng(2112)
    A = torch.from_numpy(np.argsort(rng.random((n, 64)), axis=1).astype(np.uint8)).cuda()
    B = torch.from_numpy(np.argsort(rng.random((n, 64)), axis=1).astype(np.uint8)).cuda()
    Wa = torch.from_numpy(rng.integers(-2 ** 63, 2 ** 63 - 1, size=(n, 4), dtype=np.int64)).cuda()
    Wb = torch.from_numpy(rng.integers(-2 ** 63, 2 ** 63 - 1, size=(n, 4), dtype=np.int64)).cuda()
    torch.cuda.synchronize()
    out = {"pairs": n * n}
    for name, a, b, kind in (("siftrank64", A, B, S.MATCH_RANKS), ("brief256", Wa, Wb, S.MATCH_BRIEF)):
        S.match(a, b, kind, stream)
        ms = time_calls(lambda: S.match(a, b, kind, stream), reps, stream)
        out[name] = {"ms": round(ms, 4), "g_pairs_per_s": round(n * n / (ms * 1e-3) / 1e9, 2)}
    return out


def large_volume_roofline(stream, reps):
    """The same roofline on the 512x512x384 volume (config 4), whose levels
    do not fit the last-level cache: the fused pass against HBM."""
    import torch

    import paper_2112_10258_amd as S
    from gen import phantoms as P
    vol = P.config4()
    nz, ny, nx = vol.shape
    ctx = S.Context(S.default_params(), P.pair_draws())
    plan = S.Plan(ctx, (nx, ny, nz), 1 << 17)
    buf = S.Buffers(plan)
    dvol = torch.from_numpy(vol).cuda()
    for _ in range(2):
        S.run_extract(plan, dvol, buf, stream=stream)
    torch.cuda.synchronize()
    ms = time_calls(lambda: S.run_extract(plan, dvol, buf, stream=stream), 3, stream)
    passes = plan.pyramid_passes()
    pass_ms = [time_calls(lambda i=i: plan.pyramid_pass(i, dvol, buf.ws, stream), reps, stream)
               if p[0] == 0 else 0.0 for i, p in enumerate(passes)]
    out = octave0_roofline(plan, passes, pass_ms, "config4")
    out["workload"] = "config4: 512x512x384 smoothed noise + 4000 blobs"
    out["ms_per_extraction"] = round(ms, 4)
    # uniform-filter approximation of the largest increment (sigma 3.09,
    # three passes per axis) on the same volume, beside the Gaussian pass
    # that computes that level (blur + DoG)
    box_out, box_tmp = torch.empty_like(dvol), torch.empty_like(dvol)
    h = S.box_half_width(3.09, 3)
    S.box_blur(dvol, h, 3, box_out, box_tmp, stream)
    box_ms = time_calls(lambda: S.box_blur(dvol, h, 3, box_out, box_tmp, stream), reps, stream)
    g5 = [i for i, p in enumerate(passes) if p[0] == 0 and p[1] == 5]
    out["box"] = {"sigma": 3.09, "passes": 3, "half_width": h, "ms": round(box_ms, 4),
                  "algorithmic_gb_per_s": round(3 * 8 * dvol.numel() / (box_ms * 1e-3) / 1e9, 1),
                  "gaussian_level_pass_ms": round(pass_ms[g5[0]], 4) if g5 else None}
    del box_out, box_tmp
    del buf, plan, dvol
    torch.cuda.empty_cache()
    return out


def batch_vs_plain(steps, stream, extra):
    """32 mixed-size volumes (each axis U{96..192}): one batch-plan call per step
    against 32 one-volume calls per step. Inputs resident in HBM."""
    import torch

    import paper_2112_10258_amd as S
    from gen import phantoms as P
    vols = P.config3()
    shapes = [(v.shape[2], v.shape[1], v.shape[0]) for v in vols]
    cap = 1 << 14
    ctx = S.Context(S.default_params(**extra), P.pair_draws())
    bplan = S.Plan(ctx, shapes, cap, batch=True)
    bbuf = S.Buffers(bplan)
    packed = bplan.pack_volumes(vols)
    plain = []
    for v, sh in zip(vols, shapes):
        pl = S.Plan(ctx, sh, cap)
        plain.append((pl, S.Buffers(pl), torch.from_numpy(v).cuda()))

    def batched():
        S.run_extract(bplan, packed, bbuf, stream=stream)

    def one_by_one():
        for pl, b, dv in plain:
            S.run_extract(pl, dv, b, stream=stream)

    for _ in range(2):
        batched()
        one_by_one()
    torch.cuda.synchronize()
    ms_b = time_calls(batched, steps, stream)
    ms_p = time_calls(one_by_one, steps, stream)
    n = len(vols)
    counts_b = bbuf.count.cpu().tolist()
    counts_p = [int(b.count.item()) for _, b, _ in plain]
    vox = sum(int(np.prod(sh)) for sh in shapes)
    del bbuf, plain
    torch.cuda.empty_cache()
    return {
        "workload": "config3: 32 smoothed-noise + blob volumes, each axis U{96..192}",
        "volumes": n,
        "voxels": vox,
        "batched_ms_per_call": round(ms_b, 4),
        "batched_volumes_per_s": round(n * 1000.0 / ms_b, 1),
        "plain_ms_for_all": round(ms_p, 4),
        "plain_volumes_per_s": round(n * 1000.0 / ms_p, 1),
        "batched_vs_plain": round(ms_p / ms_b, 3),
        "keypoints_total": int(sum(counts_b)),
        "same_counts_as_plain": counts_b == counts_p,
    }


def _pct(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q))


def serve_vs_plain(n_req, rate, pool_per_class, n_streams, max_inflight, max_batch, budget_gb, stream, extra):
    """The config-5 request stream through the server against a plain
    one-request-at-a-time loop: saturated throughput (all requests queued at
    once) and latency at the Poisson arrival rate. Volumes come from a pool of
    pool_per_class distinct volumes per size class, resident in HBM."""
    import threading

    import torch

    import paper_2112_10258_amd as S
    from gen import phantoms as P
    reqs = P.config5_requests(n_req, rate)
    sizes = list(P.CONFIG5_SIZES)
    pool = {}
    t0 = time.perf_counter()
    for c, sh in enumerate(sizes):
        pool[sh] = [torch.from_numpy(P.noise_blob_volume(sh, 5000 + 100 * c + j)).cuda()
                    for j in range(pool_per_class)]
    torch.cuda.synchronize()
    log(f"[bench] serve: pool of {pool_per_class} volumes per size class built in {time.perf_counter() - t0:.1f} s")
    work = [(arr, sh, pool[sh][i % pool_per_class], i % pool_per_class) for i, (arr, sh, _) in enumerate(reqs)]
    cap = 1 << 14
    ctx = S.Context(S.default_params(**extra), P.pair_draws())

    # plain path: one plan and buffer set per shape, one request per call
    plans = {sh: S.Plan(ctx, sh, cap) for sh in sizes}
    bufs = {sh: S.Buffers(plans[sh]) for sh in sizes}
    plain_counts = {}
    for sh in sizes:
        for j in range(pool_per_class):
            S.run_extract(plans[sh], pool[sh][j], bufs[sh], stream=stream)
            torch.cuda.synchronize()
            plain_counts[(sh, j)] = int(bufs[sh].count.item())

    def plain_all():
        for _, sh, dv, _ in work:
            S.run_extract(plans[sh], dv, bufs[sh], stream=stream)

    plain_all()
    torch.cuda.synchronize()
    ms_plain = time_calls(plain_all, 1, stream)

    # plain loop at the arrival rate: each request runs when it has arrived and
    # the previous one is done
    lat_plain = []
    t_begin = time.perf_counter()
    for arr, sh, dv, _ in work:
        while time.perf_counter() - t_begin < arr:
            time.sleep(min(1e-4, max(0.0, arr - (time.perf_counter() - t_begin))))
        S.run_extract(plans[sh], dv, bufs[sh], stream=stream)
        stream.synchronize()
        lat_plain.append(time.perf_counter() - t_begin - arr)
    wall_plain = time.perf_counter() - t_begin
    del bufs, plans
    torch.cuda.empty_cache()

    srv = S.Server(ctx, hbm_budget=int(budget_gb * (1 << 30)), n_streams=n_streams, max_inflight=max_inflight,
                   kp_capacity=cap, max_batch=max_batch)
    mismatch = 0

    def run(items, paced):
        """Submit items (at their arrival times if paced) from one thread while
        this one collects and releases results in order."""
        nonlocal mismatch
        tickets, times = [], []
        cv = threading.Condition()

        def submitter():
            t_begin = time.perf_counter()
            for arr, _, dv, _ in items:
                if paced:
                    while time.perf_counter() - t_begin < arr:
                        time.sleep(min(1e-4, max(0.0, arr - (time.perf_counter() - t_begin))))
                t = srv.submit(dv)
                with cv:
                    tickets.append(t)
                    cv.notify()

        sub = threading.Thread(target=submitter)
        t0 = time.perf_counter()
        sub.start()
        for k in range(len(items)):
            with cv:
                while len(tickets) <= k:
                    cv.wait()
                t = tickets[k]
            r = srv.result(t)
            if r.status != 0 or r.count != plain_counts[(items[k][1], items[k][3])]:
                mismatch += 1
            times.append((r.t_submit, r.t_start, r.t_done))
            srv.release(t)
        sub.join()
        return times, time.perf_counter() - t0

    run(work[:100], False)          # warm the plan and slot caches
    mismatch = 0
    times, _ = run(work, False)     # saturated: all requests queued at once
    served_sat = len(work) / (max(t[2] for t in times) - min(t[0] for t in times))
    times, wall_served = run(work, True)   # Poisson arrivals
    lat_served = [d - s for s, _, d in times]
    st = srv.stats()
    srv.close()
    del pool
    torch.cuda.empty_cache()
    plain_sat = len(work) * 1000.0 / ms_plain
    return {
        "workload": f"config5: {n_req} requests, Poisson {rate:g}/s, sizes {sizes} w.p. {list(P.CONFIG5_PROBS)}",
        "volumes_pool": f"{pool_per_class} distinct volumes per size class (request i uses volume i mod {pool_per_class})",
        "server": {"n_streams": n_streams, "max_inflight": max_inflight, "max_batch": max_batch,
                   "hbm_budget_gb": budget_gb, "groups": st["groups"],
                   "mean_group_size": round(st["grouped_requests"] / max(st["groups"], 1), 2),
                   "peak_allocated_gb": round(st["peak_allocated"] / 2**30, 3),
                   "slot_allocations": st["slot_allocations"], "slot_evictions": st["slot_evictions"]},
        "saturated": {"served_volumes_per_s": round(served_sat, 1), "plain_volumes_per_s": round(plain_sat, 1),
                      "served_vs_plain": round(served_sat / plain_sat, 3)},
        "poisson": {"served_p50_ms": round(_pct(lat_served, 50) * 1e3, 3),
                    "served_p99_ms": round(_pct(lat_served, 99) * 1e3, 3),
                    "served_volumes_per_s": round(len(work) / wall_served, 1),
                    "plain_p50_ms": round(_pct(lat_plain, 50) * 1e3, 3),
                    "plain_p99_ms": round(_pct(lat_plain, 99) * 1e3, 3),
                    "plain_volumes_per_s": round(len(work) / wall_plain, 1)},
        "count_mismatches_vs_plain": mismatch,
    }


def cpu_baseline(vol, kw, budget_s):
    import oracle as O
    from gen import phantoms as P
    from tests.helpers import oracle_params
    import paper_2112_10258_amd as S
    p = oracle_params(S.default_params(**kw))
    draws = P.pair_draws()
    n, t0 = 0, time.perf_counter()
    while True:
        O.extract(vol, p, draws)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 50:
            break
    return n, el, O.max_threads()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="config2", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pass-reps", type=int, default=20)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain measurement")
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--no-serve", action="store_true", help="skip the request-server measurement")
    ap.add_argument("--no-large", action="store_true", help="skip the 512x512x384 roofline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB on the device a few times (reference dispatch for counter runs)")
    ap.add_argument("--pmc-passes", type=int, default=0,
                    help="counter runs: after the warm-up, launch each octave-0 level pass this many times and exit")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the traffic summary from two rocprofv3 --pmc runs and exit (no GPU)")
    ap.add_argument("--pyramid-mode", type=int, default=None, choices=[0, 1, 2, 3],
                    help="0 = by octave size, 1 = fused streaming passes, 2 = xy + z launches, 3 = compact passes")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-pool", type=int, default=4)
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--serve-inflight", type=int, default=8)
    ap.add_argument("--serve-batch", type=int, default=8, help="largest group of same-shape requests")
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    args = ap.parse_args()
    if args.summarize_pmc:
        shapes = {"config2": (145, 174, 145), "config4": (512, 512, 384)}
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], {args.workload: shapes[args.workload]},
                      PMC_SUMMARY, args.pmc_passes or 3)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); volumes are independent, "
              "a multi-GPU run would be N copies of this one", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2112_10258_amd as S
    from gen import phantoms as P

    if args.copy_calibration:
        a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()

    desc, kw = WORKLOADS[args.workload]
    extra = {} if args.pyramid_mode is None else {"pyramid_mode": args.pyramid_mode}
    kw = dict(kw, **extra)
    log(f"[bench] workload {args.workload}: {desc}")
    vol = make_volume(args.workload)
    nz, ny, nx = vol.shape
    cap = 1 << 17
    ctx = S.Context(S.default_params(**kw), P.pair_draws())
    plan = S.Plan(ctx, (nx, ny, nz), cap)
    buf = S.Buffers(plan)
    dvol = torch.from_numpy(vol).cuda()
    stream = torch.cuda.current_stream()

    def step():
        S.run_extract(plan, dvol, buf, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if args.pmc_passes:
        passes = plan.pyramid_passes()
        for i, p in enumerate(passes):
            if p[0] == 0 and p[1] > 0:
                for _ in range(args.pmc_passes):
                    plan.pyramid_pass(i, dvol, buf.ws, stream)
        torch.cuda.synchronize()
        log(f"[bench] octave-0 level passes launched {args.pmc_passes} times each for the counters")
        return
    count = int(buf.count.item())
    log(f"[bench] {plan.n_octaves} octaves, workspace {plan.workspace_bytes / 2**20:.1f} MiB, {count} keypoints")

    # timed region: K whole steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_step = time_calls(step, args.steps, stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = 1000.0 / ms_step
    log(f"[bench] {args.steps} steps: {ms_step:.4f} ms/step (events), wall {wall * 1e3 / args.steps:.4f} ms/step")

    # stage and pass breakdown (separate, after the timed region)
    reps = args.pass_reps
    st_pyr = time_calls(lambda: plan.build_pyramid(dvol, buf.ws, stream), reps, stream)
    st_det = time_calls(lambda: plan.detect(buf.ws, buf.kp, buf.count, stream), reps, stream)
    st_sr = time_calls(lambda: plan.describe(buf.ws, buf.kp, buf.count, siftrank=buf.siftrank, stream=stream),
                       reps, stream)
    st_br = time_calls(lambda: plan.describe(buf.ws, buf.kp, buf.count, brief=buf.brief, rrief=buf.rrief,
                                             stream=stream), reps, stream)
    passes = plan.pyramid_passes()
    pass_ms = []
    for i in range(len(passes)):
        pass_ms.append(time_calls(lambda i=i: plan.pyramid_pass(i, dvol, buf.ws, stream), reps, stream))
    log("[bench] stages ms: pyramid %.4f detect %.4f siftrank %.4f brief+rrief %.4f"
        % (st_pyr, st_det, st_sr, st_br))
    for (o, lev, r, sub, b, fused, vv), t in zip(passes, pass_ms):
        log(f"[bench]   pass o={o} G{lev} r={r} sub={sub}: {t * 1e3:.2f} us, {b / t / 1e6:.0f} GB/s algorithmic")

    roofline = octave0_roofline(plan, passes, pass_ms, args.workload)
    large = box = None
    if not args.no_large and args.workload != "config4":
        del buf
        torch.cuda.empty_cache()
        large = large_volume_roofline(stream, max(3, reps // 4))
        box = large.pop("box")
        log(f"[bench] roofline 512x512x384: {large}")
        log(f"[bench] box blur 512x512x384: {box}")

    match = match_throughput(stream)
    log(f"[bench] match: {match}")

    batch = None
    if not args.no_batch:
        torch.cuda.empty_cache()
        batch = batch_vs_plain(args.batch_steps, stream, extra)
        log(f"[bench] batch: {batch}")

    serve = None
    if not args.no_serve:
        serve = serve_vs_plain(args.serve_requests, args.serve_rate, args.serve_pool, args.serve_streams,
                               args.serve_inflight, args.serve_batch, args.serve_budget_gb, stream, extra)
        log(f"[bench] serve: {serve}")

    cpu = None
    if not args.no_cpu_baseline:
        n, el, cores = cpu_baseline(vol, kw, args.cpu_seconds)
        cpu = {"value": round(n / el, 4), "unit": "volumes/s", "cores": cores, "kind": "oracle",
               "sample": f"{n} full extraction(s) of the {args.workload} volume (pyramid, detection, "
                         f"SIFT-Rank, BRIEF, RRIEF) in FP64, {el:.1f} s"}
        log(f"[bench] oracle: {n} volumes in {el:.2f} s on {cores} threads")

    vox = nx * ny * nz
    out = {
        "metric": "volumes/s (plain path, one volume per call)",
        "value": round(value, 2),
        "unit": "volumes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (pyramid, detection); f64 accumulation (descriptors)",
        "data": "synthetic",
        "config": {"workload": args.workload, "shape_xyz": [nx, ny, nz], "octaves": plan.n_octaves,
                   "keypoints": count, "descriptors": ["siftrank64", "brief256", "rrief256"],
                   "parallelism": "single GPU"},
        "voxels_per_s": round(vox * value, 1),
        "stages_ms": {"pyramid": round(st_pyr, 4), "detect": round(st_det, 4), "siftrank": round(st_sr, 4),
                      "brief_rrief": round(st_br, 4)},
        "roofline": roofline,
        "roofline_large_volume": large,
        "batch": batch,
        "serve": serve,
        "match": match,
        "box": box,
        "cpu_baseline": cpu,
        "paper_context": "paper: 1.4 s CPU, 0.2 s GPU per 145x174x145 volume (~3000 keypoints, hardware unnamed)",
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
