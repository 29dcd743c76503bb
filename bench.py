#!/usr/bin/env python3
"""Benchmark of the MI355X wavefront sweep.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-batched] [--no-serving] [--no-cpu]

One step = one sweep of the 16384 x 16384 fp32 grid (min rule, full output):
one persistent kernel launch through the C ABI (wf_solve).  Inputs are
generated on the device from the seeded counter generator before timing, so
the timed region only reads and writes HBM.

Prints ONE JSON line.  Besides the contract fields it carries
  roofline:     the sweep kernel against the 8 TB/s HBM peak (algorithmic bytes:
                4 B read + 4 B written per cell), per-launch time from HIP events
                recorded on the launch stream; `traffic` is the HBM bytes per launch
                from the committed FETCH_SIZE / WRITE_SIZE summary when it was taken
                on the current kernel sources (null otherwise);
  cpu_baseline: the CPU oracle (fp64 row-major loop, one thread) on the same
                workload;
  batched:      4096 grids, m and n log-uniform in [64, 2048], one persistent
                launch (replayed hipGraph) against 4096 separate launches;
  serving:      Poisson arrivals of square grids (n log-uniform in [128, 8192])
                at 0.7x the batched capacity of that mix, 64 GiB budget,
                continuous batching: p50/p99 latency and cells/s.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "sweep16384_memory_counters.md")
KERNEL_SOURCES = ("paper_2501_05938_amd/csrc/wf_kernel.hip", "paper_2501_05938_amd/csrc/wf_internal.h")
M = N = 16384
SEED = 2


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the 65536x65536 edges-mode run")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-grids", type=int, default=256)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-load", type=float, default=0.7)
    ap.add_argument("--serve-inflight", type=int, default=4, help="server launches in flight")
    ap.add_argument("--serve-batch", type=int, default=256, help="server requests per launch at most")
    ap.add_argument("--copy-ref", action="store_true",
                    help="run one plain 1 GiB device-to-device copy first: a kernel of known HBM "
                         "traffic (1 GiB read + 1 GiB written) to scale memory counters by")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_events(torch, fn, steps, stream):
    """Run fn() `steps` times on `stream`; return per-call ms from events on that stream."""
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    for i in range(steps):
        starts[i].record(stream)
        fn()
        ends[i].record(stream)
    torch.cuda.synchronize()
    return [s.elapsed_time(e) for s, e in zip(starts, ends)]


def measured_traffic():
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE summary, or None
    when the kernel sources have changed since those counters were taken."""
    import hashlib
    try:
        text = open(COUNTERS).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() not in text:
        return None
    for line in text.splitlines():
        if line.startswith("traffic_bytes_per_launch:"):
            return float(line.split(":")[1])
    return None


def host_cpu():
    """The host's CPU model and logical CPU count, for the CPU baseline's context."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu": model, "logical_cpus": os.cpu_count()}


def cpu_baseline(seconds: float):
    """The oracle (fp64 row-major loop, one thread) over bands of the same workload
    until `seconds` of CPU time have been spent; cells/s."""
    import numpy as np

    import oracle
    import wfgen

    band = 1024
    done_cells = 0
    spent = 0.0
    top = None
    row0 = 0
    passes = 0
    while spent < seconds:
        if row0 >= M:
            row0, top = 0, None
            passes += 1
        c = wfgen.cells(SEED, M, N, "f32", row0, band)
        left = np.full(band, np.inf)
        t0 = time.process_time()
        lr, _ = oracle.sweep(c, "min", "f64", top=top, left=left, full=False)
        spent += time.process_time() - t0
        top = np.concatenate([[np.inf], lr])
        done_cells += band * N
        row0 += band
    return {"value": done_cells / spent, "unit": "cells/s", "cores": 1, "kind": "oracle", "host": host_cpu(),
            "sample": f"fp64 oracle loop over {done_cells // N} rows of the {M}x{N} seed-{SEED} grid "
                      f"in {band}-row bands ({spent:.1f} s of one core)"}


def large_edges(torch, wf, wfgen, steps=3):
    """The 65536 x 65536 grid (17 GB of fp32 input, device-resident) in edges mode: only
    the last row, last column and final cell are written."""
    m = n = 65536
    c = torch.empty((m, n), dtype=torch.float32, device="cuda")
    wfgen.fill_device(c, seed=3)
    lr = torch.empty(n, dtype=torch.float32, device="cuda")
    lc = torch.empty(m, dtype=torch.float32, device="cuda")
    fc = torch.empty(1, dtype=torch.float32, device="cuda")
    run = lambda: wf.solve(c, mode="edges", last_row=lr, last_col=lc, final_cell=fc)  # noqa: E731
    run()
    torch.cuda.synchronize()
    wf.check()
    per = time_events(torch, run, steps, torch.cuda.current_stream())
    wf.check()
    kms = sum(per) / len(per)
    alg = 4.0 * m * n + 4.0 * (m + n) + 4.0
    achieved = alg / (kms * 1e-3) / 1e9
    del c, lr, lc, fc
    torch.cuda.empty_cache()
    return {"workload": "single 65536x65536 grid, fp32, min rule, edges mode (last row, last column, final cell)",
            "seed": 3, "steps": steps, "kernel_ms": kms, "cells_per_s": m * n / (kms * 1e-3),
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "bytes_per_launch": alg, "bytes_per_cell": 4}}


def batched(torch, wf, wfgen, count):
    """4096 uneven grids: one persistent launch vs 4096 separate launches."""
    shapes = wfgen.batch_shapes(count)
    costs, outs = [], []
    for g, (m, n) in enumerate(shapes):
        t = torch.empty((m, n), dtype=torch.float32, device="cuda")
        wfgen.fill_device(t, seed=wfgen.batch_seed(g))
        costs.append(t)
        outs.append(torch.empty((m, n), dtype=torch.float32, device="cuda"))
    cells = sum(m * n for m, n in shapes)
    stream = torch.cuda.current_stream()
    # batched: graph replay of one persistent launch
    plan = wf.BatchPlan(costs, outs)  # arguments marshalled once, as a loop over fixed buffers would
    for _ in range(2):
        plan.run()
    torch.cuda.synchronize()
    wf.check()
    reps = 5
    bt = time_events(torch, plan.run, reps, stream)
    wf.check()
    # per-grid: one wf_solve launch per grid, back to back, on S streams round-robin
    # (S = 1 is one stream); the best S is the baseline.
    def per_grid(streams):
        for i, (c, o) in enumerate(zip(costs, outs)):
            wf.solve(c, out=o, stream=streams[i % len(streams)])

    per_grid_by_s = {}
    for S in (1, 4, 16):
        streams = [stream] if S == 1 else [torch.cuda.Stream() for _ in range(S)]
        per_grid(streams)
        torch.cuda.synchronize()
        best = None
        for _ in range(2):
            t0 = time.perf_counter()
            per_grid(streams)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) * 1e3
            best = dt if best is None else min(best, dt)
        wf.check()
        per_grid_by_s[S] = best
    s_best = min(per_grid_by_s, key=per_grid_by_s.get)
    b_ms = sorted(bt)[len(bt) // 2]
    p_ms = per_grid_by_s[s_best]
    return {"grids": count, "cells": cells, "batched_ms": b_ms, "per_grid_ms": p_ms,
            "per_grid_streams": s_best, "per_grid_ms_by_streams": per_grid_by_s,
            "batched_cells_per_s": cells / (b_ms * 1e-3), "per_grid_cells_per_s": cells / (p_ms * 1e-3),
            "speedup": p_ms / b_ms,
            "shapes": "m, n independently log-uniform in [64, 2048] (PCG64 seed 4), grid g seed 1000+g"}


def serving(torch, wf, wfgen, grids, requests, load, inflight=4, batch=256):
    """Poisson arrivals of square grids (n log-uniform in [128, 8192]) served under a
    64 GiB budget with continuous batching.  The arrival rate is `load` times the
    batched capacity for the same mix, measured first with one wf_solve_batched
    launch.  Latency = completion observed by the server - submission."""
    import numpy as np

    reqs = wfgen.serving_requests(requests, rate_per_s=1.0)  # unit-rate arrival pattern, rescaled below
    # `grids` distinct grids (the first draws of the recipe); request q serves grid q mod grids.
    sizes = [n for (_, n, _) in reqs[:grids]]
    costs = []
    for g, n in enumerate(sizes):
        t = torch.empty((n, n), dtype=torch.float32, device="cuda")
        wfgen.fill_device(t, seed=50000 + g)
        costs.append(t)
    torch.cuda.synchronize()
    cells = [n * n for n in sizes]
    # capacity of this mix when batched
    outs = [torch.empty_like(c) for c in costs]
    wf.solve_batched(costs, outs, use_graph=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    wf.solve_batched(costs, outs, use_graph=0)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    wf.check()
    del outs
    cap = grids / t_batch
    rate = load * cap
    arrivals = [a / rate for (a, _, _) in reqs]
    lat, cells_done = [], 0
    with wf.Server(budget_bytes=64 << 30, max_inflight=inflight, max_batch=batch) as srv:
        # warm-up: one request of each distinct grid is not needed; a short burst warms the path
        for g in range(min(8, grids)):
            tk = srv.submit(costs[g])
            while srv.poll_times(tk) is None:
                time.sleep(1e-4)
            srv.release(tk)
        outstanding = {}
        t_start = time.perf_counter()
        i = 0
        first_submit, last_done = None, 0.0
        lag = []
        while i < len(arrivals) or outstanding:
            now = time.perf_counter()
            while i < len(arrivals) and t_start + arrivals[i] <= now:
                g = i % grids
                tk = srv.submit(costs[g])
                outstanding[tk] = (g, t_start + arrivals[i])
                i += 1
            progressed = False
            for tk in list(outstanding)[:32]:
                ts = srv.poll_times(tk)
                if ts is None:
                    continue
                g, t_arr = outstanding.pop(tk)
                srv.release(tk)
                lat.append(ts[3] - ts[0])
                lag.append(ts[0] - t_arr)
                cells_done += cells[g]
                first_submit = ts[0] if first_submit is None else min(first_submit, ts[0])
                last_done = max(last_done, ts[3])
                progressed = True
            if not progressed and (i >= len(arrivals) or t_start + arrivals[i] > time.perf_counter() + 2e-4):
                time.sleep(1e-4)
        peak = srv.memory()[1]
        # results served in the mix equal the same grids swept alone
        checked = 0
        for g in range(min(4, grids)):
            tks = [srv.submit(costs[(g + h) % grids]) for h in range(5)]  # g with 4 companions
            while any(srv.poll_times(t) is None for t in tks):
                time.sleep(1e-4)
            r = srv.poll(tks[0])
            alone = wf.solve(costs[g])
            same = torch.equal(r["out"], alone)
            torch.cuda.current_stream().synchronize()
            if not same:
                raise AssertionError(f"served grid {g} differs from the grid swept alone")
            for t in tks:
                srv.release(t)
            checked += 1
    torch.cuda.synchronize()
    wf.check()
    lat = np.array(lat) * 1e3
    span = last_done - first_submit
    return {"requests": len(arrivals), "distinct_grids": grids,
            "n": "log-uniform in [128, 8192] (PCG64 seed 5), grid g seed 50000+g, request q serves grid q mod %d" % grids,
            "batched_capacity_req_per_s": cap, "load": load, "rate_req_per_s": rate,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "cells_per_s": cells_done / span,
            "submit_lag_p99_ms": float(np.percentile(np.array(lag) * 1e3, 99)),
            "peak_server_bytes": peak, "budget_bytes": 64 << 30, "checked_equal_alone": checked,
            "max_inflight": inflight, "max_batch": batch}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sweep's multi-GPU "
              f"row-band split is a design note, not a measured path", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2501_05938_amd as wf
    import wfgen

    if not torch.cuda.is_available():
        print("no GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    log(f"[bench] device {torch.cuda.get_device_name(0)}; filling {M}x{N} fp32 input on the device")
    cost = torch.empty((M, N), dtype=torch.float32, device=dev)
    wfgen.fill_device(cost, seed=SEED)
    out = torch.empty((M, N), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()

    if args.copy_ref:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] reference copy: 1 GiB read + 1 GiB written")
    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        wf.solve(cost, out=out)
    torch.cuda.synchronize()
    wf.check()

    log(f"[bench] timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per = time_events(torch, lambda: wf.solve(cost, out=out), args.steps, stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    wf.check()
    ms_per_step = wall * 1e3 / args.steps
    kernel_ms = sum(per) / len(per)
    cells = M * N
    value = cells * args.steps / wall
    alg_bytes = 8.0 * cells
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    result = {
        "metric": "grid cells/s + % HBM roofline at n=16384; batched vs per-grid; p99 latency",
        "value": value,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (SplitMix64 uniform [0,1) fp32 inputs generated on the device)",
        "config": {"workload": "single 16384x16384 grid, fp32, min rule, default boundary, full output",
                   "m": M, "n": N, "seed": SEED, "rule": "min", "mode": "full"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel_ms": kernel_ms, "kernel_ms_min": min(per),
                     "bytes_per_launch": alg_bytes, "bytes_per_cell": 8},
    }
    if not args.no_large:
        log("[bench] 65536x65536 edges mode")
        try:
            result["large_edges"] = large_edges(torch, wf, wfgen)
        except Exception as e:  # report, do not lose the main line
            result["large_edges"] = {"error": repr(e)}
    if not args.no_batched:
        log(f"[bench] batched: {args.batch_count} grids")
        try:
            result["batched"] = batched(torch, wf, wfgen, args.batch_count)
        except Exception as e:  # report, do not lose the main line
            result["batched"] = {"error": repr(e)}
    if not args.no_serving:
        log(f"[bench] serving: {args.serve_requests} requests over {args.serve_grids} grids")
        try:
            result["serving"] = serving(torch, wf, wfgen, args.serve_grids, args.serve_requests, args.serve_load,
                                        args.serve_inflight, args.serve_batch)
        except Exception as e:  # report, do not lose the main line
            result["serving"] = {"error": repr(e)}
        # The same mix at a light and a heavy load (half as many requests each).
        others = {}
        for load in (0.3, 0.9):
            log(f"[bench] serving at load {load}")
            try:
                r = serving(torch, wf, wfgen, args.serve_grids, max(args.serve_requests // 2, 1), load,
                            args.serve_inflight, args.serve_batch)
                others[str(load)] = {k: r[k] for k in ("requests", "rate_req_per_s", "p50_ms", "p99_ms", "cells_per_s")}
            except Exception as e:  # report, do not lose the main line
                others[str(load)] = {"error": repr(e)}
        result["serving"]["other_loads"] = others
    if not args.no_cpu:
        log(f"[bench] cpu baseline ({args.cpu_seconds:.0f} s of one core)")
        result["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
