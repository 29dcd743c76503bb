#!/usr/bin/env python3
"""Benchmark of the MI355X wavefront sweep.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-large] [--no-batched]
                    [--no-serving] [--no-copy-serving] [--no-fp64] [--no-dtw] [--no-cpu]

One step = one sweep of the 16384 x 16384 fp32 grid (min rule, full output):
one persistent kernel launch through the C ABI (wf_solve).  Inputs are
generated on the device from the seeded counter generator before timing, so
the timed region only reads and writes HBM.

Prints ONE JSON line.  Besides the contract fields it carries
  roofline:     the sweep kernel against the 8 TB/s HBM peak (algorithmic bytes:
                4 B read + 4 B written per cell), per-launch time from HIP events
                recorded on the launch stream; `traffic` is the HBM bytes per launch
                from the committed FETCH_SIZE / WRITE_SIZE summary when it was taken
                on the current kernel sources (null otherwise); `latency` is the
                second bound: m + n - 1 dependent steps of the walk's chain, each
                as long as the device measures it;
  cpu_baseline: the CPU oracle (fp64 row-major loop, one pinned core) on the same
                workload;
  large_edges:  the 65536 x 65536 grid in edges mode;
  fp64:         the 16384 x 16384 grid in fp64 (16 B per cell);
  dtw:          dynamic time warping of two 16384-long sequences (inputs |x_i - y_j|
                computed on the device), edges mode and full mode;
  traceback:    the path back from the last cell of the 16384 x 16384 grid;
  batched:      4096 grids, m and n log-uniform in [64, 2048], one persistent
                launch (replayed hipGraph) against 4096 separate launches on 1..32
                streams, with the paper's stream-count model (Sections 2.3-2.4)
                fitted to per-grid timings of this device and its choice of
                stream count beside the measured best;
  serving:      Poisson arrivals of square grids (n log-uniform in [128, 8192])
                at 0.7x the batched capacity of that mix, 64 GiB budget,
                continuous batching: p50/p99 latency (poll-observed completion
                minus scheduled arrival) and cells/s, over 10000 requests after
                500 warm-up ones;
  copy_serving: a burst of host-resident (pinned) requests served with their
                copies on the launch stream vs on copy streams that overlap
                earlier launches, with the two-stage flow-shop prediction.
"""
from __future__ import annotations

import argparse
import json
import math
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
    ap.add_argument("--no-model", action="store_true", help="skip the stream-count model calibration")
    ap.add_argument("--no-large", action="store_true", help="skip the 65536x65536 edges-mode run")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-dtw", action="store_true", help="skip dynamic time warping and the traceback")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-copy-serving", action="store_true")
    ap.add_argument("--serve-grids", type=int, default=256)
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--serve-warmup", type=int, default=500)
    ap.add_argument("--serve-load", type=float, default=0.7)
    ap.add_argument("--serve-inflight", type=int, default=2, help="server launches in flight")
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


def median(v):
    v = sorted(v)
    return v[len(v) // 2]


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
    """The oracle (fp64 row-major loop) on one host core, pinned, over bands of the same
    workload until `seconds` of CPU time have been spent; cells/s."""
    import numpy as np

    import oracle
    import wfgen

    before = os.sched_getaffinity(0)
    core = min(before)
    os.sched_setaffinity(0, {core})
    try:
        band = 1024
        done_cells = 0
        spent = 0.0
        top = None
        row0 = 0
        while spent < seconds:
            if row0 >= M:
                row0, top = 0, None
            c = wfgen.cells(SEED, M, N, "f32", row0, band)
            left = np.full(band, np.inf)
            t0 = time.process_time()
            lr, _ = oracle.sweep(c, "min", "f64", top=top, left=left, full=False)
            spent += time.process_time() - t0
            top = np.concatenate([[np.inf], lr])
            done_cells += band * N
            row0 += band
    finally:
        os.sched_setaffinity(0, before)
    return {"value": done_cells / spent, "unit": "cells/s", "cores": 1, "kind": "oracle", "host": host_cpu(),
            "pinned_core": core,
            "sample": f"fp64 oracle loop over {done_cells // N} rows of the {M}x{N} seed-{SEED} grid "
                      f"in {band}-row bands ({spent:.1f} s of one core, pinned to core {core})"}


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


def fp64_leg(torch, wf, wfgen, steps=5):
    """The 16384 x 16384 grid in fp64 (53-bit uniform [0, 1) inputs from the seeded
    generator, filled on the device): 16 B per cell of algorithmic traffic."""
    c = torch.empty((M, N), dtype=torch.float64, device="cuda")
    wfgen.fill_device(c, seed=SEED)
    out = torch.empty_like(c)
    run = lambda: wf.solve(c, out=out)  # noqa: E731
    run()
    torch.cuda.synchronize()
    wf.check()
    per = time_events(torch, run, steps, torch.cuda.current_stream())
    wf.check()
    kms = sum(per) / len(per)
    alg = 16.0 * M * N
    achieved = alg / (kms * 1e-3) / 1e9
    del c, out
    torch.cuda.empty_cache()
    return {"workload": "single 16384x16384 grid, fp64, min rule, full output", "seed": SEED, "steps": steps,
            "kernel_ms": kms, "cells_per_s": M * N / (kms * 1e-3),
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "bytes_per_launch": alg, "bytes_per_cell": 16}}


def dtw_leg(torch, wf, wfgen, step_ns, steps=5):
    """Dynamic time warping of two 16384-long sequences (cell inputs |x_i - y_j| computed on
    the device): edges mode (the distance and the last row / column; HBM traffic O(m + n),
    so the bound is the walk's latency) and full mode (the whole cost matrix written:
    4 B per cell)."""
    x = torch.empty((1, M), dtype=torch.float32, device="cuda")
    y = torch.empty((1, N), dtype=torch.float32, device="cuda")
    wfgen.fill_device(x, seed=41)
    wfgen.fill_device(y, seed=42)
    x, y = x[0], y[0]
    lr = torch.empty(N, device="cuda"); lc = torch.empty(M, device="cuda"); fc = torch.empty(1, device="cuda")
    out = torch.empty((M, N), dtype=torch.float32, device="cuda")
    res = {"workload": "dynamic time warping of two 16384-long fp32 sequences (uniform [0,1), seeds 41 and 42)",
           "steps": steps}
    floor_ms = (M + N - 1) * step_ns * 1e-6
    for mode in ("edges", "full"):
        run = (lambda: wf.dtw(x, y, mode="edges", last_row=lr, last_col=lc, final_cell=fc)) if mode == "edges" \
            else (lambda: wf.dtw(x, y, out=out))
        run()
        torch.cuda.synchronize()
        wf.check()
        kms = sum(time_events(torch, run, steps, torch.cuda.current_stream())) / steps
        wf.check()
        r = {"kernel_ms": kms, "cells_per_s": M * N / (kms * 1e-3),
             "latency": {"bound": "latency", "floor_ms": floor_ms, "frac": floor_ms / kms}}
        if mode == "full":
            alg = 4.0 * M * N
            r["roofline"] = {"bound": "hbm", "achieved": alg / (kms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": alg / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, "bytes_per_cell": 4}
        res[mode] = r
    del out
    torch.cuda.empty_cache()
    return res


def traceback_leg(torch, wf, cost, steps=3):
    """The traceback of the 16384 x 16384 benchmark grid: one wave walks back from the last
    cell through 64 x 64 blocks held in registers (a sequential path of up to m + n - 1
    cells, walked on the scalar unit; latency-bound)."""
    H = wf.solve(cost)
    torch.cuda.synchronize()
    ts = []
    for _ in range(steps):
        t0 = time.perf_counter()
        path, ex = wf.traceback(H)  # waits for the path length
        ts.append((time.perf_counter() - t0) * 1e3)
    L = int(path.shape[0])
    return {"workload": "traceback of the 16384x16384 min-rule grid (seed 2)", "path_cells": L,
            "ms": median(ts), "ns_per_cell": median(ts) * 1e6 / L, "exit": [int(v) for v in ex.cpu().tolist()]}


STREAMS = (1, 2, 4, 8, 16, 32)


def _wall(torch, fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    host = time.perf_counter() - t0
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3, host * 1e3


def stream_model(torch, wf, wfgen, costs, outs, streams_by_s, per_grid_by_s):
    """The paper's stream-count heuristic (Sections 2.3-2.4, Eqs. 3-7; selection of
    Section 3) applied to the per-grid path: jobs of G grids (the first G of the batch,
    G following the paper's size pattern 1, 2.5, 4, 5, 7.5, 8 x 10^i) timed on 1..32
    streams; `sum` (Eq. 3) is the device time of the job's launches run one after
    another; the models are fitted with shuffled 3:1 splits and the split between the
    two overhead regimes that fits the training halves best; the choice for the whole
    batch is compared with the measured best stream count."""
    counts = sorted({g for g in (10, 25, 40, 50, 75, 80, 100, 250, 400, 500, 750, 800, 1000, 2500, 4000)
                     if g < len(costs)} | {len(costs)})
    cells = [0]
    for c in costs:
        cells.append(cells[-1] + c.shape[0] * c.shape[1])
    stream0 = streams_by_s[1][0]
    samples = []
    for G in counts:
        plan = wf.EachPlan(costs[:G], outs[:G])
        # Eq. 3 analogue: per-launch device time on one stream, launches one after another
        s_ev = [torch.cuda.Event(enable_timing=True) for _ in range(G)]
        e_ev = [torch.cuda.Event(enable_timing=True) for _ in range(G)]
        sub = [wf.EachPlan([c], [o]) for c, o in zip(costs[:G], outs[:G])]
        for i in range(G):
            s_ev[i].record(stream0)
            sub[i].run([stream0])
            e_ev[i].record(stream0)
        torch.cuda.synchronize()
        sum_ms = sum(a.elapsed_time(b) for a, b in zip(s_ev, e_ev))
        t = {}
        for S in STREAMS:
            if G == len(costs) and S in per_grid_by_s:
                t[S] = per_grid_by_s[S]
                continue
            plan.run(streams_by_s[S])
            torch.cuda.synchronize()
            t[S] = min(_wall(torch, lambda: plan.run(streams_by_s[S]))[0] for _ in range(2))
        for S in STREAMS:
            samples.append((float(cells[G]), S, t[S], t[1], sum_ms))
    wf.check()
    # Split between the regimes: the candidate (a job size) with the least training error.
    sizes = sorted({s[0] for s in samples})
    best = None
    for k in range(2, len(sizes) - 2):
        split = sizes[k - 1]
        ns, nsm, nbg = wf.stream_model_groups(samples, split)
        try:
            model, rep = wf.fit_stream_model(samples, split, wfgen.permutation(41, ns), wfgen.permutation(42, nsm),
                                             wfgen.permutation(43, nbg))
        except wf.WfError:
            continue
        sse = rep[1].mse_train * rep[1].n_train + rep[2].mse_train * rep[2].n_train
        if best is None or sse < best[0]:
            best = (sse, split, model, rep)
    if best is None:
        return {"error": "no split gave a valid fit"}
    _, split, model, rep = best
    # predictions against the measured optimum for every job (the paper's Table 4, here)
    table = []
    for G in counts:
        size = float(cells[G])
        meas = {s[1]: s[2] for s in samples if s[0] == size}
        act = min(meas, key=meas.get)
        pre, _ = wf.choose_streams(model, size)
        table.append({"grids": G, "cells": int(size), "act": act, "pre": pre,
                      "t_act_ms": meas[act], "t_pre_ms": meas[pre]})
    pre_all, gaps = wf.choose_streams(model, float(cells[len(costs)]))

    def fit(r):
        return {"r2_train": r.r2_train, "r2_test": r.r2_test, "mse_train": r.mse_train, "mse_test": r.mse_test,
                "n_train": r.n_train, "n_test": r.n_test}

    return {"samples": len(samples), "jobs": counts, "split_size": split,
            "sum_model": {"slope_ms_per_cell": model.sum_slope, "intercept_ms": model.sum_intercept, **fit(rep[0])},
            "overhead_small": {"coef": list(model.small), **fit(rep[1])},
            "overhead_big": {"coef": list(model.big), **fit(rep[2])},
            "predicted_streams": pre_all, "gaps_ms": dict(zip([str(s) for s in STREAMS], gaps)),
            "correct": sum(1 for r in table if r["act"] == r["pre"]), "table": table}


def batched(torch, wf, wfgen, count, with_model=True):
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
    host_us = []
    for _ in range(reps):
        t0 = time.perf_counter()
        plan.run()
        host_us.append((time.perf_counter() - t0) * 1e6)
    torch.cuda.synchronize()
    # per-grid: one launch per grid (wf_solve_each), on S streams round-robin; best S wins
    streams_by_s = {S: [stream] + [torch.cuda.Stream() for _ in range(S - 1)] for S in STREAMS}
    each = wf.EachPlan(costs, outs)
    per_grid_by_s, per_grid_host_us = {}, {}
    for S in STREAMS:
        each.run(streams_by_s[S])
        torch.cuda.synchronize()
        runs = [_wall(torch, lambda: each.run(streams_by_s[S])) for _ in range(2)]
        per_grid_by_s[S] = min(r[0] for r in runs)
        per_grid_host_us[S] = min(r[1] for r in runs) * 1e3 / count
    wf.check()
    s_best = min(per_grid_by_s, key=per_grid_by_s.get)
    b_ms = median(bt)
    p_ms = per_grid_by_s[s_best]
    alg = 8.0 * cells
    res = {"grids": count, "cells": cells, "batched_ms": b_ms, "batched_host_us_per_call": median(host_us),
           "per_grid_ms": p_ms, "per_grid_streams": s_best,
           "per_grid_ms_by_streams": {str(k): v for k, v in per_grid_by_s.items()},
           "per_grid_host_us_per_launch": {str(k): v for k, v in per_grid_host_us.items()},
           "batched_cells_per_s": cells / (b_ms * 1e-3), "per_grid_cells_per_s": cells / (p_ms * 1e-3),
           "speedup": p_ms / b_ms,
           "roofline": {"bound": "hbm", "achieved": alg / (b_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": alg / (b_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "bytes_per_cell": 8},
           "shapes": "m, n independently log-uniform in [64, 2048] (PCG64 seed 4), grid g seed 1000+g"}
    if with_model:
        try:
            mdl = stream_model(torch, wf, wfgen, costs, outs, streams_by_s, per_grid_by_s)
            res["stream_model"] = mdl
            if "predicted_streams" in mdl:
                ps = mdl["predicted_streams"]
                res["per_grid_streams_predicted"] = ps
                res["per_grid_ms_at_predicted"] = per_grid_by_s[ps]
        except Exception as e:  # report, do not lose the rest
            res["stream_model"] = {"error": repr(e)}
    return res


def serving(torch, wf, wfgen, grids, requests, warmup, load, inflight=2, batch=256, check=True):
    """Poisson arrivals of square grids (n log-uniform in [128, 8192]) served under a
    64 GiB budget with continuous batching.  The arrival rate is `load` times the
    batched capacity for the same mix, measured first with one wf_solve_batched
    launch.  Latency = completion as observed by polling - scheduled arrival."""
    import numpy as np

    total = warmup + requests
    reqs = wfgen.serving_requests(total, rate_per_s=1.0)  # unit-rate arrival pattern, rescaled below
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
    sampled = {}  # request index -> (grid, copy of the served output)
    every = max(1, requests // 200) if check else 0
    with wf.Server(budget_bytes=64 << 30, max_inflight=inflight, max_batch=batch) as srv:
        outstanding = {}
        t_start = time.perf_counter()
        i = 0
        first_done, last_done, t_meas0 = None, 0.0, None
        while i < len(arrivals) or outstanding:
            now = time.perf_counter()
            while i < len(arrivals) and t_start + arrivals[i] <= now:
                g = i % grids
                tk = srv.submit(costs[g])
                outstanding[tk] = (i, g, t_start + arrivals[i])
                i += 1
            progressed = False
            # one call lists the requests finished since the last look
            for tk in srv.done():
                if tk not in outstanding:
                    continue
                t_obs = time.perf_counter()
                r = srv.poll(tk) if (every and (outstanding[tk][0] - warmup) % every == 0
                                     and outstanding[tk][0] >= warmup) else srv.poll_times(tk)
                q, g, t_arr = outstanding.pop(tk)
                if isinstance(r, dict):
                    sampled[q] = (g, r["out"].clone())
                    # the copy runs on torch's stream: it must be done before the server may
                    # hand the released memory to a later request
                    torch.cuda.current_stream().synchronize()
                srv.release(tk)
                if q >= warmup:
                    lat.append(t_obs - t_arr)
                    cells_done += cells[g]
                    if t_meas0 is None:
                        t_meas0 = t_start + arrivals[warmup]
                    last_done = max(last_done, t_obs)
                progressed = True
            if not progressed and (i >= len(arrivals) or t_start + arrivals[i] > time.perf_counter() + 2e-4):
                time.sleep(5e-5)
        peak = srv.memory()[1]
    torch.cuda.synchronize()
    wf.check()
    # served results equal the same grids swept alone; some also equal the oracle
    checked_alone = checked_oracle = 0
    if check:
        import oracle
        for k, (q, (g, got)) in enumerate(sorted(sampled.items())):
            alone = wf.solve(costs[g])
            if not torch.equal(got, alone):
                raise AssertionError(f"served request {q} (grid {g}) differs from the grid swept alone")
            checked_alone += 1
            if k % 10 == 0:
                n = sizes[g]
                exp = oracle.sweep(wfgen.cells(50000 + g, n, n, "f32"), "min", "f32")
                if not np.array_equal(got.cpu().numpy().view(np.uint32), exp.view(np.uint32)):
                    raise AssertionError(f"served request {q} (grid {g}) differs from the oracle")
                checked_oracle += 1
        torch.cuda.synchronize()
    lat = np.array(lat) * 1e3
    span = last_done - t_meas0
    return {"requests": requests, "warmup_requests": warmup, "distinct_grids": grids,
            "n": "log-uniform in [128, 8192] (PCG64 seed 5), grid g seed 50000+g, request q serves grid q mod %d" % grids,
            "batched_capacity_req_per_s": cap, "load": load, "rate_req_per_s": rate,
            "latency": "poll-observed completion - scheduled arrival",
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "cells_per_s": cells_done / span,
            "peak_server_bytes": peak, "budget_bytes": 64 << 30,
            "checked_equal_alone": checked_alone, "checked_equal_oracle": checked_oracle,
            "max_inflight": inflight, "max_batch": batch}


def copy_serving(torch, wf, wfgen, count=256, batch=16):
    """Host-resident inputs (pinned) for a burst of `count` square requests (n
    log-uniform in [128, 2048]) on one launch stream, `batch` requests per launch:
    copies on the launch stream just before each launch vs on two copy streams started
    at admission (overlapping earlier launches).  Prediction: the two-stage flow shop
    of launches L (copy time C_L from the measured host-to-device bandwidth, sweep time
    K_L measured alone), makespan max_j (sum_{L<=j} C_L + sum_{L>=j} K_L); serialised:
    sum (C_L + K_L).  With identical launches this is the paper's streamed-time model,
    Eq. 2: the larger stage whole, the smaller hidden but for one launch's share."""
    reqs = wfgen.serving_requests(count, rate_per_s=1.0, lo=128, hi=2048, seed=6)
    hosts = [torch.from_numpy(wfgen.cells(seed, n, n, "f32")).pin_memory() for (_, n, seed) in reqs]
    devs = [h.to("cuda", non_blocking=False) for h in hosts]
    # host-to-device bandwidth with one large pinned copy
    big = torch.empty(256 << 20, dtype=torch.uint8).pin_memory()
    dbig = torch.empty_like(big, device="cuda")
    dbig.copy_(big)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        dbig.copy_(big)
    torch.cuda.synchronize()
    h2d = 3 * big.numel() / (time.perf_counter() - t0)
    del big, dbig
    # per-launch sweep time alone (the server packs requests in submission order)
    launches = [list(range(k, min(k + batch, count))) for k in range(0, count, batch)]
    K = []
    for L in launches:
        cs = [devs[q] for q in L]
        os_ = [torch.empty_like(c) for c in cs]
        wf.solve_batched(cs, os_, waves_per_wg=1, order=1, use_graph=-1)
        torch.cuda.synchronize()
        K.append(min(_wall(torch, lambda: wf.solve_batched(cs, os_, waves_per_wg=1, order=1, use_graph=-1))[0]
                     for _ in range(2)))
    C = [sum(hosts[q].numel() * 4 for q in L) / h2d * 1e3 for L in launches]
    serial = sum(C) + sum(K)
    flow = max(sum(C[:j + 1]) + sum(K[j:]) for j in range(len(launches)))
    res = {"requests": count, "per_launch": batch, "h2d_GBps": h2d / 1e9, "copy_ms": sum(C), "sweep_ms": sum(K),
           "predicted_serial_ms": serial, "predicted_overlap_ms": flow, "predicted_gain": serial / flow}
    for copy_streams in (0, 2):
        best = None
        for _ in range(2):
            with wf.Server(budget_bytes=16 << 30, max_inflight=1, max_batch=batch, copy_streams=copy_streams) as srv:
                t0 = time.perf_counter()
                tks = [srv.submit(h) for h in hosts]
                pending = set(tks)
                while pending:
                    for tk in srv.done():
                        if tk in pending and srv.poll_times(tk) is not None:
                            pending.discard(tk)
                            srv.release(tk)
                    time.sleep(2e-5)
                dt = (time.perf_counter() - t0) * 1e3
            best = dt if best is None else min(best, dt)
        res["measured_ms_copy_streams_%d" % copy_streams] = best
    res["measured_gain"] = res["measured_ms_copy_streams_0"] / res["measured_ms_copy_streams_2"]
    return res


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
    step_ns = wf.measure_step_ns()
    floor_ms = (M + N - 1) * step_ns * 1e-6
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
                     "bytes_per_launch": alg_bytes, "bytes_per_cell": 8,
                     "latency": {"bound": "latency", "steps": M + N - 1, "step_ns": step_ns,
                                 "floor_ms": floor_ms, "frac": floor_ms / kernel_ms,
                                 "what": "m+n-1 dependent steps of the walk's chain (DPP move, min, add), "
                                         "each as long as one wave alone measures it"}},
    }
    del out
    legs = []
    if not args.no_large:
        legs.append(("large_edges", lambda: large_edges(torch, wf, wfgen)))
    if not args.no_fp64:
        legs.append(("fp64", lambda: fp64_leg(torch, wf, wfgen)))
    if not args.no_dtw:
        legs.append(("dtw", lambda: dtw_leg(torch, wf, wfgen, step_ns)))
        legs.append(("traceback", lambda: traceback_leg(torch, wf, cost)))
    if not args.no_batched:
        legs.append(("batched", lambda: batched(torch, wf, wfgen, args.batch_count, not args.no_model)))
    if not args.no_serving:
        legs.append(("serving", lambda: serving(torch, wf, wfgen, args.serve_grids, args.serve_requests,
                                                args.serve_warmup, args.serve_load, args.serve_inflight,
                                                args.serve_batch)))
    if not args.no_copy_serving:
        legs.append(("copy_serving", lambda: copy_serving(torch, wf, wfgen)))
    for name, fn in legs:
        log(f"[bench] {name}")
        try:
            result[name] = fn()
        except Exception as e:  # report, do not lose the main line
            result[name] = {"error": repr(e)}
        torch.cuda.empty_cache()
    if not args.no_serving and "error" not in result.get("serving", {}):
        # The same mix at a light and a heavy load (half as many requests each, no checks).
        others = {}
        for load in (0.3, 0.9):
            log(f"[bench] serving at load {load}")
            try:
                r = serving(torch, wf, wfgen, args.serve_grids, max(args.serve_requests // 2, 1), args.serve_warmup,
                            load, args.serve_inflight, args.serve_batch, check=False)
                others[str(load)] = {k: r[k] for k in ("requests", "rate_req_per_s", "p50_ms", "p99_ms", "cells_per_s")}
            except Exception as e:  # report, do not lose the main line
                others[str(load)] = {"error": repr(e)}
        result["serving"]["other_loads"] = others
    if not args.no_cpu:
        log(f"[bench] cpu baseline ({args.cpu_seconds:.0f} s of one pinned core)")
        result["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
