"""GPU tests of the serving front end (wf_server_* through the C ABI).

Each served result must be bit-identical to the same grid swept alone with
wf_solve (and, for a few, to the CPU oracle): admission, batching with other
requests and overlap with other launches must not change a single bit.

While the server has launches in flight the tests wait on torch's own stream
only (never a device-wide synchronize), as a serving client would.
"""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_2501_05938_amd as wf  # noqa: E402
import wfgen  # noqa: E402

DEV = torch.device("cuda:0")


def _wait_all(srv, tickets, timeout_s=60.0):
    done = {}
    t0 = time.time()
    while len(done) < len(tickets):
        for t in tickets:
            if t not in done:
                r = srv.poll(t)
                if r is not None:
                    done[t] = r
        if time.time() - t0 > timeout_s:
            raise TimeoutError(f"{len(tickets) - len(done)} requests still pending")
        time.sleep(0.0005)
    return done


def _sync():
    torch.cuda.current_stream().synchronize()


def _bits(t):
    _sync()
    a = t.cpu().numpy()
    return a.view(np.uint32) if a.dtype == np.float32 else a


def test_mix_equals_alone():
    """Requests of mixed size, dtype, rule, mode and input kind, submitted together."""
    rng = np.random.default_rng(7)
    specs = []
    for q in range(24):
        m = int(rng.integers(1, 700))
        n = int(rng.integers(1, 900))
        dt = "f32" if q % 3 else "i32"
        rule = "min" if q % 4 else "max"
        mode = "full" if q % 5 else "edges"
        host = q % 2 == 1
        specs.append((m, n, dt, rule, mode, host, 60000 + q))
    print(f"[serving] mix of {len(specs)} requests", flush=True)
    inputs, tickets = [], []
    with wf.Server(budget_bytes=1 << 30, max_inflight=4, max_batch=8) as srv:
        for (m, n, dt, rule, mode, host, seed) in specs:
            c = wfgen.cells(seed, m, n, dt)
            x = c if host else torch.from_numpy(c).to(DEV)
            inputs.append(c)
            tickets.append(srv.submit(x, rule=rule, mode=mode))  # the binding keeps x alive
        res = _wait_all(srv, tickets)
        for (m, n, dt, rule, mode, host, seed), c, t in zip(specs, inputs, tickets):
            r = res[t]
            alone = wf.solve(torch.from_numpy(c).to(DEV), rule=rule)
            exp = _bits(alone)
            if mode == "full":
                assert np.array_equal(_bits(r["out"]), exp), (m, n, dt, rule, mode)
            assert np.array_equal(_bits(r["last_row"]), exp[-1]), (m, n, dt, rule, mode)
            assert np.array_equal(_bits(r["last_col"]), exp[:, -1]), (m, n, dt, rule, mode)
            assert _bits(r["final_cell"])[0] == exp[-1, -1]
            assert r["t_submit"] <= r["t_admit"] <= r["t_launch"] <= r["t_done"]
            srv.release(t)
        assert srv.memory()[0] == 0
    _sync()


def test_served_results_match_oracle_and_alone_at_scale():
    """250 requests of the serving mix's shape (square, n log-uniform, smaller here so the
    oracle keeps up) submitted in a burst through a small budget, so admission, batching
    and overlapping launches all happen: all 250 bit-equal to the grid swept alone, 25 of
    them to the fp32 oracle as well."""
    reqs = wfgen.serving_requests(250, rate_per_s=1.0, lo=64, hi=700, seed=55)
    grids = [wfgen.cells(seed, n, n, "f32") for (_, n, seed) in reqs]
    devs = [torch.from_numpy(g).to(DEV) for g in grids]
    _sync()
    print(f"[serving] {len(reqs)} requests", flush=True)
    with wf.Server(budget_bytes=96 << 20, max_inflight=4, max_batch=32) as srv:
        tickets = [srv.submit(d) for d in devs]
        res = _wait_all(srv, tickets, timeout_s=120)
        for q, (t, d) in enumerate(zip(tickets, devs)):
            alone = wf.solve(d)
            assert np.array_equal(_bits(res[t]["out"]), _bits(alone)), q
            if q % 10 == 0:
                assert np.array_equal(_bits(res[t]["out"]), oracle.sweep(grids[q], "min", "f32").view(np.uint32)), q
            srv.release(t)
        assert srv.memory()[0] == 0


def test_host_inputs_on_copy_streams():
    """Host inputs (pageable numpy and pinned CPU tensors) copied at admission on two copy
    streams, overlapping earlier launches: results equal the oracle."""
    specs = [(int(m), int(n)) for m, n in np.random.default_rng(8).integers(1, 600, size=(30, 2))]
    cs = [wfgen.cells(80 + q, m, n, "f32") for q, (m, n) in enumerate(specs)]
    print("[serving] copy streams", flush=True)
    with wf.Server(budget_bytes=256 << 20, max_inflight=3, max_batch=4, copy_streams=2,
                   staging_bytes=8 << 20) as srv:
        tickets = []
        for q, c in enumerate(cs):
            x = c if q % 2 == 0 else torch.from_numpy(c).pin_memory()
            tickets.append(srv.submit(x, mode="full" if q % 3 else "edges"))
        res = _wait_all(srv, tickets)
        for q, (t, c) in enumerate(zip(tickets, cs)):
            exp = oracle.sweep(c, "min", "f32").view(np.uint32)
            if q % 3:
                assert np.array_equal(_bits(res[t]["out"]), exp), q
            assert np.array_equal(_bits(res[t]["last_row"]), exp[-1]), q
            assert np.array_equal(_bits(res[t]["last_col"]), exp[:, -1]), q
            srv.release(t)


def test_seeded_requests_match_generator_and_oracle():
    """WF_INPUT_SEED: the server generates the inputs on the device; results equal the
    oracle on the host generator's grid (f32 and i32)."""
    print("[serving] seeded", flush=True)
    with wf.Server(budget_bytes=64 << 20) as srv:
        specs = [(300, 513, 91, "f32", "min"), (65, 7, 92, "i32", "max"), (129, 200, 93, "f32", "max")]
        tickets = [srv.submit_seeded(m, n, seed, dt, rule) for (m, n, seed, dt, rule) in specs]
        res = _wait_all(srv, tickets)
        for (m, n, seed, dt, rule), t in zip(specs, tickets):
            c = wfgen.cells(seed, m, n, dt)
            exp = oracle.sweep(c, rule, "f32").view(np.uint32) if dt == "f32" else \
                oracle.sweep(c, rule, "i64").astype(np.int32)
            assert np.array_equal(_bits(res[t]["out"]), exp), (m, n, dt, rule)
            srv.release(t)


def test_device_input_written_asynchronously_before_submit():
    """A device input still being written on the caller's stream when it is submitted:
    the launch waits for it on the device (ready event), with no host synchronization."""
    m = n = 1500
    exp = oracle.sweep(wfgen.cells(94, m, n, "f32"), "min", "f32").view(np.uint32)
    print("[serving] ready event", flush=True)
    with wf.Server(budget_bytes=128 << 20) as srv:
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            x = torch.zeros((m, n), dtype=torch.float32, device=DEV)
            for _ in range(20):  # keep the stream busy so the fill lands late
                x.add_(1.0)
            wfgen.fill_device(x, seed=94, stream=side)
            t = srv.submit(x)  # records the ready event on `side`, the current stream here
        r = _wait_all(srv, [t])[t]
        got = _bits(r["out"])
        srv.release(t)
    assert np.array_equal(got, exp)


def test_budget_limits_admission():
    """A budget that holds only a few requests at once: all complete, the peak stays
    within the budget, and memory returns to zero after release."""
    m = n = 512
    per = m * n * 4 * 2  # output + rounding slack per request, roughly
    budget = 3 * per
    with wf.Server(budget_bytes=budget, max_inflight=2, max_batch=4) as srv:
        cs = [torch.from_numpy(wfgen.cells(70 + q, m, n, "f32")).to(DEV) for q in range(10)]
        tickets = [srv.submit(c) for c in cs]
        pending = set(tickets)
        t0 = time.time()
        while pending:
            for t in list(pending):
                r = srv.poll(t)
                if r is not None:
                    exp = wf.solve(cs[tickets.index(t)])
                    same = torch.equal(r["out"], exp)
                    _sync()
                    assert same
                    srv.release(t)  # frees memory so later requests are admitted
                    pending.discard(t)
            assert time.time() - t0 < 60, "admission stalled"
            time.sleep(0.0005)
        in_use, peak = srv.memory()
        assert in_use == 0
        assert 0 < peak <= budget


def test_oversized_and_invalid_requests():
    with wf.Server(budget_bytes=1 << 20) as srv:
        with pytest.raises(wf.WfError) as e:
            srv.submit(torch.zeros((1024, 1024), dtype=torch.float32, device=DEV))
        assert e.value.status == -3  # WF_E2BIG
        with pytest.raises(wf.WfError) as e:
            srv.poll(12345)
        assert e.value.status == -6  # WF_ENOTFOUND
        t = srv.submit(torch.zeros((0, 5), dtype=torch.float32, device=DEV))
        r = srv.poll(t)
        assert r is not None and r["out"] is None
        srv.release(t)


def test_done_reports_each_finished_ticket_once():
    """wf_server_done lists every finished ticket exactly once, and only finished ones
    (wf_poll already has its result); results match the grids swept alone."""
    grids = []
    for q in range(40):
        m, n = 64 + 37 * q, 80 + 29 * q
        c = torch.empty((m, n), dtype=torch.float32, device=DEV)
        wfgen.fill_device(c, seed=900 + q)
        grids.append(c)
    _sync()
    with wf.Server(budget_bytes=8 << 30) as srv:
        tickets = [srv.submit(c) for c in grids]
        seen = []
        t0 = time.time()
        while len(seen) < len(tickets):
            for tk in srv.done():
                assert srv.poll_times(tk) is not None, "reported before it finished"
                seen.append(tk)
            if time.time() - t0 > 60.0:
                raise TimeoutError(f"{len(tickets) - len(seen)} requests never reported")
            time.sleep(0.0005)
        assert sorted(seen) == sorted(tickets) and len(set(seen)) == len(seen)
        assert srv.done() == []
        for tk, c in zip(tickets, grids):
            got = srv.poll(tk)["out"].clone()
            _sync()
            assert torch.equal(got, wf.solve(c))
            srv.release(tk)
