"""GPU parity of the batched sweep: many uneven grids in one persistent launch.

Every grid of a batch must be bit-identical to the CPU oracle (fp32 / int32),
for every configuration the autotuner can pick (band shapes of one or two
compute waves of one row per lane, or one wave of two rows per lane;
grid-major and interleaved work order), on graph replay, and in edges mode.
"""
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


def _batch(count, lo, hi, dtype="f32", seed=4):
    shapes = wfgen.batch_shapes(count, lo=lo, hi=hi, seed=seed)
    hs = [wfgen.cells(wfgen.batch_seed(g), m, n, dtype) for g, (m, n) in enumerate(shapes)]
    return shapes, hs, [torch.from_numpy(h).to(DEV) for h in hs]


def _expect(h, rule, dtype):
    if dtype == "f32":
        return oracle.sweep(h, rule, "f32").view(np.uint32)
    return oracle.sweep(h, rule, "i64").astype(np.int32)


def _bits(t):
    a = t.cpu().numpy()
    return a.view(np.uint32) if a.dtype == np.float32 else a


@pytest.mark.parametrize("W,R", [(1, 1), (2, 1), (1, 2)])
@pytest.mark.parametrize("order", [1, 2])
def test_every_configuration(W, R, order):
    print(f"[batched] W={W} R={R} order={order}", flush=True)
    shapes, hs, ds = _batch(40, 1, 700, seed=11)
    outs = wf.solve_batched(ds, waves_per_wg=W, rows_per_lane=R, order=order, use_graph=0)
    torch.cuda.synchronize()
    wf.check()
    for (m, n), h, o in zip(shapes, hs, outs):
        assert np.array_equal(_bits(o), _expect(h, "min", "f32")), (m, n, W, R, order)


def test_autotuned_graph_replay_and_alone():
    """Autotuned, captured once, replayed twice; each grid equals the grid swept alone."""
    shapes, hs, ds = _batch(64, 64, 1024, seed=12)
    outs = [torch.full_like(d, float("nan")) for d in ds]
    for rep in range(3):
        print(f"[batched] autotuned replay {rep}", flush=True)
        for o in outs:
            o.fill_(float("nan"))
        wf.solve_batched(ds, outs)
        torch.cuda.synchronize()
        wf.check()
        for (m, n), h, d, o in zip(shapes, hs, ds, outs):
            if rep == 0:
                assert np.array_equal(_bits(o), _expect(h, "min", "f32")), (m, n)
            else:
                assert torch.equal(o, wf.solve(d)), (m, n, rep)


@pytest.mark.parametrize("rule", ["min", "max"])
def test_int32_batch(rule):
    shapes, hs, ds = _batch(24, 1, 600, dtype="i32", seed=13)
    outs = wf.solve_batched(ds, rule=rule, use_graph=0)
    torch.cuda.synchronize()
    for (m, n), h, o in zip(shapes, hs, outs):
        assert np.array_equal(_bits(o), _expect(h, rule, "i32")), (m, n, rule)


def test_edges_batch():
    shapes, hs, ds = _batch(24, 1, 900, seed=14)
    outs = wf.solve_batched(ds, mode="edges", use_graph=0)
    torch.cuda.synchronize()
    for (m, n), h, (lr, lc, fc) in zip(shapes, hs, outs):
        exp = oracle.sweep(h, "min", "f32")
        assert np.array_equal(_bits(lr), exp[-1].view(np.uint32)), (m, n)
        assert np.array_equal(_bits(lc), exp[:, -1].view(np.uint32)), (m, n)
        assert _bits(fc)[0] == exp[-1, -1].view(np.uint32)


def test_mixed_dtype_batch_is_rejected():
    a = torch.zeros((4, 4), dtype=torch.float32, device=DEV)
    b = torch.zeros((4, 4), dtype=torch.int32, device=DEV)
    with pytest.raises(wf.WfError) as e:
        wf.solve_batched([a, b])
    assert e.value.status == -8  # WF_EUNSUPPORTED


@pytest.mark.slow
def test_benchmark_batch_every_grid_both_modes():
    """The 4096-grid benchmark batch (sizes log-uniform in [64, 2048]) launched as the
    benchmark launches it (autotuned, graph-replayed) in full mode, and again in edges
    mode: every grid bit-exact against the fp32 oracle in both."""
    from concurrent.futures import ThreadPoolExecutor
    shapes = wfgen.batch_shapes(4096)
    ds = []
    for g, (m, n) in enumerate(shapes):
        t = torch.empty((m, n), dtype=torch.float32, device=DEV)
        wfgen.fill_device(t, seed=wfgen.batch_seed(g))
        ds.append(t)
    print("[batched] 4096 grids, full mode", flush=True)
    full = wf.solve_batched(ds)
    torch.cuda.synchronize()
    wf.check()
    print("[batched] 4096 grids, edges mode", flush=True)
    edges = wf.solve_batched(ds, mode="edges")
    torch.cuda.synchronize()
    wf.check()

    def check(g):
        m, n = shapes[g]
        exp = oracle.sweep(wfgen.cells(wfgen.batch_seed(g), m, n, "f32"), "min", "f32").view(np.uint32)
        return (np.array_equal(_bits(full[g]), exp), np.array_equal(_bits(edges[g][0]), exp[-1]),
                np.array_equal(_bits(edges[g][1]), exp[:, -1]), _bits(edges[g][2])[0] == exp[-1, -1])

    bad = []
    with ThreadPoolExecutor(12) as pool:
        for g, ok in enumerate(pool.map(check, range(len(shapes)))):
            if not all(ok):
                bad.append((g, shapes[g], ok))
    assert not bad, bad[:10]


def test_three_waves_per_workgroup_is_rejected():
    a = torch.zeros((4, 4), dtype=torch.float32, device=DEV)
    with pytest.raises(wf.WfError) as e:
        wf.solve_batched([a], waves_per_wg=3)
    assert e.value.status == -1  # WF_EINVAL


def test_graph_replay_after_single_solves_of_another_dtype():
    """A replayed batch whose launch slot was used meanwhile by single-grid int32
    solves (other handoff-row sentinel, possibly larger rows) is still exact."""
    shapes, hs, ds = _batch(16, 64, 300, seed=15)
    outs = [torch.empty_like(d) for d in ds]
    plan = wf.BatchPlan(ds, outs)
    plan.run()
    torch.cuda.synchronize()
    ci = torch.from_numpy(wfgen.cells(16, 700, 700, "i32")).to(DEV)
    for _ in range(10):  # cycles through every launch slot of the context
        wf.solve(ci)
    torch.cuda.synchronize()
    for rep in range(2):
        print(f"[batched] replay after int32 solves {rep}", flush=True)
        for o in outs:
            o.fill_(float("nan"))
        plan.run()
        torch.cuda.synchronize()
        wf.check()
        for (m, n), h, o in zip(shapes, hs, outs):
            assert np.array_equal(_bits(o), _expect(h, "min", "f32")), (m, n, rep)


def test_per_grid_path_on_several_streams():
    """wf_solve_each: one launch per grid, spread over 1, 3 and 8 streams; every grid
    bit-exact against the oracle, and more launches in flight than the context had
    slots before."""
    shapes, hs, ds = _batch(80, 1, 500, seed=17)
    for S in (1, 3, 8):
        print(f"[per-grid] {S} streams", flush=True)
        streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(S - 1)]
        plan = wf.EachPlan(ds)
        for o in plan.outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        plan.run(streams)
        torch.cuda.synchronize()
        wf.check()
        for (m, n), h, o in zip(shapes, hs, plan.outs):
            assert np.array_equal(_bits(o), _expect(h, "min", "f32")), (m, n, S)


def test_replays_pipeline_and_follow_new_buffers():
    """A graph-replayed plan run several times back to back without waiting (two lanes in
    flight), then with the same shapes on new buffers: every run exact."""
    shapes, hs, ds = _batch(24, 64, 400, seed=18)
    outs = [torch.empty_like(d) for d in ds]
    plan = wf.BatchPlan(ds, outs, waves_per_wg=1, order=2, use_graph=1)
    for rep in range(4):
        plan.run()
    torch.cuda.synchronize()
    wf.check()
    for (m, n), h, o in zip(shapes, hs, outs):
        assert np.array_equal(_bits(o), _expect(h, "min", "f32")), (m, n)
    ds2 = [d.clone() for d in ds]
    outs2 = [torch.full_like(d, float("nan")) for d in ds]
    wf.BatchPlan(ds2, outs2, waves_per_wg=1, order=2, use_graph=1).run()
    torch.cuda.synchronize()
    wf.check()
    for (m, n), h, o in zip(shapes, hs, outs2):
        assert np.array_equal(_bits(o), _expect(h, "min", "f32")), (m, n)
