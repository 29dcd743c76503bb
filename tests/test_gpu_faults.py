"""Failure handling on the GPU, forced from the host so every kernel still exits
normally: the WF_FAULT test hook makes one band of a context's first launch keep
its bottom row to itself, the band below waits on it, and a short watchdog (set
with wf_set_watchdog) makes the launch give up and drain.  The error must be
reported as WF_ETIMEDOUT, and the next launch on the same context -- which reuses
the aborted launch's handoff rows -- must be bit-exact again."""
import ctypes
import os

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
ETIMEDOUT = -5


def _fault_ctx(band):
    lib = wf.load_library()
    os.environ["WF_FAULT"] = f"drop_hand:{band}"
    try:
        h = ctypes.c_void_p()
        assert lib.wf_init(0, ctypes.byref(h)) == 0
    finally:
        del os.environ["WF_FAULT"]
    assert lib.wf_set_watchdog(h, 20) == 0
    return h


def test_watchdog_reports_and_rearms():
    lib = wf.load_library()
    torch.cuda.synchronize()
    h = _fault_ctx(1)
    try:
        m, n = 300, 513
        c = wfgen.cells(95, m, n, "f32")
        cd = torch.from_numpy(c).to(DEV)
        out = torch.empty_like(cd)
        p = wf.make_problem(cd, out)
        torch.cuda.synchronize()
        print("[faults] launch with a dropped handoff", flush=True)
        assert lib.wf_solve(h, ctypes.byref(p), None) == 0
        assert lib.wf_check(h) == ETIMEDOUT
        print("[faults] next launch on the same context", flush=True)
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        assert lib.wf_solve(h, ctypes.byref(p), None) == 0
        assert lib.wf_check(h) == 0
        assert np.array_equal(out.cpu().numpy().view(np.uint32), oracle.sweep(c, "min", "f32").view(np.uint32))
    finally:
        lib.wf_destroy(h)


def test_server_reports_a_failed_launch_and_recovers():
    lib = wf.load_library()
    h = _fault_ctx(2)
    try:
        c = wfgen.cells(96, 400, 300, "f32")
        print("[faults] served request with a dropped handoff", flush=True)
        with wf.Server(budget_bytes=64 << 20, max_inflight=1, ctx=h) as srv:
            t = srv.submit(c)
            import time
            t0 = time.time()
            with pytest.raises(wf.WfError) as e:
                while srv.poll(t) is None:
                    assert time.time() - t0 < 30
                    time.sleep(0.001)
            assert e.value.status == ETIMEDOUT
            srv.release(t)
            t2 = srv.submit(c)
            while (r := srv.poll(t2)) is None:
                assert time.time() - t0 < 60
                time.sleep(0.001)
            got = r["out"].cpu().numpy().view(np.uint32)
            srv.release(t2)
        assert np.array_equal(got, oracle.sweep(c, "min", "f32").view(np.uint32))
    finally:
        lib.wf_destroy(h)


def test_watchdog_bounds():
    lib = wf.load_library()
    ctx = wf.context(0)
    assert lib.wf_set_watchdog(ctx, -1) == -1
    assert lib.wf_set_watchdog(None, 5) == -1
    assert lib.wf_set_watchdog(ctx, 2000) == 0
