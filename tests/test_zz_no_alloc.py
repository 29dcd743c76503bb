"""The allocation-free entry point (wf_solve_noalloc) against wf_solve, through the C ABI.

Both run the same kernels; the allocation-free call keeps its control words and
handoff rows in a fixed device array.  Two calls in a row, the second on a smaller
grid (so it runs on what the first left in the array), must each equal wf_solve's
result bit for bit; so must the largest benchmark grid the array holds and an
int32 grid.  A problem larger than the array is refused before anything is
enqueued.
"""
import ctypes

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


def _pair(m, n, seed, dtype="f32", rule="min"):
    print(f"[noalloc] m={m} n={n} seed={seed} dtype={dtype} rule={rule}", flush=True)
    c = torch.from_numpy(wfgen.cells(seed, m, n, dtype)).to(DEV)
    want = wf.solve(c, rule=rule)
    got = torch.full_like(c, -1)
    wf.solve_noalloc(c, got, rule=rule)
    torch.cuda.synchronize()
    wf.check()
    return c, got, want


def _bits_equal(a, b):
    return torch.equal(a.view(torch.int32), b.view(torch.int32))


def test_two_calls_in_a_row_second_smaller():
    for (m, n, seed) in ((2100, 1000, 61), (300, 513, 62)):
        c, got, want = _pair(m, n, seed)
        assert _bits_equal(got, want), (m, n)
        ref = oracle.sweep(c.cpu().numpy(), "min", "f32")
        assert np.array_equal(got.cpu().numpy().view(np.uint32), ref.view(np.uint32)), (m, n)


def test_int32_max_rule_and_edges_mode():
    _, got, want = _pair(700, 333, 63, dtype="i32", rule="max")
    assert torch.equal(got, want)
    m, n = 1000, 777
    c = torch.from_numpy(wfgen.cells(64, m, n, "f32")).to(DEV)
    lr, lc, fc = (torch.empty(n, device=DEV), torch.empty(m, device=DEV), torch.empty(1, device=DEV))
    wf.solve_noalloc(c, None, mode="edges", last_row=lr, last_col=lc, final_cell=fc)
    H = wf.solve(c)
    torch.cuda.synchronize()
    assert _bits_equal(lr, H[-1]) and _bits_equal(lc, H[:, -1].contiguous()) and _bits_equal(fc, H[-1, -1:])


def test_benchmark_grid_16384():
    c, got, want = _pair(16384, 16384, 2)
    assert _bits_equal(got, want)


def test_oversized_problem_is_refused_before_any_launch():
    c = torch.zeros((64, 64), device=DEV)
    p = wf.make_problem(c, c)
    p.m = p.n = 65536  # needs ~268 MB of handoff rows; the array holds 32 MiB
    p.ld_cost = p.ld_out = 65536
    st = wf.load_library().wf_solve_noalloc(wf.context(0), ctypes.byref(p), None)
    assert st == -3  # WF_E2BIG
    assert b"fixed workspace" in wf.load_library().wf_last_error()
    # the context is still usable
    _, got, want = _pair(129, 300, 65)
    assert _bits_equal(got, want)
