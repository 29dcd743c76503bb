"""GPU parity of dynamic time warping (cell inputs |x_i - y_j| computed on the device)
and of the traceback kernel, through the C ABI, against the CPU oracle.

Bar: bit-exact.  DTW in fp32 is one rounding for the difference and one for the sum,
so the device result is unique; the traceback is a deterministic walk over exact
comparisons of stored values, so the whole path and its exit must be equal.
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


def _seq(seed, k):
    return (wfgen.vector(seed, k, "f32") * 4.0 - 2.0).astype(np.float32)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _bits(t):
    torch.cuda.synchronize()
    a = t.cpu().numpy()
    return a.view(np.uint32) if a.dtype == np.float32 else a


DTW_SHAPES = [(1, 1), (1, 300), (300, 1), (65, 65), (129, 300), (700, 333), (2100, 1000), (4097, 65)]


@pytest.mark.parametrize("m,n", DTW_SHAPES)
@pytest.mark.parametrize("W,R", [(1, 1), (2, 1), (1, 2)])
def test_dtw_full(m, n, W, R):
    print(f"[dtw] m={m} n={n} W={W} R={R}", flush=True)
    x, y = _seq(m, m), _seq(n + 7, n)
    got = wf.dtw(_dev(x), _dev(y), waves_per_wg=W, rows_per_lane=R)
    want = oracle.dtw(x, y)
    assert np.array_equal(_bits(got), want.view(np.uint32))
    wf.check()


@pytest.mark.parametrize("m,n", [(1, 1), (300, 513), (2100, 333)])
def test_dtw_edges_and_max_rule(m, n):
    print(f"[dtw] edges/max m={m} n={n}", flush=True)
    x, y = _seq(3 * m, m), _seq(5 * n, n)
    lr, lc, fc = wf.dtw(_dev(x), _dev(y), mode="edges")
    r, c = oracle.dtw(x, y, full=False)
    assert np.array_equal(_bits(lr), r.view(np.uint32)) and np.array_equal(_bits(lc), c.view(np.uint32))
    assert _bits(fc)[0] == r.view(np.uint32)[-1]
    cost = np.abs(x[:, None] - y[None, :]).astype(np.float32)
    got = wf.dtw(_dev(x), _dev(y), rule="max")
    assert np.array_equal(_bits(got), oracle.sweep(cost, "max", "f32").view(np.uint32))


@pytest.mark.slow
def test_dtw_16384_edges():
    """The 16384 x 16384 DTW as the benchmark runs it (edges mode), against the oracle."""
    m = n = 16384
    print("[dtw] 16384^2 edges", flush=True)
    x, y = _seq(41, m), _seq(42, n)
    lr, lc, fc = wf.dtw(_dev(x), _dev(y), mode="edges")
    r, c = oracle.dtw(x, y, full=False)
    assert np.array_equal(_bits(lr), r.view(np.uint32)) and np.array_equal(_bits(lc), c.view(np.uint32))


TB_SHAPES = [(1, 1), (1, 200), (200, 1), (63, 63), (64, 64), (65, 130), (300, 513), (1000, 1000), (2100, 333)]


def _tb_case(m, n, rule, dtype, seed, explicit=False):
    print(f"[traceback] m={m} n={n} rule={rule} dtype={dtype} explicit={explicit}", flush=True)
    c = wfgen.cells(seed, m, n, dtype)
    if dtype == "i32":
        c = (c % 3).astype(np.int32)  # many equal values: the tie-break decides
    top = left = None
    if explicit:
        top = (wfgen.vector(seed + 1, n + 1, dtype) * (3 if dtype == "f32" else 1)).astype(c.dtype)
        left = (wfgen.vector(seed + 2, m, dtype) * (3 if dtype == "f32" else 1)).astype(c.dtype)
    td = None if top is None else _dev(top)
    ld = None if left is None else _dev(left)
    H = wf.solve(_dev(c), rule=rule, top=td, left=ld)
    path, ex = wf.traceback(H, rule, top=td, left=ld)
    if dtype == "f32":
        Ho = oracle.sweep(c, rule, "f32", top=top, left=left)
    else:
        Ho = oracle.sweep(c, rule, "i64", top=None if top is None else top.astype(np.int64),
                          left=None if left is None else left.astype(np.int64)).astype(np.int32)
    assert np.array_equal(_bits(H), Ho.view(np.uint32) if dtype == "f32" else Ho)
    want_path, want_ex = oracle.traceback(Ho, rule, top=top, left=left)
    assert np.array_equal(path.cpu().numpy(), want_path), (m, n)
    assert np.array_equal(ex.cpu().numpy(), want_ex)


@pytest.mark.parametrize("m,n", TB_SHAPES)
@pytest.mark.parametrize("rule", ["min", "max"])
def test_traceback_f32(m, n, rule):
    _tb_case(m, n, rule, "f32", seed=m + n)


@pytest.mark.parametrize("m,n", [(1, 1), (65, 130), (300, 513), (1000, 1000)])
@pytest.mark.parametrize("rule", ["min", "max"])
def test_traceback_i32_with_ties(m, n, rule):
    _tb_case(m, n, rule, "i32", seed=7 * m + n)


@pytest.mark.parametrize("m,n", [(5, 9), (300, 513)])
@pytest.mark.parametrize("rule", ["min", "max"])
def test_traceback_explicit_boundary(m, n, rule):
    _tb_case(m, n, rule, "f32", seed=3, explicit=True)


def test_traceback_of_dtw_identical_sequences():
    x = _seq(77, 1500)
    path, ex = wf.traceback(wf.dtw(_dev(x), _dev(x)))
    assert np.array_equal(path.cpu().numpy(), np.stack([np.arange(1499, -1, -1)] * 2, axis=1))
    assert tuple(ex.cpu().numpy()) == (-1, -1)


@pytest.mark.slow
def test_traceback_16384():
    m = n = 16384
    print("[traceback] 16384^2", flush=True)
    cd = torch.empty((m, n), dtype=torch.float32, device=DEV)
    wfgen.fill_device(cd, seed=2)
    H = wf.solve(cd)
    path, ex = wf.traceback(H)
    want_path, want_ex = oracle.traceback(oracle.sweep(cd.cpu().numpy(), "min", "f32"), "min")
    assert np.array_equal(path.cpu().numpy(), want_path) and np.array_equal(ex.cpu().numpy(), want_ex)
