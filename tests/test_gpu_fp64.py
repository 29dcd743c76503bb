"""GPU parity of the fp64 sweep (the paper's own precision) through the C ABI.

Bar: bit-exact against the oracle's fp64 loop over fp64 inputs (one fp64 rounding
per cell after an exact min/max, so the result does not depend on evaluation order).
Inputs use all 53 bits of the mantissa.  Shapes cover single rows and columns,
several bands, ragged tails, explicit boundaries, row padding holding the handoff
sentinel's bit pattern, edges mode, batches, the allocation-free entry point's shape
rule, the traceback, and the 1024 x 1024 and 16384 x 16384 grids.
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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _bits(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def _case(m, n, rule="min", seed=1, explicit=False, ld_pad=0, pad_bits=0):
    print(f"[fp64] m={m} n={n} rule={rule} seed={seed} explicit={explicit} ld_pad={ld_pad}", flush=True)
    c = wfgen.cells(seed, m, n, "f64")
    top = left = None
    if explicit:
        top = wfgen.vector(seed + 100, n + 1, "f64") * 3
        left = wfgen.vector(seed + 200, m, "f64") * 3
    if ld_pad:
        cb = np.full((m, n + ld_pad), pad_bits, np.uint64).view(np.float64)
        cb[:, :n] = c
        cd = _dev(cb)[:, :n]
    else:
        cd = _dev(c)
    H = wf.solve(cd, rule=rule, top=None if top is None else _dev(top), left=None if left is None else _dev(left))
    got = _bits(H)
    wf.check()
    want = oracle.sweep(c, rule, "d64", top=top, left=left).view(np.uint64)
    bad = np.argwhere(got != want)
    assert bad.size == 0, f"{len(bad)} cells differ; first {bad[:5].tolist()}"
    return H


SHAPES = [(1, 1), (1, 100), (100, 1), (3, 5), (63, 63), (64, 64), (65, 65), (64, 1000), (129, 300), (300, 513),
          (2100, 333), (4097, 65), (64, 4099)]


@pytest.mark.parametrize("m,n", SHAPES)
@pytest.mark.parametrize("rule", ["min", "max"])
def test_fp64_shapes(m, n, rule):
    _case(m, n, rule, seed=m + 3 * n)


@pytest.mark.parametrize("m,n", [(1, 1), (7, 9), (129, 300), (2100, 333)])
@pytest.mark.parametrize("rule", ["min", "max"])
def test_fp64_explicit_boundary(m, n, rule):
    _case(m, n, rule, seed=5, explicit=True)


@pytest.mark.parametrize("m,n", [(65, 65), (300, 513)])
def test_fp64_row_padding_holding_the_sentinel(m, n):
    _case(m, n, seed=9, ld_pad=5, pad_bits=0xFFFFFFFFFFFFFFFF)
    _case(m, n, "max", seed=9, ld_pad=3, pad_bits=0xFFFFFFFF00000000)


def test_fp64_1024():
    a = _case(1024, 1024, seed=1)
    b = _case(1024, 1024, seed=1)
    assert torch.equal(a, b)


# (64, 1000), (128, 300), (192, 4099): the last band is full, so its interior chunks
# write the last row from their 16-byte quads.
@pytest.mark.parametrize("m,n", [(1, 1), (70, 300), (2100, 333), (64, 1000), (128, 300), (192, 4099)])
def test_fp64_edges(m, n):
    c = wfgen.cells(8, m, n, "f64")
    lr, lc, fc = wf.solve(_dev(c), mode="edges")
    want = oracle.sweep(c, "min", "d64")
    assert np.array_equal(_bits(lr), want[-1].view(np.uint64))
    assert np.array_equal(_bits(lc), np.ascontiguousarray(want[:, -1]).view(np.uint64))
    assert _bits(fc)[0] == want[-1:, -1].view(np.uint64)[0]


def test_fp64_batch_and_traceback():
    shapes = wfgen.batch_shapes(24, lo=1, hi=600, seed=21)
    hs = [wfgen.cells(wfgen.batch_seed(g), m, n, "f64") for g, (m, n) in enumerate(shapes)]
    outs = wf.solve_batched([_dev(h) for h in hs], use_graph=0)
    torch.cuda.synchronize()
    for (m, n), h, o in zip(shapes, hs, outs):
        assert np.array_equal(_bits(o), oracle.sweep(h, "min", "d64").view(np.uint64)), (m, n)
    m, n = 700, 333
    c = wfgen.cells(31, m, n, "f64")
    H = wf.solve(_dev(c))
    path, ex = wf.traceback(H)
    want_path, want_ex = oracle.traceback(oracle.sweep(c, "min", "d64"), "min")
    assert np.array_equal(path.cpu().numpy(), want_path) and np.array_equal(ex.cpu().numpy(), want_ex)


def test_fp64_rejections():
    a = torch.zeros((4, 4), dtype=torch.float64, device=DEV)
    with pytest.raises(wf.WfError) as e:
        wf.solve(a, rows_per_lane=2)
    assert e.value.status == -8  # WF_EUNSUPPORTED
    with pytest.raises(wf.WfError) as e:
        wf.solve(a, waves_per_wg=2)
    assert e.value.status == -8
    with wf.Server(budget_bytes=1 << 20) as srv:
        with pytest.raises(wf.WfError) as e:
            srv.submit(a)
        assert e.value.status == -8


@pytest.mark.slow
def test_fp64_16384():
    """The 16384 x 16384 fp64 grid as the benchmark runs it (device-filled input), whole
    grid bit-exact against the oracle's fp64 loop."""
    m = n = 16384
    print("[fp64] 16384^2", flush=True)
    cd = torch.empty((m, n), dtype=torch.float64, device=DEV)
    wfgen.fill_device(cd, seed=2)
    H = wf.solve(cd)
    got = _bits(H)
    want = oracle.sweep(cd.cpu().numpy(), "min", "d64").view(np.uint64)
    assert np.array_equal(got, want)
