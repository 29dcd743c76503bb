"""GPU parity: the HIP sweep (through the C ABI) against the CPU oracle, element
by element, on seeded inputs.

Bar: bit-exact for fp32 against the fp32 oracle loop (the result of
"one rounding after an exact min/max" does not depend on evaluation order) and
bit-exact for int32; against the fp64 oracle every cell must satisfy
|H32 - H64| <= gamma_{i+j+1} * |H64| (the rounding bound pinned in
test_oracle_pins.py).  Shapes cover one row/column, several bands of every
band shape (64-row bands; 128-row bands of two compute waves chained through
LDS, or of one wave whose lanes own two rows each), ragged tails and leading
dimensions larger than n.
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_2501_05938_amd as wf  # noqa: E402
import wfgen  # noqa: E402

U = 2.0 ** -24
DEV = torch.device("cuda:0")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _gamma_bound(H64):
    m, n = H64.shape
    k = (np.arange(m)[:, None] + np.arange(n)[None, :] + 1).astype(np.float64)
    return k * U / (1 - k * U) * np.abs(H64)


def _case(m, n, rule="min", dtype="f32", seed=1, explicit=False, ld_pad=0, pad_value=0, waves_per_wg=0,
          rows_per_lane=0, sides="both"):
    print(f"[parity] m={m} n={n} rule={rule} dtype={dtype} seed={seed} explicit={explicit} ld_pad={ld_pad} "
          f"pad_value={pad_value} W={waves_per_wg} R={rows_per_lane}", flush=True)
    c = wfgen.cells(seed, m, n, dtype)
    top = left = None
    if explicit:
        top = (wfgen.vector(seed + 100, n + 1, dtype) * (3 if dtype == "f32" else 2)).astype(c.dtype)
        left = (wfgen.vector(seed + 200, m, dtype) * (3 if dtype == "f32" else 2)).astype(c.dtype)
        if sides == "top":
            left = None
        elif sides == "left":
            top = None
    if ld_pad:
        cb = np.full((m, n + ld_pad), pad_value, np.uint32).view(c.dtype)
        cb[:, :n] = c
        cd = _dev(cb)[:, :n]
        out = torch.full((m, n + ld_pad), float("nan") if dtype == "f32" else -7, dtype=cd.dtype, device=DEV)[:, :n]
    else:
        cd = _dev(c)
        out = torch.full((m, n), float("nan") if dtype == "f32" else -7, dtype=cd.dtype, device=DEV)
    H = wf.solve(cd, out=out, rule=rule, top=None if top is None else _dev(top),
                 left=None if left is None else _dev(left), waves_per_wg=waves_per_wg,
                 rows_per_lane=rows_per_lane)
    got = _host(H)
    wf.check()
    if dtype == "f32":
        exp32 = oracle.sweep(c, rule, "f32", top=top, left=left)
        bad = np.argwhere(got.view(np.uint32) != exp32.view(np.uint32))
        assert bad.size == 0, f"{len(bad)} cells differ; first {bad[:5].tolist()} got {got[tuple(bad[0])]} want {exp32[tuple(bad[0])]}"
        exp64 = oracle.sweep(c, rule, "f64", top=None if top is None else top.astype(np.float64),
                             left=None if left is None else left.astype(np.float64))
        assert (np.abs(got.astype(np.float64) - exp64) <= _gamma_bound(exp64)).all()
    else:
        exp = oracle.sweep(c, rule, "i64", top=None if top is None else top.astype(np.int64),
                           left=None if left is None else left.astype(np.int64))
        assert np.array_equal(got.astype(np.int64), exp)
    return got


SMALL = [(1, 1), (1, 2), (2, 1), (1, 100), (100, 1), (3, 5), (5, 3), (63, 63), (64, 64), (65, 65),
         (64, 1000), (100, 37), (37, 100), (128, 128), (129, 300)]
MEDIUM = [(256, 256), (300, 513), (511, 700), (512, 512), (700, 129), (1024, 1024)]
TALL = [(2047, 100), (2048, 77), (2100, 333), (4097, 65), (64, 4099)]


@pytest.mark.parametrize("m,n", SMALL)
def test_small_shapes_f32_min(m, n):
    _case(m, n)


@pytest.mark.parametrize("m,n", MEDIUM + TALL)
def test_banded_shapes_f32_min(m, n):
    _case(m, n, seed=2)


@pytest.mark.parametrize("m,n", [(1, 1), (65, 65), (300, 513), (2100, 333)])
def test_max_rule(m, n):
    _case(m, n, rule="max", seed=3)


@pytest.mark.parametrize("m,n", [(1, 7), (65, 65), (300, 513), (2100, 333)])
@pytest.mark.parametrize("rule", ["min", "max"])
def test_int32(m, n, rule):
    _case(m, n, rule=rule, dtype="i32", seed=4)


@pytest.mark.parametrize("m,n", [(1, 1), (7, 9), (129, 300), (2100, 333)])
@pytest.mark.parametrize("dtype", ["f32", "i32"])
def test_explicit_boundary(m, n, dtype):
    _case(m, n, dtype=dtype, seed=5, explicit=True)
    _case(m, n, rule="max", dtype=dtype, seed=6, explicit=True)


@pytest.mark.parametrize("m,n", [(65, 65), (600, 1000)])
def test_leading_dimension(m, n):
    _case(m, n, seed=7, ld_pad=13)


@pytest.mark.parametrize("m,n", [(65, 65), (300, 513), (130, 1000)])
@pytest.mark.parametrize("dtype", ["f32", "i32"])
def test_row_padding_holding_the_sentinel(m, n, dtype):
    """Row padding (ld_cost > n) that holds the handoff sentinel's bit pattern (0xFFFFFFFF
    for fp32, INT32_MIN for int32) must neither change a cell nor stall a band."""
    pad = 0xFFFFFFFF if dtype == "f32" else 0x80000000
    _case(m, n, dtype=dtype, seed=9, ld_pad=5, pad_value=pad)
    _case(m, n, rule="max", dtype=dtype, seed=9, ld_pad=5, pad_value=pad, waves_per_wg=2)
    _case(m, n, dtype=dtype, seed=9, ld_pad=5, pad_value=pad, rows_per_lane=1)


@pytest.mark.parametrize("m,n", [(1, 1), (65, 65), (129, 300), (300, 513), (2100, 333), (1024, 1024)])
@pytest.mark.parametrize("rule", ["min", "max"])
def test_two_compute_waves_per_workgroup(m, n, rule):
    """wf_solve_tuned with bands of 128 rows: two compute waves chained through LDS."""
    _case(m, n, rule=rule, seed=10, waves_per_wg=2)


@pytest.mark.parametrize("m,n", [(1, 1), (1, 300), (63, 63), (64, 64), (65, 65), (127, 5), (128, 128), (129, 300),
                                 (300, 513), (2100, 333), (1024, 1024), (4097, 65)])
@pytest.mark.parametrize("rule", ["min", "max"])
def test_one_row_per_lane(m, n, rule):
    """wf_solve_tuned with 64-row bands given explicitly (the shape wf_solve picks)."""
    _case(m, n, rule=rule, seed=12, rows_per_lane=1)


@pytest.mark.parametrize("m,n", [(1, 1), (2, 3), (63, 63), (64, 64), (65, 65), (127, 5), (128, 128), (129, 300),
                                 (255, 700), (256, 256), (257, 1000), (2100, 333)])
@pytest.mark.parametrize("dtype", ["f32", "i32"])
def test_two_rows_per_lane(m, n, dtype):
    """wf_solve_tuned with 128-row bands of one wave whose lanes own two rows, from one
    row to several bands, with ragged last bands."""
    _case(m, n, dtype=dtype, seed=13, rows_per_lane=2)
    _case(m, n, rule="max", dtype=dtype, seed=14, explicit=True, rows_per_lane=2)


@pytest.mark.parametrize("m,n", [(65, 65), (300, 513), (2100, 333)])
@pytest.mark.parametrize("sides", ["top", "left"])
@pytest.mark.parametrize("R", [1, 2])
def test_one_sided_explicit_boundary(m, n, sides, R):
    """An explicit top with the default left boundary takes the first chunks without
    per-cell selection (the cells left of column 0 stay absent by themselves); an explicit
    left boundary takes them with it.  Both bit-exact, both rules."""
    _case(m, n, seed=15, explicit=True, sides=sides, rows_per_lane=R)
    _case(m, n, rule="max", seed=16, explicit=True, sides=sides, rows_per_lane=R)


def test_two_waves_of_two_rows_is_rejected():
    a = torch.zeros((4, 4), dtype=torch.float32, device=DEV)
    with pytest.raises(wf.WfError) as e:
        wf.solve(a, waves_per_wg=2, rows_per_lane=2)
    assert e.value.status == -8  # WF_EUNSUPPORTED


def test_config_small_grid_1024_and_repeatability():
    """The 1024 x 1024 configuration, twice, bit-identical both times."""
    a = _case(1024, 1024, seed=1)
    b = _case(1024, 1024, seed=1)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("m,n", [(1, 1), (70, 300), (2100, 333)])
def test_edges_mode(m, n):
    print(f"[edges] m={m} n={n}", flush=True)
    c = wfgen.cells(8, m, n, "f32")
    lr, lc, fc = wf.solve(_dev(c), mode="edges")
    exp = oracle.sweep(c, "min", "f32")
    assert np.array_equal(_host(lr).view(np.uint32), exp[-1].view(np.uint32))
    assert np.array_equal(_host(lc).view(np.uint32), exp[:, -1].view(np.uint32))
    assert _host(fc)[0] == exp[-1, -1]


def test_device_fill_matches_host_generator():
    for dtype, tdt in (("f32", torch.float32), ("i32", torch.int32)):
        t = torch.empty((300, 517), dtype=tdt, device=DEV)
        wfgen.fill_device(t, seed=123, row0=40)
        exp = wfgen.cells(123, 340, 517, dtype, 40, 300)
        assert np.array_equal(_host(t), exp)


def test_empty_grid_is_a_no_op():
    c = torch.empty((0, 5), dtype=torch.float32, device=DEV)
    out = wf.solve(c)
    assert out.shape == (0, 5)


@pytest.mark.slow
def test_full_size_16384_against_fp32_oracle():
    """The 16384 x 16384 configuration, launched as the benchmark launches it:
    device-filled input, whole output compared bit-exactly with the fp32 oracle."""
    m = n = 16384
    print("[parity] 16384^2 full grid", flush=True)
    cd = torch.empty((m, n), dtype=torch.float32, device=DEV)
    wfgen.fill_device(cd, seed=2)
    H = wf.solve(cd)
    got = _host(H)
    wf.check()
    c = wfgen.cells(2, m, n, "f32")
    exp = oracle.sweep(c, "min", "f32")
    bad = np.count_nonzero(got.view(np.uint32) != exp.view(np.uint32))
    assert bad == 0, f"{bad} cells differ"
    # fp64 bound on rows 0, 1, n/2, n-2, n-1 and 64 seeded random rows (final cell included)
    rows = [0, 1, n // 2, m - 2, m - 1] + [int(r) for r in np.random.default_rng(2).choice(m, 64, replace=False)]
    del exp
    _, _, want = oracle.sweep_banded(lambda r0, k: c[r0:r0 + k], m, n, "min", "f64", band=2048, want_rows=rows)
    for r in rows:
        k = (r + np.arange(n) + 1).astype(np.float64)
        assert (np.abs(got[r].astype(np.float64) - want[r]) <= k * U / (1 - k * U) * want[r]).all(), r


@pytest.mark.slow
def test_full_size_65536_edges_against_fp32_oracle():
    """The 65536 x 65536 configuration (17 GB input, device-resident) in edges mode, as
    the benchmark launches it: last row, last column and final cell bit-exact against
    the fp32 oracle, swept band by band on the host from the same generated input."""
    m = n = 65536
    print("[parity] 65536^2 edges", flush=True)
    cd = torch.empty((m, n), dtype=torch.float32, device=DEV)
    wfgen.fill_device(cd, seed=3)
    lr, lc, fc = wf.solve(cd, mode="edges")
    got_lr, got_lc, got_fc = _host(lr), _host(lc), _host(fc)
    wf.check()

    def rows(row0, nrows):
        return cd[row0:row0 + nrows].cpu().numpy()

    # fp32 (bit-exact) and fp64 (rounding bound) oracles band by band, on two threads over
    # the same host copy of each band (the oracle's C loop runs without the GIL).
    from concurrent.futures import ThreadPoolExecutor
    band = 2048
    last32 = last64 = None
    lc32 = np.empty(m, np.float32)
    lc64 = np.empty(m, np.float64)
    with ThreadPoolExecutor(2) as pool:
        for row0 in range(0, m, band):
            cb = rows(row0, band)
            t32 = None if last32 is None else np.concatenate([[np.inf], last32]).astype(np.float32)
            t64 = None if last64 is None else np.concatenate([[np.inf], last64])
            l32 = np.full(band, np.inf, np.float32)
            l64 = np.full(band, np.inf)
            f32 = pool.submit(oracle.sweep, cb, "min", "f32", t32, l32, False)
            f64 = pool.submit(oracle.sweep, cb, "min", "f64", t64, l64, False)
            (last32, c32), (last64, c64) = f32.result(), f64.result()
            lc32[row0:row0 + band], lc64[row0:row0 + band] = c32, c64
    assert np.array_equal(got_lr.view(np.uint32), last32.view(np.uint32))
    assert np.array_equal(got_lc.view(np.uint32), lc32.view(np.uint32))
    assert got_fc.view(np.uint32)[0] == last32.view(np.uint32)[-1]
    j = np.arange(n, dtype=np.float64)
    k = (m - 1) + j + 1
    assert (np.abs(got_lr.astype(np.float64) - last64) <= k * U / (1 - k * U) * last64).all()
    i = np.arange(m, dtype=np.float64)
    k = i + (n - 1) + 1
    assert (np.abs(got_lc.astype(np.float64) - lc64) <= k * U / (1 - k * U) * lc64).all()
