"""Pins for the CPU oracle: checks against things other than the oracle itself.

- brute-force enumeration of every monotone lattice path (steps S, E, SE) on
  tiny grids, with default and with explicit boundaries (min and max rules,
  float and integer inputs);
- a graph-library shortest/longest path on the cell DAG (scipy Dijkstra and
  Bellman-Ford) for medium grids;
- closed forms: zero and constant inputs, identical rows/columns;
- the streamed-time model of the paper (Eq. 2, Section 2.2), which is the
  identical-rows closed form of the max rule with the three copy/compute
  engines as columns, exact when the H2D stage dominates and a lower bound
  otherwise;
- invariants: transpose, scaling by powers of two, monotonicity, block
  composition through explicit boundaries, first row = sequential prefix sum;
- the fp32 error bound |H32 - H64| <= gamma_{i+j} * H64 for c >= 0, which
  follows from rounding being monotone (fl(c + min(a,b,d)) equals the min of
  the rounded path sums) and the classic bound for a rounded sum of
  non-negative terms.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse
import scipy.sparse.csgraph

import oracle
import wfgen

U = 2.0 ** -24  # unit roundoff of fp32


# ---------------------------------------------------------------- brute force
def _paths_value(c, rule, top=None, left=None):
    """Min (max) over all S/E/SE paths that start at a boundary cell and run
    through interior cells only, of boundary value + sum of c on the path.
    Default boundary: only the corner (value 0) exists."""
    m, n = c.shape
    best = np.full((m, n), np.nan)
    pick = min if rule == "min" else max

    # starts: (row, col, value) of boundary cells; interior successors of a
    # boundary cell (-1, jj) are (0, jj) [S] and (0, jj+1) [SE]; of (ii, -1):
    # (ii, 0) [E] and (ii+1, 0) [SE]; corner (-1,-1): (0,0) [SE].
    starts = []
    if top is None and left is None:
        starts.append(((0, 0), 0.0))
    else:
        top = np.asarray(top, dtype=np.float64) if top is not None else None
        left = np.asarray(left, dtype=np.float64) if left is not None else None
        corner = top[0] if top is not None else 0.0
        starts.append(((0, 0), corner))
        if top is not None:
            for jj in range(n):  # boundary cell (-1, jj) has value top[jj+1]
                v = top[jj + 1]
                starts.append(((0, jj), v))
                if jj + 1 < n:
                    starts.append(((0, jj + 1), v))
        if left is not None:
            for ii in range(m):
                v = left[ii]
                starts.append(((ii, 0), v))
                if ii + 1 < m:
                    starts.append(((ii + 1, 0), v))

    def walk(i, j, acc):
        acc = acc + float(c[i, j])
        cur = best[i, j]
        best[i, j] = acc if np.isnan(cur) else pick(cur, acc)
        for di, dj in ((1, 0), (0, 1), (1, 1)):
            a, b = i + di, j + dj
            if a < m and b < n:
                walk(a, b, acc)

    for (i, j), v in starts:
        if np.isfinite(v):
            walk(i, j, v)
    return best


@pytest.mark.parametrize("rule", ["min", "max"])
def test_bruteforce_default_boundary_float(rule):
    for m, n in itertools.product(range(1, 6), range(1, 6)):
        c = wfgen.cells(100 + 7 * m + n, m, n, "f32")
        H = oracle.sweep(c, rule, "f64")
        B = _paths_value(c.astype(np.float64), rule)
        # inputs are multiples of 2^-24 below 1 and paths have <= 9 cells: every sum is exact in fp64
        assert np.array_equal(H, B), (m, n)


@pytest.mark.parametrize("rule", ["min", "max"])
def test_bruteforce_default_boundary_int(rule):
    for m, n in itertools.product(range(1, 6), range(1, 6)):
        c = wfgen.cells(200 + 7 * m + n, m, n, "i32")
        H = oracle.sweep(c, rule, "i64")
        B = _paths_value(c.astype(np.float64), rule)
        assert np.array_equal(H.astype(np.float64), B), (m, n)


@pytest.mark.parametrize("rule", ["min", "max"])
def test_bruteforce_explicit_boundary(rule):
    for m, n in itertools.product(range(1, 5), range(1, 5)):
        c = wfgen.cells(300 + 7 * m + n, m, n, "f32")
        top = wfgen.vector(400 + m, n + 1, "f32").astype(np.float64) * 3.0
        left = wfgen.vector(500 + n, m, "f32").astype(np.float64) * 3.0
        H = oracle.sweep(c, rule, "f64", top=top, left=left)
        B = _paths_value(c.astype(np.float64), rule, top=top, left=left)
        assert np.array_equal(H, B), (m, n)
        # integer flavour with the same structure
        ci = wfgen.cells(600 + 7 * m + n, m, n, "i32")
        ti = wfgen.vector(700 + m, n + 1, "i32").astype(np.int64) * 2
        li = wfgen.vector(800 + n, m, "i32").astype(np.int64) * 2
        Hi = oracle.sweep(ci, rule, "i64", top=ti, left=li)
        Bi = _paths_value(ci.astype(np.float64), rule, top=ti, left=li)
        assert np.array_equal(Hi.astype(np.float64), Bi), (m, n)


# --------------------------------------------------------- graph library pin
def _dag(c):
    """Cell DAG with edge weight c[target]; node m*n is a source feeding (0,0)."""
    m, n = c.shape
    idx = np.arange(m * n).reshape(m, n)
    src, dst = [m * n], [0]
    for di, dj in ((1, 0), (0, 1), (1, 1)):
        a = idx[: m - di, : n - dj].ravel()
        b = idx[di:, dj:].ravel()
        src.extend(a.tolist())
        dst.extend(b.tolist())
    src = np.array(src)
    dst = np.array(dst)
    w = c.ravel()[dst].astype(np.float64)
    return src, dst, w, m * n + 1


def test_dijkstra_min_rule():
    m, n = 37, 53
    c = wfgen.cells(11, m, n, "f32")
    src, dst, w, N = _dag(c)
    # scipy treats explicit zeros as absent edges; inputs are in [0,1) so shift
    # every weight by +1 and undo it with the path length, which is not unique
    # per target -- instead keep weights as is and replace exact zeros by a
    # tiny positive epsilon whose total effect is far below the tolerance.
    w = np.where(w == 0.0, 1e-300, w)
    G = scipy.sparse.csr_matrix((w, (src, dst)), shape=(N, N))
    dist = scipy.sparse.csgraph.dijkstra(G, directed=True, indices=m * n)[: m * n].reshape(m, n)
    H = oracle.sweep(c, "min", "f64")
    np.testing.assert_allclose(H, dist, rtol=1e-12, atol=1e-250)


def test_bellman_ford_max_rule():
    m, n = 23, 31
    c = wfgen.cells(12, m, n, "f32")
    src, dst, w, N = _dag(c)
    w = -np.where(w == 0.0, 1e-300, w)
    G = scipy.sparse.csr_matrix((w, (src, dst)), shape=(N, N))
    dist = scipy.sparse.csgraph.bellman_ford(G, directed=True, indices=m * n)[: m * n].reshape(m, n)
    H = oracle.sweep(c, "max", "f64")
    np.testing.assert_allclose(H, -dist, rtol=1e-12, atol=1e-250)


# --------------------------------------------------------------- closed forms
@pytest.mark.parametrize("arith", ["f64", "f32"])
def test_zero_input(arith):
    c = np.zeros((40, 70), np.float32)
    for rule in ("min", "max"):
        assert not oracle.sweep(c, rule, arith).any()


@pytest.mark.parametrize("arith", ["f64", "f32"])
def test_constant_input(arith):
    m, n = 90, 130
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    for k in (1.0, 0.5, 2.0 ** -10, 3.0):
        c = np.full((m, n), k, np.float32)
        # min rule: the diagonal steps give max(i,j)+1 cells; max rule: all S/E steps, i+j+1 cells
        assert np.array_equal(oracle.sweep(c, "min", arith), k * (np.maximum(i, j) + 1)), k
        assert np.array_equal(oracle.sweep(c, "max", arith), k * (i + j + 1)), k


def test_identical_rows_closed_form():
    m, n = 60, 45
    p = wfgen.vector(21, n, "f32").astype(np.float64)
    c = np.tile(p.astype(np.float32), (m, 1))
    H = oracle.sweep(c, "min", "f64")
    Hmax = oracle.sweep(c, "max", "f64")
    csum = np.cumsum(p)
    cmin = np.minimum.accumulate(p)
    cmax = np.maximum.accumulate(p)
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    exp_min = csum[None, :] + np.maximum(0, i - j) * cmin[None, :]
    exp_max = csum[None, :] + i * cmax[None, :]
    np.testing.assert_allclose(H, exp_min, rtol=1e-14)
    np.testing.assert_allclose(Hmax, exp_max, rtol=1e-14)
    # identical columns by transposition
    Ht = oracle.sweep(np.ascontiguousarray(c.T), "min", "f64")
    np.testing.assert_allclose(Ht, exp_min.T, rtol=1e-14)


def test_streamed_time_model_eq2():
    """Max rule on an (s chunks) x (3 engines: H2D, COMP, D2H) grid with every
    chunk taking 1/s of each stage time is the flow-shop makespan; its last
    cell is sum(p) + (s-1)*max(p).  When H2D dominates this is
    T_H2D + (T_COMP + T_D2H)/s, the Stage-1 bracket of the streamed model
    (Eq. 2); otherwise Eq. 2 is a lower bound, as the paper remarks."""
    for s in (1, 2, 4, 8, 16, 32):
        for (a, b, d) in ((1.0, 0.25, 0.125), (0.75, 0.5, 0.0625), (0.25, 0.5, 0.125)):
            p = np.array([a, b, d], np.float64) / s
            c = np.tile(p.astype(np.float32), (s, 1))
            H = oracle.sweep(c, "max", "f64")
            last = H[-1, -1]
            assert last == pytest.approx(p.sum() + (s - 1) * p.max(), rel=1e-14)
            eq2 = a + (b + d) / s
            if a >= max(b, d):
                assert last == pytest.approx(eq2, rel=1e-14)
            else:
                assert last >= eq2 - 1e-15


# ----------------------------------------------------------------- invariants
@pytest.mark.parametrize("arith", ["f64", "f32"])
def test_transpose_and_scaling(arith):
    c = wfgen.cells(31, 77, 121, "f32")
    for rule in ("min", "max"):
        H = oracle.sweep(c, rule, arith)
        Ht = oracle.sweep(np.ascontiguousarray(c.T), rule, arith)
        assert np.array_equal(H, Ht.T)
        for e in (-3, 5):
            Hs = oracle.sweep((c * np.float32(2.0 ** e)).astype(np.float32), rule, arith)
            assert np.array_equal(Hs, H * (2.0 ** e))


def test_monotone():
    c = wfgen.cells(32, 50, 60, "f32")
    bump = (wfgen.cells(33, 50, 60, "f32") * np.float32(0.25)).astype(np.float32)
    for rule in ("min", "max"):
        H = oracle.sweep(c, rule, "f64")
        H2 = oracle.sweep((c + bump).astype(np.float32), rule, "f64")
        assert (H2 >= H).all()


@pytest.mark.parametrize("arith", ["f64", "f32", "i64"])
def test_block_composition(arith):
    m, n, mb, nb = 70, 90, 33, 41
    dt = "i32" if arith == "i64" else "f32"
    c = wfgen.cells(34, m, n, dt)
    for rule in ("min", "max"):
        H = oracle.sweep(c, rule, arith)
        odt = H.dtype
        absent = (1 << 62) if arith == "i64" else np.inf
        if rule == "max":
            absent = -absent
        G = np.empty_like(H)
        for r0, r1 in ((0, mb), (mb, m)):
            for c0, c1 in ((0, nb), (nb, n)):
                if r0 == 0:
                    top = np.full(c1 - c0 + 1, absent, odt)
                    top[0] = 0 if c0 == 0 else absent
                else:
                    corner = G[r0 - 1, c0 - 1] if c0 > 0 else absent
                    top = np.concatenate([[corner], G[r0 - 1, c0:c1]]).astype(odt)
                left = G[r0:r1, c0 - 1].astype(odt) if c0 > 0 else np.full(r1 - r0, absent, odt)
                G[r0:r1, c0:c1] = oracle.sweep(np.ascontiguousarray(c[r0:r1, c0:c1]), rule, arith,
                                               top=top, left=left)
        assert np.array_equal(G, H), rule


def test_first_row_is_sequential_prefix_sum():
    c = wfgen.cells(35, 20, 3000, "f32")
    H32 = oracle.sweep(c, "min", "f32")
    assert np.array_equal(H32[0], np.add.accumulate(c[0], dtype=np.float32))
    assert np.array_equal(H32[:, 0], np.add.accumulate(c[:, 0], dtype=np.float32))
    H64 = oracle.sweep(c, "max", "f64")
    assert np.array_equal(H64[0], np.add.accumulate(c[0].astype(np.float64)))


def test_banded_sweep_matches_whole():
    m, n = 300, 200
    c = wfgen.cells(36, m, n, "f32")
    H = oracle.sweep(c, "min", "f32")
    lr, lc, rows = oracle.sweep_banded(lambda r0, k: wfgen.cells(36, m, n, "f32", r0, k), m, n, "min", "f32",
                                       band=64, want_rows=(0, 131, 299))
    assert np.array_equal(lr, H[-1]) and np.array_equal(lc, H[:, -1])
    for r in (0, 131, 299):
        assert np.array_equal(rows[r], H[r])


# --------------------------------------------------------------- error bound
def _gamma(k):
    return k * U / (1 - k * U)


def test_fp32_error_bound():
    m, n = 400, 500
    c = wfgen.cells(37, m, n, "f32")
    for rule in ("min", "max"):
        H32 = oracle.sweep(c, rule, "f32").astype(np.float64)
        H64 = oracle.sweep(c, rule, "f64")
        i = np.arange(m)[:, None]
        j = np.arange(n)[None, :]
        bound = _gamma(i + j + 1) * H64
        assert (np.abs(H32 - H64) <= bound).all(), rule


def test_int_matches_float_on_integer_inputs():
    c = wfgen.cells(38, 80, 90, "i32")
    Hi = oracle.sweep(c, "min", "i64")
    Hf = oracle.sweep(c.astype(np.float32), "min", "f64")
    assert np.array_equal(Hi.astype(np.float64), Hf)


def test_empty_and_degenerate_shapes():
    for m, n in ((0, 5), (5, 0), (0, 0)):
        H = oracle.sweep(np.zeros((m, n), np.float32), "min", "f64")
        assert H.shape == (m, n)
    c = wfgen.cells(39, 1, 50, "f32")
    assert np.array_equal(oracle.sweep(c, "min", "f32")[0], np.add.accumulate(c[0], dtype=np.float32))


# ------------------------------------------------------- pins detect mistakes
def test_pins_reject_a_planted_mistake():
    """A variant with the NW term dropped differs from the brute force, so the
    brute-force pin would catch that mistake in the oracle."""
    m, n = 4, 4
    c = np.array([[0.5, 0.9, 0.9, 0.9],
                  [0.9, 0.1, 0.9, 0.9],
                  [0.9, 0.9, 0.1, 0.9],
                  [0.9, 0.9, 0.9, 0.1]], np.float32)
    B = _paths_value(c.astype(np.float64), "min")
    wrong = np.zeros((m, n))
    for i in range(m):
        for j in range(n):
            cands = []
            if i > 0:
                cands.append(wrong[i - 1, j])
            if j > 0:
                cands.append(wrong[i, j - 1])
            wrong[i, j] = float(c[i, j]) + (min(cands) if cands else 0.0)
    assert not np.array_equal(wrong, B)
    assert np.array_equal(oracle.sweep(c, "min", "f64"), B)
