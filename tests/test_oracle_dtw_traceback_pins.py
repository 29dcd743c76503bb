"""Pins for the oracle's fp64-input sweep, its dynamic time warping and its
traceback, each against something other than the oracle itself:

- brute force over every monotone lattice path on tiny grids, with exact
  (dyadic) inputs, and with the path sums rounded step by step along the path
  (which must reproduce the one-rounding-per-cell loop bit for bit, because
  rounding is monotone);
- exact rational arithmetic (fractions) and the classic error bound for fp64;
- closed forms for constant inputs and constant sequences;
- a textbook memoised recursion for DTW, symmetry D(y, x) = D(x, y)^T and
  D(x, x) = 0 on the diagonal;
- for the traceback: the path re-summed from its boundary cell reproduces the
  final cell exactly, every step satisfies the cell rule with the chosen
  predecessor, brute-force optimal paths with the NW > N > W preference, and
  the closed-form path of a constant grid.
"""
import functools
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle


# ------------------------------------------------------------------ helpers
def _monotone_paths(m, n):
    """Every S/E/SE path from (0,0) to (m-1,n-1), as lists of cells."""
    out = []

    def rec(i, j, acc):
        acc = acc + [(i, j)]
        if (i, j) == (m - 1, n - 1):
            out.append(acc)
            return
        for di, dj in ((1, 0), (0, 1), (1, 1)):
            a, b = i + di, j + dj
            if a < m and b < n:
                rec(a, b, acc)

    rec(0, 0, [])
    return out


def _paths_to(i, j):
    return _monotone_paths(i + 1, j + 1)


def _dyadic(rng, shape, bits=8, hi=4):
    return (rng.integers(0, hi << bits, size=shape) / float(1 << bits)).astype(np.float64)


# ------------------------------------------------------------- fp64 inputs
@pytest.mark.parametrize("rule", ["min", "max"])
@pytest.mark.parametrize("m,n", [(1, 1), (2, 3), (3, 2), (4, 4), (5, 3)])
def test_d64_brute_force_exact_inputs(rule, m, n):
    c = _dyadic(np.random.default_rng(m * 10 + n), (m, n))
    H = oracle.sweep(c, rule, "d64")
    pick = min if rule == "min" else max
    for i in range(m):
        for j in range(n):
            want = pick(sum(Fraction(float(c[a, b])) for a, b in p) for p in _paths_to(i, j))
            assert Fraction(float(H[i, j])) == want, (i, j)


@pytest.mark.parametrize("rule", ["min", "max"])
def test_d64_equals_min_of_stepwise_rounded_path_sums(rule):
    """With arbitrary doubles, H[i][j] is the min (max) over paths of the path sum
    rounded after every step: one fp64 rounding per cell, nothing else."""
    rng = np.random.default_rng(7)
    m, n = 4, 5
    c = rng.random((m, n)) * 3.0
    H = oracle.sweep(c, rule, "d64")
    pick = min if rule == "min" else max
    for i in range(m):
        for j in range(n):
            sums = []
            for p in _paths_to(i, j):
                acc = 0.0
                for a, b in p:
                    acc = float(np.float64(c[a, b]) + np.float64(acc))
                sums.append(acc)
            assert H[i, j] == pick(sums), (i, j)


def test_d64_error_bound_against_exact_rationals():
    rng = np.random.default_rng(8)
    m, n = 5, 5
    c = rng.random((m, n))
    H = oracle.sweep(c, "min", "d64")
    u = Fraction(1, 2 ** 53)
    for i in range(m):
        for j in range(n):
            exact = min(sum(Fraction(float(c[a, b])) for a, b in p) for p in _paths_to(i, j))
            k = i + j + 1
            gamma = k * u / (1 - k * u)
            assert abs(Fraction(float(H[i, j])) - exact) <= gamma * exact


@pytest.mark.parametrize("k", [0.0, 0.75, 3.0, 1.0 / 1024])
def test_d64_constant_closed_forms(k):
    m, n = 37, 53
    c = np.full((m, n), k)
    ii, jj = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
    assert np.array_equal(oracle.sweep(c, "min", "d64"), k * (np.maximum(ii, jj) + 1))
    assert np.array_equal(oracle.sweep(c, "max", "d64"), k * (ii + jj + 1))


# ---------------------------------------------------------------------- DTW
def _textbook_dtw(x, y):
    """Memoised recursion of the DTW definition, in float32 arithmetic."""
    x = [np.float32(v) for v in x]
    y = [np.float32(v) for v in y]

    @functools.lru_cache(maxsize=None)
    def D(i, j):
        if i < 0 and j < 0:
            return np.float32(0.0)
        if i < 0 or j < 0:
            return np.float32(np.inf)
        best = min(D(i - 1, j), D(i, j - 1), D(i - 1, j - 1))
        return np.float32(np.abs(np.float32(x[i] - y[j])) + best)

    return np.array([[D(i, j) for j in range(len(y))] for i in range(len(x))], dtype=np.float32)


@pytest.mark.parametrize("m,n", [(1, 1), (1, 5), (5, 1), (4, 6), (7, 7), (9, 4)])
def test_dtw_textbook_recursion(m, n):
    rng = np.random.default_rng(m * 31 + n)
    x = rng.standard_normal(m).astype(np.float32)
    y = rng.standard_normal(n).astype(np.float32)
    want = _textbook_dtw(x, y)
    assert np.array_equal(oracle.dtw(x, y).view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("m,n", [(2, 3), (4, 4), (3, 5)])
def test_dtw_brute_force_warping_paths(m, n):
    rng = np.random.default_rng(m + 100 * n)
    x = rng.integers(-8, 9, m).astype(np.float32)
    y = rng.integers(-8, 9, n).astype(np.float32)
    D = oracle.dtw(x, y)
    for i in range(m):
        for j in range(n):
            want = min(sum(abs(float(x[a]) - float(y[b])) for a, b in p) for p in _paths_to(i, j))
            assert D[i, j] == want, (i, j)


def test_dtw_symmetry_identity_and_constants():
    rng = np.random.default_rng(3)
    x = rng.standard_normal(200).astype(np.float32)
    y = rng.standard_normal(150).astype(np.float32)
    Dxy, Dyx = oracle.dtw(x, y), oracle.dtw(y, x)
    assert np.array_equal(Dxy.view(np.uint32), Dyx.T.view(np.uint32))
    Dxx = oracle.dtw(x, x)
    assert np.all(np.diag(Dxx) == 0.0) and np.all(Dxx >= 0)
    a, b = np.float32(1.25), np.float32(-0.5)
    Dc = oracle.dtw(np.full(30, a, np.float32), np.full(40, b, np.float32))
    ii, jj = np.meshgrid(np.arange(30), np.arange(40), indexing="ij")
    assert np.array_equal(Dc, np.float32(1.75) * (np.maximum(ii, jj) + 1).astype(np.float32))


def test_dtw_equals_sweep_of_materialised_cost():
    rng = np.random.default_rng(4)
    x = rng.random(123).astype(np.float32)
    y = rng.random(77).astype(np.float32)
    c = np.abs(x[:, None] - y[None, :]).astype(np.float32)  # numpy rounds the difference once in fp32
    assert np.array_equal(oracle.dtw(x, y).view(np.uint32), oracle.sweep(c, "min", "f32").view(np.uint32))
    lr, lc = oracle.dtw(x, y, full=False)
    D = oracle.dtw(x, y)
    assert np.array_equal(lr, D[-1]) and np.array_equal(lc, D[:, -1])


# ---------------------------------------------------------------- traceback
def _resum(c, path, exit_, H, rule, top=None, left=None, dtype=np.float32):
    """Re-add c along the path (start to end) from the boundary value it left through."""
    ei, ej = int(exit_[0]), int(exit_[1])
    absent = np.inf if rule == "min" else -np.inf
    if ei == -1:
        v = top[ej + 1] if top is not None else (0.0 if ej == -1 else absent)
    else:
        v = left[ei] if left is not None else absent
    acc = dtype(v)
    for (i, j) in path[::-1]:
        acc = dtype(dtype(c[i, j]) + acc)
    return acc


@pytest.mark.parametrize("rule", ["min", "max"])
@pytest.mark.parametrize("m,n", [(1, 1), (1, 9), (9, 1), (40, 70), (70, 40), (128, 128)])
def test_traceback_resum_and_cell_rule(rule, m, n):
    rng = np.random.default_rng(m * n + (rule == "max"))
    c = rng.random((m, n)).astype(np.float32)
    H = oracle.sweep(c, rule, "f32")
    path, ex = oracle.traceback(H, rule)
    assert tuple(path[0]) == (m - 1, n - 1)
    assert len(path) <= m + n - 1
    assert _resum(c, path, ex, H, rule) == H[-1, -1]
    # every step is a move to NW, N or W, and the cell rule holds with that predecessor
    steps = np.vstack([path, ex[None, :]])
    d = steps[:-1] - steps[1:]
    assert all(tuple(s) in ((1, 1), (1, 0), (0, 1)) for s in d)
    for (i, j), (pi, pj) in zip(steps[:-1], steps[1:]):
        if pi >= 0 and pj >= 0:
            assert H[i, j] == np.float32(c[i, j] + H[pi, pj])


@pytest.mark.parametrize("rule", ["min", "max"])
def test_traceback_explicit_boundary_resum(rule):
    rng = np.random.default_rng(11)
    m, n = 33, 47
    c = rng.random((m, n)).astype(np.float32)
    top = (rng.random(n + 1) * 3).astype(np.float32)
    left = (rng.random(m) * 3).astype(np.float32)
    H = oracle.sweep(c, rule, "f32", top=top, left=left)
    path, ex = oracle.traceback(H, rule, top=top, left=left)
    assert ex[0] == -1 or ex[1] == -1
    assert _resum(c, path, ex, H, rule, top, left) == H[-1, -1]


def _brute_force_traceback(c, rule):
    """Optimal path values from brute force (exact integers); then from the end,
    step to the first of NW, N, W that lies on an optimal path to here."""
    m, n = c.shape
    pick = min if rule == "min" else max
    best = {}
    for i in range(m):
        for j in range(n):
            best[(i, j)] = pick(sum(int(c[a, b]) for a, b in p) for p in _paths_to(i, j))
    path = [(m - 1, n - 1)]
    i, j = m - 1, n - 1
    while True:
        nxt = None
        for di, dj in ((-1, -1), (-1, 0), (0, -1)):
            a, b = i + di, j + dj
            if (a, b) == (-1, -1) and (i, j) == (0, 0):
                nxt = (a, b)
                break
            if a >= 0 and b >= 0 and best[(a, b)] + int(c[i, j]) == best[(i, j)]:
                nxt = (a, b)
                break
        i, j = nxt
        if i < 0 or j < 0:
            return np.array(path, dtype=np.int32), np.array([i, j], dtype=np.int32)
        path.append((i, j))


@pytest.mark.parametrize("rule", ["min", "max"])
@pytest.mark.parametrize("m,n,seed", [(3, 3, 1), (4, 5, 2), (5, 4, 3), (5, 5, 4), (2, 6, 5)])
def test_traceback_brute_force_with_ties(rule, m, n, seed):
    c = np.random.default_rng(seed).integers(0, 3, (m, n)).astype(np.int32)  # many equal values
    H = oracle.sweep(c, rule, "i64").astype(np.int32)
    path, ex = oracle.traceback(H, rule)
    want_path, want_ex = _brute_force_traceback(c, rule)
    assert np.array_equal(path, want_path) and np.array_equal(ex, want_ex)


@pytest.mark.parametrize("m,n", [(7, 7), (9, 4), (4, 9), (1, 5)])
def test_traceback_constant_grid_closed_form(m, n):
    """c == 1: NW ties with N (or W) everywhere off the diagonal, so the path takes
    min(m, n) - 1 diagonal steps, then runs straight to (0, 0) and leaves through the corner."""
    H = oracle.sweep(np.ones((m, n), np.float32), "min", "f32")
    path, ex = oracle.traceback(H, "min")
    k = min(m, n) - 1
    want = [(m - 1 - t, n - 1 - t) for t in range(k + 1)]
    i, j = want[-1]
    while (i, j) != (0, 0):
        i, j = (i - 1, j) if i > 0 else (i, j - 1)
        want.append((i, j))
    assert [tuple(p) for p in path] == want
    assert tuple(ex) == (-1, -1)


def test_traceback_of_dtw_identical_sequences_is_the_diagonal():
    x = np.random.default_rng(9).standard_normal(64).astype(np.float32)
    path, ex = oracle.traceback(oracle.dtw(x, x), "min")
    assert [tuple(p) for p in path] == [(i, i) for i in range(63, -1, -1)]
    assert tuple(ex) == (-1, -1)


def _python_traceback(H, order):
    """A copy of the traceback rule in Python with a given preference order, for the
    planted-mistake check below."""
    m, n = H.shape
    i, j, path = m - 1, n - 1, []
    moves = {"NW": (-1, -1), "N": (-1, 0), "W": (0, -1)}
    while i >= 0 and j >= 0:
        path.append((i, j))
        vals = {}
        for name, (di, dj) in moves.items():
            a, b = i + di, j + dj
            vals[name] = (0.0 if (a, b) == (-1, -1) else np.inf) if (a < 0 or b < 0) else float(H[a, b])
        best = min(vals[o] for o in order)
        pick = next(o for o in order if vals[o] == best)
        i, j = i + moves[pick][0], j + moves[pick][1]
    return path


def test_planted_tiebreak_mistake_is_caught():
    """Preferring N over NW (a plausible slip) changes the path on a constant grid, where
    the closed-form pin above fixes the diagonal first; the oracle's own order passes it."""
    H = oracle.sweep(np.ones((9, 4), np.float32), "min", "f32")
    path, _ = oracle.traceback(H, "min")
    assert _python_traceback(H, ("NW", "N", "W")) == [tuple(p) for p in path]
    assert _python_traceback(H, ("N", "NW", "W")) != [tuple(p) for p in path]
