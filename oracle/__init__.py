"""CPU oracle for the anti-diagonal wavefront sweep.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check in
__graft_entry__.py and by the cpu_baseline leg of bench.py.  The product
library never imports, links or loads anything from here, and this package
imports nothing from the product package.

The arithmetic lives in wf_oracle.c (a plain row-major double loop, built with
gcc into liboracle.so); this module only marshals numpy arrays.  See the
header of wf_oracle.c for the cell rule and boundary convention.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

RULES = {"min": 0, "max": 1}


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
               "-std=c99", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        p = ctypes.c_void_p
        i64 = ctypes.c_int64
        for name in ("oracle_sweep_f64", "oracle_sweep_f32", "oracle_sweep_i64", "oracle_sweep_d64"):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [ctypes.c_int, i64, i64, p, i64, p, p, p, i64, p, p]
        lib.oracle_dtw_f32.restype = ctypes.c_int
        lib.oracle_dtw_f32.argtypes = [i64, i64, p, p, p, i64, p, p]
        for name in ("oracle_traceback_f32", "oracle_traceback_f64", "oracle_traceback_i32"):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [ctypes.c_int, i64, i64, p, i64, p, p, p, p]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def sweep(c: np.ndarray, rule: str = "min", arith: str | None = None, top=None, left=None,
          full: bool = True):
    """Sweep the grid `c` (2-D, float32 or int32).

    arith: "f64" (default for float32 inputs), "f32" (bit-exact fp32 reference),
           "i64" (only for int32 inputs) or "d64" (float64 inputs, fp64 loop: the
           bit-exact fp64 reference; the default for float64 inputs).
    top:   n+1 boundary values (top[0] = corner) or None for the default.
    left:  m boundary values or None for the default.
    Returns H (m x n) if full, else (last_row, last_col).
    """
    c = np.ascontiguousarray(c)
    if c.ndim != 2:
        raise ValueError("c must be 2-D")
    m, n = c.shape
    if arith is None:
        arith = {np.dtype(np.int32): "i64", np.dtype(np.float64): "d64"}.get(c.dtype, "f64")
    if arith in ("f64", "f32") and c.dtype != np.float32:
        raise ValueError("float arithmetic needs float32 inputs")
    if arith == "i64" and c.dtype != np.int32:
        raise ValueError("integer arithmetic needs int32 inputs")
    if arith == "d64" and c.dtype != np.float64:
        raise ValueError("d64 arithmetic needs float64 inputs")
    odt = {"f64": np.float64, "f32": np.float32, "i64": np.int64, "d64": np.float64}[arith]
    if top is not None:
        top = np.ascontiguousarray(top, dtype=odt)
        if top.shape != (n + 1,):
            raise ValueError("top must have n+1 entries")
    if left is not None:
        left = np.ascontiguousarray(left, dtype=odt)
        if left.shape != (m,):
            raise ValueError("left must have m entries")
    lib = _load()
    fn = {"f64": lib.oracle_sweep_f64, "f32": lib.oracle_sweep_f32, "i64": lib.oracle_sweep_i64,
          "d64": lib.oracle_sweep_d64}[arith]
    if full:
        H = np.empty((m, n), dtype=odt)
        rc = fn(RULES[rule], m, n, _ptr(c), n, _ptr(top), _ptr(left), _ptr(H), n, None, None)
        if rc != 0:
            raise RuntimeError(f"oracle returned {rc}")
        return H
    last_row = np.empty(n, dtype=odt)
    last_col = np.empty(m, dtype=odt)
    rc = fn(RULES[rule], m, n, _ptr(c), n, _ptr(top), _ptr(left), None, 0, _ptr(last_row), _ptr(last_col))
    if rc != 0:
        raise RuntimeError(f"oracle returned {rc}")
    return last_row, last_col


def dtw(x: np.ndarray, y: np.ndarray, full: bool = True):
    """Dynamic time warping of float32 sequences x (m) and y (n) in fp32: the min rule
    with c[i][j] = |x[i] - y[j]| and the default boundary (see oracle_dtw_f32).
    Returns D (m x n) if full, else (last_row, last_col)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    m, n = len(x), len(y)
    lib = _load()
    if full:
        H = np.empty((m, n), dtype=np.float32)
        rc = lib.oracle_dtw_f32(m, n, _ptr(x), _ptr(y), _ptr(H), n, None, None)
        if rc != 0:
            raise RuntimeError(f"oracle returned {rc}")
        return H
    last_row = np.empty(n, dtype=np.float32)
    last_col = np.empty(m, dtype=np.float32)
    rc = lib.oracle_dtw_f32(m, n, _ptr(x), _ptr(y), None, 0, _ptr(last_row), _ptr(last_col))
    if rc != 0:
        raise RuntimeError(f"oracle returned {rc}")
    return last_row, last_col


def traceback(H: np.ndarray, rule: str = "min", top=None, left=None):
    """Path of predecessor choices through the computed grid H (float32, float64 or
    int32) from (m-1, n-1) back to the boundary, preferring NW, then N, then W on equal
    values (see oracle_traceback_*).  Returns (path, exit): path is an (L, 2) int32 array
    of visited cells, (m-1, n-1) first; exit is the outside predecessor it ended on."""
    H = np.ascontiguousarray(H)
    m, n = H.shape
    lib = _load()
    fn = {np.dtype(np.float32): lib.oracle_traceback_f32, np.dtype(np.float64): lib.oracle_traceback_f64,
          np.dtype(np.int32): lib.oracle_traceback_i32}[H.dtype]
    if top is not None:
        top = np.ascontiguousarray(top, dtype=H.dtype)
    if left is not None:
        left = np.ascontiguousarray(left, dtype=H.dtype)
    path = np.empty((m + n + 1, 2), dtype=np.int32)
    ln = ctypes.c_int64(0)
    rc = fn(RULES[rule], m, n, _ptr(H), n, _ptr(top), _ptr(left), _ptr(path), ctypes.byref(ln))
    if rc != 0:
        raise RuntimeError(f"oracle returned {rc}")
    L = ln.value
    return path[:L].copy(), path[L].copy()


def sweep_banded(rows_fn, m: int, n: int, rule: str = "min", arith: str = "f64", band: int = 256,
                 want_rows=()):
    """Sweep an m x n grid band by band with O(band * n) memory.

    rows_fn(row0, rows) must return the input rows [row0, row0+rows).
    Each band is solved with the explicit boundary taken from the band above
    (top = [corner] + previous last row, where the corner is the previous
    band's last left-boundary value, i.e. the default for that row).
    Returns (last_row, last_col, {r: row r for r in want_rows}).
    """
    odt = {"f64": np.float64, "f32": np.float32, "i64": np.int64}[arith]
    absent = {"min": np.inf, "max": -np.inf}[rule]
    if arith == "i64":
        absent = (1 << 62) if rule == "min" else -(1 << 62)
    want = set(int(r) for r in want_rows)
    got = {}
    last_col = np.empty(m, dtype=odt)
    top = None
    for row0 in range(0, m, band):
        rows = min(band, m - row0)
        c = rows_fn(row0, rows)
        left = np.full(rows, absent, dtype=odt)
        need_full = any(row0 <= r < row0 + rows for r in want)
        if need_full:
            H = sweep(c, rule, arith, top=top, left=left, full=True)
            lr, lc = H[-1].copy(), H[:, -1].copy()
            for r in want:
                if row0 <= r < row0 + rows:
                    got[r] = H[r - row0].copy()
        else:
            lr, lc = sweep(c, rule, arith, top=top, left=left, full=False)
        last_col[row0:row0 + rows] = lc
        top = np.concatenate([np.array([absent], dtype=odt), lr])
    return lr, last_col, got


if __name__ == "__main__":  # pragma: no cover - manual build helper
    print(build(force="--force" in sys.argv))
