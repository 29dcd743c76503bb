"""Seeded synthetic inputs for the wavefront sweep (shared by the oracle side
and the GPU side; holds none of the sweep's arithmetic).

Every per-cell input is a pure function of (seed, linear index k = i*n + j),
so a grid can be generated in any order, in bands, or on the device, and the
CPU and GPU copies are bit-identical.

Generator: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014).  The k-th output of a SplitMix64 stream
seeded with `seed` is  mix64(seed + (k+1) * GAMMA)  with
    mix64(z): z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
              z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31
(all arithmetic mod 2^64).

Mapping to cell values:
  float32: top 24 bits, (x >> 40) * 2^-24   -> uniform on [0, 1), exact in fp32
  float64: top 53 bits, (x >> 11) * 2^-53   -> uniform on [0, 1), exact in fp64
  int32:   low 8 bits,  x & 255             -> uniform on {0, ..., 255}

Workload recipes (sizes, seeds, arrival times) for the benchmark
configurations also live here, because they are input generation too.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, k: np.ndarray) -> np.ndarray:
    """k-th outputs (uint64 array) of the SplitMix64 stream seeded with `seed`."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(int(seed) & 0xFFFFFFFFFFFFFFFF) + (k + np.uint64(1)) * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def _to_dtype(x: np.ndarray, dtype: str) -> np.ndarray:
    if dtype == "f32":
        return ((x >> np.uint64(40)).astype(np.float64) * (2.0 ** -24)).astype(np.float32)
    if dtype == "i32":
        return (x & np.uint64(255)).astype(np.int32)
    if dtype == "f64":
        return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    raise ValueError(f"unknown dtype {dtype!r}")


def cells(seed: int, m: int, n: int, dtype: str = "f32", row0: int = 0, rows: int | None = None) -> np.ndarray:
    """Rows [row0, row0+rows) of the m x n input grid for `seed` (row-major, C-contiguous)."""
    if rows is None:
        rows = m - row0
    if not (0 <= row0 and rows >= 0 and row0 + rows <= m):
        raise ValueError("row band out of range")
    i = np.arange(row0, row0 + rows, dtype=np.uint64)[:, None]
    j = np.arange(n, dtype=np.uint64)[None, :]
    k = i * np.uint64(n) + j
    return _to_dtype(splitmix64(seed, k), dtype)


def vector(seed: int, length: int, dtype: str = "f32") -> np.ndarray:
    """A seeded 1-D vector (used for explicit top/left boundaries in tests)."""
    return _to_dtype(splitmix64(seed, np.arange(length, dtype=np.uint64)), dtype)


def batch_shapes(count: int = 4096, lo: int = 64, hi: int = 2048, seed: int = 4):
    """(m, n) pairs, each drawn independently log-uniform on [lo, hi]:
    floor(exp(U[ln lo, ln(hi+1)))).  Uses numpy's PCG64 so the recipe is
    reproducible from (count, lo, hi, seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(math.log(lo), math.log(hi + 1), size=(count, 2))
    mn = np.floor(np.exp(u)).astype(np.int64)
    mn = np.clip(mn, lo, hi)
    return [(int(a), int(b)) for a, b in mn]


def batch_seed(g: int) -> int:
    """Seed of grid g in a batch."""
    return 1000 + g


def serving_requests(count: int, rate_per_s: float, lo: int = 128, hi: int = 8192, seed: int = 5):
    """Poisson arrivals of square grids: returns [(t_arrival_s, n, seed_of_grid)].
    Inter-arrival times are exponential with mean 1/rate; n is log-uniform on
    [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps) - gaps[0]
    u = rng.uniform(math.log(lo), math.log(hi + 1), size=count)
    ns = np.clip(np.floor(np.exp(u)).astype(np.int64), lo, hi)
    return [(float(a), int(b), 50000 + q) for q, (a, b) in enumerate(zip(t, ns))]


# ------------------------------------------------------------- device fill
import ctypes as _ctypes
import os as _os
import subprocess as _subprocess

_HERE = _os.path.dirname(_os.path.abspath(__file__))
_FILL_SRC = _os.path.join(_HERE, "wfgen_fill.hip")
FILL_LIB = _os.path.join(_HERE, "libwfgen.so")
_fill_lib = None


def build_fill(force: bool = True) -> str:
    """Compile libwfgen.so (the device-side fill) for gfx950."""
    if force or not _os.path.exists(FILL_LIB):
        cmd = ["/opt/rocm/bin/hipcc", "-O3", "-fPIC", "-shared", "--offload-arch=gfx950",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-o", FILL_LIB + ".tmp", _FILL_SRC]
        _subprocess.run(cmd, check=True, stderr=_subprocess.DEVNULL)
        _os.replace(FILL_LIB + ".tmp", FILL_LIB)
    return FILL_LIB


def fill_device(t, seed: int, row0: int = 0, n_cols: int | None = None, stream=None):
    """Fill a 2-D device tensor (rows x n, unit column stride) with the same values
    cells(seed, ..., row0, rows) would give, for a grid of n_cols columns (default n)."""
    import torch
    global _fill_lib
    if _fill_lib is None:
        if not _os.path.exists(FILL_LIB):
            raise RuntimeError("libwfgen.so not built; call wfgen.build_fill()")
        lib = _ctypes.CDLL(FILL_LIB)
        lib.wfgen_fill.restype = _ctypes.c_int
        lib.wfgen_fill.argtypes = [_ctypes.c_void_p, _ctypes.c_int, _ctypes.c_int64, _ctypes.c_int64,
                                   _ctypes.c_int64, _ctypes.c_uint64, _ctypes.c_int64, _ctypes.c_void_p]
        _fill_lib = lib
    rows, n = t.shape
    if n_cols is not None and n_cols != n:
        raise ValueError("a band must span the full grid width")
    if t.stride(1) != 1:
        raise ValueError("unit column stride required")
    dt = {torch.float32: 0, torch.int32: 1, torch.float64: 2}[t.dtype]
    s = stream if stream is not None else torch.cuda.current_stream()
    rc = _fill_lib.wfgen_fill(t.data_ptr(), dt, rows, n, t.stride(0), seed & 0xFFFFFFFFFFFFFFFF, row0,
                              s.cuda_stream)
    if rc != 0:
        raise RuntimeError(f"wfgen_fill failed with HIP error {rc}")
    return t


def permutation(seed: int, n: int) -> np.ndarray:
    """A seeded shuffle of range(n) (numpy PCG64): the random draw behind a
    shuffled train/test split."""
    return np.random.Generator(np.random.PCG64(seed)).permutation(n)
