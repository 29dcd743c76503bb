"""Oracle of the paper's stream-count heuristic (arXiv 2501.05938, Sections 2.3 and
2.4, Eqs. 3-7, and the selection rule restated at the start of Section 3).

TEST INFRASTRUCTURE ONLY: imported by tests/ and by the benchmark's model
check.  The library (libwf.so) has its own C++ implementation of the same
fits and selection (wf_stream_model_fit / wf_stream_model_choose); the two
share no code.  Random draws (the shuffled 3:1 split) are inputs here: the
caller passes the permutation, made by the seeded input generator.

Plain numpy, in the paper's order:

  Eq. 3   sum = T1_COMP + T1_D2H + T3_H2D + T3_COMP, the operations whose time
          the streams overlap.
  S. 2.3  the earlier heuristic: per-stream overhead tau, optimum sqrt(sum / tau).
  Eq. 4   sum modelled as a straight line in the problem size, fitted by least
          squares on a shuffled 3:1 train/test split.
  Eq. 5   T_overhead = (T_str - T_non_str) + (s - 1)/s * sum.
  Eq. 6   a stream count s is worth using when T_overhead < (s - 1)/s * sum;
          among those, the one with the largest gap wins.
  Eq. 7   T_overhead modelled in two size regimes:
            small: a*N + b*log10(s) + c
            big:   (a*N + b)*log2(s^(4/3)) + c
          both linear in (a, b, c), fitted by least squares on a shuffled 3:1
          split of each regime's samples.
  S. 3    candidates are 1, 2, 4, ..., 32 streams; s = 1 is scored like the
          others (its gap is -T_overhead(N, 1)), and when no candidate has a
          positive gap one stream is used.

Readings where the paper is silent (stated again in the design notes):
  * the split puts the first ceil(n/4) entries of the permutation in the test
    set and the rest in the training set (the layout of scikit-learn's
    shuffled split, which the paper names);
  * the overhead models are fitted on samples with s >= 2 (at s = 1 Eq. 5 is
    zero by definition, so those samples carry no information);
  * metrics are R^2 = 1 - SS_res / SS_tot and MSE = SS_res / n.
"""
from __future__ import annotations

import math

import numpy as np

CANDIDATES = (1, 2, 4, 8, 16, 32)


# ------------------------------------------------------------------ Eq. 3, S. 2.3
def overlappable_sum(t1_comp, t1_d2h, t3_h2d, t3_comp):
    """Eq. 3."""
    return t1_comp + t1_d2h + t3_h2d + t3_comp


def earlier_heuristic_streams(sum_ms, tau_ms):
    """Section 2.3: overhead s * tau, so dT/ds = -sum/s^2 + tau = 0 at s = sqrt(sum / tau)."""
    return math.sqrt(sum_ms / tau_ms)


# ------------------------------------------------------------------ Eqs. 5 and 6
def overhead(t_str, t_non_str, sum_ms, s):
    """Eq. 5."""
    return (t_str - t_non_str) + (s - 1) / s * sum_ms


def gap(sum_ms, t_ov, s):
    """Right-hand side of Eq. 6 minus its left-hand side: positive when s streams pay."""
    return (s - 1) / s * sum_ms - t_ov


# ------------------------------------------------------------------ splits and fits
def split_3_1(n, perm):
    """(train indices, test indices) of n samples from a permutation of range(n)."""
    perm = np.asarray(perm, dtype=np.int64)
    if sorted(perm.tolist()) != list(range(n)):
        raise ValueError("perm must be a permutation of range(n)")
    n_test = int(math.ceil(n / 4))
    return perm[n_test:], perm[:n_test]


def least_squares(X, y):
    """Coefficients minimising ||X b - y||_2 (numpy's SVD-based solver)."""
    b, *_ = np.linalg.lstsq(np.asarray(X, np.float64), np.asarray(y, np.float64), rcond=None)
    return b


def metrics(y, yhat):
    y = np.asarray(y, np.float64)
    yhat = np.asarray(yhat, np.float64)
    ss_res = float(((y - yhat) ** 2).sum())
    ss_tot = float(((y - y.mean()) ** 2).sum())
    return {"r2": 1.0 - ss_res / ss_tot if ss_tot > 0 else float("nan"), "mse": ss_res / len(y), "n": len(y)}


def sum_features(size):
    size = np.asarray(size, np.float64)
    return np.stack([size, np.ones_like(size)], axis=1)


def small_features(size, s):
    size = np.asarray(size, np.float64)
    s = np.asarray(s, np.float64)
    return np.stack([size, np.log10(s), np.ones_like(size)], axis=1)


def big_features(size, s):
    size = np.asarray(size, np.float64)
    L = np.log2(np.asarray(s, np.float64) ** (4.0 / 3.0))
    return np.stack([size * L, L, np.ones_like(size)], axis=1)


def fit_sum(sizes, sums, perm):
    """Eq. 4 on one (size, sum) sample per problem size.  Returns (slope, intercept),
    {"train": metrics, "test": metrics}."""
    tr, te = split_3_1(len(sizes), perm)
    X, y = sum_features(sizes), np.asarray(sums, np.float64)
    b = least_squares(X[tr], y[tr])
    return (float(b[0]), float(b[1])), {"train": metrics(y[tr], X[tr] @ b), "test": metrics(y[te], X[te] @ b)}


def fit_overhead(sizes, streams, t_ov, perm, regime):
    """Eq. 7 for one regime ("small" or "big") on its (size, s, T_overhead) samples.
    Returns (a, b, c), {"train": ..., "test": ...}."""
    feats = small_features if regime == "small" else big_features
    tr, te = split_3_1(len(sizes), perm)
    X, y = feats(sizes, streams), np.asarray(t_ov, np.float64)
    b = least_squares(X[tr], y[tr])
    return tuple(float(v) for v in b), {"train": metrics(y[tr], X[tr] @ b), "test": metrics(y[te], X[te] @ b)}


# ------------------------------------------------------------------ models and choice
def sum_model(coef, size):
    return coef[0] * size + coef[1]


def overhead_model(small, big, split_size, size, s):
    if size <= split_size:
        a, b, c = small
        return a * size + b * math.log10(s) + c
    a, b, c = big
    return (a * size + b) * math.log2(s ** (4.0 / 3.0)) + c


def choose_streams(sum_coef, small, big, split_size, size, candidates=CANDIDATES):
    """Section 3's selection: (best s, {s: gap})."""
    S = sum_model(sum_coef, size)
    gaps = {s: gap(S, overhead_model(small, big, split_size, size, s), s) for s in candidates}
    best, best_gap = 1, None
    for s in candidates:
        if gaps[s] > 0 and (best_gap is None or gaps[s] > best_gap):
            best, best_gap = s, gaps[s]
    return best, gaps
