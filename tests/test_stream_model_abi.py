"""The library's stream-count model (wf_stream_model_* in the C ABI; host-only, no GPU)
against the oracle of oracle/stream_model.py: the paper's own coefficients must
give Table 4's predictions, and fits of seeded synthetic timing sets must give
the oracle's coefficients, metrics and choices."""
import ctypes
import json
import math
import os

import numpy as np
import pytest

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2501_05938_amd", "libwf.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libwf.so not built")

from oracle import stream_model as sm  # noqa: E402
import wfgen  # noqa: E402

GOLD = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                   "paper_stream_tables.json")))


def _paper_model(wf):
    m = wf.StreamModel()
    m.sum_slope, m.sum_intercept = GOLD["eq4"]["slope"], GOLD["eq4"]["intercept"]
    m.split_size = GOLD["eq7"]["split_size"]
    for k, key in enumerate("abc"):
        m.small[k] = GOLD["eq7"]["small"][key]
        m.big[k] = GOLD["eq7"]["big"][key]
    return m


def test_paper_coefficients_reproduce_table4():
    import paper_2501_05938_amd as wf
    m = _paper_model(wf)
    for r in GOLD["table4"]["rows"]:
        best, gaps = wf.choose_streams(m, r["size"])
        assert best == r["pre"], r
        small = tuple(GOLD["eq7"]["small"][k] for k in "abc")
        big = tuple(GOLD["eq7"]["big"][k] for k in "abc")
        _, og = sm.choose_streams((m.sum_slope, m.sum_intercept), small, big, m.split_size, r["size"])
        assert np.allclose(gaps, [og[s] for s in sm.CANDIDATES], rtol=1e-12, atol=1e-12)


def _synthetic(seed, split):
    """A seeded timing set shaped like the paper's: sum linear in size, overhead
    logarithmic in s in two regimes, plus noise."""
    rng = np.random.default_rng(seed)
    sizes = [m * 10.0 ** i for i in range(3, 8) for m in (1, 2.5, 4, 5, 7.5, 8)] + [1e8]
    out = []
    for N in sizes:
        S = 2.2e-6 * N + 0.15 + rng.normal(0, 0.01)
        t_non = S + 0.3 * S + 0.05
        for s in (1, 2, 4, 8, 16, 32):
            if N <= split:
                ov = 2.2e-7 * N + 0.6 * math.log10(s) - 0.06 + rng.normal(0, 0.05)
            else:
                ov = (3.6e-8 * N + 0.05) * math.log2(s ** (4 / 3)) + 0.39 + rng.normal(0, 0.3)
            t_str = t_non if s == 1 else t_non - (s - 1) / s * S + ov
            out.append((N, s, t_str, t_non, S))
    return out


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_fit_matches_oracle(seed):
    import paper_2501_05938_amd as wf
    split = 1e6
    samples = _synthetic(seed, split)
    ns, nsm, nbg = wf.stream_model_groups(samples, split)
    ps, psm, pbg = wfgen.permutation(10 + seed, ns), wfgen.permutation(20 + seed, nsm), wfgen.permutation(30 + seed, nbg)
    model, rep = wf.fit_stream_model(samples, split, ps, psm, pbg)
    # oracle: the same groups, built plainly
    sizes = list(dict.fromkeys(s[0] for s in samples))
    sums = [np.mean([s[4] for s in samples if s[0] == N]) for N in sizes]
    coef, met = sm.fit_sum(np.array(sizes), np.array(sums), ps)
    assert model.sum_slope == pytest.approx(coef[0], rel=1e-9)
    assert model.sum_intercept == pytest.approx(coef[1], rel=1e-9)
    assert rep[0].r2_train == pytest.approx(met["train"]["r2"], rel=1e-9)
    assert rep[0].mse_test == pytest.approx(met["test"]["mse"], rel=1e-7)
    ov = [(s[0], s[1], sm.overhead(s[2], s[3], s[4], s[1])) for s in samples if s[1] >= 2]
    small = [o for o in ov if o[0] <= split]
    big = [o for o in ov if o[0] > split]
    cs, ms = sm.fit_overhead(*map(np.array, zip(*small)), psm, "small")
    cb, mb = sm.fit_overhead(*map(np.array, zip(*big)), pbg, "big")
    assert np.allclose(list(model.small), cs, rtol=1e-8, atol=1e-14)
    assert np.allclose(list(model.big), cb, rtol=1e-8, atol=1e-14)
    assert (rep[1].n_train, rep[1].n_test) == (ms["train"]["n"], ms["test"]["n"])
    assert rep[2].r2_test == pytest.approx(mb["test"]["r2"], rel=1e-8)
    for N in np.geomspace(1e3, 1e8, 41):
        best, gaps = wf.choose_streams(model, N)
        ob, og = sm.choose_streams(coef, cs, cb, split, N)
        assert best == ob, N
        assert np.allclose(gaps, [og[s] for s in sm.CANDIDATES], rtol=1e-9, atol=1e-9)


def test_errors():
    import paper_2501_05938_amd as wf
    samples = _synthetic(4, 1e6)
    ns, nsm, nbg = wf.stream_model_groups(samples, 1e6)
    bad = list(range(ns))
    bad[0] = bad[1]
    with pytest.raises(wf.WfError) as e:
        wf.fit_stream_model(samples, 1e6, bad, range(nsm), range(nbg))
    assert e.value.status == -1
    # every overhead sample at one size: the size column is constant, so the small fit is degenerate
    flat = [(1e4, s, 1.0, 1.0, 0.5) for s in (1, 2, 4, 8)] + [(2e4, 1, 1.0, 1.0, 0.6)]
    with pytest.raises(wf.WfError):
        wf.fit_stream_model(flat, 1e6, range(2), range(3), [])
    lib = wf.load_library()
    assert lib.wf_stream_model_choose(None, 1.0, None, 0, None, None) == -1
    assert math.isnan(lib.wf_stream_model_overhead(None, 1.0, 2))
