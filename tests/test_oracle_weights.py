"""Pins of the per-call weight resampling law of the co-occurrence experiment
(Section 9.2) in its integer form: the cumulative threshold table of
`workloads.resampled_weight_cdf` and the oracle's draw from it.

Independent references: scipy's normal distribution for the rounded and
clipped Gaussian law, the zero-spread limit (round and clip), a degenerate
table that must reproduce the fixed-weight law exactly, and the empirical
frequencies of the oracle's draws (Hoeffding).
"""
import numpy as np
import pytest
from scipy.stats import norm

import oracle as O
from paper_2605_14743_amd import workloads as W


def test_table_matches_rounded_clipped_gaussian():
    w0 = np.array([1, 2, 5, 17, 30, 31])
    w_max, rm, rs = 31, 0.1, 0.2
    T = W.resampled_weight_cdf(w0, w_max, rm, rs)
    assert np.all(np.diff(T.astype(np.int64), axis=1) >= 0) and np.all(T[:, -1] == 2 ** 32)
    for e, a in enumerate(w0):
        mu, sd = a + rm * (w_max - a), rs * (w_max - a)
        pm = np.diff(np.concatenate([[0], T[e].astype(np.float64)])) / 2 ** 32
        for v in range(1, w_max + 1):
            if v < a:
                ref = 0.0
            elif sd == 0.0:
                ref = 1.0 if v == a else 0.0
            elif v == a:
                ref = norm.cdf(a + 0.5, mu, sd)                   # all mass below w0 lands on w0
            elif v == w_max:
                ref = norm.sf(w_max - 0.5, mu, sd)                # all mass above w_max lands on w_max
            else:
                ref = norm.cdf(v + 0.5, mu, sd) - norm.cdf(v - 0.5, mu, sd)
            assert pm[v - 1] == pytest.approx(ref, abs=1e-9), (e, v)


def test_zero_spread_is_round_and_clip():
    w0 = np.array([1, 4, 10, 20])
    T = W.resampled_weight_cdf(w0, 25, 0.37, 0.0)
    for e, a in enumerate(w0):
        target = int(np.clip(np.floor(a + 0.37 * (25 - a) + 0.5), a, 25))
        pm = np.diff(np.concatenate([[0], T[e].astype(np.int64)]))
        assert pm[target - 1] == 2 ** 32 and pm.sum() == 2 ** 32


def test_degenerate_table_reproduces_the_fixed_law():
    g = W.powerlaw_weighted_graph(77, 254, 2.5, 3.0, 31, 0)
    T = np.zeros((g.m, 31), np.uint64)
    for e, a in enumerate(g.w0):
        T[e, a - 1:] = 2 ** 32
    a = O.sweep(g.n, g.eu, g.ev, seed=3, R=60, alpha=0.15, k_min=5, want_next=True, p_fail=0.1, weight="fixed",
                w0=g.w0)
    b = O.sweep(g.n, g.eu, g.ev, seed=3, R=60, alpha=0.15, k_min=5, want_next=True, p_fail=0.1, weight="table",
                w_cdf=T)
    assert np.array_equal(a["counts"], b["counts"]) and np.array_equal(a["next_table"], b["next_table"])
    assert np.array_equal(a["bsum"], b["bsum"])


def test_draw_frequencies_follow_the_table():
    g = W.powerlaw_weighted_graph(77, 254, 2.5, 3.0, 31, 0)
    T = W.resampled_weight_cdf(g.w0, 31, 0.1, 0.2)
    R = 3000
    counts = np.zeros((g.m, 31))
    for r in range(R):
        _, w = O.realize(g.n, g.eu, g.ev, 11, r, p_fail=0.0, weight="table", w_cdf=T)
        counts[np.arange(g.m), w - 1] += 1
    pm = np.diff(np.concatenate([np.zeros((g.m, 1)), T.astype(np.float64)], axis=1), axis=1) / 2 ** 32
    bound = np.sqrt(np.log(2 * g.m * 31 / 1e-6) / (2 * R))
    assert np.abs(counts / R - pm).max() < bound
    assert np.all(counts[pm == 0] == 0)                                # never below w0
