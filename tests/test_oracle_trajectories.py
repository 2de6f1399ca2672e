"""Pins of the oracle's trajectory simulator (Section 4.3): episodes of the
network process, each step a fresh network state anchored at the current node.

Independent references: the exact crossroads kernel of Section 2.1 (every world
of its three stochastic spokes enumerated) for the length-biased estimators of
the uniform-step equivalence and for the law of one step; a star graph with no
failures, where every valid step reports the hub, for exact visit, switch and
length bookkeeping; the geometric law of the absorption time when only the stop
coin absorbs; and the prefix property of truncated episodes.
"""
import numpy as np
import pytest

import oracle as O
from paper_2605_14743_amd import workloads as W
from test_oracle_montecarlo import exact_kernel, hoeffding


def _batch_se(num, den, batches):
    """Standard error of a ratio estimator sum(num) / sum(den) from batch means."""
    nb = np.array([a.sum(0) for a in np.array_split(num, batches)])
    db = np.array([a.sum() for a in np.array_split(den, batches)])
    est = nb / db[:, None] if nb.ndim == 2 else nb / db
    return est.std(axis=0, ddof=1) / np.sqrt(batches)


def test_crossroads_length_biased_estimators_match_exact_chain():
    g, pf = W.crossroads()
    P, _, _, _ = exact_kernel(g, pf, 0.1, 3)
    ch = O.chain(P[:, :10], np.full(10, 0.1))
    f = np.linspace(0.5, 2.0, g.n)
    E = 30000
    x0 = np.arange(E) % g.n                         # s uniform, stratified
    res = O.trajectories(g.n, g.eu, g.ev, seed=21, x0=x0, alpha=0.1, k_min=3, f=f, want_paths=True,
                         p_fail=0.0, p_fail_edge=pf, weight="unit")
    T = res["lengths"].astype(float)
    assert res["truncated"] == 0 and res["total_steps"] == int(T.sum())
    b_hat = res["visits"] / res["total_steps"]       # Proposition on uniform-step equivalence
    per_ep = np.zeros((E, g.n))
    for e in range(E):
        np.add.at(per_ep[e], res["paths"][e, :res["lengths"][e]], 1.0)
    se = _batch_se(per_ep, T, 50)
    assert np.all(np.abs(b_hat - ch["b"]) <= 5 * se)
    assert T.mean() == pytest.approx(ch["ET"], abs=5 * T.std() / np.sqrt(E))
    # node reward: sum f(X_t) / sum T estimates b . f (eq. mr-inner-product)
    fb = ch["b"] @ f
    assert res["reward_f"] / res["total_steps"] == pytest.approx(fb, abs=5 * (per_ep @ f / T.mean()).std() /
                                                                 np.sqrt(E) + 1e-3)
    # survival-weighted decomposition: w_t = P(T > t) / E[T] sums to one
    w = np.array([(res["lengths"] > t).sum() for t in range(res["lengths"].max())]) / res["total_steps"]
    assert w.sum() == pytest.approx(1.0, abs=1e-12)


def test_crossroads_first_step_follows_the_row_law():
    g, pf = W.crossroads()
    P, _, _, _ = exact_kernel(g, pf, 0.1, 3)
    E = 20000
    hub = 9
    res = O.trajectories(g.n, g.eu, g.ev, seed=5, x0=np.full(E, hub), alpha=0.1, k_min=3, want_paths=True,
                         max_steps=4, p_fail=0.0, p_fail_edge=pf, weight="unit")
    nxt = np.where(res["lengths"] >= 2, res["paths"][:, 1], g.n)          # bottom = column n
    emp = np.bincount(nxt, minlength=g.n + 1) / E
    assert np.abs(emp - P[hub]).max() < hoeffding(E, g.n + 1)


def test_star_without_failures_bookkeeping_is_exact():
    hub, n = 3, 7
    g = W.canonical(n, [(min(hub, v), max(hub, v)) for v in range(n) if v != hub])
    E = 2000
    x0 = np.arange(E) % n
    res = O.trajectories(n, g.eu, g.ev, seed=9, x0=x0, alpha=0.3, k_min=1, want_paths=True, max_steps=200,
                         p_fail=0.0, weight="unit")
    L = res["lengths"]
    for e in range(E):                                   # X_0 = x0, then the hub until absorption
        path = res["paths"][e, :L[e]]
        assert path[0] == x0[e] and np.all(path[1:] == hub)
        assert np.all(res["paths"][e, L[e]:] == -1)
    assert res["visits"][hub] == (L - (x0 != hub)).sum()
    assert res["switches"] == int(((x0 != hub) & (L >= 2)).sum())
    # only the stop coin absorbs: T is geometric with mean 1 / alpha
    alpha_eff = O.prob_threshold(0.3) / 2 ** 32
    assert L.mean() == pytest.approx(1 / alpha_eff, abs=5 * np.sqrt(1 - alpha_eff) / alpha_eff / np.sqrt(E))
    surv = np.array([(L > t).mean() for t in range(8)])
    assert np.allclose(surv, (1 - alpha_eff) ** np.arange(8), atol=5 * 0.5 / np.sqrt(E))


def test_truncated_episodes_are_prefixes():
    wl = W.config_er20()
    g = wl.graph
    x0 = np.arange(200) % g.n
    full = O.trajectories(g.n, g.eu, g.ev, seed=3, x0=x0, want_paths=True, max_steps=1024, **wl.model())
    cut = O.trajectories(g.n, g.eu, g.ev, seed=3, x0=x0, want_paths=True, max_steps=3, **wl.model())
    assert np.array_equal(cut["lengths"], np.minimum(full["lengths"], 3))
    assert cut["truncated"] == int((full["lengths"] > 3).sum())
    assert np.array_equal(cut["paths"], full["paths"][:, :3])
