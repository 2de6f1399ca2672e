"""End-to-end pins of the oracle's Monte Carlo sweep (Alg. 1 for every anchor,
counted as in Alg. 2) and its tail.

Exact kernels come from enumerating every world of the stochastic edges
(2^k worlds, Section 8.1 notes this is only possible for tiny k); the sweep's
empirical rows must fall within the Hoeffding bound of Section 8.4, and the
crossroads example must reproduce the values the paper prints (Section 2.1).
"""
import itertools

import numpy as np
import pytest

import oracle as O
from paper_2605_14743_amd import workloads as W


def exact_kernel(g, p_fail_edge, alpha, k_min, tau=1e-9, pool=None, w0=None):
    """Row law of Alg. 1 by enumerating every world of the stochastic edges.
    Event probabilities use the integer mapping floor(p 2^32) / 2^32."""
    n = g.n
    T = lambda p: O.prob_threshold(p) / 2 ** 32
    stoch = [e for e in range(g.m) if 0.0 < T(p_fail_edge[e]) < 1.0]
    base_alive = np.array([1 if T(p) == 0.0 else 0 for p in p_fail_edge], np.uint8)
    a_eff = T(alpha)
    P = np.zeros((n, n + 1))
    Pw = np.zeros((n, n + 1))
    p1 = np.zeros(n)
    Bavg = np.zeros(n)
    unit = w0 is None
    w = np.ones(g.m, np.uint32) if unit else np.asarray(w0, np.uint32)
    for bits in itertools.product([0, 1], repeat=len(stoch)):
        alive = base_alive.copy()
        pr = 1.0
        for e, bit in zip(stoch, bits):
            alive[e] = bit
            pr *= (1.0 - T(p_fail_edge[e])) if bit else T(p_fail_edge[e])
        B = O.betweenness(n, g.eu, g.ev, alive, w, unit)
        comp, size = O.components(n, g.eu, g.ev, alive)
        Bavg += pr * B
        p1[O.band_argmax(B, np.ones(n, np.uint8), tau)[0]] += pr
        for i in range(n):
            if size[i] < k_min:
                P[i, n] += pr
                Pw[i, n] += pr
                continue
            mem = (comp == comp[i]).astype(np.uint8)
            c = O.band_argmax(B, mem, tau)[0]
            P[i, c] += pr * (1 - a_eff)
            P[i, n] += pr * a_eff
            if pool is not None:
                mw = mem.copy()
                mw[[v for v in range(n) if v not in set(pool)]] = 0
                cw = O.band_argmax(B, mw, tau)[0]
                Pw[i, cw if cw >= 0 else n] += pr * (1 - a_eff)
                Pw[i, n] += pr * a_eff
    return P, Pw, p1, Bavg


def hoeffding(R, entries, delta=1e-6):
    return np.sqrt(np.log(2 * entries / delta) / (2 * R))


def test_crossroads_exact_values(golden):
    ref = golden("crossroads.json")
    g, pf = W.crossroads()
    P, _, _, Bavg = exact_kernel(g, pf, 0.1, 3)
    assert np.allclose(P.sum(1), 1.0)                                     # Lemma (row normalisation)
    ch = O.chain(P[:, :10], np.full(10, 0.1))
    assert np.allclose(ch["b"], ref["afc_b"], atol=5e-4)
    assert ch["ET"] == pytest.approx(ref["expected_length"], abs=5e-3)
    share = Bavg / Bavg.sum()
    for k, v in ref["averaged_bc_share"].items():
        if k != "interior":
            assert share[int(k) - 1] == pytest.approx(v, abs=5e-4)
    hub = P[9] / 0.9                                                       # undo the stop coin
    assert hub[9] == pytest.approx(ref["hub_row"]["two_or_more_spokes"], abs=1e-8)
    assert hub[[0, 3, 6]].sum() == pytest.approx(ref["hub_row"]["one_spoke_moves_to_gateway"], abs=1e-8)
    valid = 1 - ref["hub_row"]["hub_isolated"]
    for k, v in ref["hub_single_spoke_conditionals"].items():
        assert hub[int(k) - 1] / valid == pytest.approx(v, abs=5e-4)
    assert hub[9] / valid == pytest.approx(0.5435, abs=1e-4)             # printed as 0.544
    interior = [1, 2, 4, 5, 7, 8]
    assert np.allclose(ch["b"][interior], 0.1 / ch["ET"], rtol=1e-12)     # never reported: s_v / E[T]
    assert np.all(P[:, interior] == 0)


def test_crossroads_monte_carlo_within_hoeffding():
    g, pf = W.crossroads()
    P, _, _, Bavg = exact_kernel(g, pf, 0.1, 3)
    R = 20000
    res = O.sweep(g.n, g.eu, g.ev, seed=42, R=R, alpha=0.1, k_min=3, p_fail=0.0, p_fail_edge=pf, weight="unit")
    C = res["counts"]
    assert np.all(C.sum(1) == R)
    assert np.abs(C / R - P).max() < hoeffding(R, g.n * (g.n + 1))
    bmax = 54.0
    assert np.abs(res["bsum"] / R - Bavg).max() < bmax * hoeffding(R, g.n)


@pytest.mark.parametrize("trial", range(4))
def test_random_tiny_graphs_monte_carlo_within_hoeffding(trial):
    rng = np.random.default_rng(100 + trial)
    n = int(rng.integers(6, 10))
    while True:
        pairs = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < 0.45]
        g = W.canonical(n, pairs)
        if 6 <= g.m <= 16:
            break
    pf = np.where(rng.random(g.m) < 0.6, rng.uniform(0.1, 0.6, g.m), 0.0)
    if int((pf > 0).sum()) > 10:
        pf[np.flatnonzero(pf > 0)[10:]] = 0.0
    weighted = trial % 2 == 1
    w0 = rng.integers(1, 4, size=g.m).astype(np.uint32) if weighted else None
    pool = np.sort(rng.choice(n, size=3, replace=False))
    alpha, k_min = 0.15, 3
    P, Pw, p1, _ = exact_kernel(g, pf, alpha, k_min, pool=pool, w0=w0)
    R = 8000
    model = dict(p_fail=0.0, p_fail_edge=pf, weight="fixed" if weighted else "unit", w0=w0)
    res = O.sweep(g.n, g.eu, g.ev, seed=trial, R=R, alpha=alpha, k_min=k_min, pool=pool, want_next=True, **model)
    eps = hoeffding(R, n * (n + 1))
    assert np.abs(res["counts"] / R - P).max() < eps
    assert np.abs(res["counts_w"] / R - Pw).max() < eps
    p_hat = np.bincount(res["center_global"], minlength=n) / R          # eq. oneshot-p, Freq-argmax
    assert np.abs(p_hat - p1).max() < hoeffding(R, n)
    nt = res["next_table"]
    for i in range(n):                                                    # counts are the next table tallied
        assert np.array_equal(np.bincount(np.where(nt[:, i] < 0, n, nt[:, i]), minlength=n + 1),
                              res["counts"][i])
    in_pool = np.isin(res["next_table_w"], pool) | (res["next_table_w"] < 0)
    assert np.all(in_pool)


def test_split_ranges_add_up():
    g = W.config_er20().graph
    kw = dict(seed=3, alpha=0.15, k_min=5, p_fail=0.1, weight="uniform", w_lo=1, w_hi=5, want_next=True)
    full = O.sweep(g.n, g.eu, g.ev, R=60, **kw)
    a = O.sweep(g.n, g.eu, g.ev, R=25, r_begin=0, **kw)
    b = O.sweep(g.n, g.eu, g.ev, R=35, r_begin=25, **kw)
    assert np.array_equal(full["counts"], a["counts"] + b["counts"])
    assert np.array_equal(full["next_table"], np.vstack([a["next_table"], b["next_table"]]))
    assert np.array_equal(full["center_global"], np.r_[a["center_global"], b["center_global"]])


def test_work_accounting_matches_components():
    """n_K, A_K and D_K summed over (r, s) from scipy components."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    g = W.er_graph(80, 2.0 / 80, 1)
    R = 5
    res = O.sweep(g.n, g.eu, g.ev, seed=7, R=R, alpha=0.15, k_min=5, p_fail=0.3, weight="unit")
    deg = g.degrees()
    tot = np.zeros(3, dtype=np.int64)
    for r in range(R):
        alive, _ = O.realize(g.n, g.eu, g.ev, 7, r, p_fail=0.3, weight="unit")
        a = alive == 1
        A = csr_matrix((np.ones(int(a.sum())), (g.eu[a], g.ev[a])), shape=(g.n, g.n))
        k, lab = connected_components(A, directed=False)
        sz = np.bincount(lab, minlength=k)
        alive_slots = np.bincount(lab[g.eu[a]], minlength=k) * 2
        dsum = np.bincount(lab, weights=deg, minlength=k)
        tot += [int(sz[lab].sum()), int(alive_slots[lab].sum()), int(dsum[lab].sum())]
    st = res["stats"]
    assert st["units"] == R * g.n
    assert [st["sum_nK"], st["sum_AK"], st["sum_DK"]] == tot.tolist()
