"""Pins of the oracle's finite-k local Top-k rows: the component ranking and the
Top-k step rewards (Sections 3.3, 6.2, 6.3), the finite-k pool selector
(Section 7.1), the reward-AFCs (Proposition on reward-AFC), the fallback
kernel (Section 7.3) and the censored profile (Section 7.4).

Independent references: exact-rational betweenness by path enumeration with
an exact sort of every component, a closed form for k = 1, the per-draw
classification of the fallback selector, and simulated trajectories of the
estimated chains (the length-biased uniform pre-absorption representation).
"""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

import oracle as O
from paper_2605_14743_amd import workloads as W
from test_oracle_brandes import brute_force


def _components(n, g, alive):
    e = np.flatnonzero(alive)
    A = csr_matrix((np.ones(len(e)), (g.eu[e], g.ev[e])), shape=(n, n))
    _, lab = connected_components(A, directed=False)
    label = np.zeros(n, np.int64)
    for c in np.unique(lab):
        mem = np.flatnonzero(lab == c)
        label[mem] = mem.min()
    return label


def exact_topk_reference(g, model, seed, R, k, alpha, k_min, pool, gamma):
    """psi, psi_w and the finite-k pool counts from exact betweenness."""
    n = g.n
    gam = np.ones(n) if gamma is None else np.asarray(gamma, float)
    inW = np.zeros(n, bool)
    inW[np.asarray(pool)] = True
    psi = np.zeros(n)
    psi_w = np.zeros(n)
    cw = np.zeros((n, n + 1), np.uint32)
    for r in range(R):
        alive, w = O.realize(n, g.eu, g.ev, seed, r, **model)
        B, _, _ = brute_force(n, g.eu, g.ev, alive, w)
        lab = _components(n, g, alive)
        top = {}
        for c in np.unique(lab):
            mem = sorted(np.flatnonzero(lab == c), key=lambda v: (-B[v], v))   # exact order, ties to the index
            top[c] = mem[:k]
        for i in range(n):
            coin = O.stop_coin(seed, r, i, alpha)
            valid = (not coin) and np.count_nonzero(lab == lab[i]) >= k_min
            sel = -1
            if valid:
                C = top[lab[i]]
                psi[i] += gam[C].sum()
                psi_w[i] += gam[[v for v in C if inW[v]]].sum()
                inpool = [v for v in C if inW[v]]
                sel = inpool[0] if inpool else -1
            cw[i, sel if sel >= 0 else n] += 1
    return psi, psi_w, cw


@pytest.mark.parametrize("trial", range(4))
def test_topk_rewards_and_selector_match_exact_ranking(trial):
    rng = np.random.default_rng(100 + trial)
    n = int(rng.integers(5, 9))
    pairs = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < 0.45]
    g = W.canonical(n, pairs)
    weighted = trial % 2 == 1
    model = ({"p_fail": 0.2, "weight": "uniform", "w_lo": 1, "w_hi": 3} if weighted
             else {"p_fail": 0.2, "weight": "unit"})
    pool = np.sort(rng.choice(n, size=3, replace=False))
    gamma = rng.random(n) + 0.5
    for k in (1, 2, 3, n):
        R = 12
        res = O.sweep(n, g.eu, g.ev, seed=7 + trial, R=R, alpha=0.2, k_min=2, pool=pool, topk=k, gamma=gamma,
                      **model)
        psi, psi_w, cw = exact_topk_reference(g, model, 7 + trial, R, k, 0.2, 2, pool, gamma)
        assert np.allclose(res["psi"], psi, rtol=1e-13, atol=0), k
        assert np.allclose(res["psi_w"], psi_w, rtol=1e-13, atol=0), k
        assert np.array_equal(res["counts_w"], cw), k


def test_k1_unit_reward_counts_valid_draws_and_closed_form():
    # with k = 1 every valid draw reports exactly one candidate: psi_i = R - C_i,bottom,
    # and b_{1,1} = s N (1 - r) / s N 1 = 1 - 1 / E[T] (absorption is certain)
    wl = W.config_er20()
    g = wl.graph
    R = 400
    res = O.sweep(g.n, g.eu, g.ev, seed=3, R=R, alpha=wl.alpha, k_min=wl.k_min, topk=1, **wl.model())
    assert np.array_equal(res["psi"], (R - res["counts"][:, g.n]).astype(float))
    t = O.tail(res["counts"], R, eta=0.0, psi=res["psi"])
    assert t["b_k"] == pytest.approx(1.0 - 1.0 / t["ET"], rel=1e-12)


def test_large_k_reward_is_component_size():
    # k >= n: C_k(i) is the whole component, so with unit values psi_i adds |K(i;H_r)| on valid draws
    wl = W.config_er20()
    g = wl.graph
    R = 60
    res = O.sweep(g.n, g.eu, g.ev, seed=5, R=R, alpha=wl.alpha, k_min=wl.k_min, topk=g.n, want_next=True,
                  **wl.model())
    ref = np.zeros(g.n)
    for r in range(R):
        alive, _ = O.realize(g.n, g.eu, g.ev, 5, r, **wl.model())
        lab = _components(g.n, g, alive)
        size = np.array([np.count_nonzero(lab == lab[i]) for i in range(g.n)])
        valid = res["next_table"][r] >= 0
        ref += np.where(valid, size, 0)
    assert np.array_equal(res["psi"], ref)


def test_pool_of_every_vertex_selects_the_centre():
    wl = W.config_er20()
    g = wl.graph
    for k in (1, 3):
        res = O.sweep(g.n, g.eu, g.ev, seed=9, R=200, alpha=wl.alpha, k_min=wl.k_min, topk=k,
                      pool=np.arange(g.n), **wl.model())
        assert np.array_equal(res["counts_w"], res["counts"])


def _simulate(Q, r, s, reward, episodes, rng, visit_mask=None):
    """Trajectories of the absorbing chain (Q, r) from s: total reward / total steps, and the
    share of steps spent on each state (optionally among the steps outside a mask)."""
    n = len(s)
    P = np.hstack([Q, r[:, None]])
    cum = np.cumsum(P, axis=1)
    cum[:, -1] = 1.0
    x = rng.choice(n, size=episodes, p=s)
    alive = np.ones(episodes, bool)
    tot_reward, tot_steps = 0.0, 0
    visits = np.zeros(n)
    while alive.any():
        xs = x[alive]
        tot_reward += reward[xs].sum()
        tot_steps += len(xs)
        np.add.at(visits, xs, 1)
        u = rng.random(len(xs))
        nxt = (cum[xs] < u[:, None]).sum(axis=1)
        x[alive] = np.minimum(nxt, n - 1)
        alive[np.flatnonzero(alive)[nxt == n]] = False
    return tot_reward / tot_steps, visits


def test_reward_afc_equals_uniform_pre_absorption_average():
    wl = W.config_er20()
    g = wl.graph
    R = 500
    pool = np.array([1, 4, 7, 11, 15])
    gamma = 0.5 + 1.5 * np.random.default_rng(2).random(g.n)
    res = O.sweep(g.n, g.eu, g.ev, seed=11, R=R, alpha=wl.alpha, k_min=wl.k_min, topk=3, pool=pool, gamma=gamma,
                  **wl.model())
    t = O.tail(res["counts"], R, psi=res["psi"], psi_w=res["psi_w"])
    Q, rr = O.counts_to_kernel(res["counts"], R, 0.1 / np.sqrt(R))
    s = np.full(g.n, 1.0 / g.n)
    rng = np.random.default_rng(0)
    est, _ = _simulate(Q, rr, s, res["psi"] / R, 200000, rng)
    est_w, _ = _simulate(Q, rr, s, res["psi_w"] / R, 200000, rng)
    assert est == pytest.approx(t["b_k"], rel=0.01)
    assert est_w == pytest.approx(t["b_kw"], rel=0.03)


def test_fallback_kernel_from_per_draw_selection_and_censoring():
    wl = W.config_er20()
    g = wl.graph
    R = 500
    pool = np.array([2, 5, 8, 13])
    fb_set = np.array([0, 19])
    fb_node = 19
    res = O.sweep(g.n, g.eu, g.ev, seed=13, R=R, alpha=wl.alpha, k_min=wl.k_min, topk=2, pool=pool,
                  want_next=True, **wl.model())
    t = O.tail(res["counts"], R, pool=pool, counts_w=res["counts_w"], fb_node=fb_node, fb_set=fb_set)
    # the selector of Section 7.3 draw by draw: the pool pick, else v_fb on a valid draw, else bottom
    n = g.n
    cf = np.zeros((n, n + 1), np.uint32)
    for r in range(R):
        for i in range(n):
            nw, nx = res["next_table_w"][r, i], res["next_table"][r, i]
            j = nw if nw >= 0 else (fb_node if nx >= 0 else n)
            cf[i, j] += 1
    Q, rr = O.counts_to_kernel(cf, R, 0.1 / np.sqrt(R))
    N = O.fundamental(Q)
    mu, ET, b = O.visits(N, np.full(n, 1.0 / n))
    assert np.allclose(t["b_fb"], b, rtol=0, atol=1e-12 * b.max())
    assert t["ET_fb"] == pytest.approx(ET, rel=1e-12)
    assert t["m_w_fb"] == pytest.approx(b[pool].sum(), rel=1e-12)
    # censoring: the uniform pre-absorption step conditioned on leaving V_fb
    assert np.all(t["b_cens"][fb_set] == 0.0)
    assert t["b_cens"].sum() == pytest.approx(1.0, rel=1e-12)
    _, visits = _simulate(Q, rr, np.full(n, 1.0 / n), np.zeros(n), 200000, np.random.default_rng(1))
    off = np.ones(n, bool)
    off[fb_set] = False
    share = visits[off] / visits[off].sum()
    assert np.allclose(share, t["b_cens"][off], atol=0.004)


def test_fallback_equals_pool_kernel_when_the_pool_is_everything():
    wl = W.config_er20()
    g = wl.graph
    R = 300
    pool = np.arange(1, g.n)             # every vertex but the fallback representative
    res = O.sweep(g.n, g.eu, g.ev, seed=17, R=R, alpha=wl.alpha, k_min=wl.k_min, topk=g.n, pool=pool,
                  **wl.model())
    # with k = n every valid draw's Top-k set holds a pool member (components of >= 2 vertices)
    t = O.tail(res["counts"], R, pool=pool, counts_w=res["counts_w"], fb_node=0, fb_set=[0])
    assert np.allclose(t["b_fb"], t["b_w"], rtol=0, atol=1e-15)
