"""Pins of the oracle's anchored r-hop neighbourhoods (Section 9.2): each
anchor's step ranks the betweenness of the subgraph induced by the vertices
within r surviving hops of the anchor.

Independent references: exact-rational betweenness of each induced subgraph by
path enumeration; a radius covering the whole graph reduces to the row-wise
component centres; a star graph solved by hand.
"""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

import oracle as O
from paper_2605_14743_amd import workloads as W
from test_oracle_brandes import brute_force


def exact_anchored(g, model, seed, R, radius, alpha, k_min, pool=None):
    n = g.n
    cnt = np.zeros((n, n + 1), np.uint32)
    cw = np.zeros((n, n + 1), np.uint32)
    for r in range(R):
        alive, w = O.realize(n, g.eu, g.ev, seed, r, **model)
        e = np.flatnonzero(alive)
        A = csr_matrix((np.ones(len(e)), (g.eu[e], g.ev[e])), shape=(n, n))
        hops = shortest_path(A, directed=False, unweighted=True)
        for i in range(n):
            S = np.flatnonzero(hops[i] <= radius)
            inS = np.zeros(n, bool)
            inS[S] = True
            aliveS = (alive.astype(bool) & inS[g.eu] & inS[g.ev]).astype(np.uint8)
            B, _, _ = brute_force(n, g.eu, g.ev, aliveS, w)
            order = sorted(S, key=lambda v: (-B[v], v))
            coin = O.stop_coin(seed, r, i, alpha)
            valid = (not coin) and len(S) >= k_min
            cnt[i, order[0] if valid else n] += 1
            if pool is not None:
                inpool = [v for v in order if v in set(pool)]
                cw[i, inpool[0] if (valid and inpool) else n] += 1
    return cnt, cw


@pytest.mark.parametrize("trial", range(3))
def test_anchored_counts_match_exact_induced_betweenness(trial):
    rng = np.random.default_rng(300 + trial)
    n = 8
    pairs = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < 0.4]
    g = W.canonical(n, pairs)
    model = {"p_fail": 0.15, "weight": "uniform", "w_lo": 1, "w_hi": 3}
    pool = [1, 4, 6]
    for radius in (1, 2):
        res = O.sweep(n, g.eu, g.ev, seed=trial, R=10, alpha=0.2, k_min=2, hop_radius=radius, pool=pool, **model)
        cnt, cw = exact_anchored(g, model, trial, 10, radius, 0.2, 2, pool)
        assert np.array_equal(res["counts"], cnt), radius
        assert np.array_equal(res["counts_w"], cw), radius


def test_radius_beyond_the_graph_is_the_row_wise_chain():
    wl = W.config_er20()
    g = wl.graph
    a = O.sweep(g.n, g.eu, g.ev, seed=4, R=80, alpha=wl.alpha, k_min=wl.k_min, want_next=True, pool=[2, 9, 11],
                **wl.model())
    b = O.sweep(g.n, g.eu, g.ev, seed=4, R=80, alpha=wl.alpha, k_min=wl.k_min, want_next=True, pool=[2, 9, 11],
                hop_radius=g.n, **wl.model())
    assert np.array_equal(a["counts"], b["counts"]) and np.array_equal(a["next_table"], b["next_table"])
    assert np.array_equal(a["counts_w"], b["counts_w"])


def test_star_by_hand():
    hub, n = 2, 6
    g = W.canonical(n, [(min(hub, v), max(hub, v)) for v in range(n) if v != hub])
    res = O.sweep(n, g.eu, g.ev, seed=1, R=50, alpha=0.2, k_min=3, hop_radius=1, want_next=True, p_fail=0.0,
                  weight="unit")
    nt = res["next_table"]
    leaves = [v for v in range(n) if v != hub]
    assert np.all(nt[:, leaves] == -1)                    # S_1(leaf) = {leaf, hub}: too small
    coins = np.array([[O.stop_coin(1, r, hub, 0.2) for r in range(50)]])[0]
    assert np.array_equal(nt[:, hub], np.where(coins, -1, hub))
    # radius 1 with k_min 2: a leaf's subgraph is one edge (no intermediate vertex, B = 0 on both),
    # so the tie rule reports the smaller index of the pair
    res2 = O.sweep(n, g.eu, g.ev, seed=1, R=50, alpha=0.2, k_min=2, hop_radius=1, want_next=True, p_fail=0.0,
                   weight="unit")
    for v in leaves:
        c = [O.stop_coin(1, r, v, 0.2) for r in range(50)]
        assert np.array_equal(res2["next_table"][:, v], np.where(c, -1, min(v, hub)))
