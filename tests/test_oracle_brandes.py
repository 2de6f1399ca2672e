"""Pins of the oracle's distances, exact path counts, betweenness, components
and tie-broken argmax (Section 3.1 and Section 3.2 of the paper).

Independent references: brute-force enumeration of all simple paths with exact
rationals, Floyd-Warshall (scipy), networkx's betweenness, closed forms, the
two-clique example of Fig. 1 and the crossroads base graph of Section 2.1.
"""
import itertools
import math
from fractions import Fraction

import networkx as nx
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components, shortest_path

import oracle as O
from paper_2605_14743_amd import workloads as W


def _adj(n, eu, ev, alive, w):
    adj = [dict() for _ in range(n)]
    for e, (u, v) in enumerate(zip(eu, ev)):
        if alive[e]:
            adj[u][v] = int(w[e])
            adj[v][u] = int(w[e])
    return adj


def brute_force(n, eu, ev, alive, w):
    """Exact B_v by enumerating every simple s-t path (exact rationals)."""
    adj = _adj(n, eu, ev, alive, w)
    dist = np.full((n, n), -1, dtype=np.int64)
    sig = np.zeros((n, n), dtype=object)
    B = [Fraction(0)] * n
    for s in range(n):
        paths = {t: [] for t in range(n)}
        stack = [(s, [s], 0)]
        while stack:
            x, path, L = stack.pop()
            paths[x].append((L, path))
            for y, wt in adj[x].items():
                if y not in path:
                    stack.append((y, path + [y], L + wt))
        for t in range(n):
            if t == s:
                dist[s, t] = 0
                sig[s, t] = 1
                continue
            if not paths[t]:
                continue
            best = min(L for L, _ in paths[t])
            sp = [p for L, p in paths[t] if L == best]
            dist[s, t] = best
            sig[s, t] = len(sp)
            for v in range(n):
                if v in (s, t):
                    continue
                through = sum(1 for p in sp if v in p[1:-1])
                B[v] += Fraction(through, len(sp))
    return B, dist, sig


def _random_tiny(rng, n, p, weighted):
    pairs = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p]
    g = W.canonical(n, pairs)
    alive = (rng.random(g.m) < 0.85).astype(np.uint8)
    w = rng.integers(1, 4, size=g.m).astype(np.uint32) if weighted else np.ones(g.m, np.uint32)
    return g, alive, w


@pytest.mark.parametrize("weighted", [False, True])
def test_brandes_equals_brute_force_tiny(weighted):
    rng = np.random.default_rng(11 + weighted)
    for trial in range(60):
        n = int(rng.integers(2, 8))
        g, alive, w = _random_tiny(rng, n, 0.55, weighted)
        B = O.betweenness(n, g.eu, g.ev, alive, w, unit=not weighted)
        Bp = O.betweenness(n, g.eu, g.ev, alive, w, unit=not weighted, pairs=True)
        ex, dist, sig = brute_force(n, g.eu, g.ev, alive, w)
        assert np.allclose(B, [float(x) for x in ex], rtol=1e-13, atol=1e-13), (trial, B, ex)
        assert np.allclose(Bp, [float(x) for x in ex], rtol=1e-13, atol=1e-13)
        for s in range(n):
            d, sg, _ = O.sssp(n, g.eu, g.ev, alive, w, not weighted, s)
            reach = dist[s] >= 0
            assert np.array_equal(d[reach].astype(np.int64), dist[s][reach])
            assert np.all(d[~reach] == np.iinfo(np.uint64).max)
            assert [int(x) for x in sg[reach]] == [int(x) for x in sig[s][reach]]
            assert np.all(sg[~reach] == 0)


def test_all_small_connected_graphs_atlas():
    """Every graph of the networkx atlas with 3..6 vertices, unit weights."""
    for G in nx.graph_atlas_g()[3:209]:
        n = G.number_of_nodes()
        g = W.canonical(n, list(G.edges()))
        one = np.ones(g.m, np.uint8)
        B = O.betweenness(n, g.eu, g.ev, one, None, True)
        ex, _, _ = brute_force(n, g.eu, g.ev, one, np.ones(g.m, np.uint32))
        assert np.allclose(B, [float(x) for x in ex], rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("n", [2, 3, 5, 9])
def test_closed_forms_path_star_complete(n):
    path = W.canonical(n, [(i, i + 1) for i in range(n - 1)])
    B = O.betweenness(n, path.eu, path.ev)
    # ordered pairs: vertex k (1-based) separates (k-1) vertices from (n-k)
    assert np.allclose(B, [2 * (k - 1) * (n - k) for k in range(1, n + 1)])
    star = W.canonical(n, [(0, i) for i in range(1, n)])
    B = O.betweenness(n, star.eu, star.ev)
    assert B[0] == (n - 1) * (n - 2) and np.all(B[1:] == 0)
    kn = W.canonical(n, [(u, v) for u in range(n) for v in range(u + 1, n)])
    B = O.betweenness(n, kn.eu, kn.ev)
    assert np.all(B == 0)
    assert O.band_argmax(B, np.ones(n, np.uint8))[0] == 0   # all tie -> smallest index


def test_two_cliques_bridge_fig1():
    """Fig. 1: vertex 5 is the unique maximiser; every cross-clique ordered pair
    (4 x 4 x 2 = 32) passes it, while 1 and 6 each carry 3 x 5 x 2 = 30."""
    g = W.two_cliques_bridge()
    B = O.betweenness(g.n, g.eu, g.ev)
    assert B[4] == 32 and B[0] == 30 and B[5] == 30
    assert O.band_argmax(B, np.ones(g.n, np.uint8))[0] == 4
    deg = g.degrees()                                       # walk stationary law: 2/28 vs 4/28
    assert deg[4] / deg.sum() == pytest.approx(2 / 28) and deg[0] / deg.sum() == pytest.approx(4 / 28)


def test_crossroads_base_graph_shares(golden):
    ref = golden("crossroads.json")["base_bc_share"]
    g, _ = W.crossroads()
    B = O.betweenness(g.n, g.eu, g.ev)
    share = B / B.sum()
    for v in (0, 3, 6):
        assert share[v] == pytest.approx(ref["gateways"], abs=5e-4)
    assert share[9] == pytest.approx(ref["hub"], abs=5e-4)
    assert np.all(share[[1, 2, 4, 5, 7, 8]] == 0)


def test_hop_identity_unweighted():
    """sum_v B_v = sum over connected ordered pairs (s != t) of (hops - 1)."""
    rng = np.random.default_rng(3)
    for trial in range(6):
        n = int(rng.integers(30, 90))
        g = W.er_graph(n, 3.0 / n, int(rng.integers(1 << 30)))
        alive = (rng.random(g.m) < 0.9).astype(np.uint8)
        B = O.betweenness(n, g.eu, g.ev, alive, None, True)
        A = csr_matrix((np.ones(2 * int(alive.sum())), (np.r_[g.eu[alive == 1], g.ev[alive == 1]],
                                                          np.r_[g.ev[alive == 1], g.eu[alive == 1]])), shape=(n, n))
        D = shortest_path(A, unweighted=True)
        fin = np.isfinite(D) & (D > 0)
        assert B.sum() == pytest.approx(float((D[fin] - 1).sum()), rel=1e-12)


def test_against_networkx_weighted():
    rng = np.random.default_rng(5)
    for trial in range(4):
        g = W.ws_graph(120, 6, 0.2, trial)
        alive, w = O.realize(g.n, g.eu, g.ev, trial, 3, p_fail=0.15, weight="uniform", w_lo=1, w_hi=6)
        B = O.betweenness(g.n, g.eu, g.ev, alive, w, unit=False)
        G = nx.Graph()
        G.add_nodes_from(range(g.n))
        for e in range(g.m):
            if alive[e]:
                G.add_edge(int(g.eu[e]), int(g.ev[e]), weight=int(w[e]))
        ref = nx.betweenness_centrality(G, normalized=False, weight="weight")
        # networkx counts each unordered pair once on undirected graphs
        assert np.allclose(B, [2 * ref[v] for v in range(g.n)], rtol=1e-10, atol=1e-9)


def test_pair_definition_equals_brandes_medium():
    rng = np.random.default_rng(9)
    g = W.er_graph(60, 0.08, 2)
    alive, w = O.realize(g.n, g.eu, g.ev, 4, 0, p_fail=0.1, weight="uniform", w_lo=1, w_hi=4)
    for unit in (True, False):
        B = O.betweenness(g.n, g.eu, g.ev, alive, w, unit)
        Bp = O.betweenness(g.n, g.eu, g.ev, alive, w, unit, pairs=True)
        assert np.allclose(B, Bp, rtol=1e-12, atol=1e-12)


def test_distances_against_floyd_warshall():
    g = W.ws_graph(80, 6, 0.3, 1)
    alive, w = O.realize(g.n, g.eu, g.ev, 1, 5, p_fail=0.1, weight="uniform", w_lo=1, w_hi=9)
    a = alive == 1
    A = csr_matrix((np.r_[w[a], w[a]].astype(float), (np.r_[g.eu[a], g.ev[a]], np.r_[g.ev[a], g.eu[a]])),
                   shape=(g.n, g.n))
    D = shortest_path(A, method="FW", directed=False)
    for s in range(0, g.n, 7):
        d, _, _ = O.sssp(g.n, g.eu, g.ev, alive, w, False, s)
        fin = np.isfinite(D[s])
        assert np.array_equal(d[fin].astype(np.int64), D[s][fin].astype(np.int64))
        assert np.all(d[~fin] == np.iinfo(np.uint64).max)


def _grid(a, b):
    idx = lambda i, j: i * b + j
    pairs = [(idx(i, j), idx(i, j + 1)) for i in range(a) for j in range(b - 1)]
    pairs += [(idx(i, j), idx(i + 1, j)) for i in range(a - 1) for j in range(b)]
    return W.canonical(a * b, pairs)


def test_sigma_binomials_on_grid():
    g = _grid(12, 17)
    d, sg, _ = O.sssp(g.n, g.eu, g.ev, np.ones(g.m, np.uint8), np.ones(g.m, np.uint32), True, 0)
    for i in range(12):
        for j in range(17):
            assert int(sg[i * 17 + j]) == math.comb(i + j, i)
            assert int(d[i * 17 + j]) == i + j


def test_sigma_overflow_is_reported():
    ok = _grid(34, 34)        # C(66, 33) ~ 7.2e18 < 2^64
    d, sg, _ = O.sssp(ok.n, ok.eu, ok.ev, np.ones(ok.m, np.uint8), np.ones(ok.m, np.uint32), True, 0)
    assert int(sg[-1]) == math.comb(66, 33)
    bad = _grid(35, 35)       # C(68, 34) ~ 2.8e19 > 2^64
    with pytest.raises(O.OracleError) as ei:
        O.sssp(bad.n, bad.eu, bad.ev, np.ones(bad.m, np.uint8), np.ones(bad.m, np.uint32), True, 0)
    assert ei.value.rc == O.E_SIGMA
    with pytest.raises(O.OracleError):
        O.sssp(bad.n, bad.eu, bad.ev, np.ones(bad.m, np.uint8), np.ones(bad.m, np.uint32), False, 0)


def test_components_against_scipy():
    rng = np.random.default_rng(21)
    for trial in range(5):
        g = W.er_graph(300, 1.2 / 300, trial)
        alive = (rng.random(g.m) < 0.7).astype(np.uint8)
        comp, size = O.components(g.n, g.eu, g.ev, alive)
        a = alive == 1
        A = csr_matrix((np.ones(int(a.sum())), (g.eu[a], g.ev[a])), shape=(g.n, g.n))
        k, lab = connected_components(A, directed=False)
        for c in range(k):
            mem = np.flatnonzero(lab == c)
            assert np.all(comp[mem] == mem.min()) and np.all(size[mem] == len(mem))


def test_band_argmax_matches_exact_rational_argmax():
    rng = np.random.default_rng(17)
    for trial in range(80):
        n = int(rng.integers(3, 8))
        g, alive, w = _random_tiny(rng, n, 0.5, bool(trial % 2))
        ex, _, _ = brute_force(n, g.eu, g.ev, alive, w)
        B = O.betweenness(n, g.eu, g.ev, alive, w, unit=not (trial % 2))
        comp, _ = O.components(n, g.eu, g.ev, alive)
        for c in set(comp.tolist()):
            mem = comp == c
            best = max(ex[v] for v in range(n) if mem[v])
            exact = min(v for v in range(n) if mem[v] and ex[v] == best)
            assert O.band_argmax(B, mem.astype(np.uint8))[0] == exact
    assert O.band_argmax(np.zeros(3), np.zeros(3, np.uint8))[0] == -1


def test_band_rule_on_rounding_ties():
    B = np.array([1.0, 0.9999999999999999, 3.0 - 1e-13, 3.0, 2.0])
    assert O.band_argmax(B, np.array([1, 1, 0, 0, 0], np.uint8))[0] == 0
    assert O.band_argmax(B, np.array([0, 0, 1, 1, 1], np.uint8))[0] == 2
    assert O.band_argmax(B, np.array([0, 0, 1, 1, 1], np.uint8), tau=1e-15)[0] == 3


@pytest.mark.parametrize("n", [5, 6, 9, 12])
def test_closed_form_cycle(n):
    """Cycle C_n, ordered pairs: with k = floor(n/2), every vertex has B =
    k(k-1) for odd n; for even n the antipodal pairs split over two paths,
    giving (k-1)^2.  Checked against brute-force path enumeration as well."""
    c = W.canonical(n, [(i, i + 1) for i in range(n - 1)] + [(0, n - 1)])
    B = O.betweenness(n, c.eu, c.ev)
    k = n // 2
    want = k * (k - 1) if n % 2 else (k - 1) ** 2
    assert np.allclose(B, want, rtol=1e-14, atol=0)
    one = np.ones(c.m, np.uint8)
    ex, _, _ = brute_force(n, c.eu, c.ev, one, np.ones(c.m, np.uint32))
    assert [float(x) for x in ex] == [float(want)] * n
    assert O.band_argmax(B, np.ones(n, np.uint8))[0] == 0
