"""Pins of the oracle's Wasserstein-1 on the hop metric of the base topology
(robust experiment of Section 9.1).

Independent references: the closed forms on a path (cumulative sums) and on a
tree (mass below every edge), the dual over integer 1-Lipschitz potentials by
exhaustive search on small graphs (exact because the edge-node incidence
matrix is totally unimodular), scipy's LP solver on the transport problem
over the all-pairs hop distances, point masses (W1 = the hop distance), and
the metric axioms."""
import itertools

import numpy as np
import pytest
from scipy.optimize import linprog
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import shortest_path

import oracle as O


def random_profile(n, rng, zeros=0.3):
    x = rng.random(n) * (rng.random(n) > zeros)
    if x.sum() == 0:
        x[0] = 1.0
    return x / x.sum()


def connected_graph(n, extra, rng):
    """A random spanning tree plus `extra` random chords, canonical edge list."""
    edges = set()
    for v in range(1, n):
        u = int(rng.integers(0, v))
        edges.add((u, v))
    while len(edges) < n - 1 + extra and len(edges) < n * (n - 1) // 2:
        u, v = sorted(rng.choice(n, 2, replace=False).tolist())
        edges.add((u, v))
    e = np.array(sorted(edges), dtype=np.int32).reshape(-1, 2)
    return e[:, 0], e[:, 1]


def hop_distances(n, eu, ev):
    A = coo_matrix((np.ones(len(eu)), (eu, ev)), shape=(n, n))
    return shortest_path(A, directed=False, unweighted=True)


def test_path_closed_form():
    rng = np.random.default_rng(0)
    for n in (2, 3, 10, 57):
        eu = np.arange(n - 1, dtype=np.int32)
        ev = eu + 1
        p, q = random_profile(n, rng), random_profile(n, rng)
        expect = np.abs(np.cumsum(p - q)[:-1]).sum()
        assert O.w1(n, eu, ev, p, q) == pytest.approx(expect, rel=1e-13, abs=1e-16)


def test_tree_closed_form():
    rng = np.random.default_rng(1)
    for n in (5, 30, 200):
        parent = np.array([-1] + [int(rng.integers(0, v)) for v in range(1, n)])
        eu, ev = parent[1:].astype(np.int32), np.arange(1, n, dtype=np.int32)
        order = np.lexsort((ev, eu))
        p, q = random_profile(n, rng), random_profile(n, rng)
        below = p - q                                     # mass of each subtree, children before parents
        for v in range(n - 1, 0, -1):
            below[parent[v]] += below[v]
        expect = np.abs(below[1:]).sum()
        assert O.w1(n, eu[order], ev[order], p, q) == pytest.approx(expect, rel=1e-12, abs=1e-16)


def brute_dual(n, eu, ev, d):
    """max sum phi_v d_v over integer phi with phi_0 = 0 and |phi_u - phi_v| <= 1 on edges."""
    adj = [[] for _ in range(n)]
    for a, b in zip(eu, ev):
        adj[a].append(b)
        adj[b].append(a)
    order, par, seen = [0], {0: None}, {0}
    for x in order:
        for y in adj[x]:
            if y not in seen:
                seen.add(y)
                par[y] = x
                order.append(y)
    best = -np.inf
    for steps in itertools.product((-1, 0, 1), repeat=n - 1):
        phi = np.zeros(n)
        for v, st in zip(order[1:], steps):
            phi[v] = phi[par[v]] + st
        if np.all(np.abs(phi[eu] - phi[ev]) <= 1):
            best = max(best, float(phi @ d))
    return best


def test_dual_by_exhaustive_search():
    rng = np.random.default_rng(2)
    for trial in range(12):
        n = int(rng.integers(3, 9))
        eu, ev = connected_graph(n, int(rng.integers(0, n)), rng)
        p, q = random_profile(n, rng), random_profile(n, rng)
        assert O.w1(n, eu, ev, p, q) == pytest.approx(brute_dual(n, eu, ev, p - q), rel=1e-12, abs=1e-15)


def test_transport_lp():
    rng = np.random.default_rng(3)
    for trial in range(6):
        n = int(rng.integers(6, 26))
        eu, ev = connected_graph(n, int(rng.integers(0, 2 * n)), rng)
        D = hop_distances(n, eu, ev)
        p, q = random_profile(n, rng), random_profile(n, rng)
        A_eq = np.vstack([np.kron(np.eye(n), np.ones(n)), np.kron(np.ones(n), np.eye(n))])
        lp = linprog(D.ravel(), A_eq=A_eq, b_eq=np.concatenate([p, q]), bounds=(0, None), method="highs")
        assert lp.status == 0
        assert O.w1(n, eu, ev, p, q) == pytest.approx(lp.fun, rel=1e-9, abs=1e-12)


def test_point_masses_and_axioms():
    rng = np.random.default_rng(4)
    n = 40
    eu, ev = connected_graph(n, 30, rng)
    D = hop_distances(n, eu, ev)
    for u, v in ((0, 39), (5, 6), (17, 3)):
        p, q = np.eye(n)[u], np.eye(n)[v]
        assert O.w1(n, eu, ev, p, q) == D[u, v]
    a, b, c = (random_profile(n, rng) for _ in range(3))
    assert O.w1(n, eu, ev, a, a) == 0.0
    assert O.w1(n, eu, ev, a, b) == pytest.approx(O.w1(n, eu, ev, b, a), rel=1e-12)
    assert O.w1(n, eu, ev, a, c) <= O.w1(n, eu, ev, a, b) + O.w1(n, eu, ev, b, c) + 1e-12


def test_unbalanced_components_are_rejected():
    eu = np.array([0, 2], dtype=np.int32)
    ev = np.array([1, 3], dtype=np.int32)
    with pytest.raises(Exception):
        O.w1(4, eu, ev, np.array([1.0, 0, 0, 0]), np.array([0, 0, 1.0, 0]))
    # balanced components are fine: each moves inside its own component
    assert O.w1(4, eu, ev, np.array([0.5, 0, 0.5, 0]), np.array([0, 0.5, 0, 0.5])) == pytest.approx(1.0)


# --------------------------------------------------------------------------- weighted ground metric
def weighted_distances(n, eu, ev, c):
    A = coo_matrix((c.astype(float), (eu, ev)), shape=(n, n)).tocsr()
    return shortest_path(A, directed=False)


def test_weighted_path_and_tree_closed_forms():
    """On a tree every unit of the mass below an edge crosses it once:
    W1 = sum over edges of c_e |mass below e|."""
    rng = np.random.default_rng(5)
    for n in (2, 9, 64):
        eu = np.arange(n - 1, dtype=np.int32)
        ev = eu + 1
        c = rng.integers(1, 12, n - 1).astype(np.uint32)
        p, q = random_profile(n, rng), random_profile(n, rng)
        expect = (c * np.abs(np.cumsum(p - q)[:-1])).sum()
        assert O.w1(n, eu, ev, p, q, cost=c) == pytest.approx(expect, rel=1e-13, abs=1e-16)
    n = 120
    parent = np.array([-1] + [int(rng.integers(0, v)) for v in range(1, n)])
    eu, ev = parent[1:].astype(np.int32), np.arange(1, n, dtype=np.int32)
    c = rng.integers(1, 31, n - 1).astype(np.uint32)
    order = np.lexsort((ev, eu))
    p, q = random_profile(n, rng), random_profile(n, rng)
    below = p - q
    for v in range(n - 1, 0, -1):
        below[parent[v]] += below[v]
    expect = (c * np.abs(below[1:])).sum()
    assert O.w1(n, eu[order], ev[order], p, q, cost=c[order]) == pytest.approx(expect, rel=1e-12, abs=1e-16)


def test_weighted_transport_lp():
    """Transport problem over the weighted all-pairs distances (scipy's
    Dijkstra and HiGHS), on graphs with cycles where paths of fewer hops can
    be longer."""
    rng = np.random.default_rng(6)
    for trial in range(6):
        n = int(rng.integers(6, 26))
        eu, ev = connected_graph(n, int(rng.integers(0, 2 * n)), rng)
        c = rng.integers(1, 32, len(eu)).astype(np.uint32)
        D = weighted_distances(n, eu, ev, c)
        p, q = random_profile(n, rng), random_profile(n, rng)
        A_eq = np.vstack([np.kron(np.eye(n), np.ones(n)), np.kron(np.ones(n), np.eye(n))])
        lp = linprog(D.ravel(), A_eq=A_eq, b_eq=np.concatenate([p, q]), bounds=(0, None), method="highs")
        assert lp.status == 0
        assert O.w1(n, eu, ev, p, q, cost=c) == pytest.approx(lp.fun, rel=1e-9, abs=1e-12)
        # unit lengths give the hop metric back
        assert O.w1(n, eu, ev, p, q, cost=np.ones(len(eu), np.uint32)) == pytest.approx(O.w1(n, eu, ev, p, q),
                                                                                          rel=1e-13)


def test_weighted_point_masses():
    rng = np.random.default_rng(7)
    n = 30
    eu, ev = connected_graph(n, 25, rng)
    c = rng.integers(1, 9, len(eu)).astype(np.uint32)
    D = weighted_distances(n, eu, ev, c)
    for u, v in ((0, 29), (4, 11), (20, 2)):
        assert O.w1(n, eu, ev, np.eye(n)[u], np.eye(n)[v], cost=c) == D[u, v]
