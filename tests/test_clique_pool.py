"""The 3-clique target pool of the structure-constrained experiment
(Section 9), checked by brute force over all vertex triples."""
import itertools

import numpy as np

from paper_2605_14743_amd import workloads as W


def brute(g, S):
    E = set(zip(g.eu.tolist(), g.ev.tolist()))
    deg = g.degrees()
    tri = [(a, b, c) for a, b, c in itertools.combinations(range(g.n), 3)
           if (a, b) in E and (a, c) in E and (b, c) in E]
    tri.sort(key=lambda t: (-int(deg[list(t)].sum()), t))
    return tri[:S]


def test_against_brute_force():
    for seed in range(6):
        g = W.er_graph(24, 0.3, seed)
        for S in (1, 3, 8, 1000):
            Wp, fb, chosen = W.clique_pool(g, S)
            ref = brute(g, S)
            assert chosen == ref
            assert np.array_equal(Wp, sorted({v for t in ref for v in t}))
            assert fb == (ref[0][0] if ref else -1)


def test_two_cliques_bridge():
    # Fig. 1: the triangles live inside the two 4-cliques; the clique holding the
    # bridge end (degree 4) scores highest
    g = W.two_cliques_bridge()
    Wp, fb, chosen = W.clique_pool(g, 2)
    deg = g.degrees()
    assert all(deg[list(t)].sum() == max(deg[list(u)].sum() for u in brute(g, 100)) for t in chosen[:1])
    assert len(brute(g, 100)) == 8                         # 4 triangles in each 4-clique
    assert fb == chosen[0][0] and fb in Wp


def test_triangle_free_graph():
    g = W.canonical(6, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5)])
    Wp, fb, chosen = W.clique_pool(g, 8)
    assert len(Wp) == 0 and fb == -1 and chosen == []
