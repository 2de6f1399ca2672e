"""GPU parity of the Wasserstein-1 leg of the robust tail (amc_robust with a
base topology, on the hop metric or on integer edge lengths; robust
experiments of Sections 9.1 and 9.2) against the oracle: W1 of
every sampled profile from b0 within 1e-11 of the largest (two exact
transshipment solvers that push along different shortest paths), the
maximiser identical unless the two largest are that close, and the AFC at
the maximiser within 1e-12 of its max norm."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2605_14743_amd import amc
from paper_2605_14743_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = amc.Context(0)
    yield c
    c.close()


def random_kernel(n, seed, leak=0.2, density=0.5):
    rng = np.random.default_rng(seed)
    Q = rng.random((n, n)) * (rng.random((n, n)) < density)
    Q[np.arange(n), rng.integers(0, n, n)] += 0.1
    return Q / Q.sum(1, keepdims=True) * (1 - leak)


def connected_graph(n, extra, seed):
    rng = np.random.default_rng(seed)
    edges = {(int(rng.integers(0, v)), v) for v in range(1, n)}
    while len(edges) < n - 1 + extra and len(edges) < n * (n - 1) // 2:
        u, v = sorted(rng.choice(n, 2, replace=False).tolist())
        edges.add((u, v))
    e = np.array(sorted(edges), dtype=np.int32).reshape(-1, 2)
    return e[:, 0], e[:, 1]


def oracle_w1(Q0, eu, ev, samples, delta, r_min, seed, only=None, cost=None):
    n = Q0.shape[0]
    s = np.full(n, 1.0 / n)
    b0 = O.chain(Q0, s)["b"]
    out = {}
    for k in (range(samples) if only is None else only):
        bk = O.chain(O.perturbed_kernel(Q0, seed, k, delta, r_min), s)["b"]
        out[k] = (O.w1(n, eu, ev, bk, b0, cost=cost), bk)
    return out


def check(g, o, what):
    w = np.array([o[k][0] for k in sorted(o)])
    scale = max(w.max(), 1e-300)
    assert np.abs(g["w1"] - w).max() <= 1e-11 * scale, f"{what}: w1"
    top2 = np.sort(w)[-2:] if len(w) > 1 else w
    if len(w) == 1 or top2[1] - top2[0] > 1e-10 * scale:
        assert g["w1_arg"] == int(np.argmax(w)), what
    bw = o[g["w1_arg"]][1]
    assert np.abs(g["b_w1"] - bw).max() <= 1e-12 * np.abs(bw).max(), f"{what}: b_w1"


@pytest.mark.parametrize("n,extra,samples", [(2, 0, 5), (7, 4, 12), (64, 40, 12), (130, 300, 12), (20, 10, 130)])
def test_random_topologies(ctx, n, extra, samples):
    Q0 = random_kernel(n, n)
    eu, ev = connected_graph(n, extra, n)
    say(f"[gpu] robust w1 n={n} m={len(eu)} samples={samples}")
    g = amc.robust(ctx, Q0, samples=samples, delta=0.4, r_min=0.05, seed=n, topology=(eu, ev))
    o = oracle_w1(Q0, eu, ev, samples, 0.4, 0.05, n)
    check(g, o, f"n={n}")
    # the KL / TV legs are unchanged by the topology
    g0 = amc.robust(ctx, Q0, samples=samples, delta=0.4, r_min=0.05, seed=n)
    assert np.array_equal(g0["kl"], g["kl"]) and np.array_equal(g0["tv"], g["tv"])
    assert g0["w1_arg"] == -1


def test_tree_topology(ctx):
    # a path: W1 is the sum of the absolute cumulative differences
    n = 50
    Q0 = random_kernel(n, 5)
    eu = np.arange(n - 1, dtype=np.int32)
    ev = eu + 1
    say("[gpu] robust w1 on a path")
    g = amc.robust(ctx, Q0, samples=8, delta=0.5, r_min=0.05, seed=3, topology=(eu, ev))
    o = oracle_w1(Q0, eu, ev, 8, 0.5, 0.05, 3)
    check(g, o, "path")
    for k in range(8):
        expect = np.abs(np.cumsum(o[k][1] - g["b0"])[:-1]).sum()
        assert g["w1"][k] == pytest.approx(expect, rel=1e-11)


def test_long_path_past_the_lds_cache(ctx):
    # n = 2500 on a path: 20 n + 5 m bytes exceed the LDS cache of the edges, so
    # the ends and flow signs are read from HBM; W1 of the maximiser against the
    # cumulative-sum closed form
    n = 2500
    Q0 = random_kernel(n, 9, density=0.004)
    eu = np.arange(n - 1, dtype=np.int32)
    ev = eu + 1
    say("[gpu] robust w1 on a path of 2500 vertices")
    g = amc.robust(ctx, Q0, samples=3, delta=0.5, r_min=0.05, seed=2, topology=(eu, ev))
    k = g["w1_arg"]
    expect = np.abs(np.cumsum(g["b_w1"] - g["b0"])[:-1]).sum()
    assert g["w1"][k] == pytest.approx(expect, rel=1e-10)
    assert np.all(g["w1"] >= g["tv"] * (1 - 1e-12))


def test_ws1000_estimated_kernel(ctx):
    # the kernel estimated from the WS(1000) run, its own base topology, 100 samples
    wl = W.config_ws1000()
    gr = wl.graph
    G = amc.Graph(ctx, gr.n, gr.eu, gr.ev, gr.w0)
    res = amc.run(ctx, G, wl.model(), seed=wl.seed, R=wl.R, alpha=wl.alpha, k_min=wl.k_min)
    G.close()
    say("[gpu] robust w1 on the ws1000 kernel, 100 samples")
    g = amc.robust(ctx, res["Q"], samples=100, delta=0.5, r_min=0.05, seed=1, topology=(gr.eu, gr.ev))
    assert 0 <= g["w1_arg"] < 100 and g["w1"][g["w1_arg"]] == g["w1"].max()
    for k in (g["w1_arg"], 17):
        say(f"[gpu]   oracle sample {k}")
        o = oracle_w1(res["Q"], gr.eu, gr.ev, 100, 0.5, 0.05, 1, only=[k])
        assert g["w1"][k] == pytest.approx(o[k][0], rel=1e-11)
    # on a graph metric the moved mass (total variation) costs at least 1 and at most the diameter per unit
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import shortest_path
    D = shortest_path(coo_matrix((np.ones(gr.m), (gr.eu, gr.ev)), shape=(gr.n, gr.n)), directed=False,
                      unweighted=True)
    assert np.all(g["w1"] >= g["tv"] * (1 - 1e-12)) and np.all(g["w1"] <= D.max() * g["tv"] * (1 + 1e-12))


def test_topology_arguments(ctx):
    n = 6
    Q0 = random_kernel(n, 1)
    eu, ev = connected_graph(n, 2, 1)
    bad = [(np.array([0, 2], np.int32), np.array([1, 3], np.int32)),      # disconnected
           (ev, eu),                                                      # eu > ev
           (eu[::-1].copy(), ev[::-1].copy()),                            # not increasing
           (np.array([0, 1, 2, 3, 4, 4], np.int32), np.array([1, 2, 3, 4, 5, 6], np.int32))]   # out of range
    for t in bad:
        with pytest.raises(amc.AmcError) as ei:
            amc.robust(ctx, Q0, samples=3, topology=t)
        assert ei.value.rc == amc.E_INVALID_ARG
    N = amc.MAX_W1_N + 1
    Qb = np.zeros((N, N))
    Qb[np.arange(N), (np.arange(N) + 1) % N] = 0.5
    path = (np.arange(N - 1, dtype=np.int32), np.arange(1, N, dtype=np.int32))
    with pytest.raises(amc.AmcError) as ei:
        amc.robust(ctx, Qb, samples=1, topology=path)
    assert ei.value.rc == amc.E_UNSUPPORTED
    # no samples: nothing to measure, no maximiser
    g = amc.robust(ctx, Q0, samples=0, topology=(eu, ev))
    assert g["w1_arg"] == -1


# ---- integer edge lengths (the weighted ground metric) ----

@pytest.mark.parametrize("n,extra,samples,w_hi", [(7, 4, 12, 9), (64, 40, 12, 100), (130, 300, 12, 65535),
                                                  (20, 10, 130, 3)])
def test_weighted_random_topologies(ctx, n, extra, samples, w_hi):
    Q0 = random_kernel(n, n + 1)
    eu, ev = connected_graph(n, extra, n + 1)
    w = np.random.default_rng(n).integers(1, w_hi + 1, len(eu)).astype(np.uint32)
    say(f"[gpu] robust w1 weighted n={n} m={len(eu)} lengths 1..{w_hi} samples={samples}")
    g = amc.robust(ctx, Q0, samples=samples, delta=0.4, r_min=0.05, seed=n, topology=(eu, ev, w))
    o = oracle_w1(Q0, eu, ev, samples, 0.4, 0.05, n, cost=w)
    check(g, o, f"weighted n={n}")
    g0 = amc.robust(ctx, Q0, samples=samples, delta=0.4, r_min=0.05, seed=n, topology=(eu, ev))
    assert np.array_equal(g0["kl"], g["kl"]) and np.array_equal(g0["tv"], g["tv"])
    # every length at least 1: never below the hop metric, never above w_hi times it
    assert np.all(g["w1"] >= g0["w1"] * (1 - 1e-12)) and np.all(g["w1"] <= w_hi * g0["w1"] * (1 + 1e-12))


def test_unit_lengths_are_the_hop_metric(ctx):
    n = 64
    Q0 = random_kernel(n, 4)
    eu, ev = connected_graph(n, 40, 4)
    say("[gpu] robust w1 with explicit unit lengths")
    g1 = amc.robust(ctx, Q0, samples=12, delta=0.4, r_min=0.05, seed=4,
                    topology=(eu, ev, np.ones(len(eu), np.uint32)))
    g0 = amc.robust(ctx, Q0, samples=12, delta=0.4, r_min=0.05, seed=4, topology=(eu, ev))
    assert np.array_equal(g1["w1"], g0["w1"]) and g1["w1_arg"] == g0["w1_arg"]


@pytest.mark.parametrize("n", [50, 2500])
def test_weighted_path_closed_form(ctx, n):
    # on a path with lengths w_i, W1 = sum_i w_i |cumulative difference up to i|;
    # n = 2500 takes the kernel that reads ends, lengths and signs from HBM
    Q0 = random_kernel(n, 11, density=0.5 if n < 100 else 0.004)
    eu = np.arange(n - 1, dtype=np.int32)
    ev = eu + 1
    w = np.random.default_rng(n).integers(1, 1000, n - 1).astype(np.uint32)
    samples = 8 if n < 100 else 3
    say(f"[gpu] robust w1 on a weighted path of {n} vertices")
    g = amc.robust(ctx, Q0, samples=samples, delta=0.5, r_min=0.05, seed=6, topology=(eu, ev, w))
    if n < 100:
        o = oracle_w1(Q0, eu, ev, samples, 0.5, 0.05, 6, cost=w)
        check(g, o, "weighted path")
    k = g["w1_arg"]
    expect = (w * np.abs(np.cumsum(g["b_w1"] - g["b0"])[:-1])).sum()
    assert g["w1"][k] == pytest.approx(expect, rel=1e-10)


@pytest.mark.parametrize("n,weighted", [(3500, True), (6000, True), (amc.MAX_W1_N, False)])
def test_tree_closed_form_past_64k_lds(ctx, n, weighted):
    # on a tree every edge carries the net mass of the subtree below it, so
    # W1 = sum over edges of w_e |sum of p - q over that subtree|; from n = 3500
    # on the solver's node arrays alone take more than 64 KB of LDS
    rng = np.random.default_rng(n)
    par = np.array([int(rng.integers(0, v)) for v in range(1, n)], np.int64)   # random recursive tree
    order = np.lexsort((np.arange(1, n), par))
    eu = par[order].astype(np.int32)
    ev = np.arange(1, n, dtype=np.int32)[order]
    w = rng.integers(1, 1000, n - 1).astype(np.uint32) if weighted else np.ones(n - 1, np.uint32)
    Q0 = random_kernel(n, 12, density=0.004)
    say(f"[gpu] robust w1 on a random tree of {n} vertices, weighted={weighted}")
    topo = (eu, ev, w) if weighted else (eu, ev)
    g = amc.robust(ctx, Q0, samples=3, delta=0.5, r_min=0.05, seed=7, topology=topo)
    k = g["w1_arg"]
    sub = g["b_w1"] - g["b0"]
    for v in range(n - 1, 0, -1):          # parents precede their children
        sub[par[v - 1]] += sub[v]
    wv = np.empty(n)
    wv[ev] = w
    expect = (wv[1:] * np.abs(sub[1:])).sum()
    assert g["w1"][k] == pytest.approx(expect, rel=1e-10)
    assert np.all(g["w1"] >= g["tv"] * (1 - 1e-12))


def test_cooc77_fixed_weights(ctx):
    # the 77-node weighted co-occurrence stand-in with its own fixed weights as
    # the ground metric, on the kernel estimated from its run
    wl = W.config_cooc77()
    gr = wl.graph
    G = amc.Graph(ctx, gr.n, gr.eu, gr.ev, gr.w0)
    res = amc.run(ctx, G, wl.model(), seed=wl.seed, R=2000, alpha=wl.alpha, k_min=wl.k_min)
    G.close()
    say("[gpu] robust w1 on the cooc77 kernel with its weights, 40 samples")
    g = amc.robust(ctx, res["Q"], samples=40, delta=0.5, r_min=0.05, seed=2, topology=(gr.eu, gr.ev, gr.w0))
    o = oracle_w1(res["Q"], gr.eu, gr.ev, 40, 0.5, 0.05, 2, cost=gr.w0)
    check(g, o, "cooc77 weighted")


def test_edge_length_arguments(ctx):
    n = 6
    Q0 = random_kernel(n, 1)
    eu, ev = connected_graph(n, 2, 1)
    for bad in (0, 65536):
        w = np.ones(len(eu), np.uint32)
        w[len(eu) // 2] = bad
        with pytest.raises(amc.AmcError) as ei:
            amc.robust(ctx, Q0, samples=3, topology=(eu, ev, w))
        assert ei.value.rc == amc.E_INVALID_ARG
