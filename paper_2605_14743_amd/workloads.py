"""Seeded synthetic inputs: base graphs, candidate pools, rewards, query mixes.

This module holds no arithmetic of the method; it only draws the inputs that
the GPU library and the CPU oracle both consume.  Every generator is a pure
function of its arguments (numpy ``default_rng`` streams).

The paper's experiments use Erdos-Renyi and Watts-Strogatz base graphs and a
weighted co-occurrence network (Section 9); the workloads below reproduce
their shapes.  The co-occurrence network itself is not used: a synthetic
power-law graph with the same vertex and edge counts and integer weights in
[1, 31] stands in for it.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math

import numpy as np


@dataclasses.dataclass
class Graph:
    """Undirected simple base graph as a canonical edge list (u < v, sorted)."""
    n: int
    eu: np.ndarray                      # int32[m]
    ev: np.ndarray                      # int32[m]
    w0: np.ndarray | None = None        # uint32[m] fixed integer weights, or None
    name: str = ""

    @property
    def m(self) -> int:
        return int(len(self.eu))

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        h.update(self.eu.astype(np.int32).tobytes())
        h.update(self.ev.astype(np.int32).tobytes())
        if self.w0 is not None:
            h.update(self.w0.astype(np.uint32).tobytes())
        return h.hexdigest()

    def degrees(self) -> np.ndarray:
        return np.bincount(np.concatenate([self.eu, self.ev]), minlength=self.n)


def canonical(n: int, pairs, w0=None, name: str = "") -> Graph:
    """Canonical form: u < v, lexicographically sorted, no self-loops or repeats."""
    a = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    if len(a) == 0:
        return Graph(n, np.zeros(0, np.int32), np.zeros(0, np.int32),
                     None if w0 is None else np.zeros(0, np.uint32), name)
    if np.any(a[:, 0] == a[:, 1]):
        raise ValueError("self-loop")
    u = np.minimum(a[:, 0], a[:, 1])
    v = np.maximum(a[:, 0], a[:, 1])
    key = u * n + v
    order = np.argsort(key, kind="stable")
    key = key[order]
    if np.any(key[1:] == key[:-1]):
        raise ValueError("repeated edge")
    ww = None if w0 is None else np.asarray(w0, dtype=np.uint32)[order]
    return Graph(n, u[order].astype(np.int32), v[order].astype(np.int32), ww, name)


def er_graph(n: int, p: float, seed: int) -> Graph:
    """G(n, p): every unordered pair present independently with probability p."""
    rng = np.random.default_rng(seed)
    us, vs = [], []
    for u in range(n - 1):
        hit = np.flatnonzero(rng.random(n - u - 1) < p)
        us.append(np.full(len(hit), u))
        vs.append(hit + u + 1)
    if not us:
        return canonical(n, [], name=f"er({n},{p},{seed})")
    pairs = np.stack([np.concatenate(us), np.concatenate(vs)], axis=1)
    return canonical(n, pairs, name=f"er({n},{p:.6g},{seed})")


def ws_graph(n: int, k: int, beta: float, seed: int) -> Graph:
    """Watts-Strogatz: ring lattice with k/2 neighbours per side, each lattice
    edge (u, u+j) rewired with probability beta to (u, w), w uniform among the
    vertices that are neither u nor already adjacent to u."""
    rng = np.random.default_rng(seed)
    half = k // 2
    adj = [set() for _ in range(n)]
    for u in range(n):
        for j in range(1, half + 1):
            v = (u + j) % n
            adj[u].add(v)
            adj[v].add(u)
    for j in range(1, half + 1):
        for u in range(n):
            v = (u + j) % n
            if rng.random() >= beta:
                continue
            if len(adj[u]) >= n - 1:
                continue
            while True:
                w = int(rng.integers(n))
                if w != u and w not in adj[u]:
                    break
            adj[u].discard(v)
            adj[v].discard(u)
            adj[u].add(w)
            adj[w].add(u)
    pairs = [(u, v) for u in range(n) for v in adj[u] if u < v]
    return canonical(n, pairs, name=f"ws({n},{k},{beta:.6g},{seed})")


def powerlaw_weighted_graph(n: int, m: int, exponent: float, w_mean: float, w_max: int, seed: int) -> Graph:
    """Sparse weighted power-law graph (Chung-Lu style): vertex weights
    proportional to (v + v0)^(-1/(exponent-1)); distinct pairs drawn with
    probability proportional to the product of their weights until exactly m
    edges exist; redrawn with the next sub-seed until connected.  Integer edge
    weights are geometric on {1, 2, ...} with mean w_mean, clipped at w_max."""
    sub = 0
    while True:
        rng = np.random.default_rng([seed, sub])
        x = (np.arange(n) + 3.0) ** (-1.0 / (exponent - 1.0))
        prob = x / x.sum()
        edges = set()
        while len(edges) < m:
            a = rng.choice(n, size=2 * m, p=prob)
            b = rng.choice(n, size=2 * m, p=prob)
            for u, v in zip(a, b):
                if u == v:
                    continue
                e = (min(u, v), max(u, v))
                if e not in edges:
                    edges.add(e)
                    if len(edges) == m:
                        break
        pairs = sorted(edges)
        if _connected(n, pairs):
            w = np.minimum(rng.geometric(1.0 / w_mean, size=m), w_max).astype(np.uint32)
            return canonical(n, pairs, w0=w, name=f"powerlaw({n},{m},{exponent},{seed})")
        sub += 1


def _connected(n, pairs) -> bool:
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for u, v in pairs:
        parent[find(u)] = find(v)
    return len({find(v) for v in range(n)}) == 1


def resampled_weight_cdf(w0: np.ndarray, w_max: int, rho_mu: float, rho_sigma: float) -> np.ndarray:
    """Per-edge law of the per-call resampled weight of the co-occurrence
    experiment (Section 9.2): x ~ N(mu_e, sigma_e^2) with mu_e = w0 + rho_mu
    (w_max - w0), sigma_e = rho_sigma (w_max - w0), rounded and clipped to
    [w0, w_max].  Returned as cumulative thresholds T[e, v-1] =
    floor(P(w <= v) 2^32) for v = 1..w_max (T[e, w_max-1] = 2^32), the integer
    form both the library and the oracle draw from (x1 < T means w <= v)."""
    w0 = np.asarray(w0, dtype=np.int64)
    m = len(w0)
    T = np.zeros((m, w_max), dtype=np.uint64)
    for e in range(m):
        a = int(w0[e])
        mu = a + rho_mu * (w_max - a)
        sd = rho_sigma * (w_max - a)
        for v in range(1, w_max + 1):
            if v < a:
                c = 0.0
            elif v >= w_max:
                c = 1.0
            elif sd == 0.0:
                c = 1.0 if mu < v + 0.5 else 0.0              # round half up, no spread
            else:
                c = 0.5 * math.erfc(-(v + 0.5 - mu) / (sd * math.sqrt(2.0)))
            T[e, v - 1] = min(int(math.floor(c * 4294967296.0)), 4294967296)
        T[e, w_max - 1] = 4294967296
    return T


def pool(n: int, size: int, seed: int) -> np.ndarray:
    """Candidate pool W: `size` distinct vertices, sorted."""
    rng = np.random.default_rng([seed, 2])
    return np.sort(rng.choice(n, size=min(size, n), replace=False)).astype(np.int32)


def rewards(n: int, members: np.ndarray, lo: float, hi: float, seed: int) -> np.ndarray:
    """Node values: uniform in [lo, hi] on the pool members, 0 elsewhere."""
    rng = np.random.default_rng([seed, 3])
    f = np.zeros(n, dtype=np.float64)
    f[members] = rng.uniform(lo, hi, size=len(members))
    return f


def clique_pool(g: Graph, S: int = 8) -> tuple[np.ndarray, int, list]:
    """Target pool of the structure-constrained experiment (Section 9): every
    3-clique {a < b < c} of the base graph scored by its degree sum, the S
    best taken (ties to the lexicographically smaller triple); W = their
    union (sorted), the fallback v_fb = the smallest vertex of the first
    chosen clique.  Returns (W, v_fb, chosen triples)."""
    deg = g.degrees()
    nbr = [set() for _ in range(g.n)]
    for a, b in zip(g.eu.tolist(), g.ev.tolist()):
        nbr[a].add(b)
        nbr[b].add(a)
    tri = []
    for a, b in zip(g.eu.tolist(), g.ev.tolist()):           # a < b
        for c in sorted(nbr[a] & nbr[b]):
            if c > b:
                tri.append((-int(deg[a] + deg[b] + deg[c]), a, b, c))
    tri.sort()
    chosen = [t[1:] for t in tri[:S]]
    if not chosen:
        return np.zeros(0, dtype=np.int32), -1, []
    W = np.array(sorted({v for t in chosen for v in t}), dtype=np.int32)
    return W, int(chosen[0][0]), chosen


# ----------------------------------------------------------------------------- worked examples of the paper
def two_cliques_bridge() -> Graph:
    """Two 4-cliques {1,2,3,4}, {6,7,8,9} joined by the path 1-5-6 (Fig. 1);
    vertex k of the figure is index k-1."""
    pairs = []
    for c in ([0, 1, 2, 3], [5, 6, 7, 8]):
        pairs += [(a, b) for i, a in enumerate(c) for b in c[i + 1:]]
    pairs += [(0, 4), (4, 5)]
    return canonical(9, pairs, name="two-cliques-bridge")


def crossroads() -> tuple[Graph, np.ndarray]:
    """Asymmetric crossroads (Section 2.1, Fig. 2): triangles {1,2,3}, {4,5,6},
    {7,8,9} and hub 10 with spokes 10-1, 10-4, 10-7 present with probability
    0.8, 0.5, 0.2; vertex k of the figure is index k-1.  Returns the graph and
    the per-edge failure probability (0 for triangle edges)."""
    pairs = [(0, 1), (0, 2), (1, 2), (3, 4), (3, 5), (4, 5), (6, 7), (6, 8), (7, 8), (0, 9), (3, 9), (6, 9)]
    g = canonical(10, pairs, name="crossroads")
    p_on = {(0, 9): 0.8, (3, 9): 0.5, (6, 9): 0.2}
    p_fail = np.array([1.0 - p_on.get((int(u), int(v)), 1.0) for u, v in zip(g.eu, g.ev)])
    return g, p_fail


def hop_distances(g: Graph, src: int) -> np.ndarray:
    """Hop counts from src over the base graph's edges (-1 = unreachable)."""
    adj = [[] for _ in range(g.n)]
    for u, v in zip(g.eu.tolist(), g.ev.tolist()):
        adj[u].append(v)
        adj[v].append(u)
    d = np.full(g.n, -1, dtype=np.int64)
    d[src] = 0
    frontier = [src]
    while frontier:
        nxt = []
        for u in frontier:
            for v in adj[u]:
                if d[v] < 0:
                    d[v] = d[u] + 1
                    nxt.append(v)
        frontier = nxt
    return d


def multi_reward(g: Graph, hubs: int = 3, R: float = 10.0, beta: float = 0.6) -> np.ndarray:
    """Node values of the multi-reward experiment (Section 9.1): the `hubs`
    vertices of largest base-graph degree (ties to the smaller index) carry
    reward R each, and f(v) = max over hubs h of R beta^{d(v, h)}, d the hop
    distance in the base graph; f(v) = 0 when no hub reaches v."""
    deg = np.bincount(np.concatenate([g.eu, g.ev]), minlength=g.n)
    order = sorted(range(g.n), key=lambda v: (-int(deg[v]), v))[:hubs]
    f = np.zeros(g.n)
    for h in order:
        d = hop_distances(g, h)
        f = np.maximum(f, np.where(d >= 0, R * beta ** np.maximum(d, 0), 0.0))
    return f


# ----------------------------------------------------------------------------- the five workloads
@dataclasses.dataclass
class Workload:
    graph: Graph
    seed: int = 0
    R: int = 1000
    p_fail: float = 0.1
    weight: str = "uniform"              # unit | uniform | fixed
    w_lo: int = 1
    w_hi: int = 1
    alpha: float = 0.15
    k_min: int = 5
    pool: np.ndarray | None = None
    reward: np.ndarray | None = None
    eps: float = 0.0
    r_lower: float = 0.05
    cert_topk: int = 5
    name: str = ""
    w_cdf: np.ndarray | None = None         # per-edge resampling law ("table" weights)
    hop_radius: int = 0                      # anchored r-hop neighbourhoods

    def model(self) -> dict:
        d = {"p_fail": self.p_fail, "weight": self.weight, "w_lo": self.w_lo, "w_hi": self.w_hi}
        if self.weight == "fixed":
            d["w0"] = self.graph.w0
        if self.weight == "table":
            d["w_cdf"] = self.w_cdf
        return d


def config_er20() -> Workload:
    """ER G(20, 0.2) from seed 0; failure 0.1; weights U{1..5}; 1,000 realizations."""
    g = er_graph(20, 0.2, 0)
    return Workload(g, seed=0, R=1000, p_fail=0.1, weight="uniform", w_lo=1, w_hi=5, name="er20-w5-R1000")


def config_ws1000() -> Workload:
    """WS(1000, 10, 0.1) from seed 0; failure 0.05; weights U{1..10}; 10,000 realizations."""
    g = ws_graph(1000, 10, 0.1, 0)
    return Workload(g, seed=0, R=10000, p_fail=0.05, weight="uniform", w_lo=1, w_hi=10,
                    name="ws1000-k10-w10-R10000")


def config_er5000() -> Workload:
    """ER n = 5000, mean degree 8, unit weights; failure 0.1; 4,096 realizations;
    pool of 50 random vertices with rewards U[0.5, 2]."""
    g = er_graph(5000, 8.0 / 4999.0, 0)
    W = pool(5000, 50, 0)
    return Workload(g, seed=0, R=4096, p_fail=0.1, weight="unit", pool=W, reward=rewards(5000, W, 0.5, 2.0, 0),
                    name="er5000-d8-unit-R4096-pool50")


def config_cooc77() -> Workload:
    """Co-occurrence stand-in (n = 77, m = 254, power-law degrees, geometric
    weights clipped at 31) with the per-call weight resampling and anchored
    2-hop neighbourhoods of Section 9.2 (rho_mu = 0.1, rho_sigma = 0.2; the
    topology is fixed)."""
    g = powerlaw_weighted_graph(77, 254, 2.5, 3.0, 31, 0)
    return Workload(g, seed=0, R=2000, p_fail=0.0, weight="table", w_cdf=resampled_weight_cdf(g.w0, 31, 0.1, 0.2),
                    hop_radius=2, name="cooc77-resampled-hop2-R2000")


def config_mixed_batch(count: int = 64, R: int = 2048, seed: int = 0) -> list[Workload]:
    """Uneven-size batch: a synthetic power-law co-occurrence-style graph
    (n = 77, m = 254, weights geometric with mean 3, at most 31) plus ER / WS
    graphs with n uniform in [200, 3000] and mean degree uniform in {4..12};
    failure probability U[0.02, 0.2]; radius eps in {0.01, 0.05}."""
    rng = np.random.default_rng([seed, 4])
    out = []
    g0 = powerlaw_weighted_graph(77, 254, 2.5, 3.0, 31, seed)
    out.append(Workload(g0, seed=seed, R=R, p_fail=float(rng.uniform(0.02, 0.2)), weight="fixed",
                        eps=float(rng.choice([0.01, 0.05])), name="cooc77"))
    for gi in range(1, count):
        n = int(rng.integers(200, 3001))
        deg = int(rng.integers(4, 13))
        if gi % 2 == 1:
            g = er_graph(n, deg / (n - 1), seed * 1000 + gi)
        else:
            k = max(2, deg - deg % 2)
            g = ws_graph(n, k, 0.1, seed * 1000 + gi)
        out.append(Workload(g, seed=seed * 1000 + gi, R=R, p_fail=float(rng.uniform(0.02, 0.2)), weight="uniform",
                            w_lo=1, w_hi=10, eps=float(rng.choice([0.01, 0.05])), name=f"mix{gi}-{g.name}"))
    return out


def serving_trace(count: int = 256, rate: float = 200.0, seed: int = 0, n_lo: int = 50, n_hi: int = 4000,
                  logR_lo: int = 8, logR_hi: int = 14):
    """Poisson arrivals of queries: ER or WS (50/50), n log-uniform in
    [n_lo, n_hi], mean degree U[4, 12], R = 2^U{logR_lo..logR_hi}, failure
    U[0.05, 0.2], weights U{1..10}, eps = 0.05.  Returns (arrival_s, Workload)."""
    rng = np.random.default_rng([seed, 5])
    t = 0.0
    out = []
    for q in range(count):
        t += float(rng.exponential(1.0 / rate))
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        deg = float(rng.uniform(4, 12))
        if rng.random() < 0.5:
            g = er_graph(n, min(1.0, deg / (n - 1)), seed * 100000 + q)
        else:
            k = max(2, int(round(deg)) - int(round(deg)) % 2)
            g = ws_graph(n, k, 0.1, seed * 100000 + q)
        R = 2 ** int(rng.integers(logR_lo, logR_hi + 1))
        out.append((t, Workload(g, seed=seed * 100000 + q, R=R, p_fail=float(rng.uniform(0.05, 0.2)),
                                weight="uniform", w_lo=1, w_hi=10, eps=0.05, name=f"q{q}-{g.name}")))
    return out
