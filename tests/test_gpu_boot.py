"""GPU parity of the bootstrap of b (amc_bootstrap, Section 8.4) against the
CPU oracle.

Tolerances: b of the draws and every replicate's b within 1e-12 of the max
norm (FP64 Gauss-Jordan against LU with pivoting, both on diagonally dominant
I - Q); mean within 1e-12 of the max norm, standard deviation within 1e-9
relative plus 1e-15 of the max norm (cancellation in the centred sum), the
order statistics within 1e-12 of the max norm (an order statistic moves at
most as far as the largest input does).  The redrawn counts are integers, so
any difference in the resampling shows up far beyond these bounds."""
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


def draws_from_kernel(P, R, seed):
    """next(t, i) drawn from row i of P (columns 0..n-1 transient, n = bottom)."""
    rng = np.random.default_rng(seed)
    n = P.shape[0]
    cum = np.cumsum(P, axis=1)
    cum[:, -1] = 1.0
    u = rng.random((R, n))
    nxt = np.array([np.searchsorted(cum[i], u[:, i], side="right") for i in range(n)]).T
    return np.where(nxt >= n, -1, nxt).astype(np.int32)


def random_kernel(n, seed, leak=0.2, density=0.6):
    rng = np.random.default_rng(seed)
    Q = rng.random((n, n)) * (rng.random((n, n)) < density)
    Q[np.arange(n), rng.integers(0, n, n)] += 0.1
    Q = Q / Q.sum(1, keepdims=True) * (1 - leak)
    return np.hstack([Q, np.full((n, 1), leak)])


def close(x, y, tol, what, scale=None):
    x, y = np.asarray(x, float), np.asarray(y, float)
    scale = max(np.abs(y).max(initial=0.0), 1e-300) if scale is None else scale
    err = np.abs(x - y).max(initial=0.0)
    assert err <= tol * scale, f"{what}: {err} > {tol} * {scale}"


def compare(g, o, what):
    sc = max(np.abs(o["b_rep"]).max(), 1e-300)
    close(g["b0"], o["b0"], 1e-12, f"{what} b0")
    close(g["b_rep"], o["b_rep"], 1e-12, f"{what} b_rep", sc)
    close(g["mean"], o["mean"], 1e-12, f"{what} mean", sc)
    assert np.all(np.abs(g["sd"] - o["sd"]) <= 1e-9 * o["sd"] + 1e-15 * sc), f"{what} sd"
    close(g["lo"], o["lo"], 1e-12, f"{what} lo", sc)
    close(g["hi"], o["hi"], 1e-12, f"{what} hi", sc)


@pytest.mark.parametrize("n,R,B,level", [(1, 5, 3, 0.9), (12, 300, 40, 0.9), (70, 301, 70, 0.95),
                                         (33, 64, 1, 0.5), (130, 1001, 129, 0.8), (20, 40001, 6, 0.9)])
def test_random_tables(ctx, n, R, B, level):
    # several 32 x 32 transpose tiles with ragged edges, R not a multiple of 4,
    # B past one group of 128 matrices, B = 1; R = 40001: a row's outcomes
    # (2 R bytes) no longer fit the LDS next to the counts, so the redraw
    # gathers from the cache
    nt = draws_from_kernel(random_kernel(n, n), R, R)
    say(f"[gpu] bootstrap n={n} R={R} B={B} level={level}")
    g = amc.bootstrap(ctx, nt, replicates=B, level=level, seed=n + R)
    o = O.bootstrap(nt, replicates=B, level=level, seed=n + R)
    compare(g, o, f"n={n} R={R} B={B}")
    assert g["ms"] > 0.0
    if B == 1:
        assert np.all(g["sd"] == 0.0) and np.array_equal(g["lo"], g["b_rep"][0])


def test_floor_and_initial_distribution(ctx):
    # rows 0..3 never absorb: the floor eta (default 0.1 / sqrt(R), or given)
    n, R = 9, 200
    P = random_kernel(n, 4)
    P[:4, :n] /= P[:4, :n].sum(1, keepdims=True)
    P[:4, n] = 0.0
    nt = draws_from_kernel(P, R, 5)
    s = np.linspace(1.0, 2.0, n)
    s /= s.sum()
    for eta in (-1.0, 0.05):
        say(f"[gpu] bootstrap floor eta={eta}")
        g = amc.bootstrap(ctx, nt, replicates=20, floor_eta=eta, s=s, seed=3)
        o = O.bootstrap(nt, replicates=20, eta=None if eta < 0 else eta, s=s, seed=3)
        compare(g, o, f"floor eta={eta}")


def test_degenerate_rows(ctx):
    n, R = 6, 50
    nt = np.tile(np.array([1, 2, 3, -1, 0, -1], dtype=np.int32), (R, 1))
    say("[gpu] bootstrap degenerate rows")
    g = amc.bootstrap(ctx, nt, replicates=8, seed=1)
    o = O.bootstrap(nt, replicates=8, seed=1)
    compare(g, o, "degenerate")
    assert np.all(g["sd"] <= 1e-15) and np.array_equal(g["lo"], g["b0"]) and np.array_equal(g["hi"], g["b0"])


def test_closed_class_without_floor_is_singular(ctx):
    # states 0 and 1 send every draw to each other: with the floor disabled
    # I - Q* is singular in every replicate
    nt = np.tile(np.array([1, 0, -1], dtype=np.int32), (16, 1))
    say("[gpu] bootstrap singular without the floor")
    with pytest.raises(amc.AmcError) as ei:
        amc.bootstrap(ctx, nt, replicates=4, floor_eta=0.0)
    assert ei.value.rc == amc.E_SINGULAR
    g = amc.bootstrap(ctx, nt, replicates=4)
    o = O.bootstrap(nt, replicates=4)
    compare(g, o, "closed class with the floor")


def test_sweep_next_table(ctx):
    # the table amc_run writes for the ER(20) workload, 1,000 realizations
    wl = W.config_er20()
    g = wl.graph
    G = amc.Graph(ctx, g.n, g.eu, g.ev, g.w0)
    say("[gpu] bootstrap of an er20 sweep")
    res = amc.run(ctx, G, wl.model(), seed=wl.seed, R=wl.R, alpha=wl.alpha, k_min=wl.k_min,
                  flags=amc.WANT_NEXT_TABLE)
    G.close()
    nt = res["next_table"]
    gb = amc.bootstrap(ctx, nt, replicates=100, seed=11)
    ob = O.bootstrap(nt, replicates=100, seed=11)
    compare(gb, ob, "er20 sweep")
    close(gb["b0"], res["b"], 1e-12, "b0 against the run's own b")


def test_ws1000_full_size_sampled(ctx):
    # 10,000 realizations of WS(1000): b0 and two replicates against the oracle
    # one at a time, the summaries against numpy on the device's replicates
    wl = W.config_ws1000()
    g = wl.graph
    G = amc.Graph(ctx, g.n, g.eu, g.ev, g.w0)
    say("[gpu] bootstrap of the ws1000 sweep, R=10000, B=100")
    res = amc.run(ctx, G, wl.model(), seed=wl.seed, R=wl.R, alpha=wl.alpha, k_min=wl.k_min,
                  flags=amc.WANT_NEXT_TABLE)
    G.close()
    nt = res["next_table"]
    B, level = 100, 0.95
    gb = amc.bootstrap(ctx, nt, replicates=B, level=level, seed=7)
    close(gb["b0"], res["b"], 1e-12, "b0 against the run's own b")
    eta = 0.1 / np.sqrt(wl.R)
    s = np.full(g.n, 1.0 / g.n)
    for beta in (0, 77):
        say(f"[gpu]   oracle replicate {beta}")
        Q, _ = O.counts_to_kernel(O.boot_counts(nt, 7, beta), wl.R, eta)
        close(gb["b_rep"][beta], O.chain(Q, s)["b"], 1e-12, f"replicate {beta}")
    reps = gb["b_rep"]
    sc = np.abs(reps).max()
    close(gb["mean"], reps.mean(0), 1e-13, "mean", sc)
    assert np.all(np.abs(gb["sd"] - reps.std(0, ddof=1)) <= 1e-9 * reps.std(0, ddof=1) + 1e-15 * sc)
    assert np.array_equal(gb["lo"], np.percentile(reps, 2.5, axis=0, method="inverted_cdf"))
    assert np.array_equal(gb["hi"], np.percentile(reps, 97.5, axis=0, method="inverted_cdf"))


def test_n500_batched_large_tiles(ctx):
    # n = 500, 64 replicates: the batched inversion takes its 128-wide tiles
    # (ragged last tile of 116) -- b0 and two replicates against the oracle
    n, R, B = 500, 200, 64
    nt = draws_from_kernel(random_kernel(n, 21, density=0.05), R, 22)
    say(f"[gpu] bootstrap n={n} R={R} B={B}")
    g = amc.bootstrap(ctx, nt, replicates=B, seed=4)
    eta = 0.1 / np.sqrt(R)
    s = np.full(n, 1.0 / n)
    C0 = np.zeros((n, n + 1), np.uint32)
    for i in range(n):
        col = nt[:, i]
        C0[i, :n] = np.bincount(col[col >= 0], minlength=n)
        C0[i, n] = np.count_nonzero(col < 0)
    Q, _ = O.counts_to_kernel(C0, R, eta)
    close(g["b0"], O.chain(Q, s)["b"], 1e-12, "b0")
    for beta in (0, B - 1):
        Q, _ = O.counts_to_kernel(O.boot_counts(nt, 4, beta), R, eta)
        close(g["b_rep"][beta], O.chain(Q, s)["b"], 1e-12, f"replicate {beta}")


def test_invalid_arguments(ctx):
    nt = np.zeros((4, 3), dtype=np.int32)
    for kw in ({"replicates": 0}, {"replicates": amc.MAX_BOOT_REPLICATES + 1}, {"level": 1.0}, {"level": 0.0},
               {"floor_eta": 1.0}, {"s": np.array([0.5, 0.5, 0.5])}):
        with pytest.raises(amc.AmcError) as ei:
            amc.bootstrap(ctx, nt, **kw)
        assert ei.value.rc == amc.E_INVALID_ARG, kw
    for bad in (3, -2):
        t = nt.copy()
        t[2, 1] = bad
        with pytest.raises(amc.AmcError) as ei:
            amc.bootstrap(ctx, t)
        assert ei.value.rc == amc.E_INVALID_ARG, bad
    with pytest.raises(amc.AmcError) as ei:
        amc.bootstrap(ctx, np.zeros((2, amc.MAX_BOOT_N + 1), dtype=np.int32), replicates=1)
    assert ei.value.rc == amc.E_UNSUPPORTED
