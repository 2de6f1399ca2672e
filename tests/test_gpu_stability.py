"""GPU parity of the rank-stability check (amc_stability, Section 8.4): the
estimates at M and 2M realizations against the oracle's sweep and tail at M
and 2M (counts bit-exact, b within 1e-12 of its max norm, Top-k sets equal
as sets unless the oracle's b has a near-tie at the k-th place), and at full
size against direct runs of amc_run at M and at 2M."""
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


def close(x, y, tol, what):
    x, y = np.asarray(x, float), np.asarray(y, float)
    scale = max(np.abs(y).max(initial=0.0), 1e-300)
    err = np.abs(x - y).max(initial=0.0)
    assert err <= tol * scale, f"{what}: {err} > {tol} * {scale}"


def same_topk(top_gpu, b_ref, k, what):
    """The set of the k largest of b_ref (ties to the smaller index), allowing
    either side of a gap below 1e-10 at the k-th place."""
    order = np.lexsort((np.arange(len(b_ref)), -b_ref))
    ref = set(order[:k].tolist())
    if set(np.asarray(top_gpu).tolist()) == ref:
        return
    gap = b_ref[order[k - 1]] - b_ref[order[k]]
    assert gap < 1e-10 * max(b_ref.max(), 1e-300), f"{what}: Top-{k} differs with a clear gap {gap}"


@pytest.mark.parametrize("M,k,r0", [(500, 5, 0), (333, 3, 1000), (1, 2, 7)])
def test_er20_against_the_oracle(ctx, M, k, r0):
    wl = W.config_er20()
    g = wl.graph
    G = amc.Graph(ctx, g.n, g.eu, g.ev, g.w0)
    say(f"[gpu] stability er20 M={M} k={k} r0={r0}")
    st = amc.stability(ctx, G, wl.model(), k=k, seed=wl.seed, R=M, r_begin=r0, alpha=wl.alpha, k_min=wl.k_min)
    G.close()
    refM = O.sweep(g.n, g.eu, g.ev, seed=wl.seed, R=M, r_begin=r0, alpha=wl.alpha, k_min=wl.k_min, **wl.model())
    ref2 = O.sweep(g.n, g.eu, g.ev, seed=wl.seed, R=2 * M, r_begin=r0, alpha=wl.alpha, k_min=wl.k_min,
                   **wl.model())
    assert np.array_equal(st["counts_2M"], ref2["counts"])
    tM = O.tail(refM["counts"], M, cert_topk=k)
    t2 = O.tail(ref2["counts"], 2 * M, cert_topk=k)
    close(st["b_M"], tM["b"], 1e-12, "b_M")
    close(st["b_2M"], t2["b"], 1e-12, "b_2M")
    same_topk(st["top_M"], tM["b"], k, "top_M")
    same_topk(st["top_2M"], t2["b"], k, "top_2M")
    assert st["overlap"] == len(set(st["top_M"].tolist()) & set(st["top_2M"].tolist()))
    assert st["same_set"] == (st["overlap"] == k)
    assert st["max_abs_diff"] == np.abs(st["b_2M"] - st["b_M"]).max()
    assert np.all(np.diff(st["b_M"][st["top_M"]]) <= 0)      # listed in decreasing b


def test_ws1000_full_size_against_direct_runs(ctx):
    # M = 5000: the two halves of the 10,000-realization workload
    wl = W.config_ws1000()
    g = wl.graph
    G = amc.Graph(ctx, g.n, g.eu, g.ev, g.w0)
    M = wl.R // 2
    q = dict(seed=wl.seed, alpha=wl.alpha, k_min=wl.k_min)
    say("[gpu] stability ws1000 M=5000")
    st = amc.stability(ctx, G, wl.model(), k=10, R=M, **q)
    dM = amc.run(ctx, G, wl.model(), R=M, cert_topk=10, **q)
    d2 = amc.run(ctx, G, wl.model(), R=2 * M, cert_topk=10, **q)
    G.close()
    assert np.array_equal(st["counts_2M"], d2["counts"])
    assert np.array_equal(st["b_M"], dM["b"]) and np.array_equal(st["b_2M"], d2["b"])
    assert np.array_equal(st["top_M"], dM["top"]) and np.array_equal(st["top_2M"], d2["top"])
    assert np.all(st["counts_2M"].sum(1) == 2 * M)
    assert st["sweep_ms"] > 0.0
    say(f"[gpu]   same set {st['same_set']} overlap {st['overlap']} max |db| {st['max_abs_diff']:.3g}")


def test_invalid_arguments(ctx):
    wl = W.config_er20()
    g = wl.graph
    G = amc.Graph(ctx, g.n, g.eu, g.ev, g.w0)
    for k, extra in ((0, {}), (17, {}), (20, {}), (5, {"R": 0}), (5, {"R": 2 ** 31}),
                     (5, {"r_begin": 2 ** 32 - 10, "R": 6}), (5, {"topk": 2}), (5, {"pool": np.array([1, 2])}),
                     (5, {"flags": amc.FALLBACK, "fb_node": 1})):
        q = dict(seed=0, R=10, alpha=wl.alpha, k_min=wl.k_min)
        q.update(extra)
        with pytest.raises(amc.AmcError) as ei:
            amc.stability(ctx, G, wl.model(), k=k, **q)
        assert ei.value.rc == amc.E_INVALID_ARG, (k, extra)
    G.close()
