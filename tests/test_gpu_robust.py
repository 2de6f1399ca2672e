"""GPU parity of the robust tail (amc_robust) against the CPU oracle: AFC of
the nominal and sampled kernels and the first-order AFC within 1e-12 of their
max norm, divergences within 1e-10 relative, maximisers identical (the sampled
divergences are far apart), transition rewards and norms within 1e-12."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2605_14743_amd import amc
from paper_2605_14743_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def close(x, y, tol, what):
    x, y = np.asarray(x, float), np.asarray(y, float)
    scale = max(np.abs(y).max(initial=0.0), 1e-300)
    assert np.abs(x - y).max(initial=0.0) <= tol * scale, what


def compare(g, o, what):
    close(g["b0"], o["b0"], 1e-12, f"{what} b0")
    assert g["b_sw"] == pytest.approx(o["b_sw"], rel=1e-12, abs=1e-300)
    assert g["b_imp"] == pytest.approx(o["b_imp"], rel=1e-12, abs=1e-300)
    close(g["kl"], o["kl"], 1e-10, f"{what} kl")
    close(g["tv"], o["tv"], 1e-10, f"{what} tv")
    assert g["kl_arg"] == o["kl_arg"] and g["tv_arg"] == o["tv_arg"]
    for key in ("b_kl", "b_tv", "b_lin"):
        close(g[key], o[key], 1e-12, f"{what} {key}")
    for key in ("norm_N0E", "norm_N0", "rem_bound"):
        assert g[key] == pytest.approx(o[key], rel=1e-12), key
    assert abs(g["rem_actual"] - o["rem_actual"]) <= 1e-12 * o["norm_N0"]


@pytest.mark.parametrize("n", [1, 7, 64, 130])
def test_random_kernels(ctx, n):
    Q0 = random_kernel(n, n)
    f = np.linspace(0.0, 2.0, n)
    print(f"[gpu] robust n={n}", flush=True)
    g = amc.robust(ctx, Q0, f=f, samples=12, delta=0.4, r_min=0.05, seed=n)
    o = O.robust(Q0, f=f, samples=12, delta=0.4, r_min=0.05, seed=n)
    compare(g, o, f"random n={n}")
    assert g["tail_ms"] > 0.0


def test_more_samples_than_one_group(ctx):
    # 130 sampled kernels: inverted in groups of 64, 64 and 2
    Q0 = random_kernel(20, 77)
    f = np.linspace(1.0, 0.0, 20)
    print("[gpu] robust 130 samples", flush=True)
    g = amc.robust(ctx, Q0, f=f, samples=130, delta=0.3, r_min=0.05, seed=11)
    o = O.robust(Q0, f=f, samples=130, delta=0.3, r_min=0.05, seed=11)
    compare(g, o, "130 samples")


def test_estimated_kernel_of_a_run(ctx):
    wl = W.config_er20()
    g = wl.graph
    G = amc.Graph(ctx, g.n, g.eu, g.ev)
    sys.stdout.write("[gpu] robust on an estimated kernel\n")
    res = amc.run(ctx, G, wl.model(), seed=wl.seed, R=wl.R, alpha=wl.alpha, k_min=wl.k_min)
    G.close()
    f = np.arange(g.n, dtype=float) % 5
    gr = amc.robust(ctx, res["Q"], f=f, samples=20, delta=0.5, r_min=0.05, seed=3)
    o = O.robust(res["Q"], f=f, samples=20, delta=0.5, r_min=0.05, seed=3)
    compare(gr, o, "er20 estimated")
    close(gr["b0"], res["b"], 1e-12, "b0 equals the run's b")


def test_robust_arguments(ctx):
    Q0 = random_kernel(5, 1)
    bad_rows = Q0.copy()
    bad_rows[0] *= 1.0 / bad_rows[0].sum()                # row sum 1: no absorption
    for kw in ({"samples": -1}, {"samples": 5000}, {"delta": -0.1}, {"r_min": 0.0}, {"f": -np.ones(5)},
               {"s": np.full(5, 0.3)}):
        with pytest.raises(amc.AmcError) as ei:
            amc.robust(ctx, Q0, **kw)
        assert ei.value.rc == amc.E_INVALID_ARG, kw
    with pytest.raises(amc.AmcError) as ei:
        amc.robust(ctx, bad_rows)
    assert ei.value.rc == amc.E_INVALID_ARG


def test_multi_reward_value_of_section_9_1(ctx):
    # the multi-reward experiment: f(v) = max over the three largest-degree
    # hubs of 10 * 0.6^hops (0 when unreachable) on a WS(200) estimate; the
    # node-reward AFC b . f of the run, and the switching and improvement
    # transition reward-AFCs of the robust tail, against the oracle
    g = W.ws_graph(200, 6, 0.1, 4)
    f = W.multi_reward(g)
    assert f.max() == 10.0 and np.count_nonzero(f == 10.0) == 3
    model = {"p_fail": 0.15, "weight": "unit"}
    G = amc.Graph(ctx, g.n, g.eu, g.ev)
    print("[gpu] multi-reward ws200", flush=True)
    res = amc.run(ctx, G, model, seed=5, R=400, reward=f)
    G.close()
    ref = O.sweep(g.n, g.eu, g.ev, seed=5, R=400, **model)
    assert np.array_equal(res["counts"], ref["counts"])
    t = O.tail(ref["counts"], 400, f=f)
    close(res["b"], t["b"], 1e-12, "b")
    assert res["b_f"] == pytest.approx(t["b_f"], rel=1e-12)
    assert res["b_f"] == pytest.approx(float(t["b"] @ f), rel=1e-12)
    gr = amc.robust(ctx, res["Q"], f=f, samples=8, delta=0.3, r_min=0.05, seed=9)
    o = O.robust(t["Q"], f=f, samples=8, delta=0.3, r_min=0.05, seed=9)
    compare(gr, o, "multi-reward")
    assert gr["b_imp"] > 0.0 and gr["b_sw"] > 0.0
