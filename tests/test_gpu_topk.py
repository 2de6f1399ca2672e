"""GPU parity of the finite-k local Top-k rows (Sections 3.3, 6.2-6.3, 7.1,
7.3-7.4) against the CPU oracle, through the C-ABI.

Bit-exact: counts, the finite-k pool-selector counts and next table.  Floating
point: the step-reward averages psi and psi_W (sums of gamma over the draws,
positive terms, so both sides agree to (k + R) u relative), the reward-AFCs
and the fallback-kernel AFC, pool mass and censored profile within 1e-12.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2605_14743_amd import amc
from paper_2605_14743_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = amc.Context(0)
    yield c
    c.close()


def close(x, y, tol=TOL, what=""):
    x = np.asarray(x, float)
    y = np.asarray(y, float)
    scale = max(np.abs(y).max(initial=0.0), 1e-300)
    err = np.abs(x - y).max(initial=0.0)
    assert err <= tol * scale, f"{what}: max err {err:.3e} vs scale {scale:.3e}"


def run_both(ctx, g, model, R, *, topk, pool, gamma=None, fb=None, fb_set=None, seed=0, r_begin=0, alpha=0.15,
             k_min=5, tail=True, **gq):
    G = amc.Graph(ctx, g.n, g.eu, g.ev, g.w0)
    flags = amc.WANT_NEXT_TABLE | (0 if tail else amc.SKIP_TAIL)
    say(f"[gpu] topk n={g.n} R={R} k={topk} pool={len(pool)} fb={fb} {gq}")
    try:
        res = amc.run(ctx, G, model, seed=seed, R=R, r_begin=r_begin, alpha=alpha, k_min=k_min, topk=topk,
                      pool=pool, gamma=gamma, fb_node=fb, fb_set=fb_set, flags=flags, **gq)
    finally:
        G.close()
    om = dict(model)
    if om.get("weight") == "fixed":
        om["w0"] = g.w0
    ref = O.sweep(g.n, g.eu, g.ev, seed=seed, R=R, r_begin=r_begin, alpha=alpha, k_min=k_min, pool=pool,
                  topk=topk, gamma=gamma, want_next=True, **om)
    return res, ref


def check(res, ref, R, what):
    assert np.array_equal(res["counts"], ref["counts"]), f"{what}: counts"
    assert np.array_equal(res["counts_w"], ref["counts_w"]), f"{what}: finite-k pool counts"
    assert np.array_equal(res["next_table_w"], ref["next_table_w"]), f"{what}: pool table"
    close(res["psi"], ref["psi"] / R, what=f"{what} psi")
    close(res["psi_w"], ref["psi_w"] / R, what=f"{what} psi_w")


@pytest.mark.parametrize("mode,extra", [(amc.MODE_WAVE, {}), (amc.MODE_WAVE_L2, {}), (amc.MODE_BLOCK, {}),
                                        (amc.MODE_WAVE, {"tile": 3}), (amc.MODE_WAVE_L2, {"tile": 5}),
                                        (amc.MODE_BLOCK, {"tile": 7})])
def test_er20_topk_rewards_selector_and_fallback(ctx, mode, extra):
    wl = W.config_er20()
    g = wl.graph
    pool = np.array([2, 5, 8, 13, 17])
    gamma = 0.5 + 1.5 * np.random.default_rng(4).random(g.n)
    fb_set = np.array([0, 19])
    for k in (1, 3, 20):
        res, ref = run_both(ctx, g, wl.model(), wl.R, topk=k, pool=pool, gamma=gamma, fb=19, fb_set=fb_set,
                            mode=mode, **extra)
        check(res, ref, wl.R, f"er20 k={k} mode={mode} {extra}")
        t = O.tail(ref["counts"], wl.R, pool=pool, counts_w=ref["counts_w"], psi=ref["psi"], psi_w=ref["psi_w"],
                   fb_node=19, fb_set=fb_set)
        assert res["b_k"] == pytest.approx(t["b_k"], rel=TOL)
        assert res["b_kw"] == pytest.approx(t["b_kw"], rel=TOL)
        close(res["b_w"], t["b_w"], what="b_w")
        close(res["b_fb"], t["b_fb"], what="b_fb")
        close(res["b_cens"], t["b_cens"], what="b_cens")
        assert res["E_T_fb"] == pytest.approx(t["ET_fb"], rel=TOL)
        assert res["m_w_fb"] == pytest.approx(t["m_w_fb"], rel=TOL)
        assert res["c_fb"] == pytest.approx(t["c_fb"], rel=TOL)
        assert res["stats"]["topk_ms"] > 0.0


@pytest.mark.parametrize("mode,graph", [(amc.MODE_WAVE_L2, "ws200"), (amc.MODE_WAVE, "ws200"),
                                        (amc.MODE_BLOCK, "er20"), (amc.MODE_WAVE_L2, "er20")])
def test_last_realizations_split_into_kept_rows(ctx, mode, graph):
    # whole realizations (tile = n) with R = workgroups + 37 and a finite k:
    # the last 37 realizations run split into tiles that assemble their
    # B(H_r) rows and labels in place in the rows the Top-k stage reads
    g = W.config_er20().graph if graph == "er20" else W.ws_graph(200, 6, 0.1, 1)
    model = {"p_fail": 0.1, "weight": "uniform", "w_lo": 1, "w_hi": 6}
    pool = np.arange(3, g.n, 7)
    gamma = 0.5 + 1.5 * np.random.default_rng(5).random(g.n)
    G = amc.Graph(ctx, g.n, g.eu, g.ev)
    probe = amc.run(ctx, G, model, seed=3, R=32768, mode=mode, tile=g.n, topk=3, pool=pool, gamma=gamma,
                    flags=amc.SKIP_TAIL)                                 # the same plan as the run below
    G.close()
    blocks = probe["stats"]["blocks"]
    if blocks >= 32768:
        pytest.skip("more workgroup slots than the probe's realizations")
    R = blocks + 37
    res, ref = run_both(ctx, g, model, R, topk=3, pool=pool, gamma=gamma, seed=3, mode=mode, tile=g.n)
    st = res["stats"]
    assert st["tail_split"] == 37 and st["tail_tiles"] >= 2, st
    check(res, ref, R, f"{graph} mode {mode} kept rows")
    assert np.array_equal(res["counts"], ref["counts"])


def test_unit_values_and_no_pool(ctx):
    wl = W.config_er20()
    g = wl.graph
    G = amc.Graph(ctx, g.n, g.eu, g.ev)
    say("[gpu] topk without pool")
    res = amc.run(ctx, G, wl.model(), seed=2, R=300, topk=2, flags=amc.SKIP_TAIL)
    G.close()
    ref = O.sweep(g.n, g.eu, g.ev, seed=2, R=300, topk=2, **wl.model())
    assert np.array_equal(res["psi"], ref["psi"] / 300)          # integer-valued sums: exact


def test_ws1000_sampled_topk(ctx):
    wl = W.config_ws1000()
    g = wl.graph
    pool = W.pool(g.n, 50, 1)
    gamma = W.rewards(g.n, pool, 0.5, 2.0, 1)
    res, ref = run_both(ctx, g, wl.model(), 2, topk=5, pool=pool, gamma=gamma, seed=wl.seed, r_begin=4321,
                        alpha=wl.alpha, k_min=wl.k_min, tail=False)
    check(res, ref, 2, "ws1000")


def test_er5000_sampled_topk(ctx):
    wl = W.config_er5000()
    g = wl.graph
    res, ref = run_both(ctx, g, wl.model(), 1, topk=5, pool=wl.pool, gamma=wl.reward, seed=wl.seed, r_begin=99,
                        alpha=wl.alpha, k_min=wl.k_min, tail=False)
    check(res, ref, 1, "er5000")


@pytest.mark.parametrize("S,k", [(3, 3), (8, 20)])
def test_clique_pool_with_fallback_inside_the_pool(ctx, S, k):
    # structure-constrained selection (Section 9): W = the S best 3-cliques by
    # degree sum, v_fb = the smallest vertex of the first one (inside W)
    g = W.ws_graph(60, 6, 0.1, 3)
    pool, fb, chosen = W.clique_pool(g, S)
    assert len(chosen) == S and fb in pool
    model = {"p_fail": 0.1, "weight": "uniform", "w_lo": 1, "w_hi": 5}
    res, ref = run_both(ctx, g, model, 400, topk=k, pool=pool, fb=fb, seed=5)
    check(res, ref, 400, f"cliques S={S} k={k}")
    t = O.tail(ref["counts"], 400, pool=pool, counts_w=ref["counts_w"], psi=ref["psi"], psi_w=ref["psi_w"],
               fb_node=fb, fb_set=np.array([fb]))
    close(res["b_w"], t["b_w"], what="b_w")
    close(res["b_fb"], t["b_fb"], what="b_fb")
    close(res["b_cens"], t["b_cens"], what="b_cens")
    assert res["m_w_fb"] == pytest.approx(t["m_w_fb"], rel=TOL)
    assert res["c_fb"] == pytest.approx(t["c_fb"], rel=TOL)
    # every step lands in W or absorbs: the pool mass is everything off the initial spread
    assert np.all(res["counts_w"][:, np.setdiff1d(np.arange(g.n), pool)] == 0)


def test_topk_invalid_arguments(ctx):
    g = W.er_graph(12, 0.4, 1)
    G = amc.Graph(ctx, g.n, g.eu, g.ev)
    pool = np.array([1, 2, 3])
    for bad in ({"topk": amc.MAX_TOPK + 1}, {"topk": -1}, {"topk": 2, "gamma": -np.ones(12)},
                {"fb_node": 4},                                    # fallback without a pool
                {"pool": pool, "fb_node": 4, "fb_set": [5, 6]},    # v_fb outside V_fb
                {"pool": pool, "fb_node": 4, "fb_set": [4, 1]},    # V_fb meets W
                {"pool": pool, "fb_node": 12}):
        with pytest.raises(amc.AmcError) as ei:
            amc.run(ctx, G, {"p_fail": 0.1}, R=4, **bad)
        assert ei.value.rc == amc.E_INVALID_ARG, bad
    G.close()


def test_topk_beyond_the_lds(ctx):
    # n = 9000: the Top-k stage's arrays (21 n bytes) exceed the LDS and live
    # in global memory per workgroup (the sweep itself runs with its state in
    # the scratch, distances and row offsets in LDS); one realization against
    # the oracle
    g = W.er_graph(9000, 8.0 / 8999, 91)
    pool = np.arange(5, g.n, 97)
    gamma = 0.5 + 1.5 * np.random.default_rng(6).random(g.n)
    res, ref = run_both(ctx, g, {"p_fail": 0.1, "weight": "unit"}, 1, topk=4, pool=pool, gamma=gamma, seed=2,
                        tail=False)
    assert res["stats"]["state_global"] == 1, res["stats"]
    check(res, ref, 1, "n=9000 global Top-k arrays")
    assert np.array_equal(res["counts"], ref["counts"])
