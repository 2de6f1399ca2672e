"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

Bit-exact: distances, path counts, global centres, next-state tables, counts
and the work counters.  Floating point: B (summed over realizations) within
1e-12 relative; N, mu, b, rewards and certificate thresholds within 1e-12 of
the vector (row) max norm.  Both sides take the argmax decision in FP64 with
the same tie band.
"""
import sys

import numpy as np
import pytest

import oracle as O
import par_oracle as P
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


def gpu_run(ctx, g, model, **q):
    G = amc.Graph(ctx, g.n, g.eu, g.ev, g.w0)
    say(f"[gpu] run n={g.n} m={g.m} model={ {k: v for k, v in model.items() if k not in ('p_fail_edge', 'w_cdf')} } "
        f"q={ {k: v for k, v in q.items() if k not in ('pool', 'reward', 's', 'debug_pairs')} }")
    try:
        return amc.run(ctx, G, model, **q)
    finally:
        G.close()


def oracle_model(model, g):
    d = dict(model)
    if d.get("weight") == "fixed":
        d["w0"] = g.w0
    return d


def assert_close_norm(x, y, tol=TOL, what=""):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    scale = max(np.abs(y).max(initial=0.0), 1e-300)
    err = np.abs(x - y).max(initial=0.0)
    assert err <= tol * scale, f"{what}: max err {err:.3e} vs scale {scale:.3e}"


def assert_rel(x, y, tol=TOL, what=""):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    err = np.abs(x - y)
    assert np.all(err <= tol * np.maximum(np.abs(y), 1e-300) + 1e-300), \
        f"{what}: worst rel err {np.max(err / np.maximum(np.abs(y), 1e-300)):.3e}"


def check_sweep(res, ref, n, what=""):
    assert np.array_equal(res["counts"], ref["counts"]), f"{what}: counts differ"
    if "center_global" in res:
        assert np.array_equal(res["center_global"], ref["center_global"]), f"{what}: centres differ"
    if "next_table" in res:
        assert np.array_equal(res["next_table"], ref["next_table"]), f"{what}: next table differs"
    if "counts_w" in ref:
        assert np.array_equal(res["counts_w"], ref["counts_w"]), f"{what}: pool counts differ"
    if "next_table_w" in res and "next_table_w" in ref:
        assert np.array_equal(res["next_table_w"], ref["next_table_w"])
    if "bsum" in res:
        assert_rel(res["bsum"], ref["bsum"], what=f"{what} bsum")
    st, rst = res["stats"], ref["stats"]
    for k in ("units", "sum_nK", "sum_AK", "sum_DK"):
        assert st[k] == rst[k], f"{what}: stat {k} {st[k]} != {rst[k]}"


FLAGS = amc.WANT_NEXT_TABLE | amc.WANT_CENTER | amc.WANT_BSUM | amc.WANT_N


# --------------------------------------------------------------------------- config 1: full size, all modes
@pytest.mark.parametrize("mode,extra", [(amc.MODE_WAVE, {}), (amc.MODE_BLOCK, {}),
                                        (amc.MODE_WAVE, {"tile": 3}), (amc.MODE_WAVE, {"flags": amc.PLAIN_LAUNCH}),
                                        (amc.MODE_BLOCK, {"tile": 7}), (amc.MODE_WAVE, {"group": 4}),
                                        (amc.MODE_WAVE, {"group": 8}), (amc.MODE_WAVE, {"group": 16}),
                                        (amc.MODE_WAVE, {"group": 3}), (amc.MODE_WAVE_L2, {}),
                                        (amc.MODE_WAVE_L2, {"tile": 3}), (amc.MODE_WAVE_L2, {"group": 8}),
                                        (amc.MODE_WAVE_L2, {"flags": amc.PLAIN_LAUNCH}),
                                        (amc.MODE_WAVE, {"flags": amc.DIST16}),
                                        (amc.MODE_WAVE, {"group": 8, "flags": amc.DIST16}),
                                        (amc.MODE_WAVE, {"group": 3, "flags": amc.DIST16}),
                                        (amc.MODE_WAVE_L2, {"flags": amc.DIST16}),
                                        (amc.MODE_WAVE_L2, {"tile": 3, "flags": amc.DIST16}),
                                        (amc.MODE_WAVE_L2, {"flags": amc.SIGMA_GLOBAL}),
                                        (amc.MODE_WAVE_L2, {"group": 2, "flags": amc.SIGMA_GLOBAL}),
                                        (amc.MODE_WAVE_L2, {"group": 3, "flags": amc.SIGMA_GLOBAL}),
                                        (amc.MODE_WAVE_L2, {"tile": 3, "flags": amc.SIGMA_GLOBAL | amc.DIST16}),
                                        (amc.MODE_WAVE_L2, {"flags": amc.SIGMA_GLOBAL | amc.PLAIN_LAUNCH})])
def test_er20_full_against_oracle(ctx, mode, extra):
    wl = W.config_er20()
    g = wl.graph
    model = wl.model()
    flags = FLAGS | extra.pop("flags", 0)
    res = gpu_run(ctx, g, model, seed=wl.seed, R=wl.R, alpha=wl.alpha, k_min=wl.k_min, flags=flags, mode=mode,
                  cert_topk=5, eps=1e-3, r_lower=0.05, **extra)
    ref = O.sweep(g.n, g.eu, g.ev, seed=wl.seed, R=wl.R, alpha=wl.alpha, k_min=wl.k_min, want_next=True,
                  **oracle_model(model, g))
    check_sweep(res, ref, g.n, "er20")
    t = O.tail(ref["counts"], wl.R, eps=1e-3, r_lower=0.05, cert_topk=5)
    assert_close_norm(res["Q"], t["Q"], 0.0, "Q")          # same operations: exact
    assert_close_norm(res["N"], t["N"], what="N")
    assert_close_norm(res["mu"], t["mu"], what="mu")
    assert_close_norm(res["b"], t["b"], what="b")
    assert abs(res["E_T"] - t["ET"]) <= TOL * t["ET"]
    assert np.array_equal(res["top"], t["top"]) and np.array_equal(res["cert_v"], t["cert_v"])
    assert_close_norm(res["cert_gap"], t["cert_gap"], what="gap")
    assert_close_norm(res["cert_sharp"], t["cert_sharp"], what="sharp")
    assert_close_norm(res["cert_sharp_supp"], t["cert_sharp_supp"], what="sharp_supp")
    assert res["cert_crude"] == pytest.approx(t["cert_crude"], rel=1e-15)
    assert res["epsbar_supp"] == pytest.approx(t["epsbar_supp"], rel=1e-15)
    assert res["admissible"] == t["admissible"]
    st = res["stats"]
    assert st["mode"] == mode
    if flags & amc.SIGMA_GLOBAL:
        assert st["sig_global"] == 1
    if mode != amc.MODE_BLOCK:          # 16 waves fit either way: 32-bit entries unless asked otherwise
        assert st["dist_bytes"] == (2 if flags & amc.DIST16 else 4)


def test_debug_dump_distances_sigma_delta(ctx):
    wl = W.config_er20()
    g = wl.graph
    pairs = [(0, 0), (3, 7), (999, 19), (500, 11)]
    for mode, fl in ((amc.MODE_WAVE, 0), (amc.MODE_BLOCK, 0), (amc.MODE_WAVE_L2, 0), (amc.MODE_WAVE, amc.DIST16),
                     (amc.MODE_WAVE_L2, amc.DIST16), (amc.MODE_WAVE_L2, amc.SIGMA_GLOBAL),
                     (amc.MODE_WAVE_L2, amc.SIGMA_GLOBAL | amc.DIST16)):
        res = gpu_run(ctx, g, wl.model(), seed=wl.seed, R=wl.R, alpha=wl.alpha, k_min=wl.k_min, mode=mode,
                      flags=amc.SKIP_TAIL | fl, debug_pairs=pairs)
        for k, (r, s) in enumerate(pairs):
            alive, w = O.realize(g.n, g.eu, g.ev, wl.seed, r, **wl.model())
            d, sg, dl = O.sssp(g.n, g.eu, g.ev, alive, w, False, s)
            dd = np.where(d == np.iinfo(np.uint64).max, 0xFFFFFFFF, d).astype(np.uint32)
            assert np.array_equal(res["dbg_dist"][k], dd), (mode, r, s)
            assert np.array_equal(res["dbg_sigma"][k], sg), (mode, r, s)
            assert_rel(res["dbg_delta"][k], dl, what=f"delta {mode} {(r, s)}")


# --------------------------------------------------------------------------- edge cases
def _case(ctx, g, model, R, **q):
    flags = q.pop("flags", FLAGS)
    res = gpu_run(ctx, g, model, R=R, flags=flags, **q)
    ref = O.sweep(g.n, g.eu, g.ev, R=R, want_next=True, pool=q.get("pool"), seed=q.get("seed", 0),
                  r_begin=q.get("r_begin", 0), alpha=q.get("alpha", 0.15), k_min=q.get("k_min", 5),
                  **oracle_model(model, g))
    check_sweep(res, ref, g.n, str(q))
    return res, ref


@pytest.mark.parametrize("mode", [amc.MODE_WAVE, amc.MODE_BLOCK, amc.MODE_WAVE_L2, "wave-g8"])
def test_edge_cases(ctx, mode):
    if mode == "wave-g8":
        global _case
        base_case = _case

        def _case(ctx_, g_, model_, R_, **q_):
            return base_case(ctx_, g_, model_, R_, group=8, **q_)
        try:
            return test_edge_cases(ctx, amc.MODE_WAVE)
        finally:
            _case = base_case
    one = W.canonical(1, [])
    _case(ctx, one, {"p_fail": 0.1}, 5, mode=mode, k_min=1)
    empty = W.canonical(7, [])
    _case(ctx, empty, {"p_fail": 0.5}, 9, mode=mode, k_min=1)
    g = W.er_graph(40, 0.1, 3)
    _case(ctx, g, {"p_fail": 1.0, "weight": "uniform", "w_lo": 1, "w_hi": 3}, 7, mode=mode)          # all fail
    _case(ctx, g, {"p_fail": 0.0, "weight": "unit"}, 3, mode=mode, k_min=41)                      # k_min > n
    _case(ctx, g, {"p_fail": 0.2, "weight": "uniform", "w_lo": 2, "w_hi": 2}, 11, mode=mode, alpha=1.0)
    _case(ctx, g, {"p_fail": 0.2, "weight": "uniform", "w_lo": 1, "w_hi": 65535}, 5, mode=mode, seed=2 ** 40 + 7,
          r_begin=4000000000)
    path = W.canonical(60, [(i, i + 1) for i in range(59)])                                       # deep, one vertex per level
    _case(ctx, path, {"p_fail": 0.02, "weight": "uniform", "w_lo": 1, "w_hi": 4}, 6, mode=mode, k_min=2)
    cr, pf = W.crossroads()
    _case(ctx, cr, {"p_fail": 0.0, "p_fail_edge": pf}, 300, mode=mode, alpha=0.1, k_min=3)
    pw = W.powerlaw_weighted_graph(77, 254, 2.5, 3.0, 31, 0)
    _case(ctx, pw, {"p_fail": 0.1, "weight": "fixed"}, 40, mode=mode, pool=np.array([0, 5, 9, 33, 70]))


@pytest.mark.parametrize("mode,extra", [(amc.MODE_WAVE, 0), (amc.MODE_WAVE_L2, 0),
                                        (amc.MODE_WAVE_L2, amc.SIGMA_GLOBAL)])
def test_edge_cases_16bit_distances(ctx, mode, extra):
    kw = dict(mode=mode, flags=FLAGS | amc.DIST16 | extra)
    _case(ctx, W.canonical(1, []), {"p_fail": 0.1}, 5, k_min=1, **kw)
    _case(ctx, W.canonical(7, []), {"p_fail": 0.5}, 9, k_min=1, **kw)
    g = W.er_graph(40, 0.1, 3)
    _case(ctx, g, {"p_fail": 1.0, "weight": "uniform", "w_lo": 1, "w_hi": 3}, 7, **kw)
    _case(ctx, g, {"p_fail": 0.2, "weight": "uniform", "w_lo": 1, "w_hi": 1600}, 5, **kw)      # 40 * 1600 < 0xFFFF
    path = W.canonical(60, [(i, i + 1) for i in range(59)])          # one vertex per segment
    _case(ctx, path, {"p_fail": 0.02, "weight": "uniform", "w_lo": 1, "w_hi": 4}, 6, k_min=2, **kw)
    _case(ctx, path, {"p_fail": 0.0, "weight": "unit"}, 3, k_min=2, **kw)
    cr, pf = W.crossroads()
    _case(ctx, cr, {"p_fail": 0.0, "p_fail_edge": pf}, 300, alpha=0.1, k_min=3, **kw)
    pw = W.powerlaw_weighted_graph(77, 254, 2.5, 3.0, 31, 0)
    _case(ctx, pw, {"p_fail": 0.1, "weight": "fixed"}, 40, pool=np.array([0, 5, 9, 33, 70]), **kw)
    with pytest.raises(amc.AmcError) as ei:                          # 40 * 2000 >= 0xFFFF
        _case(ctx, g, {"p_fail": 0.2, "weight": "uniform", "w_lo": 1, "w_hi": 2000}, 5, **kw)
    assert ei.value.rc == amc.E_UNSUPPORTED


def test_sigma_overflow_reported(ctx):
    a = 35
    idx = lambda i, j: i * a + j
    pairs = [(idx(i, j), idx(i, j + 1)) for i in range(a) for j in range(a - 1)]
    pairs += [(idx(i, j), idx(i + 1, j)) for i in range(a - 1) for j in range(a)]
    g = W.canonical(a * a, pairs)
    G = amc.Graph(ctx, g.n, g.eu, g.ev)
    say("[gpu] sigma overflow grid 35x35")
    with pytest.raises(amc.AmcError) as ei:
        amc.run(ctx, G, {"p_fail": 0.0}, R=1, flags=amc.SKIP_TAIL)
    assert ei.value.rc == amc.E_SIGMA_OVERFLOW
    G.close()
    a = 34
    pairs = [(i * a + j, i * a + j + 1) for i in range(a) for j in range(a - 1)]
    pairs += [(i * a + j, (i + 1) * a + j) for i in range(a - 1) for j in range(a)]
    g = W.canonical(a * a, pairs)
    G = amc.Graph(ctx, g.n, g.eu, g.ev)
    say("[gpu] sigma no overflow grid 34x34")
    res = amc.run(ctx, G, {"p_fail": 0.0}, R=1, flags=amc.SKIP_TAIL, debug_pairs=[(0, 0)])
    assert int(res["dbg_sigma"][0][-1]) == 7219428434016265740    # C(66, 33)
    G.close()


def test_invalid_arguments(ctx):
    g = W.er_graph(10, 0.4, 1)
    with pytest.raises(amc.AmcError) as ei:
        amc.Graph(ctx, g.n, g.ev, g.eu)                      # not canonical
    assert ei.value.rc == amc.E_INVALID_ARG
    G = amc.Graph(ctx, g.n, g.eu, g.ev)
    for bad in ({"model": {"p_fail": 1.5}}, {"model": {"p_fail": 0.1}, "R": 0},
                {"model": {"p_fail": 0.1}, "alpha": 0.0},
                {"model": {"p_fail": 0.1, "weight": "uniform", "w_lo": 0, "w_hi": 3}},
                {"model": {"p_fail": 0.1}, "s": np.full(10, 0.2)},
                {"model": {"p_fail": 0.1}, "pool": np.array([10])},
                {"model": {"p_fail": 0.1, "weight": "fixed"}},
                {"model": {"p_fail": 0.1}, "flags": amc.DIST16 | amc.DIST32}):
        bad = dict(bad)
        model = bad.pop("model")
        bad.setdefault("R", 4)
        with pytest.raises(amc.AmcError) as ei:
            amc.run(ctx, G, model, **bad)
        assert ei.value.rc == amc.E_INVALID_ARG, bad
    G.close()


# --------------------------------------------------------------------------- configs 2 and 3 on sampled realizations
def test_ws1000_sampled_realizations(ctx):
    wl = W.config_ws1000()
    g = wl.graph
    for r0, R, fl in ((0, 3, 0), (7777, 2, 0), (7777, 2, amc.DIST16), (7777, 2, amc.DIST32),
                      (4242, 2, amc.SIGMA_GLOBAL)):
        res = gpu_run(ctx, g, wl.model(), seed=wl.seed, R=R, r_begin=r0, alpha=wl.alpha, k_min=wl.k_min,
                      flags=FLAGS | fl, cert_topk=5)
        ref = O.sweep(g.n, g.eu, g.ev, seed=wl.seed, R=R, r_begin=r0, alpha=wl.alpha, k_min=wl.k_min,
                      want_next=True, **wl.model())
        check_sweep(res, ref, g.n, f"ws1000 r0={r0}")
        t = O.tail(ref["counts"], R, cert_topk=5)
        assert_close_norm(res["b"], t["b"], what="b")
        assert_close_norm(res["N"], t["N"], what="N")


def test_er5000_sampled_realizations_with_pool(ctx):
    wl = W.config_er5000()
    g = wl.graph
    R = 2
    ref = O.sweep(g.n, g.eu, g.ev, seed=wl.seed, R=R, r_begin=1234, alpha=wl.alpha, k_min=wl.k_min,
                  want_next=True, pool=wl.pool, **wl.model())
    for mode, fl in ((amc.MODE_BLOCK, 0), (amc.MODE_WAVE_L2, 0), (amc.MODE_WAVE_L2, amc.SIGMA_GLOBAL),
                     (amc.MODE_WAVE_L2, amc.SIGMA_GLOBAL | amc.DIST32)):
        res = gpu_run(ctx, g, wl.model(), seed=wl.seed, R=R, r_begin=1234, alpha=wl.alpha, k_min=wl.k_min,
                      flags=amc.WANT_NEXT_TABLE | amc.WANT_CENTER | amc.WANT_BSUM | amc.SKIP_TAIL | fl, pool=wl.pool,
                      mode=mode)
        assert res["stats"]["mode"] == mode
        if fl & amc.SIGMA_GLOBAL:
            assert res["stats"]["sig_global"] == 1
        check_sweep(res, ref, g.n, f"er5000 mode {mode} flags {fl}")


def _er_with_hubs(n, p, hubs, spokes, seed):
    # G(n, p) plus `hubs` vertices joined to `spokes` random others each
    g = W.er_graph(n, p, seed)
    rng = np.random.default_rng(seed)
    pairs = set(zip(g.eu.tolist(), g.ev.tolist()))
    for h in range(hubs):
        for v in rng.choice(np.arange(hubs, n), spokes, replace=False).tolist():
            pairs.add((h, v))
    return W.canonical(n, sorted(pairs), name=f"er{n}+{hubs}hubs")


@pytest.mark.parametrize("graph", ["er2000-unit", "hubs1500-unit", "er2000-w3", "er4000-w2"])
@pytest.mark.parametrize("tile", [0, 700])
def test_block_mode_wide_levels_against_oracle(ctx, graph, tile):
    # levels of several hundred to over a thousand vertices: the workgroup
    # mode walks them with one or two lanes per vertex and, with unit weights,
    # orders each wide level by degree (the hubs fall in the open last
    # class); weights 1..3 give wide equal-distance segments
    if graph == "er2000-unit":
        g, model = W.er_graph(2000, 8.0 / 1999, 7), {"p_fail": 0.1, "weight": "unit"}
    elif graph == "hubs1500-unit":
        g, model = _er_with_hubs(1500, 6.0 / 1499, 3, 300, 11), {"p_fail": 0.05, "weight": "unit"}
    elif graph == "er2000-w3":
        g, model = W.er_graph(2000, 8.0 / 1999, 8), {"p_fail": 0.1, "weight": "uniform", "w_lo": 1, "w_hi": 3}
    else:   # weights 1..2: equal-distance segments of over a thousand vertices
        g, model = W.er_graph(4000, 8.0 / 3999, 9), {"p_fail": 0.1, "weight": "uniform", "w_lo": 1, "w_hi": 2}
    R = 5
    kw = dict(seed=5, R=R, r_begin=321, alpha=0.15, k_min=5)
    ref = O.sweep(g.n, g.eu, g.ev, want_next=True, **kw, **model)
    q = dict(flags=FLAGS | amc.SKIP_TAIL, mode=amc.MODE_BLOCK, **kw)
    if tile:
        q["tile"] = tile
    res = gpu_run(ctx, g, model, **q)
    assert res["stats"]["mode"] == amc.MODE_BLOCK
    check_sweep(res, ref, g.n, f"{graph} block tile {tile}")


def test_weighted_n2400_l2_mode_sampled(ctx):
    # a graph whose realized adjacency leaves room for only two wavefronts in
    # LDS mode: the planner takes the L2 mode; two realizations split over
    # several work items each
    g = W.er_graph(2400, 8.0 / 2399, 2400)
    model = {"p_fail": 0.1, "weight": "uniform", "w_lo": 1, "w_hi": 10}
    res = gpu_run(ctx, g, model, seed=3, R=2, r_begin=77, flags=amc.WANT_NEXT_TABLE | amc.WANT_CENTER |
                  amc.WANT_BSUM | amc.SKIP_TAIL)
    assert res["stats"]["mode"] == amc.MODE_WAVE_L2
    assert res["stats"]["tile"] < g.n
    ref = O.sweep(g.n, g.eu, g.ev, seed=3, R=2, r_begin=77, want_next=True, **model)
    check_sweep(res, ref, g.n, "er2400 L2")
    res1 = gpu_run(ctx, g, model, seed=3, R=2, r_begin=77, mode=amc.MODE_WAVE_L2, tile=g.n, group=3,
                   flags=amc.WANT_NEXT_TABLE | amc.WANT_CENTER | amc.WANT_BSUM | amc.SKIP_TAIL)
    assert res1["stats"]["tile"] == g.n
    check_sweep(res1, ref, g.n, "er2400 L2 whole realizations")


@pytest.mark.parametrize("n", [2400, 3000])
def test_weighted_l2_whole_realizations_default_plan(ctx, n):
    # the sizes that dominate the mixed batch, on the plan the planner picks
    # for them (L2 mode, 16-bit distances, B in the scratch when that adds a
    # wavefront), whole realizations
    g = W.er_graph(n, 8.0 / (n - 1), n + 1)
    model = {"p_fail": 0.1, "weight": "uniform", "w_lo": 1, "w_hi": 10}
    R = 12
    res = gpu_run(ctx, g, model, seed=5, R=R, r_begin=901, tile=g.n, alpha=0.15, k_min=5,
                  flags=amc.WANT_NEXT_TABLE | amc.WANT_CENTER | amc.WANT_BSUM | amc.SKIP_TAIL)
    st = res["stats"]
    assert st["mode"] == amc.MODE_WAVE_L2 and st["tile"] == g.n, st
    say(f"[cpu] oracle on er{n} R={R} in {P.workers()} threads")
    ref = P.sweep(g.n, g.eu, g.ev, seed=5, R=R, r_begin=901, alpha=0.15, k_min=5, want_next=True, **model)
    check_sweep(res, ref, g.n, f"er{n} L2 default plan")


# --------------------------------------------------------------------------- systems properties
def test_weighted_n1800_l2_mode_global_b(ctx):
    # n = 1800: B(H_r) in LDS would cost the L2 mode a wavefront, so the
    # planner keeps B in the global scratch; split and whole realizations
    # (six wavefronts; with AMC_SIGMA_GLOBAL the path counts go to the scratch)
    g = W.er_graph(1800, 8.0 / 1799, 1800)
    model = {"p_fail": 0.1, "weight": "uniform", "w_lo": 1, "w_hi": 10}
    fl = amc.WANT_NEXT_TABLE | amc.WANT_CENTER | amc.WANT_BSUM | amc.SKIP_TAIL
    ref = O.sweep(g.n, g.eu, g.ev, seed=4, R=2, r_begin=9, want_next=True, **model)
    for extra in ({}, {"tile": g.n}):
        res = gpu_run(ctx, g, model, seed=4, R=2, r_begin=9, flags=fl, mode=amc.MODE_WAVE_L2, waves=6, **extra)
        st = res["stats"]
        assert st["mode"] == amc.MODE_WAVE_L2 and st["b_global"] == 1 and st["sig_global"] == 0, st
        check_sweep(res, ref, g.n, f"er1800 L2 global B {extra}")
    res = gpu_run(ctx, g, model, seed=4, R=2, r_begin=9, flags=fl | amc.SIGMA_GLOBAL)
    assert res["stats"]["mode"] == amc.MODE_WAVE_L2 and res["stats"]["sig_global"] == 1, res["stats"]
    check_sweep(res, ref, g.n, "er1800 path counts in the scratch")
    res = gpu_run(ctx, W.er_graph(2400, 8.0 / 2399, 2400), model, seed=3, R=1, flags=fl, mode=amc.MODE_WAVE_L2,
                  waves=5)
    assert res["stats"]["mode"] == amc.MODE_WAVE_L2 and res["stats"]["b_global"] == 0


def test_n6000_auto_picks_a_mode_that_fits(ctx):
    # the workgroup-per-source mode does not fit n = 6000; AUTO takes the L2
    # mode (16-bit distances, B in the global scratch)
    g = W.er_graph(6000, 8.0 / 5999, 6000)
    model = {"p_fail": 0.1, "weight": "uniform", "w_lo": 1, "w_hi": 10}
    res = gpu_run(ctx, g, model, seed=8, R=1, flags=amc.WANT_NEXT_TABLE | amc.WANT_CENTER | amc.SKIP_TAIL)
    st = res["stats"]
    assert st["mode"] == amc.MODE_WAVE_L2 and st["dist_bytes"] == 2 and st["b_global"] == 1, st
    ref = O.sweep(g.n, g.eu, g.ev, seed=8, R=1, want_next=True, **model)
    check_sweep(res, ref, g.n, "er6000 auto")


def test_split_ranges_and_determinism(ctx):
    wl = W.config_er20()
    g = wl.graph
    G = amc.Graph(ctx, g.n, g.eu, g.ev)
    kw = dict(seed=5, alpha=0.15, k_min=5, flags=amc.WANT_NEXT_TABLE | amc.SKIP_TAIL)
    say("[gpu] split ranges")
    full = amc.run(ctx, G, wl.model(), R=300, **kw)
    a = amc.run(ctx, G, wl.model(), R=120, r_begin=0, **kw)
    b = amc.run(ctx, G, wl.model(), R=180, r_begin=120, **kw)
    again = amc.run(ctx, G, wl.model(), R=300, **kw)
    assert np.array_equal(full["counts"], a["counts"] + b["counts"])
    assert np.array_equal(full["next_table"], np.vstack([a["next_table"], b["next_table"]]))
    assert np.array_equal(full["counts"], again["counts"])
    assert np.array_equal(full["next_table"], again["next_table"])
    G.close()


@pytest.mark.parametrize("mode,graph,extra", [(amc.MODE_WAVE_L2, "er20", {}), (amc.MODE_WAVE_L2, "ws200", {}),
                                              (amc.MODE_WAVE, "ws200", {}),
                                              (amc.MODE_WAVE_L2, "ws200", {"flags": amc.DIST16, "pool": True}),
                                              (amc.MODE_WAVE_L2, "ws200", {"flags": amc.SIGMA_GLOBAL, "pool": True}),
                                              (amc.MODE_WAVE, "ws200", {"pool": True}),
                                              (amc.MODE_BLOCK, "er20", {}), (amc.MODE_BLOCK, "ws200", {"pool": True})])
def test_last_realizations_split_into_tiles(ctx, mode, graph, extra):
    # whole realizations (tile = n) with R = workgroups + 37: the last 37 run
    # split into tiles through a second descriptor over the same counts
    g = W.config_er20().graph if graph == "er20" else W.ws_graph(200, 6, 0.1, 1)
    model = {"p_fail": 0.1, "weight": "uniform", "w_lo": 1, "w_hi": 6}
    G = amc.Graph(ctx, g.n, g.eu, g.ev)
    pool = np.arange(3, g.n, 7) if extra.get("pool") else None
    probe = amc.run(ctx, G, model, seed=3, R=32768, mode=mode, tile=g.n, pool=pool,
                    flags=amc.SKIP_TAIL | extra.get("flags", 0))          # the same plan as the run below
    G.close()
    blocks = probe["stats"]["blocks"]
    if blocks >= 32768:
        pytest.skip("more workgroup slots than the probe's realizations")
    R = blocks + 37
    res = gpu_run(ctx, g, model, seed=3, R=R, alpha=0.15, k_min=5, flags=FLAGS | extra.get("flags", 0), mode=mode,
                  tile=g.n, pool=pool)
    st = res["stats"]
    assert st["tail_split"] == 37 and st["tail_tiles"] >= 2, st
    ref = O.sweep(g.n, g.eu, g.ev, seed=3, R=R, alpha=0.15, k_min=5, want_next=True, pool=pool, **model)
    check_sweep(res, ref, g.n, f"{graph} tail split")
    t = O.tail(ref["counts"], R)
    assert_close_norm(res["b"], t["b"], what="b")


def test_result_buffers_reused(ctx):
    # out= lends the arrays of an earlier result: same objects, same values
    wl = W.config_er20()
    g = wl.graph
    G = amc.Graph(ctx, g.n, g.eu, g.ev)
    kw = dict(seed=9, R=300, alpha=0.15, k_min=5, flags=amc.WANT_NEXT_TABLE, cert_topk=3, r_lower=0.05)
    say("[gpu] result buffers reused")
    first = amc.run(ctx, G, wl.model(), **kw)
    keep = {k: v.copy() for k, v in first.items() if isinstance(v, np.ndarray)}
    second = amc.run(ctx, G, wl.model(), out=first, **dict(kw, seed=10))
    third = amc.run(ctx, G, wl.model(), out=second, **kw)
    assert second["counts"] is first["counts"] and third["Q"] is first["Q"]
    for k, v in keep.items():
        assert np.array_equal(third[k], v), k
    old_table = third["next_table"]
    other = amc.run(ctx, G, wl.model(), out=third, **dict(kw, R=200))      # next table of another shape
    G.close()
    assert other["next_table"].shape == (200, g.n) and other["next_table"] is not old_table
    assert other["counts"] is first["counts"]


# --------------------------------------------------------------------------- tail alone (amc_chain)
def test_chain_appendix_b(ctx, golden):
    ref = golden("appendix_b.json")
    Q0 = np.array(ref["Q0"])
    say("[gpu] chain appendix B")
    res = amc.chain(ctx, Q0, s=np.array(ref["s"]), flags=amc.WANT_N, eps=ref["eps_entry"], r_lower=ref["r_min"],
                    cert_topk=1)
    o = O.chain(Q0, np.array(ref["s"]))
    assert_close_norm(res["N"], o["N"], what="N")
    assert_close_norm(res["mu"], o["mu"], what="mu")
    assert np.allclose(res["mu"], ref["mu"], atol=5e-5)
    # top-1 is vertex 2 (index 1): boundary pairs (2,1) and (2,3)
    assert list(res["top"]) == [1]
    g21, _, s21 = O.pair_certificate(o["N"], o["mu"], ref["epsbar"], ref["r_min"], 1, 0)
    assert res["cert_gap"][0, 0] == pytest.approx(g21, abs=1e-15)
    assert res["cert_sharp"][0, 0] == pytest.approx(s21, rel=1e-12)
    assert res["cert_sharp"][0, 0] == pytest.approx(ref["sharp_thresholds"]["2,1"], abs=5e-5)
    assert res["cert_crude"] == pytest.approx(ref["crude_threshold"], abs=5e-5)
    # which orders each threshold certifies, as printed for the three pairs:
    # top-1 gives the pairs (2,1), (2,3); top-2 (nodes 2, 1) gives (2,3), (1,3)
    res2 = amc.chain(ctx, Q0, s=np.array(ref["s"]), eps=ref["eps_entry"], r_lower=ref["r_min"], cert_topk=2)
    assert list(res2["top"]) == [1, 0]
    for r, pairs in ((res, [("2,1", 0, 0), ("2,3", 0, 1)]), (res2, [("2,3", 0, 0), ("1,3", 1, 0)])):
        for name, a, c in pairs:
            ok = int(r["cert_ok"][a, c])
            assert bool(ok & 1) == ref["sharp_certifies"][name], name
            assert bool(ok & 4) == ref["crude_certifies"][name], name


@pytest.mark.parametrize("n", [1, 2, 31, 33, 64, 97, 300])
def test_chain_random_kernels(ctx, n):
    rng = np.random.default_rng(n)
    Q = rng.random((n, n)) * (rng.random((n, n)) < 0.4)
    rr = 0.1 + 0.4 * rng.random(n)
    Q = Q / np.maximum(Q.sum(1, keepdims=True), 1e-300) * (1 - rr)[:, None]
    s = rng.dirichlet(np.ones(n))
    f = rng.random(n)
    say(f"[gpu] chain random n={n}")
    res = amc.chain(ctx, Q, s=s, reward=f, flags=amc.WANT_N, eps=1e-4, r_lower=0.1, cert_topk=min(3, n - 1))
    o = O.chain(Q, s)
    assert_close_norm(res["N"], o["N"], what="N")
    assert_close_norm(res["b"], o["b"], what="b")
    assert res["E_T"] == pytest.approx(o["ET"], rel=TOL)
    assert res["b_f"] == pytest.approx(float(o["b"] @ f), rel=1e-12)
    # the certificate bits are the strict comparisons of the returned gaps and thresholds
    if n > 1:
        g, ok = res["cert_gap"], res["cert_ok"].astype(int)
        assert np.array_equal(ok & 1, (g > res["cert_sharp"]).astype(int))
        assert np.array_equal((ok >> 1) & 1, (g > res["cert_sharp_supp"]).astype(int))
        assert np.array_equal((ok >> 2) & 1, (g > res["cert_crude"]).astype(int))


# --------------------------------------------------------------------------- per-call weight resampling (Section 9.2)
@pytest.mark.parametrize("mode", [amc.MODE_WAVE, amc.MODE_WAVE_L2, amc.MODE_BLOCK, "wave-g8"])
def test_resampled_weight_table(ctx, mode):
    g = W.powerlaw_weighted_graph(77, 254, 2.5, 3.0, 31, 0)
    T = W.resampled_weight_cdf(g.w0, 31, 0.1, 0.2)
    model = {"p_fail": 0.05, "weight": "table", "w_cdf": T}
    q = dict(mode=amc.MODE_WAVE, group=8) if mode == "wave-g8" else dict(mode=mode)
    res = gpu_run(ctx, g, model, seed=5, R=400, alpha=0.15, k_min=5, flags=FLAGS, **q)
    ref = O.sweep(g.n, g.eu, g.ev, seed=5, R=400, alpha=0.15, k_min=5, want_next=True, **model)
    check_sweep(res, ref, g.n, f"table law {mode}")
    er = W.config_er20().graph
    T2 = W.resampled_weight_cdf(np.full(er.m, 2), 9, 0.3, 0.25)
    model2 = {"p_fail": 0.1, "weight": "table", "w_cdf": T2}
    res = gpu_run(ctx, er, model2, seed=6, R=300, flags=FLAGS, **q)
    ref = O.sweep(er.n, er.eu, er.ev, seed=6, R=300, want_next=True, **model2)
    check_sweep(res, ref, er.n, f"table law er20 {mode}")


def test_weight_table_arguments(ctx):
    g = W.er_graph(10, 0.4, 1)
    G = amc.Graph(ctx, g.n, g.eu, g.ev)
    good = W.resampled_weight_cdf(np.full(g.m, 1), 5, 0.2, 0.3)
    bad_last = good.copy()
    bad_last[0, -1] = 2 ** 32 - 1
    bad_order = good.copy()
    bad_order[1, 0], bad_order[1, 1] = good[1, 1], good[1, 0] - 1
    for T in (bad_last, bad_order):
        with pytest.raises(amc.AmcError) as ei:
            amc.run(ctx, G, {"p_fail": 0.1, "weight": "table", "w_cdf": T}, R=4)
        assert ei.value.rc == amc.E_INVALID_ARG
    G.close()


# --------------------------------------------------------------------------- anchored r-hop neighbourhoods (Section 9.2)
@pytest.mark.parametrize("radius,extra", [(1, {}), (2, {}), (3, {"tile": 5}), (2, {"waves": 3})])
def test_anchored_neighbourhoods(ctx, radius, extra):
    g = W.powerlaw_weighted_graph(77, 254, 2.5, 3.0, 31, 0)
    T = W.resampled_weight_cdf(g.w0, 31, 0.1, 0.2)
    pool = np.array([0, 3, 9, 21, 40, 66])
    for model in ({"p_fail": 0.0, "weight": "table", "w_cdf": T}, {"p_fail": 0.1, "weight": "fixed"}):
        res = gpu_run(ctx, g, model, seed=7, R=120, alpha=0.15, k_min=5, hop_radius=radius, pool=pool,
                      flags=amc.WANT_NEXT_TABLE | amc.WANT_N, **extra)
        ref = O.sweep(g.n, g.eu, g.ev, seed=7, R=120, alpha=0.15, k_min=5, hop_radius=radius, pool=pool,
                      want_next=True, **oracle_model(model, g))
        check_sweep(res, ref, g.n, f"anchored r={radius} {model['weight']}")
        t = O.tail(ref["counts"], 120)
        assert_close_norm(res["b"], t["b"], what="anchored b")
    er = W.config_er20().graph
    res = gpu_run(ctx, er, W.config_er20().model(), seed=2, R=200, hop_radius=radius, flags=amc.WANT_NEXT_TABLE,
                  **extra)
    ref = O.sweep(er.n, er.eu, er.ev, seed=2, R=200, hop_radius=radius, want_next=True, **W.config_er20().model())
    check_sweep(res, ref, er.n, f"anchored er20 r={radius}")


def test_anchored_arguments(ctx):
    g = W.er_graph(10, 0.4, 1)
    G = amc.Graph(ctx, g.n, g.eu, g.ev)
    for bad in ({"hop_radius": -1}, {"hop_radius": 2, "topk": 2}, {"hop_radius": 2, "flags": amc.WANT_CENTER},
                {"hop_radius": 2, "flags": amc.WANT_BSUM}, {"hop_radius": 2, "mode": amc.MODE_BLOCK}):
        with pytest.raises(amc.AmcError) as ei:
            amc.run(ctx, G, {"p_fail": 0.1}, R=4, **bad)
        assert ei.value.rc == amc.E_INVALID_ARG, bad
    G.close()


# --------------------------------------------------------------------------- the benchmark's own launch plan
# ws1000 (Watts-Strogatz n = 1000, k = 10, beta = 0.1; failure 0.05; weights
# U{1..10}; R = 10000) as the benchmark runs it: L2 mode, whole realizations
# (tile = n), 11 wavefronts, one lane per vertex, 16-bit adjacency entries,
# 32-bit distances, B(H_r) in LDS; the last R mod 256 + 256 realizations split
# into tiles.
BENCH_PLAN = {"mode": amc.MODE_WAVE_L2, "tile": 1000, "waves": 11, "group": 1, "adj_bytes": 2, "dist_bytes": 4,
              "b_global": 0}


def _assert_bench_plan(st):
    for k, v in BENCH_PLAN.items():
        assert st[k] == v, f"plan field {k}: {st[k]} != {v} ({st})"


def _oracle_rows(g, wl, rs):
    """Oracle next-state rows and global centres of single realizations."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(P.workers()) as ex:
        outs = list(ex.map(lambda r: O.sweep(g.n, g.eu, g.ev, seed=wl.seed, R=1, r_begin=int(r), alpha=wl.alpha,
                                             k_min=wl.k_min, want_next=True, want_bsum=False, **wl.model()), rs))
    return outs


def test_ws1000_bench_plan_full_R_sampled(ctx):
    # the full R = 10000 launch exactly as timed by the benchmark; sampled
    # realizations from both the whole-realization descriptor and the split
    # last realizations against the oracle, one realization at a time
    wl = W.config_ws1000()
    g = wl.graph
    res = gpu_run(ctx, g, wl.model(), seed=wl.seed, R=wl.R, alpha=wl.alpha, k_min=wl.k_min,
                  flags=amc.WANT_NEXT_TABLE | amc.WANT_CENTER | amc.SKIP_TAIL)
    st = res["stats"]
    _assert_bench_plan(st)
    assert st["blocks"] == 256 and st["tail_split"] == wl.R % 256 + 256 and st["tail_tiles"] >= 16, st
    R0 = wl.R - st["tail_split"]
    # counts are the histogram of the next-state table
    nt = res["next_table"]
    hist = np.zeros((g.n, g.n + 1), dtype=np.int64)
    cols = np.where(nt >= 0, nt, g.n)
    np.add.at(hist, (np.broadcast_to(np.arange(g.n), nt.shape), cols), 1)
    assert np.array_equal(hist, res["counts"].astype(np.int64))
    assert st["units"] == wl.R * g.n
    rs = [0, 1, 255, 256, 2500, 7777, R0 - 1, R0, R0 + 100, 9990, 9999]
    say(f"[cpu] oracle on {len(rs)} sampled ws1000 realizations")
    for r, o in zip(rs, _oracle_rows(g, wl, rs)):
        assert np.array_equal(nt[r], o["next_table"][0]), f"next table row r={r}"
        assert res["center_global"][r] == o["center_global"][0], f"centre r={r}"


def test_ws1000_bench_plan_against_oracle(ctx):
    # the benchmark's plan forced on R = 256 + 37 realizations: 256 whole
    # realizations on the benchmark's instantiation, the last 37 split into
    # tiles; everything against the oracle over the same range
    wl = W.config_ws1000()
    g = wl.graph
    plan = {k: BENCH_PLAN[k] for k in ("mode", "tile", "waves", "group")}
    R = 256 + 37
    res = gpu_run(ctx, g, wl.model(), seed=wl.seed, R=R, alpha=wl.alpha, k_min=wl.k_min, flags=FLAGS, cert_topk=5,
                  **plan)
    st = res["stats"]
    _assert_bench_plan(st)
    assert st["blocks"] == 256 and st["tail_split"] == 37, st
    say(f"[cpu] oracle on ws1000 R={R} in {P.workers()} threads")
    ref = P.sweep(g.n, g.eu, g.ev, seed=wl.seed, R=R, alpha=wl.alpha, k_min=wl.k_min, want_next=True, **wl.model())
    check_sweep(res, ref, g.n, "ws1000 bench plan")
    assert st["near_band"] == ref["stats"]["near_band"]
    t = O.tail(ref["counts"], R, cert_topk=5)
    assert_close_norm(res["N"], t["N"], what="N")
    assert_close_norm(res["mu"], t["mu"], what="mu")
    assert_close_norm(res["b"], t["b"], what="b")
    assert abs(res["E_T"] - t["ET"]) <= TOL * t["ET"]
    # whole realizations only, at spread realization indices
    for r0 in (2500, 7777, 9990):
        res = gpu_run(ctx, g, wl.model(), seed=wl.seed, R=2, r_begin=r0, alpha=wl.alpha, k_min=wl.k_min,
                      flags=FLAGS | amc.SKIP_TAIL, **plan)
        _assert_bench_plan(res["stats"])
        assert res["stats"]["tail_split"] == 0
        ref = O.sweep(g.n, g.eu, g.ev, seed=wl.seed, R=2, r_begin=r0, alpha=wl.alpha, k_min=wl.k_min,
                      want_next=True, **wl.model())
        check_sweep(res, ref, g.n, f"ws1000 bench plan r0={r0}")


def test_er5000_bench_plan_against_oracle(ctx):
    # the n = 5000 unit-weight workload on its benchmark plan: the
    # workgroup-per-source mode, 16 wavefronts, every source of a realization
    # in one work item (its wide levels ordered by degree), with its pool;
    # 40 whole realizations against the oracle over the same range
    wl = W.config_er5000()
    g = wl.graph
    R = 40
    res = gpu_run(ctx, g, wl.model(), seed=wl.seed, R=R, r_begin=4000, alpha=wl.alpha, k_min=wl.k_min,
                  flags=amc.WANT_NEXT_TABLE | amc.WANT_CENTER | amc.WANT_BSUM | amc.SKIP_TAIL, pool=wl.pool,
                  mode=amc.MODE_BLOCK, tile=g.n)
    st = res["stats"]
    assert st["mode"] == amc.MODE_BLOCK and st["tile"] == g.n and st["waves"] == 16 and st["tail_split"] == 0, st
    say(f"[cpu] oracle on er5000 R={R} in {P.workers()} threads")
    ref = P.sweep(g.n, g.eu, g.ev, seed=wl.seed, R=R, r_begin=4000, alpha=wl.alpha, k_min=wl.k_min, want_next=True,
                  pool=wl.pool, **wl.model())
    check_sweep(res, ref, g.n, "er5000 bench plan")
    assert st["near_band"] == ref["stats"]["near_band"]


# --------------------------------------------------------------------------- exact ties with nonzero betweenness
# Vertex-transitive graphs without failures: every vertex has the same B, so
# every realization's centres are vertex 0 (the smallest index, Corollary on
# deterministic tie-breaking), whatever order the FP64 additions took.
def _cycle(n):
    return W.canonical(n, [(i, i + 1) for i in range(n - 1)] + [(0, n - 1)], name=f"C{n}")


def _complete(n):
    return W.canonical(n, [(i, j) for i in range(n) for j in range(i + 1, n)], name=f"K{n}")


def _cycle_b(n):
    """B of every vertex of the cycle C_n over ordered pairs (Section 3.1): with
    k = floor(n / 2), k (k - 1) for odd n and (k - 1)^2 for even n (the two
    antipodal paths share each pair's weight)."""
    k = n // 2
    return float(k * (k - 1)) if n % 2 else float((k - 1) ** 2)


# K_29 is the largest complete graph whose per-edge staging (one byte per
# edge) fits the workgroup-per-source mode's 28 n bytes of LDS
_TIE_GRAPHS = {"C1001": lambda: _cycle(1001), "C1000": lambda: _cycle(1000), "K29": lambda: _complete(29),
               "ring1000": lambda: W.ws_graph(1000, 10, 0.0, 0)}
_TIE_MODES = [(amc.MODE_WAVE, {}), (amc.MODE_WAVE, {"group": 2}), (amc.MODE_WAVE, {"group": 3}),
              (amc.MODE_WAVE, {"group": 8}), (amc.MODE_WAVE, {"tile": 333}), (amc.MODE_WAVE, {"flags": amc.DIST16}),
              (amc.MODE_WAVE_L2, {}), (amc.MODE_WAVE_L2, {"group": 8}), (amc.MODE_WAVE_L2, {"flags": amc.DIST16}),
              (amc.MODE_WAVE_L2, {"flags": amc.SIGMA_GLOBAL}), (amc.MODE_BLOCK, {})]
_tie_ref = {}


@pytest.mark.parametrize("weights", ["unit", "const3"])
@pytest.mark.parametrize("graph", sorted(_TIE_GRAPHS))
def test_symmetric_ties_every_mode(ctx, graph, weights):
    g = _TIE_GRAPHS[graph]()
    model = {"p_fail": 0.0, "weight": "unit"} if weights == "unit" else \
        {"p_fail": 0.0, "weight": "uniform", "w_lo": 3, "w_hi": 3}
    R = 24
    kw = dict(seed=11, R=R, alpha=0.15, k_min=5)
    key = (graph, weights)
    if key not in _tie_ref:
        _tie_ref[key] = P.sweep(g.n, g.eu, g.ev, want_next=True, **kw, **model)
    ref = _tie_ref[key]
    # the oracle itself: every valid anchor moves to vertex 0, every centre is 0
    assert np.all(ref["center_global"] == 0)
    assert np.all((ref["next_table"] == 0) | (ref["next_table"] == -1))
    bv = ref["bsum"] / R
    if graph.startswith("C"):
        assert_rel(bv, np.full(g.n, _cycle_b(g.n)), what="cycle closed form")
    elif graph.startswith("K"):
        assert np.all(bv == 0.0)
    else:
        assert_rel(bv, np.full(g.n, bv[0]), what="ring lattice symmetry")
    for mode, extra in _TIE_MODES:
        extra = dict(extra)
        fl = FLAGS | amc.SKIP_TAIL | extra.pop("flags", 0)
        if (fl & amc.DIST16) and weights == "const3" and g.n * 3 >= 0xFFFF:
            continue
        res = gpu_run(ctx, g, model, flags=fl, mode=mode, **kw, **extra)
        assert res["stats"]["mode"] == mode
        check_sweep(res, ref, g.n, f"{graph} {weights} mode {mode} {extra}")


# --------------------------------------------------------------------------- state in the global scratch
@pytest.mark.parametrize("graph,model,extra", [
    ("er20", {"p_fail": 0.1, "weight": "uniform", "w_lo": 1, "w_hi": 5}, {}),
    ("er20", {"p_fail": 0.1, "weight": "unit"}, {"tile": 7}),
    ("ws200", {"p_fail": 0.1, "weight": "uniform", "w_lo": 1, "w_hi": 6}, {"pool": True}),
    ("er2000", {"p_fail": 0.1, "weight": "unit"}, {}),
    ("er2000", {"p_fail": 0.1, "weight": "uniform", "w_lo": 1, "w_hi": 3}, {"tile": 700}),
])
def test_workgroup_mode_state_in_global_scratch(ctx, graph, model, extra):
    # the workgroup-per-source mode with every source's state in the global
    # scratch (forced here on graphs whose state fits LDS) against the oracle
    g = {"er20": lambda: W.config_er20().graph, "ws200": lambda: W.ws_graph(200, 6, 0.1, 1),
         "er2000": lambda: W.er_graph(2000, 8.0 / 1999, 7)}[graph]()
    extra = dict(extra)
    pool = np.arange(3, g.n, 7) if extra.pop("pool", False) else None
    R = 40 if g.n >= 2000 else 300
    res = gpu_run(ctx, g, model, seed=5, R=R, alpha=0.15, k_min=5, flags=FLAGS | amc.STATE_GLOBAL,
                  pool=pool, **extra)
    st = res["stats"]
    assert st["mode"] == amc.MODE_BLOCK and st["state_global"] == 2 and st["lds_bytes"] == 0, st
    ref = (P if g.n >= 2000 else O).sweep(g.n, g.eu, g.ev, seed=5, R=R, alpha=0.15, k_min=5, want_next=True,
                                          pool=pool, **oracle_model(model, g))
    check_sweep(res, ref, g.n, f"{graph} state in global scratch {extra}")
    t = O.tail(ref["counts"], R)
    assert_close_norm(res["b"], t["b"], what="b")


def test_graph_beyond_every_lds_layout_runs_with_global_state(ctx):
    # n = 9000 (unit weights): no wavefront layout and no LDS workgroup layout
    # holds it; the planner moves the workgroup mode's state to the global
    # scratch, distances and row offsets staying in LDS.  One realization
    # against the oracle (split into tiles), and sampled sources' distances,
    # path counts and dependencies
    g = W.er_graph(9000, 8.0 / 8999, 90)
    model = {"p_fail": 0.1, "weight": "unit"}
    pairs = [(0, 0), (0, 4500), (0, 8999)]
    res = gpu_run(ctx, g, model, seed=3, R=1, alpha=0.15, k_min=5,
                  flags=amc.WANT_NEXT_TABLE | amc.WANT_CENTER | amc.WANT_BSUM | amc.SKIP_TAIL, debug_pairs=pairs)
    st = res["stats"]
    assert st["mode"] == amc.MODE_BLOCK and st["state_global"] == 1 and st["lds_bytes"] > 0, st
    for k, (r, s) in enumerate(pairs):
        alive, w = O.realize(g.n, g.eu, g.ev, 3, r, **model)
        d, sg, dl = O.sssp(g.n, g.eu, g.ev, alive, w, True, s)
        dd = np.where(d == np.iinfo(np.uint64).max, 0xFFFFFFFF, d).astype(np.uint32)
        assert np.array_equal(res["dbg_dist"][k], dd), (r, s)
        assert np.array_equal(res["dbg_sigma"][k], sg), (r, s)
        assert_rel(res["dbg_delta"][k], dl, what=f"delta {(r, s)}")
    say(f"[cpu] oracle on n={g.n} R=1")
    ref = O.sweep(g.n, g.eu, g.ev, seed=3, R=1, alpha=0.15, k_min=5, want_next=True, **model)
    check_sweep(res, ref, g.n, "n=9000 global state")


def test_weighted_workgroup_mode_beyond_lds_keeps_distances_in_lds(ctx):
    # weighted n = 6000 asked for in the workgroup mode: its 28 n bytes of
    # state exceed the LDS, distances and row offsets (8 n) stay there; two
    # realizations against the oracle
    g = W.er_graph(6000, 8.0 / 5999, 60)
    model = {"p_fail": 0.1, "weight": "uniform", "w_lo": 1, "w_hi": 10}
    res = gpu_run(ctx, g, model, seed=4, R=2, alpha=0.15, k_min=5, mode=amc.MODE_BLOCK,
                  flags=amc.WANT_NEXT_TABLE | amc.WANT_CENTER | amc.WANT_BSUM | amc.SKIP_TAIL)
    st = res["stats"]
    assert st["mode"] == amc.MODE_BLOCK and st["state_global"] == 1, st
    say(f"[cpu] oracle on n={g.n} R=2 in {P.workers()} threads")
    ref = P.sweep(g.n, g.eu, g.ev, seed=4, R=2, alpha=0.15, k_min=5, want_next=True, **model)
    check_sweep(res, ref, g.n, "weighted n=6000 hybrid placement")


def test_tail_at_n9000(ctx):
    # the FP64 tail of a 9000-vertex query (N is 9000 x 9000): N inverts I - Q
    # on sampled columns, mu = s N for the uniform s, E[T] = sum mu and
    # b = mu / E[T], all from the returned Q and N
    n = 9000
    g = W.er_graph(n, 8.0 / (n - 1), 90)
    res = gpu_run(ctx, g, {"p_fail": 0.1, "weight": "unit"}, seed=3, R=8, alpha=0.15, k_min=5, flags=amc.WANT_N)
    st = res["stats"]
    assert st["mode"] == amc.MODE_BLOCK and st["state_global"] == 1, st
    Q, N, mu, b = res["Q"], res["N"], res["mu"], res["b"]
    cols = np.random.default_rng(9).choice(n, 16, replace=False)
    resid = N[:, cols] - Q @ N[:, cols]
    resid[cols, np.arange(len(cols))] -= 1.0
    assert np.abs(resid).max() <= 1e-10 * max(np.abs(N).max(), 1.0)
    assert_close_norm(mu, np.full(n, 1.0 / n) @ N, tol=1e-10, what="mu = s N")
    assert abs(res["E_T"] - mu.sum()) <= 1e-10 * mu.sum()
    assert_close_norm(b, mu / mu.sum(), tol=1e-10, what="b")
