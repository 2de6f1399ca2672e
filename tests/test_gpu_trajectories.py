"""GPU parity of the trajectory simulator (Section 4.3) against the CPU oracle,
through the C-ABI: episode paths, lengths, visits, switches, truncation and
the survival weights bit-exact; the node-reward total within 1e-12.  Every
layout is covered: the realized graph in LDS, or in the workgroup's global
scratch with B(H) in LDS or in that scratch, 32- and 16-bit distances."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2605_14743_amd import amc
from paper_2605_14743_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = amc.Context(0)
    yield c
    c.close()


def both(ctx, g, model, *, x0, seed=0, alpha=0.15, k_min=5, max_steps=64, f=None, **gq):
    G = amc.Graph(ctx, g.n, g.eu, g.ev, g.w0)
    say(f"[gpu] trajectories n={g.n} E={len(x0)} max_steps={max_steps} {gq}")
    try:
        res = amc.trajectories(ctx, G, model, seed=seed, x0=x0, alpha=alpha, k_min=k_min, max_steps=max_steps, f=f,
                               want_paths=True, **gq)
    finally:
        G.close()
    om = dict(model)
    if om.get("weight") == "fixed":
        om["w0"] = g.w0
    ref = O.trajectories(g.n, g.eu, g.ev, seed=seed, x0=x0, alpha=alpha, k_min=k_min, max_steps=max_steps, f=f,
                         want_paths=True, **om)
    return res, ref


def check(res, ref, what):
    assert np.array_equal(res["paths"], ref["paths"]), f"{what}: paths"
    assert np.array_equal(res["lengths"], ref["lengths"]), f"{what}: lengths"
    assert np.array_equal(res["visits"], ref["visits"]), f"{what}: visits"
    for key in ("switches", "total_steps", "truncated"):
        assert res[key] == ref[key], f"{what}: {key}"
    tot = ref["total_steps"]
    assert np.array_equal(res["b_hat"], ref["visits"] / tot), f"{what}: b_hat"
    surv = np.array([(ref["lengths"] > t).sum() for t in range(len(res["survival"]))]) / tot
    assert np.array_equal(res["survival"], surv), f"{what}: survival"
    if ref["reward_f"]:
        assert res["reward_f"] == pytest.approx(ref["reward_f"], rel=1e-12)


@pytest.mark.parametrize("group", [0, 1, 3, 8])
def test_er20_trajectories(ctx, group):
    wl = W.config_er20()
    g = wl.graph
    x0 = np.arange(600) % g.n
    f = np.linspace(0.5, 2.0, g.n)
    res, ref = both(ctx, g, wl.model(), x0=x0, seed=11, f=f, group=group)
    check(res, ref, f"er20 group {group}")
    assert res["sources"] > res["total_steps"]


def test_unit_weights_truncation_and_crossroads(ctx):
    g = W.er_graph(60, 0.06, 3)
    x0 = np.arange(300) % g.n
    res, ref = both(ctx, g, {"p_fail": 0.05, "weight": "unit"}, x0=x0, seed=4, alpha=0.05, k_min=2, max_steps=6)
    check(res, ref, "er60 unit, truncated")
    assert res["truncated"] > 0
    cr, pf = W.crossroads()
    x0 = np.arange(2000) % cr.n
    res, ref = both(ctx, cr, {"p_fail": 0.0, "p_fail_edge": pf, "weight": "unit"}, x0=x0, seed=8, alpha=0.1,
                    k_min=3, max_steps=256)
    check(res, ref, "crossroads")


LAYOUTS = {
    "lds": dict(mode=amc.MODE_WAVE),
    "l2-b-lds": dict(mode=amc.MODE_WAVE_L2, flags=amc.TRAJ_B_LDS | amc.DIST32),
    "l2-b-global": dict(mode=amc.MODE_WAVE_L2, flags=amc.TRAJ_B_GLOBAL | amc.DIST32),
    "l2-b-global-d16": dict(mode=amc.MODE_WAVE_L2, flags=amc.TRAJ_B_GLOBAL | amc.DIST16),
    "l2-b-lds-d16": dict(mode=amc.MODE_WAVE_L2, flags=amc.TRAJ_B_LDS | amc.DIST16),
}


def check_layout(res, layout):
    spec = LAYOUTS[layout]
    assert res["mode"] == spec["mode"], layout
    if spec["mode"] == amc.MODE_WAVE_L2:
        assert res["b_global"] == int("b-global" in layout), layout
        assert res["dist16"] == int(layout.endswith("d16")), layout


@pytest.mark.parametrize("layout", list(LAYOUTS))
def test_ws1000_sampled_episodes(ctx, layout):
    wl = W.config_ws1000()
    g = wl.graph
    res, ref = both(ctx, g, wl.model(), x0=np.array([0, 17, 512, 999]), seed=wl.seed, alpha=wl.alpha,
                    k_min=wl.k_min, max_steps=6, **LAYOUTS[layout])
    check(res, ref, f"ws1000 {layout}")
    check_layout(res, layout)


@pytest.mark.parametrize("layout", ["l2-b-lds", "l2-b-global"])
def test_shared_steps_ws1000(ctx, layout):
    # eight ws1000 episodes on eight workgroups: the workgroups whose episodes
    # end first run sources of the steps still open, reading the owner's
    # realized graph and adding into its B through the shared sums
    wl = W.config_ws1000()
    g = wl.graph
    res, ref = both(ctx, g, wl.model(), x0=np.arange(0, 1000, 125), seed=wl.seed + 3, alpha=wl.alpha,
                    k_min=wl.k_min, max_steps=12, **LAYOUTS[layout])
    check(res, ref, f"ws1000 shared steps {layout}")
    check_layout(res, layout)
    say(f"[gpu] lengths {res['lengths'].tolist()} shared sources {res['shared_sources']} of {res['sources']}")
    if res["lengths"].max() >= res["lengths"].min() + 2:
        assert res["shared_sources"] > 0


def test_ws1000_placements_agree_at_scale(ctx):
    # 2000 episodes on all 256 workgroups: the steps shared with workgroups
    # out of episodes (a large share in the last rounds) leave every episode,
    # visit count, switch and node-reward total as the LDS placement has them,
    # whose episodes the oracle pins on samples
    wl = W.config_ws1000()
    g = wl.graph
    G = amc.Graph(ctx, g.n, g.eu, g.ev, g.w0)
    x0 = np.arange(2000) % g.n
    f = np.linspace(0.0, 1.0, g.n)
    kw = dict(seed=wl.seed + 7, x0=x0, alpha=wl.alpha, k_min=wl.k_min, max_steps=256, f=f)
    runs = {}
    try:
        for layout in ("lds", "l2-b-lds", "l2-b-global"):
            say(f"[gpu] ws1000 2000 episodes {layout}")
            runs[layout] = amc.trajectories(ctx, G, wl.model(), **kw, **LAYOUTS[layout])
    finally:
        G.close()
    base = runs["lds"]
    assert base["shared_sources"] == 0
    for layout in ("l2-b-lds", "l2-b-global"):
        r = runs[layout]
        check_layout(r, layout)
        assert r["shared_sources"] > 0, layout
        assert np.array_equal(r["lengths"], base["lengths"]), layout
        assert np.array_equal(r["visits"], base["visits"]), layout
        for key in ("switches", "total_steps", "sources", "truncated"):
            assert r[key] == base[key], (layout, key)
        assert r["reward_f"] == pytest.approx(base["reward_f"], rel=1e-12), layout


@pytest.mark.parametrize("layout", ["l2-b-lds", "l2-b-global", "l2-b-lds-d16"])
@pytest.mark.parametrize("group", [1, 2, 3])
def test_er20_l2_layouts(ctx, layout, group):
    # every wavefront count up to the 16 a workgroup holds sees a component
    # of at most 20 sources; the fixed group covers each lane mapping
    wl = W.config_er20()
    g = wl.graph
    x0 = np.arange(300) % g.n
    f = np.linspace(0.5, 2.0, g.n)
    res, ref = both(ctx, g, wl.model(), x0=x0, seed=13, f=f, group=group, **LAYOUTS[layout])
    check(res, ref, f"er20 {layout} group {group}")
    check_layout(res, layout)


def test_l2_request_on_a_small_graph(ctx):
    # n = 20 defaults to eight lanes per vertex; asking for the L2 layout
    # without a mapping takes one lane per vertex
    wl = W.config_er20()
    g = wl.graph
    res, ref = both(ctx, g, wl.model(), x0=np.arange(100) % g.n, seed=17, mode=amc.MODE_WAVE_L2)
    check(res, ref, "er20 L2 default mapping")
    assert res["mode"] == amc.MODE_WAVE_L2


@pytest.mark.parametrize("layout", ["l2-b-lds", "l2-b-global"])
def test_fixed_weights_and_truncation_l2(ctx, layout):
    # the graph's own weights (1 .. 40) and episodes cut at four states, in
    # both L2 placements: truncated episodes are prefixes, as in the LDS one
    base = W.ws_graph(300, 6, 0.2, 9)
    w0 = (np.random.default_rng(9).integers(1, 41, len(base.eu))).astype(np.uint32)
    g = W.canonical(base.n, np.stack([base.eu, base.ev], axis=1), w0=w0, name="ws300-fixed")
    x0 = np.arange(0, 300, 7)
    res, ref = both(ctx, g, {"p_fail": 0.08, "weight": "fixed"}, x0=x0, seed=21, alpha=0.05, max_steps=4,
                    group=1, **LAYOUTS[layout])
    check(res, ref, f"ws300 fixed weights {layout}")
    check_layout(res, layout)
    assert res["truncated"] > 0


def test_graph_beyond_the_lds_layout(ctx):
    # n = 3500, mean degree 8, weights 1..10: the LDS layout does not hold the
    # realized graph and two wavefront regions, the L2 layout holds three
    g = W.er_graph(3500, 8.0 / 3499, 21)
    model = {"p_fail": 0.1, "weight": "uniform", "w_lo": 1, "w_hi": 10}
    res, ref = both(ctx, g, model, x0=np.array([0, 1750, 3499]), seed=5, alpha=0.3, max_steps=3)
    check(res, ref, "er3500 automatic layout")
    assert res["mode"] == amc.MODE_WAVE_L2 and res["waves"] >= 2
    G = amc.Graph(ctx, g.n, g.eu, g.ev)
    with pytest.raises(amc.AmcError) as ei:
        amc.trajectories(ctx, G, model, x0=[0], mode=amc.MODE_WAVE)
    assert ei.value.rc == amc.E_UNSUPPORTED
    G.close()


def test_trajectory_arguments(ctx):
    g = W.er_graph(12, 0.4, 1)
    G = amc.Graph(ctx, g.n, g.eu, g.ev)
    for bad in ({"x0": [0, 12]}, {"x0": [-1]}, {"x0": [1], "max_steps": 0}, {"x0": [1], "alpha": 0.0},
                {"x0": [1], "f": -np.ones(12)}, {"x0": [1], "mode": amc.MODE_BLOCK},
                {"x0": [1], "flags": amc.DIST16 | amc.DIST32}, {"x0": [1], "flags": amc.TRAJ_B_LDS | amc.TRAJ_B_GLOBAL},
                {"x0": [1], "mode": amc.MODE_WAVE, "flags": amc.TRAJ_B_GLOBAL}, {"x0": [1], "flags": 1 << 20}):
        kw = dict(bad)
        x0 = kw.pop("x0")
        with pytest.raises(amc.AmcError) as ei:
            amc.trajectories(ctx, G, {"p_fail": 0.1}, x0=x0, **kw)
        assert ei.value.rc == amc.E_INVALID_ARG, bad
    G.close()
    # a path of 7000 vertices: two wavefront regions and the component list
    # exceed the LDS in every layout
    n = 7000
    H = amc.Graph(ctx, n, np.arange(n - 1), np.arange(1, n))
    with pytest.raises(amc.AmcError) as ei:
        amc.trajectories(ctx, H, {"p_fail": 0.1, "weight": "unit"}, x0=[0])
    assert ei.value.rc == amc.E_UNSUPPORTED
    H.close()


def test_er5000_l2_layout(ctx):
    # the n = 5000 workload graph (unit weights) fits only the L2 layout with
    # B in the global scratch, with two wavefronts
    wl = W.config_er5000()
    g = wl.graph
    res, ref = both(ctx, g, {"p_fail": 0.1, "weight": "unit"}, x0=np.array([0, 4999]), seed=3, alpha=0.3,
                    max_steps=2)
    check(res, ref, "er5000")
    assert (res["mode"], res["b_global"], res["waves"]) == (amc.MODE_WAVE_L2, 1, 2)
