"""GPU systems checks: the persistent fused batch (hipGraph replays) and the
serving loop give, for every query, exactly what a standalone amc_run gives,
and every member of the mixes agrees with the CPU oracle (counts, next-state
tables and centres bit-exact; sums of B within 1e-12 relative; the tail
within 1e-12 of the max norm)."""
import sys
import time

import numpy as np
import pytest

import oracle as O
import par_oracle as P
from paper_2605_14743_amd import amc
from paper_2605_14743_amd import workloads as W

pytestmark = pytest.mark.gpu

FLAGS = amc.WANT_NEXT_TABLE | amc.WANT_CENTER | amc.WANT_BSUM


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = amc.Context(0)
    yield c
    c.close()


def mixed_items(ctx, count, R, seed=0):
    wls = W.config_mixed_batch(count=count, R=R, seed=seed)
    # keep the graphs small enough for a quick test, mixing the three sweep modes
    out, graphs = [], []
    for k, wl in enumerate(wls):
        g = wl.graph
        model = wl.model()
        if g.n > 1400 and k % 3:
            g = W.er_graph(300 + 37 * k, 6.0 / (300 + 37 * k), 900 + k)
            wl.graph = g
        if k == 2:                                   # realized graph crowds the LDS: L2 mode
            g = W.er_graph(3500, 10.0 / 3499, 77)
            wl.graph = g
            wl.R = 8
        if k == 4:                                   # unit weights, n = 4600: workgroup per source
            g = W.er_graph(4600, 8.0 / 4599, 78)
            wl.graph = g
            wl.R = 4
            model = {"p_fail": 0.1, "weight": "unit"}
        G = amc.Graph(ctx, g.n, g.eu, g.ev, g.w0)
        q = dict(seed=wl.seed, R=wl.R, alpha=wl.alpha, k_min=wl.k_min, eps=wl.eps, r_lower=wl.r_lower,
                 cert_topk=3, flags=FLAGS)
        if k == 3:
            q["pool"] = np.arange(0, g.n, 7, dtype=np.int32)
        if k == 6:                                   # anchored r-hop neighbourhoods (small graph)
            g = W.er_graph(150, 6.0 / 149, 606)
            wl.graph = g
            G.close()
            G = amc.Graph(ctx, g.n, g.eu, g.ev, g.w0)
            q.update(hop_radius=2, flags=amc.WANT_NEXT_TABLE)
        if k == 5:                                   # finite-k Top-k rewards and selector
            q.update(topk=3, pool=np.arange(1, g.n, 5, dtype=np.int32), gamma=np.linspace(0.5, 2.0, g.n))
        out.append((G, model, q))
        graphs.append(g)
    return out, graphs


def oracle_check(g, model, q, res, what):
    """One member of a mix against the oracle over the same realizations.
    Members whose full oracle run would take long are checked on sampled
    realizations (their next-state rows and centres against the oracle's,
    one realization at a time) and their counts against the histogram of the
    next-state table; the tail (up to n = 1200) is checked against the
    oracle's tail of the same counts either way."""
    pool = q.get("pool")
    R = q["R"]
    kw = dict(seed=q["seed"], alpha=q["alpha"], k_min=q["k_min"], want_next=True, pool=pool, topk=q.get("topk", 0),
              gamma=q.get("gamma"), hop_radius=q.get("hop_radius", 0), **model)
    cost = float(R) * g.n * (g.m + g.n)
    if cost <= 3e8 or "next_table" not in res:
        say(f"[cpu] oracle {what}: n={g.n} R={R}")
        ref = P.sweep(g.n, g.eu, g.ev, R=R, **kw)
        for key in ("counts", "counts_w", "next_table", "center_global"):
            if key in res and key in ref:
                assert np.array_equal(res[key], ref[key]), f"{what}: {key} differs from the oracle"
        for key in ("bsum", "psi", "psi_w"):
            if key in res and key in ref:
                assert np.allclose(res[key], ref[key] / (R if key != "bsum" else 1), rtol=1e-12, atol=0), \
                    f"{what}: {key} differs from the oracle"
        for key in ("units", "sum_nK", "sum_AK", "sum_DK"):
            assert res["stats"][key] == ref["stats"][key], f"{what}: {key}"
        counts_w = ref.get("counts_w")
    else:
        rs = sorted({0, R - 1, R // 3, (2 * R) // 3})
        say(f"[cpu] oracle {what}: n={g.n}, realizations {rs} of {R}")
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(len(rs)) as ex:
            outs = list(ex.map(lambda r: O.sweep(g.n, g.eu, g.ev, R=1, r_begin=r, **kw), rs))
        for r, o in zip(rs, outs):
            assert np.array_equal(res["next_table"][r], o["next_table"][0]), f"{what}: next table row {r}"
            if "center_global" in res:
                assert res["center_global"][r] == o["center_global"][0], f"{what}: centre {r}"
        nt = res["next_table"]
        hist = np.zeros((g.n, g.n + 1), dtype=np.int64)
        np.add.at(hist, (np.broadcast_to(np.arange(g.n), nt.shape), np.where(nt >= 0, nt, g.n)), 1)
        assert np.array_equal(hist, res["counts"].astype(np.int64)), f"{what}: counts vs next table"
        counts_w = res.get("counts_w")
    if g.n > 1200:          # the oracle's dense LU is single-threaded O(n^3); the tail is pinned elsewhere
        return
    t = O.tail(res["counts"], R, pool=pool, counts_w=counts_w, eps=q["eps"], r_lower=q["r_lower"],
               cert_topk=q["cert_topk"])
    for key in ("b", "mu"):
        scale = np.abs(t[key]).max()
        assert np.abs(res[key] - t[key]).max() <= 1e-12 * scale, f"{what}: {key} differs from the oracle"


def same(a, b, what):
    for key in ("counts", "next_table", "center_global", "counts_w"):
        if key in a:
            assert np.array_equal(a[key], b[key]), f"{what}: {key}"
    if "bsum" in a:
        assert np.allclose(a["bsum"], b["bsum"], rtol=1e-12, atol=0), f"{what}: bsum"
    for key in ("psi", "psi_w"):
        if key in a:
            assert np.allclose(a[key], b[key], rtol=1e-12, atol=0), f"{what}: {key}"
    for key in ("b", "mu", "Q"):
        assert np.allclose(a[key], b[key], rtol=0, atol=1e-13 * max(1.0, np.abs(b[key]).max())), f"{what}: {key}"
    for key in ("units", "sum_nK", "sum_AK", "sum_DK"):
        assert a["stats"][key] == b["stats"][key], f"{what}: {key}"


def test_batch_matches_standalone_runs_over_replays(ctx):
    items, graphs = mixed_items(ctx, 12, 96)
    say(f"[gpu] batch of {len(items)} graphs, n = {[G.n for G, _, _ in items]}")
    ref = [amc.run(ctx, G, model, **q) for G, model, q in items]
    modes = {r["stats"]["mode"] for r in ref}
    assert modes == {amc.MODE_WAVE, amc.MODE_BLOCK, amc.MODE_WAVE_L2}
    B = amc.Batch(ctx, items)
    info = B.info()
    assert info["launches"] >= 2
    for rep in range(3):                                  # replays, with eager work between them
        got = B.run()
        for k, (a, b) in enumerate(zip(got, ref)):
            same(a, b, f"replay {rep} query {k}")
        amc.run(ctx, items[0][0], items[0][1], **items[0][2])
    B.close()
    for k, ((G, model, q), g) in enumerate(zip(items, graphs)):
        oracle_check(g, model, q, got[k], f"batch member {k}")
    for G, _, _ in items:
        G.close()


def _overlap(times):
    """Most requests admitted at one time ([admit, finish] intervals)."""
    ev = sorted([(t[1], 1) for t in times] + [(t[2], -1) for t in times], key=lambda x: (x[0], x[1]))
    cur = peak = 0
    for _, d in ev:
        cur += d
        peak = max(peak, cur)
    return peak


def test_serving_results_equal_standalone(ctx):
    # the mix submitted at once: its queries are admitted together, their
    # items share epoch launches, and each result equals its standalone run
    # and the oracle
    items, graphs = mixed_items(ctx, 10, 64, seed=3)
    ref = [amc.run(ctx, G, model, **q) for G, model, q in items]
    say("[gpu] serving mix")
    sctx = amc.Context(0)
    sg = [amc.Graph(sctx, g.n, g.eu, g.ev, g.w0) for g in graphs]
    reqs = [amc.Request(sctx, G, model, **q) for G, (_, model, q) in zip(sg, items)]
    got = [r.wait() for r in reqs]
    for k, (a, b) in enumerate(zip(got, ref)):
        same(a, b, f"served query {k}")
    times = [r.times() for r in reqs]
    assert all(t[0] <= t[1] <= t[2] for t in times)
    info = amc.server_info(sctx)
    say(f"[gpu] server info {info}")
    assert info["admitted"] == info["completed"] == len(items)
    assert info["shared_launches"] >= 1 and info["max_members"] >= 2, info
    assert 0 < info["peak_in_use"] <= info["budget"]
    assert _overlap(times) >= 2
    for r in reqs:
        r.close()
    for G in sg:
        G.close()
    sctx.close()
    for k, ((G, model, q), g) in enumerate(zip(items, graphs)):
        oracle_check(g, model, q, got[k], f"served member {k}")


def test_serving_admits_arrivals_while_a_large_query_runs(ctx):
    # a large query first, then small ones submitted while it is on the
    # device: they are admitted at once, join its launches (shared epochs),
    # and finish before it; every result equals its standalone run
    sctx = amc.Context(0)
    big_g = W.ws_graph(1500, 10, 0.1, 21)
    big_m = {"p_fail": 0.05, "weight": "uniform", "w_lo": 1, "w_hi": 10}
    big_q = dict(seed=4, R=4096, alpha=0.15, k_min=5, flags=FLAGS)
    small = [(W.er_graph(60 + 40 * k, 6.0 / (59 + 40 * k), 300 + k), dict(seed=10 + k, R=256, alpha=0.15, k_min=5,
                                                                         flags=FLAGS)) for k in range(6)]
    model = {"p_fail": 0.1, "weight": "uniform", "w_lo": 1, "w_hi": 10}
    BG = amc.Graph(sctx, big_g.n, big_g.eu, big_g.ev)
    SG = [amc.Graph(sctx, g.n, g.eu, g.ev) for g, _ in small]
    say("[gpu] serving: large query, then arrivals")
    big = amc.Request(sctx, BG, big_m, **big_q)
    time.sleep(0.05)
    assert not big.poll(), "the large query finished before the arrivals were submitted"
    reqs = [amc.Request(sctx, G, model, **q) for G, (_, q) in zip(SG, small)]
    got = [r.wait() for r in reqs]
    got_big = big.wait()
    t_big = big.times()
    times = [r.times() for r in reqs]
    assert all(t[1] < t_big[2] for t in times), "an arrival was admitted only after the large query finished"
    assert sum(t[2] < t_big[2] for t in times) >= len(reqs) - 1
    info = amc.server_info(sctx)
    say(f"[gpu] server info {info}")
    assert info["shared_launches"] >= 1 and info["peak_active"] >= 2
    BR = amc.Graph(ctx, big_g.n, big_g.eu, big_g.ev)
    same(got_big, amc.run(ctx, BR, big_m, **big_q), "large query")
    BR.close()
    for k, ((g, q), a) in enumerate(zip(small, got)):
        G = amc.Graph(ctx, g.n, g.eu, g.ev)
        same(a, amc.run(ctx, G, model, **q), f"arrival {k}")
        G.close()
        ref = O.sweep(g.n, g.eu, g.ev, seed=q["seed"], R=q["R"], alpha=0.15, k_min=5, want_next=True, **model)
        assert np.array_equal(a["counts"], ref["counts"]) and np.array_equal(a["next_table"], ref["next_table"])
    big.close()
    for r in reqs:
        r.close()
    for G in SG + [BG]:
        G.close()
    sctx.close()


def test_serving_admission_by_footprint():
    probe = amc.Context(0)
    h = W.er_graph(200, 0.03, 5)
    fp = amc.footprint(amc.Graph(probe, h.n, h.eu, h.ev), R=64)
    probe.close()
    budget = 3 * fp + fp // 2                          # room for three such queries at a time
    small = amc.Context(0, budget_bytes=budget)
    g = W.er_graph(3000, 8.0 / 2999, 4)
    G = amc.Graph(small, g.n, g.eu, g.ev)
    with pytest.raises(amc.AmcError) as ei:           # n^2 tail matrices alone exceed the budget
        amc.Request(small, G, {"p_fail": 0.1}, R=8)
    assert ei.value.rc == amc.E_ADMISSION
    H = amc.Graph(small, h.n, h.eu, h.ev)
    assert amc.footprint(H, R=64) == fp
    reqs = [amc.Request(small, H, {"p_fail": 0.1}, R=64, seed=s) for s in range(6)]
    outs = [r.wait() for r in reqs]
    assert all(o["counts"].sum() == 64 * 200 for o in outs)
    info = amc.server_info(small)
    # queries ran side by side, and the admitted footprints never passed the budget
    assert fp < info["peak_in_use"] <= 3 * fp <= info["budget"] == budget, info
    for r in reqs:
        r.close()
    G.close()
    H.close()
    small.close()


def test_autotuner_choice_is_used_and_exact(ctx, tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("AMC_TUNE_CACHE", str(cache))
    c2 = amc.Context(0)                      # reads (empty) cache at creation
    g = W.ws_graph(600, 8, 0.1, 11)
    G = amc.Graph(c2, g.n, g.eu, g.ev)
    model = {"p_fail": 0.1, "weight": "uniform", "w_lo": 1, "w_hi": 10}
    say("[gpu] autotune ws600")
    t = amc.tune(c2, G, model, probe_R=24, R=24, seed=3)
    assert t["candidates"] >= 2 and t["units_per_s"] > 0
    res = amc.run(c2, G, model, R=40, seed=3, flags=FLAGS | amc.SKIP_TAIL)
    assert res["stats"]["mode"] == t["mode"]
    if t["mode"] != amc.MODE_BLOCK:
        assert res["stats"]["group"] == t["group"]
    ref = amc.run(c2, G, model, R=40, seed=3, flags=FLAGS | amc.SKIP_TAIL, mode=amc.MODE_BLOCK)
    assert np.array_equal(res["counts"], ref["counts"]) and np.array_equal(res["next_table"], ref["next_table"])
    line = cache.read_text().split()
    assert [int(x) for x in line[:3]] == [g.n, g.m, 1]
    G.close()
    c2.close()
    c3 = amc.Context(0)                      # a new context picks the stored choice up
    H = amc.Graph(c3, g.n, g.eu, g.ev)
    res3 = amc.run(c3, H, model, R=8, seed=3, flags=amc.SKIP_TAIL)
    assert res3["stats"]["mode"] == t["mode"]
    H.close()
    c3.close()
