"""amc_sweep_static (the sweep without any device allocation) against
amc_run's sweep on the same queries: counts and global centres bit-exact,
work counters and launch plan equal; two calls in a row, the second on a
smaller input, then a query whose plan needs more than the static scratch."""
import sys

import numpy as np
import pytest
import torch

from paper_2605_14743_amd import amc
from paper_2605_14743_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def static_vs_run(ctx, g, model, **q):
    G = amc.Graph(ctx, g.n, g.eu, g.ev, g.w0)
    R = q["R"]
    # outputs are caller-owned device buffers, filled with garbage first
    counts = torch.full((g.n * (g.n + 1),), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
    center = torch.full((R,), -7, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    say(f"[gpu] static sweep n={g.n} m={g.m} R={R}")
    st = amc.sweep_static(ctx, G, model, counts.data_ptr(), center.data_ptr(), **q)
    say(f"[gpu] amc_run sweep n={g.n} R={R}")
    ref = amc.run(ctx, G, model, flags=amc.SKIP_TAIL | amc.WANT_CENTER | q.pop("flags", 0), **q)
    G.close()
    got = counts.cpu().numpy().view(np.uint32).reshape(g.n, g.n + 1)
    assert np.array_equal(got, ref["counts"]), "counts differ from amc_run"
    assert np.array_equal(center.cpu().numpy(), ref["center_global"]), "centres differ from amc_run"
    for k in ("units", "sum_nK", "sum_AK", "sum_DK", "near_band", "mode", "waves", "tile", "blocks", "lds_bytes",
              "group", "adj_bytes", "dist_bytes", "b_global", "tail_split", "tail_tiles"):
        assert st[k] == ref["stats"][k], f"{k}: {st[k]} != {ref['stats'][k]}"
    assert st["sweep_ms"] > 0.0
    return st


def test_static_sweep_equals_amc_run_twice_then_smaller():
    ctx = amc.Context(0)
    ws = W.config_ws1000()
    # the benchmark's workload and plan (L2 mode, whole realizations, split
    # last realizations), then a smaller graph in the LDS mode with tiles
    st = static_vs_run(ctx, ws.graph, ws.model(), seed=ws.seed, R=600, alpha=ws.alpha, k_min=ws.k_min)
    assert st["mode"] == amc.MODE_WAVE_L2 and st["tail_split"] > 0
    er = W.config_er20()
    st = static_vs_run(ctx, er.graph, er.model(), seed=er.seed, R=300, r_begin=17, alpha=er.alpha, k_min=er.k_min)
    assert st["units"] == 300 * er.graph.n
    # 16-bit distances, unit weights, workgroup-per-source mode
    g = W.er_graph(700, 8.0 / 699, 3)
    static_vs_run(ctx, g, {"p_fail": 0.1, "weight": "unit"}, seed=2, R=40, mode=amc.MODE_BLOCK)
    static_vs_run(ctx, g, {"p_fail": 0.1, "weight": "uniform", "w_lo": 1, "w_hi": 9}, seed=2, R=40,
                  flags=amc.DIST16)
    ctx.close()


def test_static_sweep_rejects_what_it_cannot_hold():
    ctx = amc.Context(0)
    # n = 6000, weighted: L2 mode with 4-byte adjacency entries, whose
    # per-workgroup scratch over 256 workgroups exceeds the static array
    g = W.er_graph(6000, 8.0 / 5999, 6000)
    G = amc.Graph(ctx, g.n, g.eu, g.ev)
    counts = torch.zeros(g.n * (g.n + 1), dtype=torch.int32, device="cuda")
    model = {"p_fail": 0.1, "weight": "uniform", "w_lo": 1, "w_hi": 10}
    with pytest.raises(amc.AmcError) as ei:
        amc.sweep_static(ctx, G, model, counts.data_ptr(), None, seed=8, R=1)
    assert ei.value.rc == amc.E_SCRATCH
    for bad in ({"pool": np.array([1, 2])}, {"topk": 2}, {"flags": amc.WANT_NEXT_TABLE}, {"hop_radius": 1}):
        with pytest.raises(amc.AmcError) as ei:
            amc.sweep_static(ctx, G, model, counts.data_ptr(), None, seed=8, R=1, **bad)
        assert ei.value.rc == amc.E_INVALID_ARG, bad
    G.close()
    # after the rejected calls the array serves a normal call again
    er = W.config_er20()
    static_vs_run(ctx, er.graph, er.model(), seed=1, R=64)
    ctx.close()
