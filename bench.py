"""Benchmark: realization-sources per second of the AFC hot path on one MI355X.

One step is one full estimation of the Watts-Strogatz workload (n = 1000,
k = 10, beta = 0.1, seed 0; edge failure 0.05; integer weights uniform on
{1..10}; 10,000 realizations; alpha = 0.15, k_min = 5): the realization x
source sweep (Alg. 1 for every anchor, counted as in Alg. 2) plus the FP64
tail (N, mu, b, certificates), with the graph already staged in HBM.

Printed as one JSON line:
  value        whole-job realization-sources/s (R n per step / step time)
  roofline     the resource that bounds the sweep kernel.  The traversal
               state never leaves the chip, so HBM does not bind it: the
               kernel is bound by VALU issue ("alu": wave64 VALU instructions
               per (r, s) from the SQ counter profile of the same kernel
               sources, times the units of one launch, over the launch's
               HIP-event duration, against 256 CUs x 4 SIMDs x 2.4 GHz / 4
               cycles).  Beside it: measured HBM bytes (FETCH_SIZE /
               WRITE_SIZE, calibrated by a plain copy) against the 8 TB/s
               peak, LDS-unit busy cycles against the chip's cycles, and the
               algorithmic bytes (8 D_K + 32 A_K + 64 n_K per (r, s), counted
               exactly by the kernel) as an HBM-equivalent rate.
  teps         surviving undirected edges of s's component per (r, s) / s
  plain_gpu    the same sweep as one kernel launch per realization
  er5000       one step of the n = 5000 unit-weight workload
  serving      a bounded Poisson trace through the serving loop: p50 / p99
  cpu_baseline the CPU oracle on all host cores (one process per core over
               disjoint realization ranges) on a bounded sample
Options: --serve runs the serving trace alone, --batch the mixed batch.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CUS, CLOCK_GHZ = 256, 2.4
VALU_PEAK_GIPS = CUS * 4 * CLOCK_GHZ / 4    # 614.4 G wave64 instructions/s: 4 SIMDs per CU, 4 cycles each
PLAIN_TARGET = 10.0                         # batched sweep over the one-launch-per-realization form


def algorithmic_bytes(st: dict) -> int:
    """Bytes a traversal must move per (r, s) if nothing is cached:
    8 per base slot of K (neighbour index, two passes), 32 per surviving slot
    (distance + path count forward, distance + count + dependency backward),
    64 per reached vertex (offsets, state writes, B update, queue)."""
    return 8 * st["sum_DK"] + 32 * st["sum_AK"] + 64 * st["sum_nK"]


WORKLOADS = ("ws1000", "er5000", "er20", "cooc77")


def _workload(name):
    from paper_2605_14743_amd import workloads as W
    return {"ws1000": W.config_ws1000, "er5000": W.config_er5000, "er20": W.config_er20,
            "cooc77": W.config_cooc77}[name]()


def _cpu_worker(task):
    """One oracle process over its own realization range."""
    name, r0, budget_s = task
    import oracle as O
    wl = _workload(name)
    g = wl.graph
    R = units = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        res = O.sweep(g.n, g.eu, g.ev, seed=wl.seed, R=1, r_begin=r0 + R, alpha=wl.alpha, k_min=wl.k_min,
                      want_bsum=False, want_center=False, hop_radius=wl.hop_radius, **wl.model())
        units += res["stats"]["units"]
        R += 1
    return units, R, time.perf_counter() - t0


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_cores() -> int:
    """Host cores the oracle may use: the process's CPU set, at most 16 (one
    GPU's share of a shared host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(name: str, procs: int, budget_s: float) -> dict:
    """The oracle in `procs` fresh processes (spawned, never forked from this
    GPU process) over disjoint realization ranges; rate = all units / the
    slowest process's time.  The oracle is single-threaded C as it stands."""
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(procs) as pool:
        out = pool.map(_cpu_worker, [(name, 1_000_000 * (k + 1), budget_s) for k in range(procs)])
    units = sum(u for u, _, _ in out)
    reals = sum(r for _, r, _ in out)
    dt = max(t for _, _, t in out)
    return {"value": units / dt, "unit": "realization-sources/s", "cores": procs, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{reals} realizations of the {name} workload ({units} single-source passes) in {procs} "
                      f"oracle processes over disjoint realization ranges, {dt:.1f} s"}


# Sources each kernel's counter profile depends on: the kernel, the device
# helpers it includes, and the planner / layout code that chooses its
# launch shape, tiles and split of the last realizations.
PLANNER_SOURCES = ("amc_api.cpp", "query.cpp", "amc_kernels.hpp", "amc_runtime.hpp")
KERNEL_SOURCES = {
    "sweep_wave": ("amc_dev.hpp", "sweep_common.hpp", "wave_source.hpp", "sweep_wave.hip") + PLANNER_SOURCES,
    "sweep_block": ("amc_dev.hpp", "sweep_common.hpp", "sweep_block.hip") + PLANNER_SOURCES,
}
COUNTER_RECORDS = {"ws1000": ("sweep_wave", "sweep_wave_ws1000_R10000_counters.json"),
                   "er5000": ("sweep_block", "sweep_block_er5000_R4096_counters.json")}


def kernel_source_digest(kernel: str = "sweep_wave") -> str:
    """Digest of the sources a sweep kernel and its launch plan are built from."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2605_14743_amd", "csrc")
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()


def counter_record(workload: str):
    """The committed counter profile of a workload's sweep kernel (HBM bytes,
    VALU instructions and LDS busy cycles per unit), or None when the kernel
    or its planner has changed since the counters were taken."""
    if workload not in COUNTER_RECORDS:
        return None
    kernel, fname = COUNTER_RECORDS[workload]
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_sha256") != kernel_source_digest(kernel):
        return None
    rec["source"] = "profiles/" + fname
    return rec


def roofline(st: dict, k_ms: float, rec) -> dict:
    """Roofline of one sweep launch (units st["units"], HIP-event time k_ms).

    bound "alu": wave64 VALU instructions issued per second (instructions per
    (r, s) from the SQ_INSTS_VALU profile x units / launch time) against the
    VALU issue peak.  Secondary: measured HBM bytes (calibrated FETCH_SIZE +
    WRITE_SIZE) against the HBM peak, the LDS unit's busy cycles
    (SQ_LDS_IDX_ACTIVE) against the CU cycles of the launch, and the
    algorithmic bytes as an HBM-equivalent rate (above the HBM peak when the
    state lives on chip)."""
    t = k_ms * 1e-3
    units = st["units"]
    ab = algorithmic_bytes(st)
    alg = {"bytes_per_launch": ab, "units_per_launch": units, "GBps": ab / t / 1e9,
           "frac_of_hbm_peak": ab / t / 1e9 / HBM_PEAK_GBS,
           "note": "HBM-equivalent rate of 8 D_K + 32 A_K + 64 n_K bytes per (r, s); the traversal state is "
                   "on chip, so these bytes never cross HBM"}
    out = {"bound": "alu", "achieved": None, "peak": VALU_PEAK_GIPS, "unit": "G wave64 VALU instructions/s",
           "frac": None, "traffic": None, "algorithmic": alg}
    if rec is None:
        out["note"] = "no counter profile of the current kernel sources"
        return out
    valu = rec["valu_insts_per_unit"] * units / t / 1e9
    out.update(achieved=valu, frac=valu / VALU_PEAK_GIPS, traffic=rec["hbm_bytes_per_unit"] * units,
               source=rec["source"])
    hbm = rec["hbm_bytes_per_unit"] * units / t / 1e9
    out["hbm"] = {"achieved": hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hbm / HBM_PEAK_GBS}
    if "lds_idx_active_per_unit" in rec:
        cu_cycles = CUS * CLOCK_GHZ * 1e9 * t
        busy = rec["lds_idx_active_per_unit"] * units
        out["lds"] = {"busy_cycles": busy, "cu_cycles": cu_cycles, "frac": busy / cu_cycles,
                      "bank_conflict_share": rec.get("lds_bank_conflict_per_unit", 0.0) /
                      max(rec["lds_idx_active_per_unit"], 1e-30)}
    return out


def run_workload(ctx, amc, wl, q, steps, warmup):
    """`warmup` + `steps` synchronous estimations; returns the last result,
    the mean HIP-event times and the wall time of the timed steps."""
    import torch
    G = amc.Graph(ctx, wl.graph.n, wl.graph.eu, wl.graph.ev, wl.graph.w0)
    model = wl.model()
    last = None
    for _ in range(warmup):
        last = amc.run(ctx, G, model, out=last, **q)
    torch.cuda.synchronize()
    sweep_ms, tail_ms, topk_ms = [], [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        # every step recomputes and copies back all results, into the host
        # buffers the previous step used (no fresh allocation per step)
        last = amc.run(ctx, G, model, out=last, **q)
        sweep_ms.append(last["stats"]["sweep_ms"])
        tail_ms.append(last["stats"]["tail_ms"])
        topk_ms.append(last["stats"]["topk_ms"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    G.close()
    return last, float(np.mean(sweep_ms)), float(np.mean(tail_ms)), float(np.mean(topk_ms)), dt


def base_query(wl, args=None) -> dict:
    q = dict(seed=wl.seed, R=wl.R, alpha=wl.alpha, k_min=wl.k_min, cert_topk=wl.cert_topk, eps=0.01,
             r_lower=wl.r_lower, pool=wl.pool, reward=wl.reward, hop_radius=wl.hop_radius)
    if args is not None:
        q.update(mode=args.mode, waves=args.waves, tile=args.tile, group=args.group)
    return q


def er5000_leg(ctx, amc) -> dict:
    """One step of the n = 5000 unit-weight workload (R = 4096, pool of 50
    with rewards) with its own rate, TEPS and roofline."""
    wl = _workload("er5000")
    last, k_ms, t_ms, _, dt = run_workload(ctx, amc, wl, base_query(wl), 1, 0)
    st = last["stats"]
    return {"workload": wl.name, "value": st["units"] / dt, "unit": "realization-sources/s", "ms_per_step": dt * 1e3,
            "sweep_kernel_ms": k_ms, "tail_ms": t_ms, "teps": (st["sum_AK"] / 2) / (k_ms * 1e-3),
            "near_band": st["near_band"],
            "plan": {k: st[k] for k in ("mode", "waves", "tile", "blocks", "lds_bytes", "group", "dist_bytes",
                                        "b_global", "tail_split")},
            "roofline": roofline(st, k_ms, counter_record("er5000"))}


def serving_leg(amc, queries: int, logR_hi: int, load: float) -> dict:
    """Bounded serving trace: `queries` mixed-size queries (n log-uniform in
    [50, 4000], R = 2^U{8..logR_hi}) submitted all at once to measure the
    loop's capacity, then the same queries as a Poisson trace at `load` x
    that capacity; latency = finish - submit."""
    from paper_2605_14743_amd import workloads as W
    cap = serve_trace(amc, W.serving_trace(count=queries, rate=1e9, seed=1, logR_hi=logR_hi))
    rate = load * cap["throughput_qps"]
    run = serve_trace(amc, W.serving_trace(count=queries, rate=rate, seed=1, logR_hi=logR_hi))
    return {"queries": queries, "R_max": 2 ** logR_hi, "capacity_qps": cap["throughput_qps"],
            "offered_qps": rate, "load": load, **{k: run[k] for k in ("throughput_qps", "value", "p50_ms", "p99_ms",
                                                                       "wall_s", "max_overlap", "shared_launches")},
            "saturated": {k: cap[k] for k in ("p50_ms", "p99_ms", "wall_s", "value", "max_overlap")}}


def run_bench(args):
    import torch

    from paper_2605_14743_amd import amc
    from paper_2605_14743_amd import workloads as W

    wl = _workload(args.workload)
    g = wl.graph
    if args.R:
        wl.R = args.R
    ctx = amc.Context(0)
    q = base_query(wl, args)
    if args.dist32:
        q["flags"] = amc.DIST32
    if args.topk > 0:
        # finite-k local Top-k rows: a pool of 50 nodes with values U[0.5, 2]
        pool = wl.pool if wl.pool is not None else W.pool(g.n, 50, 1)
        gamma = wl.reward if wl.reward is not None else W.rewards(g.n, pool, 0.5, 2.0, 1)
        q.update(topk=args.topk, pool=pool, gamma=gamma)
        if args.clique_pool > 0:
            # structure-constrained selection: W = the best 3-cliques by degree
            # sum, fallback to the smallest vertex of the first one
            pool, fb, _ = W.clique_pool(g, args.clique_pool)
            q.update(pool=pool, fb_node=fb, reward=None, gamma=None)
    model = wl.model()
    last, k_ms, tail_ms, topk_ms, dt = run_workload(ctx, amc, wl, q, args.steps, args.warmup)
    G = amc.Graph(ctx, g.n, g.eu, g.ev, g.w0)
    st = last["stats"]
    units = st["units"]                      # single-source passes (R n for the row-wise sweep)
    value = units * args.steps / dt
    teps = (st["sum_AK"] / 2) / (k_ms * 1e-3)
    # the recorded counters belong to the default configuration of this workload
    default_cfg = not (args.R or args.mode or args.waves or args.tile or args.group or args.dist32 or args.topk)
    rec = counter_record(args.workload) if default_cfg else None
    out = {
        "metric": "realization-sources/sec",
        "value": value,
        "unit": "realization-sources/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "graph": g.name, "n": g.n, "hop_radius": wl.hop_radius,
                   "m": g.m, "realizations": wl.R, "p_fail": wl.p_fail,
                   "weights": wl.weight if wl.weight != "uniform" else f"uniform{{{wl.w_lo}..{wl.w_hi}}}",
                   "alpha": wl.alpha, "k_min": wl.k_min, "mode": st["mode"], "waves": st["waves"],
                   "tile": st["tile"], "blocks": st["blocks"], "lds_bytes": st["lds_bytes"], "group": st["group"],
                   "adj_bytes": st["adj_bytes"], "dist_bytes": st["dist_bytes"], "b_global": st["b_global"],
                   "tail_split": st["tail_split"]},
        "sweep_kernel_ms": k_ms,
        "tail_ms": tail_ms,
        "teps": teps,
        # set members whose gap to the set maximum lies within [tau/4, 4 tau]
        # of the tie band: where the two sides' rounding could decide a tie
        "near_band": st["near_band"],
        "roofline": roofline(st, k_ms, rec),
    }
    if args.topk > 0:
        # the Top-k stage reads every realization's B row and labels once
        # (16 B per vertex) and adds one step reward per valid anchor
        tb = 16.0 * wl.R * g.n
        out["topk_stage"] = {"k": args.topk, "pool": int(len(q["pool"])), "ms": topk_ms, "bytes_read": tb,
                             "GBps": tb / (topk_ms * 1e-3) / 1e9, "b_k": last["b_k"], "b_kw": last["b_kw"],
                             "share_of_step": topk_ms / (dt / args.steps * 1e3)}
        if args.clique_pool > 0:
            out["topk_stage"].update({"clique_pool": args.clique_pool, "fb_node": int(q["fb_node"]),
                                      "m_w_fb": last["m_w_fb"], "c_fb": last["c_fb"], "E_T_fb": last["E_T_fb"],
                                      "top5_b_fb": np.argsort(-last["b_fb"], kind="stable")[:5].tolist()})
    def robust_leg():
        # robust tail on the estimated kernel: (samples + 2) Gauss-Jordan
        # inversions (2 n^3 flops each) and two n x n products (2 n^3 each);
        # node values: the multi-reward value of the robust experiment
        f = W.multi_reward(g)
        amc.robust(ctx, last["Q"], f=f, samples=2, delta=0.5, r_min=0.05, seed=1)
        rb = amc.robust(ctx, last["Q"], f=f, samples=args.robust, delta=0.5, r_min=0.05, seed=1)
        flops = (args.robust + 2) * 2.0 * g.n ** 3 + 2 * 2.0 * g.n ** 3
        w1 = {}
        if g.n <= amc.MAX_W1_N:
            # W1 on the hop metric of the base topology: one transshipment per sample
            rw = amc.robust(ctx, last["Q"], f=f, samples=args.robust, delta=0.5, r_min=0.05, seed=1,
                            topology=(g.eu, g.ev))
            w1 = {"w1_max": float(rw["w1"].max()), "w1_arg": rw["w1_arg"], "kl_arg": rw["kl_arg"],
                  "w1_ms": rw["tail_ms"] - rb["tail_ms"]}
        return {"samples": args.robust, "ms": rb["tail_ms"], "fp64_TFLOPs": flops / (rb["tail_ms"] * 1e-3)
                / 1e12, "peak_fp64_TFLOPs": 78.6, "kl_max": float(rb["kl"].max()),
                "tv_max": float(rb["tv"].max()), "norm_N0E": rb["norm_N0E"],
                "rem_bound": rb["rem_bound"], "rem_actual": rb["rem_actual"],
                "b_switch": rb["b_sw"], "b_improve": rb["b_imp"], **w1}

    if args.robust > 0:
        secondary(out, "robust_tail", robust_leg)

    def bootstrap_leg():
        # bootstrap of b from this run's draws (outside the timed region): B
        # replicates of n R redrawn indices, B + 1 Gauss-Jordan inversions
        nt = amc.run(ctx, G, model, **dict(q, flags=q.get("flags", 0) | amc.WANT_NEXT_TABLE))["next_table"]
        amc.bootstrap(ctx, nt, replicates=2, seed=1, want_reps=False)
        bs = amc.bootstrap(ctx, nt, replicates=args.bootstrap, seed=1, want_reps=False)
        flops = (args.bootstrap + 1) * 2.0 * g.n ** 3
        return {"replicates": args.bootstrap, "ms": bs["ms"],
                "fp64_TFLOPs": flops / (bs["ms"] * 1e-3) / 1e12, "peak_fp64_TFLOPs": 78.6,
                "median_sd_over_b": float(np.median(bs["sd"] / np.maximum(bs["b0"], 1e-300))),
                "widest_interval": float((bs["hi"] - bs["lo"]).max())}

    if args.bootstrap > 0:
        secondary(out, "bootstrap", bootstrap_leg)

    def stability_leg():
        # rank-stability check: Top-k by b at M = R / 2 and at 2M = R
        qs = {k: v for k, v in q.items()
              if k not in ("pool", "reward", "topk", "gamma", "flags", "cert_topk", "fb_node")}
        qs["R"] = max(wl.R // 2, 1)
        if args.dist32:
            qs["flags"] = amc.DIST32
        sb = amc.stability(ctx, G, model, k=args.stability, **qs)
        return {"k": args.stability, "M": qs["R"], "same_set": sb["same_set"], "overlap": sb["overlap"],
                "max_abs_diff": sb["max_abs_diff"], "sweep_ms": sb["sweep_ms"],
                "top_M": sb["top_M"].tolist(), "top_2M": sb["top_2M"].tolist()}

    if args.stability > 0:
        secondary(out, "stability", stability_leg)
    if args.plain_R > 0:
        qp = dict(q, R=args.plain_R, flags=amc.PLAIN_LAUNCH | amc.SKIP_TAIL)
        amc.run(ctx, G, model, **qp)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rp = amc.run(ctx, G, model, **qp)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - t1
        pv = args.plain_R * g.n / dtp
        qb = dict(q, R=args.plain_R, flags=amc.SKIP_TAIL)
        rb = amc.run(ctx, G, model, **qb)
        out["plain_gpu"] = {"value": pv, "unit": "realization-sources/s", "realizations": args.plain_R,
                            "launches": rp["stats"]["launches"], "sweep_ms": rp["stats"]["sweep_ms"],
                            "batched_sweep_ms_same_R": rb["stats"]["sweep_ms"],
                            "batched_over_plain": value / pv, "target": PLAIN_TARGET,
                            "target_met": value / pv >= PLAIN_TARGET}
    if args.traj_leg > 0:
        secondary(out, "trajectories", lambda: traj_leg(ctx, amc, wl, G, args.traj_leg, args.max_steps, last["E_T"]))
    G.close()
    if args.er5000 and args.workload == "ws1000":
        out["er5000"] = er5000_leg(ctx, amc)
    if args.copy_mib > 0:
        # calibration kernel for the HBM byte counters: a plain device copy of
        # known size on the same stream
        a = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = args.copy_mib << 20
    ctx.close()
    if args.serve_queries > 0 and args.workload == "ws1000":
        out["serving"] = serving_leg(amc, args.serve_queries, args.serve_logR_hi, args.serve_load)
    if args.cpu_s > 0:
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_procs or cpu_cores(), args.cpu_s)
    print(json.dumps(out), flush=True)


def run_batch(args):
    """Uneven-size batch (64 graphs by default) in persistent fused launches
    replayed from one hipGraph; value = realization-sources/s of a replay."""
    import torch

    from paper_2605_14743_amd import amc
    from paper_2605_14743_amd import workloads as W

    wls = W.config_mixed_batch(count=args.batch_count, R=args.R or 2048, seed=0)
    ctx = amc.Context(0)
    graphs = [amc.Graph(ctx, wl.graph.n, wl.graph.eu, wl.graph.ev, wl.graph.w0) for wl in wls]
    items = [(G, wl.model(), dict(seed=wl.seed, R=wl.R, alpha=wl.alpha, k_min=wl.k_min, eps=wl.eps,
                                  r_lower=wl.r_lower, cert_topk=5)) for G, wl in zip(graphs, wls)]
    tuned = 0
    if args.tune:
        t0 = time.perf_counter()
        for G, model, q in items:
            amc.tune(ctx, G, model, probe_R=8, **{k: v for k, v in q.items() if k != "R"}, R=8)
            tuned += 1
        print(f"# tuned {tuned} graphs in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    B = amc.Batch(ctx, items)
    t_build = time.perf_counter() - t0
    print(f"# batch built in {t_build:.1f} s: {B.info()}", file=sys.stderr, flush=True)
    for k in range(args.warmup):
        t1 = time.perf_counter()
        B.run()
        print(f"# warm-up replay {k}: {time.perf_counter() - t1:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(args.steps):
        res = B.run()
        print(f"# replay {k}: {time.perf_counter() - t1:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t1) / args.steps
    units = sum(wl.R * wl.graph.n for wl in wls)
    st = [r["stats"] for r in res]
    ab = sum(algorithmic_bytes(x) for x in st)
    graph_ms = st[0]["sweep_ms"]
    out = {"metric": "realization-sources/sec", "value": units / dt, "unit": "realization-sources/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"mixed-batch-{len(wls)}", "graphs": len(wls),
                      "n_range": [min(w.graph.n for w in wls), max(w.graph.n for w in wls)],
                      "realizations_each": wls[0].R, "units": units, "tuned": tuned, **B.info()},
           "graph_replay_ms": graph_ms, "build_s": t_build,
           "teps": sum(x["sum_AK"] for x in st) / 2 / (graph_ms * 1e-3),
           "algorithmic_GBps": ab / (graph_ms * 1e-3) / 1e9}
    B.close()
    for G in graphs:
        G.close()
    ctx.close()
    print(json.dumps(out), flush=True)


def secondary(out: dict, key: str, leg) -> None:
    """Runs a secondary leg of the bench line; an error is recorded under its
    key (the headline line is still printed), not hidden."""
    try:
        out[key] = leg()
    except Exception as e:  # noqa: BLE001 -- recorded in the line
        print(f"# {key} leg failed: {type(e).__name__}: {e}", file=sys.stderr, flush=True)
        out[key] = {"error": f"{type(e).__name__}: {e}"}


def traj_leg(ctx, amc, wl, G, E, max_steps, row_E_T):
    """Bounded trajectory leg of the bench line: E episodes of the network
    process on the workload graph (Section 4.3), X_0 stratified over the
    vertices, after a 256-episode warm-up."""
    g = wl.graph
    x0 = np.arange(E) % g.n
    kw = dict(seed=wl.seed + 1, x0=x0, alpha=wl.alpha, k_min=wl.k_min, max_steps=max_steps)
    amc.trajectories(ctx, G, wl.model(), **dict(kw, x0=x0[:min(E, 256)]))
    tr = amc.trajectories(ctx, G, wl.model(), **kw)
    ms = tr["sweep_ms"]
    return {"episodes": E, "kernel_ms": ms, "episodes_per_s": E / (ms * 1e-3),
            "realization_sources_per_s": tr["sources"] / (ms * 1e-3), "steps": tr["total_steps"],
            "mean_T": tr["total_steps"] / E, "row_wise_E_T": row_E_T, "max_T": int(tr["lengths"].max()),
            "shared_sources": tr["shared_sources"],
            "layout": {"graph": "l2" if tr["mode"] == amc.MODE_WAVE_L2 else "lds",
                       "b": "global" if tr["b_global"] else "lds", "dist_bits": 16 if tr["dist16"] else 32,
                       "waves": tr["waves"]}}


def run_traj(args):
    """Trajectory simulator (episodes of the network process, Section 4.3) on
    the workload graph, with the row-wise b beside the length-biased b_hat."""
    import torch

    from paper_2605_14743_amd import amc
    from paper_2605_14743_amd import workloads as W

    wl = {"ws1000": W.config_ws1000, "er5000": W.config_er5000, "er20": W.config_er20,
          "cooc77": W.config_cooc77}[args.workload]()
    g = wl.graph
    ctx = amc.Context(0)
    G = amc.Graph(ctx, g.n, g.eu, g.ev, g.w0)
    E = args.traj
    x0 = np.arange(E) % g.n                                      # uniform s, stratified
    kw = dict(seed=wl.seed + 1, x0=x0, alpha=wl.alpha, k_min=wl.k_min, max_steps=args.max_steps)
    amc.trajectories(ctx, G, wl.model(), **dict(kw, x0=x0[:min(E, 256)]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr = amc.trajectories(ctx, G, wl.model(), **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"# trajectories: {E} episodes in {dt:.2f} s", file=sys.stderr, flush=True)
    R = args.R or wl.R
    row = amc.run(ctx, G, wl.model(), seed=wl.seed, R=R, alpha=wl.alpha, k_min=wl.k_min)
    diff = np.abs(tr["b_hat"] - row["b"])
    out = {
        "metric": "episodes/sec", "value": E / dt, "unit": "episodes/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{wl.name}-trajectories", "episodes": E, "max_steps": args.max_steps},
        "kernel_ms": tr["sweep_ms"], "realization_sources_per_s": tr["sources"] / (tr["sweep_ms"] * 1e-3),
        "steps": tr["total_steps"], "mean_T": tr["total_steps"] / E, "max_T": int(tr["lengths"].max()),
        "truncated": tr["truncated"],
        "layout": {"graph": "l2" if tr["mode"] == amc.MODE_WAVE_L2 else "lds",
                   "b": "global" if tr["b_global"] else "lds", "dist_bits": 16 if tr["dist16"] else 32,
                   "waves": tr["waves"]},
        "row_wise_R": R, "row_wise_E_T": row["E_T"],
        "b_hat_vs_row_b": {"max_abs": float(diff.max()), "l1": float(diff.sum()),
                           "b_row_max": float(row["b"].max())},
    }
    G.close()
    ctx.close()
    print(json.dumps(out), flush=True)


def serve_trace(amc, trace, ctx_budget: int = 0, progress: bool = False) -> dict:
    """Runs a trace [(arrival_s, Workload)] through amc_submit; latency of a
    query = its finish time - its submit time.  progress: a stderr line
    about every 20 s of waiting, with the queries completed so far."""
    import torch
    ctx = amc.Context(0, budget_bytes=ctx_budget)
    graphs = [amc.Graph(ctx, wl.graph.n, wl.graph.eu, wl.graph.ev) for _, wl in trace]
    torch.cuda.synchronize()
    reqs = []
    t0 = time.perf_counter()
    for (ts, wl), G in zip(trace, graphs):
        now = time.perf_counter() - t0
        if ts > now:
            time.sleep(ts - now)
        reqs.append(amc.Request(ctx, G, wl.model(), seed=wl.seed, R=wl.R, alpha=wl.alpha, k_min=wl.k_min,
                                cert_topk=5, eps=wl.eps, r_lower=wl.r_lower))
    lat, spans = [], []
    t_note = time.perf_counter()
    for i, r in enumerate(reqs):
        while progress and not r.poll():
            time.sleep(0.05)
            if time.perf_counter() - t_note > 20.0:
                t_note = time.perf_counter()
                done = sum(x.poll() for x in reqs)
                print(f"# serving: {done} of {len(reqs)} queries completed at {t_note - t0:.0f} s", file=sys.stderr,
                      flush=True)
        r.wait()
        t = r.times()
        lat.append(t[2] - t[0])
        spans.append((t[1], t[2]))
    dt = time.perf_counter() - t0
    # most queries admitted at one time (their [admit, finish] intervals overlap)
    ev = sorted([(a, 1) for a, _ in spans] + [(b, -1) for _, b in spans], key=lambda x: (x[0], x[1]))
    cur = peak = 0
    for _, d in ev:
        cur += d
        peak = max(peak, cur)
    info = amc.server_info(ctx)
    units = sum(wl.R * wl.graph.n for _, wl in trace)
    lat = np.array(lat)
    out = {"value": units / dt, "unit": "realization-sources/s", "queries": len(trace), "wall_s": dt,
           "throughput_qps": len(trace) / dt, "p50_ms": float(np.percentile(lat, 50) * 1e3),
           "p99_ms": float(np.percentile(lat, 99) * 1e3), "max_overlap": peak, **info}
    for r in reqs:
        r.close()
    for G in graphs:
        G.close()
    ctx.close()
    return out


def run_serve(args):
    """Poisson trace of mixed-size queries through amc_submit (continuous
    batching); reports throughput and p50/p99 latency."""
    from paper_2605_14743_amd import amc
    from paper_2605_14743_amd import workloads as W

    trace = W.serving_trace(count=args.queries, rate=args.rate, seed=0, n_hi=args.n_hi, logR_hi=args.logR_hi)
    res = serve_trace(amc, trace, progress=True)
    out = {"metric": "realization-sources/sec", "n_gpus": 1, "rate": args.rate, "data": "synthetic",
           "higher_is_better": True, **res,
           "config": {"workload": "poisson-serving", "n_hi": args.n_hi, "logR_hi": args.logR_hi}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="ws1000", choices=["ws1000", "er5000", "er20", "cooc77"],
                    help="ws1000 is the benchmark line; the others are for measurement notes")
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--R", type=int, default=0, help="override the realization count (testing only)")
    ap.add_argument("--mode", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--group", type=int, default=0)
    ap.add_argument("--dist32", action="store_true", help="32-bit distance entries (comparison runs)")
    ap.add_argument("--plain-R", dest="plain_R", type=int, default=200)
    ap.add_argument("--cpu-s", dest="cpu_s", type=float, default=12.0)
    ap.add_argument("--er5000", type=int, default=1, help="1: add one step of the n = 5000 workload")
    ap.add_argument("--serve-queries", dest="serve_queries", type=int, default=32,
                    help="queries of the bounded serving leg (0 = none)")
    ap.add_argument("--serve-logR-hi", dest="serve_logR_hi", type=int, default=12)
    ap.add_argument("--serve-load", dest="serve_load", type=float, default=0.8)
    ap.add_argument("--cpu-procs", dest="cpu_procs", type=int, default=0,
                    help="also time the oracle in this many processes over disjoint realization ranges")
    ap.add_argument("--topk", type=int, default=0, help="also run the finite-k local Top-k rows with this k")
    ap.add_argument("--clique-pool", dest="clique_pool", type=int, default=0,
                    help="with --topk: pool = the best 3-cliques by degree sum, with the fallback inside it")
    ap.add_argument("--traj", type=int, default=0, help="run the trajectory simulator with this many episodes")
    ap.add_argument("--robust", type=int, default=-1,
                    help="also run the robust tail with this many sampled kernels (-1: 100 on ws1000, else 0)")
    ap.add_argument("--bootstrap", type=int, default=-1,
                    help="also bootstrap b with this many replicates (-1: 100 on ws1000, else 0)")
    ap.add_argument("--stability", type=int, default=-1,
                    help="also check the Top-k set at R/2 and R for this k (-1: 10 on ws1000, else 0)")
    ap.add_argument("--traj-leg", dest="traj_leg", type=int, default=-1,
                    help="episodes of the trajectory leg of the bench line (-1: 5000 on ws1000, else 0)")
    ap.add_argument("--max-steps", dest="max_steps", type=int, default=512)
    ap.add_argument("--copy-mib", dest="copy_mib", type=int, default=0,
                    help="also run a device copy of this many MiB (counter calibration)")
    ap.add_argument("--serve", action="store_true")
    ap.add_argument("--batch", action="store_true", help="run the mixed-size batch instead")
    ap.add_argument("--batch-count", dest="batch_count", type=int, default=64)
    ap.add_argument("--tune", action="store_true", help="autotune every graph before building the batch")
    ap.add_argument("--queries", type=int, default=64)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--n-hi", dest="n_hi", type=int, default=4000)
    ap.add_argument("--logR-hi", dest="logR_hi", type=int, default=14)
    args = ap.parse_args()
    for name, dflt in (("robust", 100), ("bootstrap", 100), ("stability", 10), ("traj_leg", 5000)):
        if getattr(args, name) < 0:
            setattr(args, name, dflt if args.workload == "ws1000" and not args.traj else 0)
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the sweep would shard across "
              f"GPUs by realization range, with one all-reduce of the counts).", file=sys.stderr)
        sys.exit(2)
    if os.environ.get("WORLD_SIZE", "1") != "1":
        print("bench.py runs as a single process on one GPU", file=sys.stderr)
        sys.exit(2)
    if args.traj > 0:
        run_traj(args)
    elif args.serve:
        run_serve(args)
    elif args.batch:
        run_batch(args)
    else:
        run_bench(args)


if __name__ == "__main__":
    main()
