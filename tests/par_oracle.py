"""Test helper: the oracle's sweep over disjoint realization ranges in threads.

Realization r is a pure function of (seed, r), so the oracle's outputs over
[r0, r0 + R) are the combination of its outputs over any partition of that
range: counts (and pool counts, step-reward sums, work counters) add up,
per-realization tables and centres concatenate, and the sum of B adds up
within rounding.  The C oracle keeps no global state and ctypes releases the
interpreter lock during the call, so the ranges run in parallel threads.
Nothing here computes any part of the method.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle as O


def workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def sweep(n, eu, ev, *, R, r_begin=0, parts=None, **kw):
    """O.sweep over [r_begin, r_begin + R) in up to `parts` ranges."""
    parts = parts or workers()
    parts = max(1, min(parts, R))
    cuts = [r_begin + (R * k) // parts for k in range(parts + 1)]
    ranges = [(cuts[k], cuts[k + 1] - cuts[k]) for k in range(parts) if cuts[k + 1] > cuts[k]]
    if len(ranges) == 1:
        return O.sweep(n, eu, ev, R=R, r_begin=r_begin, **kw)
    with ThreadPoolExecutor(len(ranges)) as ex:
        outs = list(ex.map(lambda a: O.sweep(n, eu, ev, R=a[1], r_begin=a[0], **kw), ranges))
    res = {}
    for key in ("counts", "counts_w"):
        if key in outs[0]:
            res[key] = np.sum([o[key] for o in outs], axis=0, dtype=np.uint64).astype(np.uint32)
    for key in ("center_global", "next_table", "next_table_w"):
        if key in outs[0]:
            res[key] = np.concatenate([o[key] for o in outs], axis=0)
    for key in ("bsum", "psi", "psi_w"):
        if key in outs[0]:
            res[key] = np.sum([o[key] for o in outs], axis=0)
    res["stats"] = {k: sum(o["stats"][k] for o in outs) for k in outs[0]["stats"]}
    return res
