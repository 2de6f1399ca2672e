"""CPU oracle for absorbing-frequency centrality (AFC).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, single-threaded
FP64 statement of what the GPU library computes (``amc_oracle.c``) plus a thin
ctypes wrapper.  Only the tests, the package smoke check and the benchmark's
CPU-baseline leg may import it; the product path never does, and it shares no
code with the GPU library.

Paper: Bao, Kontou, Vogiatzis, "Betweenness-Central Nodes Under Uncertainty:
An Absorbing Markov Chain Approach".  Each wrapper names the passage the C
function follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "amc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

WEIGHT_UNIT, WEIGHT_UNIFORM, WEIGHT_FIXED, WEIGHT_TABLE = 0, 1, 2, 3
_WEIGHT_KINDS = {"unit": WEIGHT_UNIT, "uniform": WEIGHT_UNIFORM, "fixed": WEIGHT_FIXED, "table": WEIGHT_TABLE}

OK, E_ARG, E_NOMEM, E_SIGMA, E_SINGULAR = 0, -1, -2, -4, -5


class OracleError(RuntimeError):
    def __init__(self, rc, what):
        super().__init__(f"oracle {what} failed with status {rc}")
        self.rc = rc


def build() -> str:
    """Compile the oracle with gcc (plain -O2, no vectorisation tricks)."""
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


class _Model(C.Structure):
    _fields_ = [("p_fail", C.c_double), ("p_fail_edge", C.POINTER(C.c_double)), ("weight_kind", C.c_int32),
                ("w_lo", C.c_uint32), ("w_hi", C.c_uint32), ("w0", C.POINTER(C.c_uint32)),
                ("w_cdf", C.POINTER(C.c_uint64))]


class _Query(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("R", C.c_uint32), ("r_begin", C.c_uint32), ("alpha", C.c_double),
                ("k_min", C.c_uint32), ("tau", C.c_double), ("pool_mask", C.POINTER(C.c_uint8)),
                ("topk", C.c_int32), ("gamma", C.POINTER(C.c_double)), ("hop_radius", C.c_int32)]


class _SweepOut(C.Structure):
    _fields_ = [("counts", C.POINTER(C.c_uint32)), ("counts_w", C.POINTER(C.c_uint32)),
                ("center_global", C.POINTER(C.c_int32)), ("next_table", C.POINTER(C.c_int32)),
                ("next_table_w", C.POINTER(C.c_int32)), ("bsum", C.POINTER(C.c_double)),
                ("stats", C.c_uint64 * 8), ("psi", C.POINTER(C.c_double)), ("psi_w", C.POINTER(C.c_double))]


class _TailIn(C.Structure):
    _fields_ = [("eta", C.c_double), ("s", C.POINTER(C.c_double)), ("f", C.POINTER(C.c_double)),
                ("pool_mask", C.POINTER(C.c_uint8)), ("eps", C.c_double), ("r_lower", C.c_double),
                ("cert_topk", C.c_int32), ("psi", C.POINTER(C.c_double)), ("psi_w", C.POINTER(C.c_double)),
                ("fb_node", C.c_int32), ("fb_mask", C.POINTER(C.c_uint8))]


class _TailOut(C.Structure):
    _fields_ = [("Q", C.POINTER(C.c_double)), ("r", C.POINTER(C.c_double)), ("N", C.POINTER(C.c_double)),
                ("mu", C.POINTER(C.c_double)), ("b", C.POINTER(C.c_double)), ("ET", C.c_double),
                ("b_f", C.c_double), ("b_w", C.POINTER(C.c_double)), ("xi", C.POINTER(C.c_double)),
                ("ET_w", C.c_double), ("m_w", C.c_double), ("b_w_f", C.c_double),
                ("b_w_bar", C.POINTER(C.c_double)), ("top", C.POINTER(C.c_int32)),
                ("cert_gap", C.POINTER(C.c_double)), ("cert_sharp", C.POINTER(C.c_double)),
                ("cert_v", C.POINTER(C.c_int32)), ("cert_crude", C.c_double), ("epsbar", C.c_double),
                ("epsbar_supp", C.c_double), ("cert_crude_supp", C.c_double),
                ("cert_sharp_supp", C.POINTER(C.c_double)), ("admissible", C.c_int32),
                ("psi_hat", C.POINTER(C.c_double)), ("psi_w_hat", C.POINTER(C.c_double)), ("b_k", C.c_double),
                ("b_kw", C.c_double), ("b_fb", C.POINTER(C.c_double)), ("b_cens", C.POINTER(C.c_double)),
                ("ET_fb", C.c_double), ("m_w_fb", C.c_double), ("c_fb", C.c_double)]


class _TrajQuery(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("episodes", C.c_int32), ("x0", C.POINTER(C.c_int32)), ("alpha", C.c_double),
                ("k_min", C.c_uint32), ("tau", C.c_double), ("max_steps", C.c_int32), ("f", C.POINTER(C.c_double))]


class _TrajOut(C.Structure):
    _fields_ = [("lengths", C.POINTER(C.c_int32)), ("paths", C.POINTER(C.c_int32)),
                ("visits", C.POINTER(C.c_uint64)), ("reward_f", C.c_double), ("switches", C.c_uint64),
                ("total_steps", C.c_uint64), ("truncated", C.c_int32)]


class _RobustIn(C.Structure):
    _fields_ = [("s", C.POINTER(C.c_double)), ("f", C.POINTER(C.c_double)), ("samples", C.c_int32),
                ("delta", C.c_double), ("r_min", C.c_double), ("seed", C.c_uint64)]


class _RobustOut(C.Structure):
    _fields_ = [("b0", C.POINTER(C.c_double)), ("b_sw", C.c_double), ("b_imp", C.c_double),
                ("kl", C.POINTER(C.c_double)), ("tv", C.POINTER(C.c_double)), ("kl_arg", C.c_int32),
                ("tv_arg", C.c_int32), ("b_kl", C.POINTER(C.c_double)), ("b_tv", C.POINTER(C.c_double)),
                ("b_lin", C.POINTER(C.c_double)), ("norm_N0E", C.c_double), ("norm_N0", C.c_double),
                ("rem_bound", C.c_double), ("rem_actual", C.c_double)]


class _BootIn(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("replicates", C.c_int32), ("level", C.c_double), ("eta", C.c_double),
                ("s", C.POINTER(C.c_double))]


class _BootOut(C.Structure):
    _fields_ = [("b0", C.POINTER(C.c_double)), ("mean", C.POINTER(C.c_double)), ("sd", C.POINTER(C.c_double)),
                ("lo", C.POINTER(C.c_double)), ("hi", C.POINTER(C.c_double)), ("b_rep", C.POINTER(C.c_double))]


def _declare(L):
    P = C.POINTER
    L.or_w1.argtypes = [C.c_int32, C.c_int64, P(C.c_int32), P(C.c_int32), P(C.c_uint32), P(C.c_double), P(C.c_double),
                        P(C.c_double)]
    L.or_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
    L.or_philox4x32_10.restype = None
    L.or_prob_threshold.argtypes = [C.c_double]
    L.or_prob_threshold.restype = C.c_uint64
    L.or_realize.argtypes = [C.c_int32, C.c_int64, P(C.c_int32), P(C.c_int32), P(_Model), C.c_uint64, C.c_uint32,
                             P(C.c_uint8), P(C.c_uint32)]
    L.or_stop_coin.argtypes = [C.c_uint64, C.c_uint32, C.c_int32, C.c_double]
    L.or_sssp.argtypes = [C.c_int32, C.c_int64, P(C.c_int32), P(C.c_int32), P(C.c_uint8), P(C.c_uint32), C.c_int,
                          C.c_int32, P(C.c_uint64), P(C.c_uint64), P(C.c_double)]
    for name in ("or_betweenness", "or_betweenness_pairs"):
        getattr(L, name).argtypes = [C.c_int32, C.c_int64, P(C.c_int32), P(C.c_int32), P(C.c_uint8), P(C.c_uint32),
                                     C.c_int, P(C.c_double)]
    L.or_components.argtypes = [C.c_int32, C.c_int64, P(C.c_int32), P(C.c_int32), P(C.c_uint8), P(C.c_int32),
                                P(C.c_int32)]
    L.or_band_argmax.argtypes = [C.c_int32, P(C.c_double), P(C.c_uint8), C.c_double, P(C.c_int64)]
    L.or_band_argmax.restype = C.c_int32
    L.or_sweep.argtypes = [C.c_int32, C.c_int64, P(C.c_int32), P(C.c_int32), P(_Model), P(_Query), P(_SweepOut)]
    L.or_counts_to_kernel.argtypes = [C.c_int32, P(C.c_uint32), C.c_uint32, C.c_double, P(C.c_double),
                                      P(C.c_double)]
    L.or_fundamental.argtypes = [C.c_int32, P(C.c_double), P(C.c_double)]
    L.or_visits.argtypes = [C.c_int32, P(C.c_double), P(C.c_double), P(C.c_double), P(C.c_double), P(C.c_double)]
    L.or_visits.restype = None
    L.or_pair_certificate.argtypes = [C.c_int32, P(C.c_double), P(C.c_double), C.c_double, C.c_double, C.c_int32,
                                      C.c_int32, P(C.c_double), P(C.c_double), P(C.c_double)]
    L.or_pair_certificate.restype = None
    L.or_tail.argtypes = [C.c_int32, P(C.c_uint32), P(C.c_uint32), C.c_uint32, P(_TailIn), P(_TailOut)]
    L.or_robust.argtypes = [C.c_int32, P(C.c_double), P(_RobustIn), P(_RobustOut)]
    L.or_bootstrap.argtypes = [C.c_int32, C.c_uint32, P(C.c_int32), P(_BootIn), P(_BootOut)]
    L.or_boot_counts.argtypes = [C.c_int32, C.c_uint32, P(C.c_int32), C.c_uint64, C.c_uint32, P(C.c_uint32)]
    L.or_boot_counts.restype = None
    L.or_perturbed_kernel.argtypes = [C.c_int32, P(C.c_double), C.c_uint64, C.c_int32, C.c_double, C.c_double,
                                      P(C.c_double)]
    L.or_perturbed_kernel.restype = None
    L.or_trajectories.argtypes = [C.c_int32, C.c_int64, P(C.c_int32), P(C.c_int32), P(_Model), P(_TrajQuery),
                                  P(_TrajOut)]


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ctype))


def _check(rc, what):
    if rc != OK:
        raise OracleError(rc, what)


def _edges(eu, ev):
    return np.ascontiguousarray(eu, dtype=np.int32), np.ascontiguousarray(ev, dtype=np.int32)


def _model(p_fail=0.0, weight="unit", w_lo=1, w_hi=1, w0=None, p_fail_edge=None, w_cdf=None):
    keep = []
    m = _Model()
    m.p_fail = float(p_fail)
    if p_fail_edge is not None:
        pe = np.ascontiguousarray(p_fail_edge, dtype=np.float64)
        keep.append(pe)
        m.p_fail_edge = _ptr(pe, C.c_double)
    m.weight_kind = _WEIGHT_KINDS[weight]
    m.w_lo, m.w_hi = int(w_lo), int(w_hi)
    if w0 is not None:
        ww = np.ascontiguousarray(w0, dtype=np.uint32)
        keep.append(ww)
        m.w0 = _ptr(ww, C.c_uint32)
    if w_cdf is not None:
        wc = np.ascontiguousarray(w_cdf, dtype=np.uint64)
        keep.append(wc)
        m.w_cdf = _ptr(wc, C.c_uint64)
        m.w_hi = wc.shape[1]
    return m, keep


# --------------------------------------------------------------------------- RNG
def philox4x32_10(ctr, key):
    """Philox4x32-10 block (Salmon et al., SC'11) on one 128-bit counter."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(o, C.c_uint32))
    return o


def prob_threshold(p):
    return int(lib().or_prob_threshold(float(p)))


def stop_coin(seed, r, i, alpha):
    return bool(lib().or_stop_coin(int(seed), int(r), int(i), float(alpha)))


def realize(n, eu, ev, seed, r, **model):
    """One network state (Section 3.1): surviving edges and integer weights."""
    eu, ev = _edges(eu, ev)
    m = len(eu)
    mod, keep = _model(**model)
    alive = np.zeros(max(m, 1), dtype=np.uint8)
    w = np.zeros(max(m, 1), dtype=np.uint32)
    _check(lib().or_realize(n, m, _ptr(eu, C.c_int32), _ptr(ev, C.c_int32), C.byref(mod), int(seed), int(r),
                            _ptr(alive, C.c_uint8), _ptr(w, C.c_uint32)), "realize")
    del keep
    return alive[:m], w[:m]


# --------------------------------------------------------------------------- Brandes
def sssp(n, eu, ev, alive, w, unit, s):
    """Distances, exact path counts and dependencies of one source (Section 3.1)."""
    eu, ev = _edges(eu, ev)
    alive = np.ascontiguousarray(alive, dtype=np.uint8)
    w = np.ascontiguousarray(w, dtype=np.uint32)
    dist = np.zeros(n, dtype=np.uint64)
    sigma = np.zeros(n, dtype=np.uint64)
    delta = np.zeros(n, dtype=np.float64)
    _check(lib().or_sssp(n, len(eu), _ptr(eu, C.c_int32), _ptr(ev, C.c_int32), _ptr(alive, C.c_uint8),
                         _ptr(w, C.c_uint32), int(bool(unit)), int(s), _ptr(dist, C.c_uint64),
                         _ptr(sigma, C.c_uint64), _ptr(delta, C.c_double)), "sssp")
    return dist, sigma, delta


def betweenness(n, eu, ev, alive=None, w=None, unit=True, pairs=False):
    """B_v(H) of Section 3.1; ``pairs=True`` evaluates the pair-sum definition."""
    eu, ev = _edges(eu, ev)
    m = len(eu)
    alive = np.ones(max(m, 1), np.uint8) if alive is None else np.ascontiguousarray(alive, dtype=np.uint8)
    w = np.ones(max(m, 1), np.uint32) if w is None else np.ascontiguousarray(w, dtype=np.uint32)
    B = np.zeros(n, dtype=np.float64)
    fn = lib().or_betweenness_pairs if pairs else lib().or_betweenness
    _check(fn(n, m, _ptr(eu, C.c_int32), _ptr(ev, C.c_int32), _ptr(alive, C.c_uint8), _ptr(w, C.c_uint32),
              int(bool(unit)), _ptr(B, C.c_double)), "betweenness")
    return B


def components(n, eu, ev, alive=None):
    eu, ev = _edges(eu, ev)
    m = len(eu)
    alive = np.ones(max(m, 1), np.uint8) if alive is None else np.ascontiguousarray(alive, dtype=np.uint8)
    comp = np.zeros(n, dtype=np.int32)
    size = np.zeros(n, dtype=np.int32)
    _check(lib().or_components(n, m, _ptr(eu, C.c_int32), _ptr(ev, C.c_int32), _ptr(alive, C.c_uint8),
                               _ptr(comp, C.c_int32), _ptr(size, C.c_int32)), "components")
    return comp, size


def band_argmax(B, member, tau=1e-9):
    B = np.ascontiguousarray(B, dtype=np.float64)
    mem = np.ascontiguousarray(member, dtype=np.uint8)
    near = C.c_int64(0)
    v = lib().or_band_argmax(len(B), _ptr(B, C.c_double), _ptr(mem, C.c_uint8), float(tau), C.byref(near))
    return int(v), int(near.value)


# --------------------------------------------------------------------------- sweep
def sweep(n, eu, ev, *, seed, R, r_begin=0, alpha=0.15, k_min=5, tau=1e-9, pool=None, want_next=False,
          want_bsum=True, want_center=True, topk=0, gamma=None, hop_radius=0, **model):
    """Alg. 1 for every anchor over realizations [r_begin, r_begin + R), counted as in Alg. 2.
    With topk > 0 also the Top-k step-reward sums psi / psi_w (Sections 6.2-6.3) and the
    finite-k pool selector (Section 7.1)."""
    eu, ev = _edges(eu, ev)
    mod, keep = _model(**model)
    q = _Query()
    q.seed, q.R, q.r_begin = int(seed), int(R), int(r_begin)
    q.alpha, q.k_min, q.tau = float(alpha), int(k_min), float(tau)
    q.topk = int(topk)
    q.hop_radius = int(hop_radius)
    if hop_radius > 0:                     # anchored steps: no realization-wide B
        want_bsum = want_center = False
    g_arr = None
    if gamma is not None:
        g_arr = np.ascontiguousarray(gamma, dtype=np.float64)
        q.gamma = _ptr(g_arr, C.c_double)
    mask = None
    if pool is not None:
        mask = np.zeros(n, dtype=np.uint8)
        mask[np.asarray(pool, dtype=np.int64)] = 1
        q.pool_mask = _ptr(mask, C.c_uint8)
    res = {"counts": np.zeros((n, n + 1), dtype=np.uint32)}
    o = _SweepOut()
    o.counts = _ptr(res["counts"], C.c_uint32)
    if pool is not None:
        res["counts_w"] = np.zeros((n, n + 1), dtype=np.uint32)
        o.counts_w = _ptr(res["counts_w"], C.c_uint32)
    if want_center:
        res["center_global"] = np.zeros(R, dtype=np.int32)
        o.center_global = _ptr(res["center_global"], C.c_int32)
    if want_next:
        res["next_table"] = np.zeros((R, n), dtype=np.int32)
        o.next_table = _ptr(res["next_table"], C.c_int32)
        if pool is not None:
            res["next_table_w"] = np.zeros((R, n), dtype=np.int32)
            o.next_table_w = _ptr(res["next_table_w"], C.c_int32)
    if want_bsum:
        res["bsum"] = np.zeros(n, dtype=np.float64)
        o.bsum = _ptr(res["bsum"], C.c_double)
    if topk > 0:
        res["psi"] = np.zeros(n, dtype=np.float64)
        o.psi = _ptr(res["psi"], C.c_double)
        if pool is not None:
            res["psi_w"] = np.zeros(n, dtype=np.float64)
            o.psi_w = _ptr(res["psi_w"], C.c_double)
    _check(lib().or_sweep(n, len(eu), _ptr(eu, C.c_int32), _ptr(ev, C.c_int32), C.byref(mod), C.byref(q),
                          C.byref(o)), "sweep")
    st = list(o.stats)
    res["stats"] = {"units": st[0], "sum_nK": st[1], "sum_AK": st[2], "sum_DK": st[3], "near_band": st[4]}
    del keep, g_arr
    return res


def trajectories(n, eu, ev, *, seed, x0, alpha=0.15, k_min=5, tau=1e-9, max_steps=1024, f=None, want_paths=False,
                 **model):
    """Episodes of the network process (Section 4.3): lengths, visits, node-reward and switch totals."""
    eu, ev = _edges(eu, ev)
    mod, keep = _model(**model)
    x0 = np.ascontiguousarray(x0, dtype=np.int32)
    E = len(x0)
    q = _TrajQuery()
    q.seed, q.episodes, q.x0 = int(seed), E, _ptr(x0, C.c_int32)
    q.alpha, q.k_min, q.tau, q.max_steps = float(alpha), int(k_min), float(tau), int(max_steps)
    fa = None
    if f is not None:
        fa = np.ascontiguousarray(f, dtype=np.float64)
        q.f = _ptr(fa, C.c_double)
    res = {"lengths": np.zeros(E, np.int32), "visits": np.zeros(n, np.uint64)}
    o = _TrajOut()
    o.lengths = _ptr(res["lengths"], C.c_int32)
    o.visits = _ptr(res["visits"], C.c_uint64)
    if want_paths:
        res["paths"] = np.zeros((E, max_steps), np.int32)
        o.paths = _ptr(res["paths"], C.c_int32)
    _check(lib().or_trajectories(n, len(eu), _ptr(eu, C.c_int32), _ptr(ev, C.c_int32), C.byref(mod), C.byref(q),
                                 C.byref(o)), "trajectories")
    res.update(reward_f=float(o.reward_f), switches=int(o.switches), total_steps=int(o.total_steps),
               truncated=int(o.truncated))
    del keep, fa
    return res


def perturbed_kernel(Q0, seed, sample, delta, r_min):
    """Sampled admissible kernel of the robust search (multiplicative radius, row cap 1 - r_min)."""
    Q0 = np.ascontiguousarray(Q0, dtype=np.float64)
    Q = np.zeros_like(Q0)
    lib().or_perturbed_kernel(Q0.shape[0], _ptr(Q0, C.c_double), int(seed), int(sample), float(delta), float(r_min),
                              _ptr(Q, C.c_double))
    return Q


def robust(Q0, *, s=None, f=None, samples=16, delta=0.5, r_min=0.05, seed=0):
    """Transition rewards, sampled KL / TV maximisers and the first-order sensitivity (Sections 5.4, 6.4)."""
    Q0 = np.ascontiguousarray(Q0, dtype=np.float64)
    n = Q0.shape[0]
    s_arr = np.full(n, 1.0 / n) if s is None else np.ascontiguousarray(s, dtype=np.float64)
    ri = _RobustIn()
    ri.s, ri.samples, ri.delta, ri.r_min, ri.seed = _ptr(s_arr, C.c_double), int(samples), float(delta), \
        float(r_min), int(seed)
    fa = None
    if f is not None:
        fa = np.ascontiguousarray(f, dtype=np.float64)
        ri.f = _ptr(fa, C.c_double)
    out = {"b0": np.zeros(n), "kl": np.zeros(max(samples, 1)), "tv": np.zeros(max(samples, 1)), "b_kl": np.zeros(n),
           "b_tv": np.zeros(n), "b_lin": np.zeros(n)}
    ro = _RobustOut()
    for key in out:
        setattr(ro, key, _ptr(out[key], C.c_double))
    _check(lib().or_robust(n, _ptr(Q0, C.c_double), C.byref(ri), C.byref(ro)), "robust")
    for key in ("b_sw", "b_imp", "norm_N0E", "norm_N0", "rem_bound", "rem_actual"):
        out[key] = float(getattr(ro, key))
    out["kl_arg"], out["tv_arg"] = int(ro.kl_arg), int(ro.tv_arg)
    out["kl"], out["tv"] = out["kl"][:samples], out["tv"][:samples]
    del fa
    return out


def boot_counts(next_table, seed, beta):
    """Counts of bootstrap replicate beta: every row's R draws redrawn with replacement (Section 8.4)."""
    nt = np.ascontiguousarray(next_table, dtype=np.int32)
    R, n = nt.shape
    counts = np.zeros((n, n + 1), dtype=np.uint32)
    lib().or_boot_counts(n, R, _ptr(nt, C.c_int32), int(seed), int(beta), _ptr(counts, C.c_uint32))
    return counts


def bootstrap(next_table, *, replicates=100, level=0.95, eta=None, s=None, seed=0):
    """Nonparametric bootstrap of b from a next table (R x n, -1 = bottom): b of the draws themselves,
    per-node mean, standard deviation and nearest-rank percentile interval over the replicates, and
    every replicate's b (Section 8.4)."""
    nt = np.ascontiguousarray(next_table, dtype=np.int32)
    R, n = nt.shape
    s_arr = np.full(n, 1.0 / n) if s is None else np.ascontiguousarray(s, dtype=np.float64)
    bi = _BootIn()
    bi.seed, bi.replicates, bi.level = int(seed), int(replicates), float(level)
    bi.eta = 0.1 / np.sqrt(R) if eta is None else float(eta)
    bi.s = _ptr(s_arr, C.c_double)
    out = {k: np.zeros(n) for k in ("b0", "mean", "sd", "lo", "hi")}
    out["b_rep"] = np.zeros((replicates, n))
    bo = _BootOut()
    for key in out:
        setattr(bo, key, _ptr(out[key], C.c_double))
    _check(lib().or_bootstrap(n, R, _ptr(nt, C.c_int32), C.byref(bi), C.byref(bo)), "bootstrap")
    return out


def w1(n, eu, ev, p, q, cost=None):
    """Wasserstein-1 between profiles p and q (n each) on the shortest-path
    metric of the graph (eu, ev) with unit edge lengths (the hop metric) or
    the integer lengths `cost`: the cheapest transshipment of p - q over its
    edges."""
    eu = np.ascontiguousarray(eu, dtype=np.int32)
    ev = np.ascontiguousarray(ev, dtype=np.int32)
    p = np.ascontiguousarray(p, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    c = None if cost is None else np.ascontiguousarray(cost, dtype=np.uint32)
    out = C.c_double(0.0)
    _check(lib().or_w1(int(n), len(eu), _ptr(eu, C.c_int32), _ptr(ev, C.c_int32), _ptr(c, C.c_uint32),
                       _ptr(p, C.c_double), _ptr(q, C.c_double), C.byref(out)), "w1")
    return float(out.value)


# --------------------------------------------------------------------------- chain algebra
def counts_to_kernel(counts, R, eta):
    counts = np.ascontiguousarray(counts, dtype=np.uint32)
    n = counts.shape[0]
    Q = np.zeros((n, n), dtype=np.float64)
    r = np.zeros(n, dtype=np.float64)
    _check(lib().or_counts_to_kernel(n, _ptr(counts, C.c_uint32), int(R), float(eta), _ptr(Q, C.c_double),
                                     _ptr(r, C.c_double)), "counts_to_kernel")
    return Q, r


def fundamental(Q):
    """N = (I - Q)^{-1} (eq. fundamental)."""
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    n = Q.shape[0]
    N = np.zeros((n, n), dtype=np.float64)
    _check(lib().or_fundamental(n, _ptr(Q, C.c_double), _ptr(N, C.c_double)), "fundamental")
    return N


def visits(N, s):
    """mu = sN, E_s[T] = mu 1, b = mu / mu 1 (eqs. visits, expected-length, afc-def)."""
    N = np.ascontiguousarray(N, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.float64)
    n = N.shape[0]
    mu = np.zeros(n)
    b = np.zeros(n)
    ET = C.c_double(0.0)
    lib().or_visits(n, _ptr(N, C.c_double), _ptr(s, C.c_double), _ptr(mu, C.c_double), C.byref(ET),
                    _ptr(b, C.c_double))
    return mu, float(ET.value), b


def chain(Q, s):
    N = fundamental(Q)
    mu, ET, b = visits(N, s)
    return {"N": N, "mu": mu, "ET": ET, "b": b}


def pair_certificate(N, mu, epsbar, r_min, u, v):
    """(G_uv, crude threshold, sharp threshold) of eq. pm-gap and eq. sharp-gap."""
    N = np.ascontiguousarray(N, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    g, c, s = C.c_double(), C.c_double(), C.c_double()
    lib().or_pair_certificate(N.shape[0], _ptr(N, C.c_double), _ptr(mu, C.c_double), float(epsbar), float(r_min),
                              int(u), int(v), C.byref(g), C.byref(c), C.byref(s))
    return float(g.value), float(c.value), float(s.value)


def tail(counts, R, *, eta=None, s=None, f=None, pool=None, counts_w=None, eps=0.0, r_lower=0.05, cert_topk=0,
         psi=None, psi_w=None, fb_node=-1, fb_set=None):
    """Counts -> stabilised kernel -> N, mu, E[T], b, rewards, pool kernel, certificates; with
    psi / psi_w the valued Top-k reward-AFCs, with fb_node the fallback kernel and censoring."""
    counts = np.ascontiguousarray(counts, dtype=np.uint32)
    n = counts.shape[0]
    if eta is None:
        eta = 0.1 / np.sqrt(R)
    s_arr = np.full(n, 1.0 / n) if s is None else np.ascontiguousarray(s, dtype=np.float64)
    ti = _TailIn()
    ti.eta, ti.s, ti.eps, ti.r_lower, ti.cert_topk = float(eta), _ptr(s_arr, C.c_double), float(eps), \
        float(r_lower), int(cert_topk)
    f_arr = None
    if f is not None:
        f_arr = np.ascontiguousarray(f, dtype=np.float64)
        ti.f = _ptr(f_arr, C.c_double)
    mask = None
    if pool is not None:
        mask = np.zeros(n, dtype=np.uint8)
        mask[np.asarray(pool, dtype=np.int64)] = 1
        ti.pool_mask = _ptr(mask, C.c_uint8)
    keep = []
    for name, arr in (("psi", psi), ("psi_w", psi_w)):
        if arr is not None:
            a = np.ascontiguousarray(arr, dtype=np.float64)
            keep.append(a)
            setattr(ti, name, _ptr(a, C.c_double))
    ti.fb_node = int(fb_node)
    fbm = None
    if fb_set is not None:
        fbm = np.zeros(n, dtype=np.uint8)
        fbm[np.asarray(fb_set, dtype=np.int64)] = 1
        ti.fb_mask = _ptr(fbm, C.c_uint8)
    k = int(cert_topk)
    out = {"Q": np.zeros((n, n)), "r": np.zeros(n), "N": np.zeros((n, n)), "mu": np.zeros(n), "b": np.zeros(n),
           "b_w": np.zeros(n), "xi": np.zeros(n), "b_w_bar": np.zeros(n), "top": np.zeros(max(k, 1), np.int32),
           "cert_gap": np.zeros((max(k, 1), max(n - k, 1))), "cert_sharp": np.zeros((max(k, 1), max(n - k, 1))),
           "cert_sharp_supp": np.zeros((max(k, 1), max(n - k, 1))), "cert_v": np.zeros(max(n - k, 1), np.int32)}
    to = _TailOut()
    for key in ("Q", "r", "N", "mu", "b", "b_w", "xi", "b_w_bar", "cert_gap", "cert_sharp", "cert_sharp_supp"):
        setattr(to, key, _ptr(out[key], C.c_double))
    to.top = _ptr(out["top"], C.c_int32)
    to.cert_v = _ptr(out["cert_v"], C.c_int32)
    for key in ("psi_hat", "psi_w_hat", "b_fb", "b_cens"):
        out[key] = np.zeros(n)
        setattr(to, key, _ptr(out[key], C.c_double))
    cw = None
    if counts_w is not None:
        cw = np.ascontiguousarray(counts_w, dtype=np.uint32)
    _check(lib().or_tail(n, _ptr(counts, C.c_uint32), _ptr(cw, C.c_uint32), int(R), C.byref(ti), C.byref(to)),
           "tail")
    for key in ("ET", "b_f", "ET_w", "m_w", "b_w_f", "cert_crude", "epsbar", "epsbar_supp", "cert_crude_supp",
                "b_k", "b_kw", "ET_fb", "m_w_fb", "c_fb"):
        out[key] = float(getattr(to, key))
    del keep, fbm
    out["admissible"] = bool(to.admissible)
    out["top"] = out["top"][:k]
    out["cert_v"] = out["cert_v"][:n - k] if k > 0 else out["cert_v"][:0]
    if k == 0:
        for key in ("cert_gap", "cert_sharp", "cert_sharp_supp"):
            out[key] = out[key][:0, :0]
    if pool is None:
        for key in ("b_w", "xi", "b_w_bar"):
            out[key] = None
    if psi is None:
        out["psi_hat"] = None
    if psi_w is None:
        out["psi_w_hat"] = None
    if fb_node < 0 or pool is None or counts_w is None:
        for key in ("b_fb", "b_cens", "ET_fb", "m_w_fb", "c_fb"):
            out[key] = None
    return out
