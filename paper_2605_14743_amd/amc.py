"""ctypes binding of the C-ABI in ``include/amc.h`` (argument marshalling only).

Every step of the estimation runs in the HIP library ``lib/libamc.so``; this
module only converts numpy arrays to pointers and back.  Importing it does not
load the library; the first call does, and raises ``RuntimeError`` when the
library has not been built (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libamc.so")

OK, E_INVALID_ARG, E_OOM, E_HIP, E_SIGMA_OVERFLOW, E_SINGULAR, E_ADMISSION, E_NOT_READY, E_UNSUPPORTED, E_SCRATCH = \
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9
WEIGHT_UNIT, WEIGHT_UNIFORM_INT, WEIGHT_FIXED, WEIGHT_TABLE = 0, 1, 2, 3
MODE_AUTO, MODE_WAVE, MODE_BLOCK, MODE_WAVE_L2 = 0, 1, 2, 3
WANT_N, WANT_BSUM, WANT_NEXT_TABLE, WANT_CENTER, WANT_DEBUG, SKIP_TAIL, PLAIN_LAUNCH, FALLBACK, DIST32, DIST16 = \
    1, 2, 4, 8, 16, 32, 64, 128, 256, 512
SIGMA_GLOBAL, STATE_GLOBAL = 1024, 2048
MAX_TOPK, MAX_TOPK_N = 64, 65535
MAX_BOOT_REPLICATES, MAX_BOOT_N = 4096, 16383
MAX_W1_N = 7500
STATIC_SCRATCH_BYTES = 64 << 20

EXPORTS = ["amc_ctx_create", "amc_ctx_destroy", "amc_ctx_set_stream", "amc_ctx_stream", "amc_graph_create",
           "amc_graph_destroy", "amc_footprint", "amc_run", "amc_submit", "amc_poll", "amc_wait",
           "amc_request_destroy", "amc_request_times", "amc_server_info", "amc_batch_create", "amc_batch_run", "amc_batch_info",
           "amc_batch_destroy", "amc_tune", "amc_trajectories", "amc_robust", "amc_bootstrap", "amc_chain",
           "amc_stability", "amc_sweep_static", "amc_strerror", "amc_version"]
WANT_PATHS, TRAJ_B_LDS, TRAJ_B_GLOBAL = 1, 2, 4

_P = C.POINTER


class AmcError(RuntimeError):
    def __init__(self, rc: int, what: str):
        msg = _lib_or_none().amc_strerror(rc).decode() if _lib_or_none() else str(rc)
        super().__init__(f"{what}: {msg} ({rc})")
        self.rc = rc


class Model(C.Structure):
    _fields_ = [("p_fail", C.c_double), ("p_fail_edge", _P(C.c_double)), ("weight_kind", C.c_int32),
                ("w_lo", C.c_uint32), ("w_hi", C.c_uint32), ("w_cdf", _P(C.c_uint64))]


class Query(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("R", C.c_uint32), ("r_begin", C.c_uint32), ("alpha", C.c_double),
                ("k_min", C.c_uint32), ("tie_tau", C.c_double), ("floor_eta", C.c_double), ("s", _P(C.c_double)),
                ("pool", _P(C.c_int32)), ("pool_size", C.c_int32), ("reward", _P(C.c_double)), ("eps", C.c_double),
                ("r_lower", C.c_double), ("cert_topk", C.c_int32), ("flags", C.c_uint32), ("mode", C.c_int32),
                ("tile", C.c_int32), ("waves", C.c_int32), ("group", C.c_int32), ("debug_pairs", _P(C.c_uint32)),
                ("n_debug", C.c_int32), ("topk", C.c_int32), ("gamma", _P(C.c_double)), ("fb_node", C.c_int32),
                ("fb_set", _P(C.c_int32)), ("fb_set_size", C.c_int32), ("hop_radius", C.c_int32)]


class TrajQuery(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("episodes", C.c_int32), ("x0", _P(C.c_int32)), ("alpha", C.c_double),
                ("k_min", C.c_uint32), ("tie_tau", C.c_double), ("max_steps", C.c_int32), ("f", _P(C.c_double)),
                ("flags", C.c_uint32), ("group", C.c_int32), ("waves", C.c_int32), ("mode", C.c_int32)]


class TrajResult(C.Structure):
    _fields_ = [("lengths", _P(C.c_int32)), ("paths", _P(C.c_int32)), ("visits", _P(C.c_uint64)),
                ("b_hat", _P(C.c_double)), ("survival", _P(C.c_double)), ("reward_f", C.c_double),
                ("switches", C.c_uint64), ("total_steps", C.c_uint64), ("sources", C.c_uint64),
                ("truncated", C.c_int32), ("sweep_ms", C.c_double), ("mode", C.c_int32), ("waves", C.c_int32),
                ("dist16", C.c_int32), ("b_global", C.c_int32), ("shared_sources", C.c_uint64)]


class RobustQuery(C.Structure):
    _fields_ = [("s", _P(C.c_double)), ("f", _P(C.c_double)), ("samples", C.c_int32), ("delta", C.c_double),
                ("r_min", C.c_double), ("seed", C.c_uint64), ("m", C.c_int64), ("eu", _P(C.c_int32)),
                ("ev", _P(C.c_int32)), ("w", _P(C.c_uint32))]


class RobustResult(C.Structure):
    _fields_ = [("b0", _P(C.c_double)), ("b_sw", C.c_double), ("b_imp", C.c_double), ("kl", _P(C.c_double)),
                ("tv", _P(C.c_double)), ("kl_arg", C.c_int32), ("tv_arg", C.c_int32), ("b_kl", _P(C.c_double)),
                ("b_tv", _P(C.c_double)), ("b_lin", _P(C.c_double)), ("norm_N0E", C.c_double),
                ("norm_N0", C.c_double), ("rem_bound", C.c_double), ("rem_actual", C.c_double),
                ("tail_ms", C.c_double), ("w1", _P(C.c_double)), ("w1_arg", C.c_int32), ("b_w1", _P(C.c_double))]


class BootQuery(C.Structure):
    _fields_ = [("s", _P(C.c_double)), ("floor_eta", C.c_double), ("replicates", C.c_int32), ("level", C.c_double),
                ("seed", C.c_uint64)]


class BootResult(C.Structure):
    _fields_ = [("b0", _P(C.c_double)), ("mean", _P(C.c_double)), ("sd", _P(C.c_double)), ("lo", _P(C.c_double)),
                ("hi", _P(C.c_double)), ("b_rep", _P(C.c_double)), ("ms", C.c_double)]


class StabilityResult(C.Structure):
    _fields_ = [("b_M", _P(C.c_double)), ("b_2M", _P(C.c_double)), ("top_M", _P(C.c_int32)),
                ("top_2M", _P(C.c_int32)), ("counts_2M", _P(C.c_uint32)), ("same_set", C.c_int32),
                ("overlap", C.c_int32), ("max_abs_diff", C.c_double), ("sweep_ms", C.c_double)]


class TuneResult(C.Structure):
    _fields_ = [("mode", C.c_int32), ("group", C.c_int32), ("waves", C.c_int32), ("units_per_s", C.c_double),
                ("candidates", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("budget", C.c_uint64), ("peak_in_use", C.c_uint64), ("admitted", C.c_uint64),
                ("completed", C.c_uint64), ("launches", C.c_uint64), ("shared_launches", C.c_uint64),
                ("peak_active", C.c_int32), ("max_members", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("units", C.c_uint64), ("sum_nK", C.c_uint64), ("sum_AK", C.c_uint64), ("sum_DK", C.c_uint64),
                ("near_band", C.c_uint64), ("sweep_ms", C.c_double), ("tail_ms", C.c_double), ("mode", C.c_int32),
                ("waves", C.c_int32), ("tile", C.c_int32), ("blocks", C.c_int32), ("lds_bytes", C.c_int32),
                ("launches", C.c_int32), ("group", C.c_int32), ("adj_bytes", C.c_int32), ("topk_ms", C.c_double),
                ("dist_bytes", C.c_int32), ("b_global", C.c_int32), ("tail_split", C.c_int32),
                ("tail_tiles", C.c_int32), ("sig_global", C.c_int32), ("state_global", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("counts", _P(C.c_uint32)), ("counts_w", _P(C.c_uint32)), ("center_global", _P(C.c_int32)),
                ("next_table", _P(C.c_int32)), ("next_table_w", _P(C.c_int32)), ("bsum", _P(C.c_double)),
                ("Q", _P(C.c_double)), ("r", _P(C.c_double)), ("N", _P(C.c_double)), ("mu", _P(C.c_double)),
                ("b", _P(C.c_double)), ("b_w", _P(C.c_double)), ("xi", _P(C.c_double)), ("b_w_bar", _P(C.c_double)),
                ("top", _P(C.c_int32)), ("cert_v", _P(C.c_int32)), ("cert_gap", _P(C.c_double)),
                ("cert_sharp", _P(C.c_double)), ("cert_sharp_supp", _P(C.c_double)), ("dbg_dist", _P(C.c_uint32)),
                ("dbg_sigma", _P(C.c_uint64)), ("dbg_delta", _P(C.c_double)), ("E_T", C.c_double),
                ("b_f", C.c_double), ("E_T_w", C.c_double), ("m_w", C.c_double), ("b_w_f", C.c_double),
                ("cert_crude", C.c_double), ("epsbar", C.c_double), ("cert_crude_supp", C.c_double),
                ("epsbar_supp", C.c_double), ("admissible", C.c_int32), ("stats", Stats),
                ("psi", _P(C.c_double)), ("psi_w", _P(C.c_double)), ("b_k", C.c_double), ("b_kw", C.c_double),
                ("b_fb", _P(C.c_double)), ("b_cens", _P(C.c_double)), ("E_T_fb", C.c_double), ("m_w_fb", C.c_double),
                ("c_fb", C.c_double), ("cert_ok", _P(C.c_uint8))]


_lib = None


def _lib_or_none():
    return _lib


def lib():
    """Loads libamc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.amc_ctx_create.argtypes = [C.c_int, C.c_uint64, _P(vp)]
        L.amc_ctx_destroy.argtypes = [vp]
        L.amc_ctx_destroy.restype = None
        L.amc_ctx_set_stream.argtypes = [vp, vp]
        L.amc_ctx_stream.argtypes = [vp]
        L.amc_ctx_stream.restype = vp
        L.amc_graph_create.argtypes = [vp, C.c_int32, C.c_int64, _P(C.c_int32), _P(C.c_int32), _P(C.c_uint32),
                                       _P(vp)]
        L.amc_graph_destroy.argtypes = [vp]
        L.amc_graph_destroy.restype = None
        L.amc_footprint.argtypes = [vp, _P(Query), _P(C.c_uint64)]
        L.amc_run.argtypes = [vp, vp, _P(Model), _P(Query), _P(Result)]
        L.amc_submit.argtypes = [vp, vp, _P(Model), _P(Query), _P(Result), _P(vp)]
        L.amc_poll.argtypes = [vp]
        L.amc_wait.argtypes = [vp]
        L.amc_request_destroy.argtypes = [vp]
        L.amc_request_destroy.restype = None
        L.amc_request_times.argtypes = [vp, _P(C.c_double)]
        L.amc_server_info.argtypes = [vp, _P(ServerStats)]
        L.amc_chain.argtypes = [vp, C.c_int32, _P(C.c_double), _P(Query), _P(Result)]
        L.amc_batch_create.argtypes = [vp, C.c_int32, _P(vp), _P(Model), _P(Query), _P(vp)]
        L.amc_batch_run.argtypes = [vp, _P(Result)]
        L.amc_batch_info.argtypes = [vp, _P(C.c_int32), _P(C.c_int32)]
        L.amc_batch_destroy.argtypes = [vp]
        L.amc_batch_destroy.restype = None
        L.amc_tune.argtypes = [vp, vp, _P(Model), _P(Query), C.c_uint32, _P(TuneResult)]
        L.amc_trajectories.argtypes = [vp, vp, _P(Model), _P(TrajQuery), _P(TrajResult)]
        L.amc_robust.argtypes = [vp, C.c_int32, _P(C.c_double), _P(RobustQuery), _P(RobustResult)]
        L.amc_bootstrap.argtypes = [vp, C.c_int32, C.c_uint32, _P(C.c_int32), _P(BootQuery), _P(BootResult)]
        L.amc_stability.argtypes = [vp, vp, _P(Model), _P(Query), C.c_int32, _P(StabilityResult)]
        L.amc_sweep_static.argtypes = [vp, vp, _P(Model), _P(Query), vp, vp, _P(Stats)]
        L.amc_strerror.argtypes = [C.c_int]
        L.amc_strerror.restype = C.c_char_p
        L.amc_version.argtypes = []
        _lib = L
    return _lib


def _ptr(a, ct):
    return None if a is None else a.ctypes.data_as(_P(ct))


def _check(rc, what):
    if rc != OK:
        raise AmcError(rc, what)


class Context:
    """amc_ctx: one device, one stream, an HBM budget for the serving loop."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        h = C.c_void_p()
        _check(lib().amc_ctx_create(int(device), int(budget_bytes), C.byref(h)), "amc_ctx_create")
        self.h = h

    def set_stream(self, stream_handle: int | None):
        _check(lib().amc_ctx_set_stream(self.h, C.c_void_p(stream_handle or 0)), "amc_ctx_set_stream")

    def stream(self) -> int:
        return lib().amc_ctx_stream(self.h) or 0

    def close(self):
        if getattr(self, "h", None):
            lib().amc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """amc_graph: a base graph G(V,E) staged on the device (canonical edge list)."""

    def __init__(self, ctx: Context, n: int, eu, ev, w0=None):
        self.ctx = ctx
        self.n = int(n)
        self.eu = np.ascontiguousarray(eu, dtype=np.int32)
        self.ev = np.ascontiguousarray(ev, dtype=np.int32)
        self.m = len(self.eu)
        self.w0 = None if w0 is None else np.ascontiguousarray(w0, dtype=np.uint32)
        h = C.c_void_p()
        _check(lib().amc_graph_create(ctx.h, self.n, self.m, _ptr(self.eu, C.c_int32), _ptr(self.ev, C.c_int32),
                                      _ptr(self.w0, C.c_uint32), C.byref(h)), "amc_graph_create")
        self.h = h

    @classmethod
    def from_workload(cls, ctx, g):
        return cls(ctx, g.n, g.eu, g.ev, g.w0)

    def close(self):
        if getattr(self, "h", None):
            lib().amc_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_WEIGHTS = {"unit": WEIGHT_UNIT, "uniform": WEIGHT_UNIFORM_INT, "fixed": WEIGHT_FIXED, "table": WEIGHT_TABLE}


def make_model(p_fail=0.0, weight="unit", w_lo=1, w_hi=1, p_fail_edge=None, w0=None, w_cdf=None):
    keep = []
    m = Model()
    m.p_fail = float(p_fail)
    if p_fail_edge is not None:
        pe = np.ascontiguousarray(p_fail_edge, dtype=np.float64)
        keep.append(pe)
        m.p_fail_edge = _ptr(pe, C.c_double)
    m.weight_kind = _WEIGHTS[weight] if isinstance(weight, str) else int(weight)
    m.w_lo, m.w_hi = int(w_lo), int(w_hi)
    if w_cdf is not None:
        wc = np.ascontiguousarray(w_cdf, dtype=np.uint64)
        keep.append(wc)
        m.w_cdf = _ptr(wc, C.c_uint64)
        m.w_hi = int(wc.shape[1])
    return m, keep


def make_query(n, *, seed=0, R=1, r_begin=0, alpha=0.15, k_min=5, tie_tau=-1.0, floor_eta=-1.0, s=None, pool=None,
               reward=None, eps=0.0, r_lower=0.05, cert_topk=0, flags=0, mode=MODE_AUTO, tile=0, waves=0, group=0,
               debug_pairs=None, topk=0, gamma=None, fb_node=None, fb_set=None, hop_radius=0):
    keep = []
    q = Query()
    q.seed, q.R, q.r_begin = int(seed), int(R), int(r_begin)
    q.alpha, q.k_min, q.tie_tau, q.floor_eta = float(alpha), int(k_min), float(tie_tau), float(floor_eta)
    if s is not None:
        sa = np.ascontiguousarray(s, dtype=np.float64)
        keep.append(sa)
        q.s = _ptr(sa, C.c_double)
    if pool is not None:
        pa = np.ascontiguousarray(pool, dtype=np.int32)
        keep.append(pa)
        q.pool = _ptr(pa, C.c_int32)
        q.pool_size = len(pa)
    if reward is not None:
        ra = np.ascontiguousarray(reward, dtype=np.float64)
        keep.append(ra)
        q.reward = _ptr(ra, C.c_double)
    q.eps, q.r_lower, q.cert_topk, q.flags = float(eps), float(r_lower), int(cert_topk), int(flags)
    q.mode, q.tile, q.waves, q.group = int(mode), int(tile), int(waves), int(group)
    if debug_pairs is not None and len(debug_pairs):
        dp = np.ascontiguousarray(np.asarray(debug_pairs, dtype=np.uint32).reshape(-1, 2))
        keep.append(dp)
        q.debug_pairs = _ptr(dp, C.c_uint32)
        q.n_debug = len(dp)
        q.flags |= WANT_DEBUG
    q.topk = int(topk)
    q.hop_radius = int(hop_radius)
    if gamma is not None:
        ga = np.ascontiguousarray(gamma, dtype=np.float64)
        keep.append(ga)
        q.gamma = _ptr(ga, C.c_double)
    if fb_node is not None:
        q.flags |= FALLBACK
        q.fb_node = int(fb_node)
        if fb_set is not None:
            fa = np.ascontiguousarray(fb_set, dtype=np.int32)
            keep.append(fa)
            q.fb_set = _ptr(fa, C.c_int32)
            q.fb_set_size = len(fa)
    return q, keep


def _alloc_result(n, q: Query, reuse=None):
    """Caller-owned result buffers for one query; `reuse` (the dict a previous
    call returned, same shapes) lends its arrays instead of fresh ones."""
    R = int(q.R)
    k = int(q.cert_topk)
    pool = q.pool_size > 0
    arr = {"counts": np.zeros((n, n + 1), np.uint32)}
    if pool:
        arr["counts_w"] = np.zeros((n, n + 1), np.uint32)
    if q.flags & WANT_CENTER:
        arr["center_global"] = np.zeros(R, np.int32)
    if q.flags & WANT_NEXT_TABLE:
        arr["next_table"] = np.zeros((R, n), np.int32)
        if pool:
            arr["next_table_w"] = np.zeros((R, n), np.int32)
    if q.flags & WANT_BSUM:
        arr["bsum"] = np.zeros(n, np.float64)
    if not (q.flags & SKIP_TAIL):
        arr.update(Q=np.zeros((n, n)), r=np.zeros(n), mu=np.zeros(n), b=np.zeros(n))
        if q.flags & WANT_N:
            arr["N"] = np.zeros((n, n))
        if pool:
            arr.update(b_w=np.zeros(n), xi=np.zeros(n), b_w_bar=np.zeros(n))
        if k > 0:
            arr.update(top=np.zeros(k, np.int32), cert_v=np.zeros(n - k, np.int32),
                       cert_gap=np.zeros((k, n - k)), cert_sharp=np.zeros((k, n - k)),
                       cert_sharp_supp=np.zeros((k, n - k)), cert_ok=np.zeros((k, n - k), np.uint8))
    if q.n_debug > 0:
        arr.update(dbg_dist=np.zeros((q.n_debug, n), np.uint32), dbg_sigma=np.zeros((q.n_debug, n), np.uint64),
                   dbg_delta=np.zeros((q.n_debug, n)))
    if q.topk > 0:
        arr["psi"] = np.zeros(n)
        if pool:
            arr["psi_w"] = np.zeros(n)
    if (q.flags & FALLBACK) and not (q.flags & SKIP_TAIL):
        arr.update(b_fb=np.zeros(n), b_cens=np.zeros(n))
    if reuse is not None:
        for key, a in arr.items():
            b = reuse.get(key)
            if isinstance(b, np.ndarray) and b.shape == a.shape and b.dtype == a.dtype and b.flags.c_contiguous \
                    and b.flags.writeable:
                arr[key] = b
    res = Result()
    types = {np.dtype(np.uint32): C.c_uint32, np.dtype(np.int32): C.c_int32, np.dtype(np.float64): C.c_double,
             np.dtype(np.uint64): C.c_uint64, np.dtype(np.uint8): C.c_uint8}
    for key, a in arr.items():
        setattr(res, key, _ptr(a, types[a.dtype]))
    return res, arr


def _collect(res: Result, arr: dict) -> dict:
    out = dict(arr)
    for key in ("E_T", "b_f", "E_T_w", "m_w", "b_w_f", "cert_crude", "epsbar", "cert_crude_supp", "epsbar_supp",
                "b_k", "b_kw", "E_T_fb", "m_w_fb", "c_fb"):
        out[key] = float(getattr(res, key))
    out["admissible"] = bool(res.admissible)
    st = res.stats
    out["stats"] = {f: getattr(st, f) for f, _ in Stats._fields_}
    return out


def run(ctx: Context, graph: Graph, model: dict, out: dict | None = None, **query) -> dict:
    """amc_run: the sweep (Alg. 1 for every anchor over R realizations, counted
    as in Alg. 2) and the tail; returns numpy arrays and scalars.  With `out`
    (a dict an earlier call returned) its arrays of matching shape receive the
    results again instead of fresh ones."""
    m, keep_m = make_model(**model)
    q, keep_q = make_query(graph.n, **query)
    res, arr = _alloc_result(graph.n, q, out)
    _check(lib().amc_run(ctx.h, graph.h, C.byref(m), C.byref(q), C.byref(res)), "amc_run")
    del keep_m, keep_q
    return _collect(res, arr)


def server_info(ctx: Context) -> dict:
    """amc_server_info: counters of the context's serving loop."""
    out = ServerStats()
    _check(lib().amc_server_info(ctx.h, C.byref(out)), "amc_server_info")
    return {f: getattr(out, f) for f, _ in ServerStats._fields_}


def sweep_static(ctx: Context, graph: Graph, model: dict, d_counts: int, d_center: int | None = None,
                 **query) -> dict:
    """amc_sweep_static: the sweep into caller-owned device buffers (addresses
    d_counts: n x (n+1) uint32, d_center: R int32 or None) without any device
    allocation; returns the run's counters and plan."""
    m, keep_m = make_model(**model)
    q, keep_q = make_query(graph.n, **query)
    st = Stats()
    _check(lib().amc_sweep_static(ctx.h, graph.h, C.byref(m), C.byref(q), C.c_void_p(int(d_counts)),
                                  C.c_void_p(int(d_center) if d_center else 0), C.byref(st)), "amc_sweep_static")
    del keep_m, keep_q
    return {f: getattr(st, f) for f, _ in Stats._fields_}


class Request:
    """amc_request: a query submitted to the serving loop."""

    def __init__(self, ctx, graph, model: dict, **query):
        self._m, self._keep_m = make_model(**model)
        self._q, self._keep_q = make_query(graph.n, **query)
        self._res, self._arr = _alloc_result(graph.n, self._q)
        self.graph = graph
        h = C.c_void_p()
        _check(lib().amc_submit(ctx.h, graph.h, C.byref(self._m), C.byref(self._q), C.byref(self._res),
                                C.byref(h)), "amc_submit")
        self.h = h

    def poll(self) -> bool:
        rc = lib().amc_poll(self.h)
        if rc == E_NOT_READY:
            return False
        _check(rc, "amc_poll")
        return True

    def wait(self) -> dict:
        _check(lib().amc_wait(self.h), "amc_wait")
        return _collect(self._res, self._arr)

    def times(self):
        t = (C.c_double * 3)()
        _check(lib().amc_request_times(self.h, t), "amc_request_times")
        return tuple(t)

    def close(self):
        if getattr(self, "h", None):
            lib().amc_request_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """amc_batch: several queries in persistent fused launches, replayed from one hipGraph."""

    def __init__(self, ctx: Context, items):
        """items: sequence of (Graph, model dict, query dict)."""
        self.graphs = [g for g, _, _ in items]
        n = len(items)
        self._models = (Model * n)()
        self._queries = (Query * n)()
        self._keep = []
        for k, (g, model, query) in enumerate(items):
            m, km = make_model(**model)
            q, kq = make_query(g.n, **query)
            self._models[k] = m
            self._queries[k] = q
            self._keep += km + kq
        handles = (C.c_void_p * n)(*[g.h for g in self.graphs])
        h = C.c_void_p()
        _check(lib().amc_batch_create(ctx.h, n, handles, self._models, self._queries, C.byref(h)), "amc_batch_create")
        self.h = h

    def run(self) -> list:
        n = len(self.graphs)
        res = (Result * n)()
        arrs = []
        for k, g in enumerate(self.graphs):
            r, a = _alloc_result(g.n, self._queries[k])
            res[k] = r
            arrs.append(a)
        _check(lib().amc_batch_run(self.h, res), "amc_batch_run")
        return [_collect(res[k], arrs[k]) for k in range(n)]

    def info(self):
        a, b = C.c_int32(), C.c_int32()
        _check(lib().amc_batch_info(self.h, C.byref(a), C.byref(b)), "amc_batch_info")
        return {"launches": a.value, "items": b.value}

    def close(self):
        if getattr(self, "h", None):
            lib().amc_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def chain(ctx: Context, Q, **query) -> dict:
    """amc_chain: the tail alone on a given transient block Q."""
    Qa = np.ascontiguousarray(Q, dtype=np.float64)
    n = Qa.shape[0]
    q, keep = make_query(n, **query)
    res, arr = _alloc_result(n, q)
    _check(lib().amc_chain(ctx.h, n, _ptr(Qa, C.c_double), C.byref(q), C.byref(res)), "amc_chain")
    out = _collect(res, arr)
    del keep
    return out


def tune(ctx: Context, graph: Graph, model: dict, probe_R: int = 16, **query) -> dict:
    """amc_tune: times the feasible sweep configurations and records the fastest."""
    m, keep_m = make_model(**model)
    q, keep_q = make_query(graph.n, **query)
    out = TuneResult()
    _check(lib().amc_tune(ctx.h, graph.h, C.byref(m), C.byref(q), int(probe_R), C.byref(out)), "amc_tune")
    del keep_m, keep_q
    return {f: getattr(out, f) for f, _ in TuneResult._fields_}


def footprint(graph: Graph, **query) -> int:
    q, keep = make_query(graph.n, **query)
    b = C.c_uint64()
    _check(lib().amc_footprint(graph.h, C.byref(q), C.byref(b)), "amc_footprint")
    return int(b.value)


def trajectories(ctx: Context, graph: Graph, model: dict, *, seed=0, x0, alpha=0.15, k_min=5, tie_tau=-1.0,
                 max_steps=1024, f=None, want_paths=False, group=0, waves=0, mode=0, flags=0) -> dict:
    """amc_trajectories: episodes of the network process (Section 4.3) and the
    length-biased estimators (b_hat, survival weights, node-reward total).
    mode: MODE_AUTO, MODE_WAVE (realized graph in LDS) or MODE_WAVE_L2 (in the
    workgroup's L2 scratch, steps shared with idle workgroups); flags may add
    TRAJ_B_LDS / TRAJ_B_GLOBAL and DIST16 / DIST32.  The result reports the
    layout used (mode, waves, dist16, b_global) and shared_sources."""
    m, keep_m = make_model(**model)
    x0 = np.ascontiguousarray(x0, dtype=np.int32)
    E = len(x0)
    n = graph.n
    q = TrajQuery()
    q.seed, q.episodes, q.x0 = int(seed), E, _ptr(x0, C.c_int32)
    q.alpha, q.k_min, q.tie_tau, q.max_steps = float(alpha), int(k_min), float(tie_tau), int(max_steps)
    fa = None
    if f is not None:
        fa = np.ascontiguousarray(f, dtype=np.float64)
        q.f = _ptr(fa, C.c_double)
    q.flags = (WANT_PATHS if want_paths else 0) | int(flags)
    q.group, q.waves, q.mode = int(group), int(waves), int(mode)
    arr = {"lengths": np.zeros(E, np.int32), "visits": np.zeros(n, np.uint64), "b_hat": np.zeros(n),
           "survival": np.zeros(max(int(max_steps), 1))}
    if want_paths:
        arr["paths"] = np.zeros((E, int(max_steps)), np.int32)
    res = TrajResult()
    types = {np.dtype(np.int32): C.c_int32, np.dtype(np.uint64): C.c_uint64, np.dtype(np.float64): C.c_double}
    for key, a in arr.items():
        setattr(res, key, _ptr(a, types[a.dtype]))
    _check(lib().amc_trajectories(ctx.h, graph.h, C.byref(m), C.byref(q), C.byref(res)), "amc_trajectories")
    out = dict(arr)
    for key in ("reward_f", "sweep_ms"):
        out[key] = float(getattr(res, key))
    for key in ("switches", "total_steps", "sources", "truncated", "mode", "waves", "dist16", "b_global",
                "shared_sources"):
        out[key] = int(getattr(res, key))
    del keep_m, fa
    return out


def robust(ctx: Context, Q0, *, s=None, f=None, samples=16, delta=0.5, r_min=0.05, seed=0, topology=None) -> dict:
    """amc_robust: transition reward-AFCs, sampled admissible kernels with their KL / TV
    (and, with topology = (eu, ev) or (eu, ev, edge lengths), W1) maximisers, and the
    first-order sensitivity with its remainder (Sections 5.1, 5.4, 6.4, 9.1, 9.2)."""
    Q0 = np.ascontiguousarray(Q0, dtype=np.float64)
    n = Q0.shape[0]
    q = RobustQuery()
    keep = []
    if s is not None:
        sa = np.ascontiguousarray(s, dtype=np.float64)
        keep.append(sa)
        q.s = _ptr(sa, C.c_double)
    if f is not None:
        fa = np.ascontiguousarray(f, dtype=np.float64)
        keep.append(fa)
        q.f = _ptr(fa, C.c_double)
    q.samples, q.delta, q.r_min, q.seed = int(samples), float(delta), float(r_min), int(seed)
    if topology is not None:
        eu = np.ascontiguousarray(topology[0], dtype=np.int32)
        ev = np.ascontiguousarray(topology[1], dtype=np.int32)
        keep += [eu, ev]
        q.m, q.eu, q.ev = len(eu), _ptr(eu, C.c_int32), _ptr(ev, C.c_int32)
        if len(topology) > 2 and topology[2] is not None:
            wa = np.ascontiguousarray(topology[2], dtype=np.uint32)
            keep.append(wa)
            q.w = _ptr(wa, C.c_uint32)
    arr = {"b0": np.zeros(n), "kl": np.zeros(max(samples, 1)), "tv": np.zeros(max(samples, 1)), "b_kl": np.zeros(n),
           "b_tv": np.zeros(n), "b_lin": np.zeros(n), "w1": np.zeros(max(samples, 1)), "b_w1": np.zeros(n)}
    res = RobustResult()
    for key, a in arr.items():
        setattr(res, key, _ptr(a, C.c_double))
    _check(lib().amc_robust(ctx.h, n, _ptr(Q0, C.c_double), C.byref(q), C.byref(res)), "amc_robust")
    out = dict(arr)
    out["kl"], out["tv"], out["w1"] = out["kl"][:samples], out["tv"][:samples], out["w1"][:samples]
    for key in ("b_sw", "b_imp", "norm_N0E", "norm_N0", "rem_bound", "rem_actual", "tail_ms"):
        out[key] = float(getattr(res, key))
    out["kl_arg"], out["tv_arg"], out["w1_arg"] = int(res.kl_arg), int(res.tv_arg), int(res.w1_arg)
    del keep
    return out


def stability(ctx: Context, graph: Graph, model: dict, k: int = 5, **query) -> dict:
    """amc_stability: the estimate at M = R and at 2M realizations and whether
    the Top-k set by b moved (Section 8.4)."""
    m, keep_m = make_model(**model)
    q, keep_q = make_query(graph.n, **query)
    n = graph.n
    arr = {"b_M": np.zeros(n), "b_2M": np.zeros(n), "top_M": np.zeros(k, np.int32), "top_2M": np.zeros(k, np.int32),
           "counts_2M": np.zeros((n, n + 1), np.uint32)}
    res = StabilityResult()
    for key, a in arr.items():
        ct = C.c_double if a.dtype == np.float64 else (C.c_int32 if a.dtype == np.int32 else C.c_uint32)
        setattr(res, key, _ptr(a, ct))
    _check(lib().amc_stability(ctx.h, graph.h, C.byref(m), C.byref(q), int(k), C.byref(res)), "amc_stability")
    out = dict(arr)
    out["same_set"], out["overlap"] = bool(res.same_set), int(res.overlap)
    out["max_abs_diff"], out["sweep_ms"] = float(res.max_abs_diff), float(res.sweep_ms)
    del keep_m, keep_q
    return out


def bootstrap(ctx: Context, next_table, *, replicates=100, level=0.95, floor_eta=-1.0, s=None, seed=0,
              want_reps=True) -> dict:
    """amc_bootstrap: resample each row's R draws with replacement, B times, and
    summarise b per node (Section 8.4).  next_table is R x n (-1 = bottom)."""
    nt = np.ascontiguousarray(next_table, dtype=np.int32)
    R, n = nt.shape
    q = BootQuery()
    keep = []
    if s is not None:
        sa = np.ascontiguousarray(s, dtype=np.float64)
        keep.append(sa)
        q.s = _ptr(sa, C.c_double)
    q.floor_eta, q.replicates, q.level, q.seed = float(floor_eta), int(replicates), float(level), int(seed)
    arr = {k: np.zeros(n) for k in ("b0", "mean", "sd", "lo", "hi")}
    if want_reps:
        arr["b_rep"] = np.zeros((max(int(replicates), 1), n))
    res = BootResult()
    for key, a in arr.items():
        setattr(res, key, _ptr(a, C.c_double))
    _check(lib().amc_bootstrap(ctx.h, n, R, _ptr(nt, C.c_int32), C.byref(q), C.byref(res)), "amc_bootstrap")
    out = dict(arr)
    out["ms"] = float(res.ms)
    del keep
    return out
