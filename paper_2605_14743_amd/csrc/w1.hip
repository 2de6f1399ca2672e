// w1.hip -- Wasserstein-1 between AFC profiles on the shortest-path metric of
// the base topology (unit edge lengths, or given integer lengths), one
// workgroup per sampled profile.
//
// Paper: Bao, Kontou, Vogiatzis, "Betweenness-Central Nodes Under
// Uncertainty: An Absorbing Markov Chain Approach" (robust experiment of
// Section 9.1: discrepancies by W1 with the shortest-path distance of the base
// topology as ground metric; W1 as an integral probability metric, Section 4).
//
// On a graph metric, W1(p, q) is the cost of the cheapest flow that moves the
// surplus p - q over the edges at cost c_e per unit on edge e (c_e = 1 for the
// hop metric).  The workgroup solves that transshipment by successive
// shortest paths, in phases:
//   - the residual graph: an edge carrying flow f from u to v offers v -> u at
//     cost -c_e (capacity f) and u -> v at cost +c_e; a flow-free edge offers
//     both directions at +c_e;
//   - a phase labels every node with (distance, hops) from the nodes with
//     surplus, by parallel Bellman-Ford passes over the edges with 64-bit LDS
//     minima on the packed label until a pass changes nothing (at most n + 1
//     passes: no residual cycle is negative while the flow is optimal for what
//     it has moved, and the lexicographic label makes the shortest walks
//     simple);
//   - every labelled node then keeps one arc that realises its label (the
//     smallest arc code), and while a node with deficit at the smallest
//     distance D* remains (smallest index first), one thread follows these
//     arcs back to a surplus node, checking each against the current flow
//     (the hop count falls by one per arc), and makes the largest push that overdraws
//     neither the surplus, the deficit, nor a cancelled flow is made; each
//     push zeroes one of those exactly (x + (-x) = 0).  A push along such arcs
//     leaves the labels a feasible potential (the reverse of a realising arc
//     realises the label back), so every later path of length D* is still a
//     shortest one; a deficit node whose walk fails is left to the next phase.
// W1 is the sum of c_e |flow| over the edges once no surplus or no deficit is
// left.  Every loop has a bound; exceeding one sets bit 4 of *err.
#include "amc_dev.hpp"
#include "amc_kernels.hpp"

namespace amc {

namespace {

constexpr int kW1Threads = 1024;
constexpr uint64_t kNoLabel = ~0ull;
// distances of simple walks stay within (n - 1) * 65535 < 2^31 (n <= 32768;
// the LDS arrays of 21 n bytes bound n well below that)
constexpr uint64_t kDistBias = 1ull << 31;

__device__ __forceinline__ uint64_t w1_label(int64_t dist, uint32_t hops) {
    return ((uint64_t)(dist + (int64_t)kDistBias) << 32) | hops;
}
__device__ __forceinline__ int64_t w1_dist(uint64_t key) { return (int64_t)(key >> 32) - (int64_t)kDistBias; }

// cost of traversing an edge whose flow has sign sg (-1, 0, +1) from its
// first endpoint (fwd) or from its second
__device__ __forceinline__ int64_t w1_cost(int sg, bool fwd) { return fwd ? (sg < 0 ? -1 : 1) : (sg > 0 ? -1 : 1); }
__device__ __forceinline__ int w1_sign(double f) { return f > 0.0 ? 1 : (f < 0.0 ? -1 : 0); }

}  // namespace

// CACHED: the edge ends (packed 16 + 16 bits), the signs of the flows and the
// edge lengths (16 bits, when given) sit in LDS next to the per-node arrays
// (when they fit), otherwise the ends and lengths are read from HBM and the
// signs from the flows.  LEN: edge lengths len[] are given (otherwise every
// edge has length 1 and len is not read).
template <bool CACHED, bool LEN>
__global__ __launch_bounds__(kW1Threads) void k_w1(int n, int m, const int32_t *eu, const int32_t *ev,
                                                   const uint32_t *len, const int32_t *rp, const int32_t *inc,
                                                   const double *P, const double *q, double *fscr, double *w1,
                                                   int *err) {
    extern __shared__ double w1_smem[];
    double *ex = w1_smem;                                   // n: remaining surplus (> 0) / deficit (< 0)
    uint64_t *key = (uint64_t *)(ex + n);                   // n: packed (distance, hops) labels
    int32_t *path = (int32_t *)(key + n);                   // n: predecessor arcs of the phase (2e + dir)
    uint8_t *tried = (uint8_t *)(path + n);                 // n: deficit nodes whose walk failed this phase
    uint32_t *ends = (uint32_t *)(tried + ((n + 3) & ~3));  // m (CACHED): eu | ev << 16
    int8_t *sgn = (int8_t *)(ends + (CACHED ? m : 0));      // m (CACHED): sign of the flow
    uint16_t *lens = (uint16_t *)(sgn + (CACHED ? ((m + 1) & ~1) : 0));   // m (CACHED, len given): lengths
    __shared__ int s_any_src, s_any_snk, s_changed, s_stop, s_pushed;
    __shared__ uint64_t s_best;
    __shared__ uint32_t s_sink;
    __shared__ double s_part[kW1Threads / 64];
    const int tid = threadIdx.x, k = blockIdx.x;
    const double *p = P + (size_t)k * n;
    double *f = fscr + (size_t)k * m;
    for (int v = tid; v < n; v += kW1Threads) ex[v] = p[v] - q[v];
    for (int e = tid; e < m; e += kW1Threads) {
        f[e] = 0.0;
        if constexpr (CACHED) {
            ends[e] = (uint32_t)eu[e] | ((uint32_t)ev[e] << 16);
            sgn[e] = 0;
            if constexpr (LEN) lens[e] = (uint16_t)len[e];
        }
    }
    auto end_a = [&](int e) { return CACHED ? (int)(ends[e] & 0xFFFFu) : eu[e]; };
    auto end_b = [&](int e) { return CACHED ? (int)(ends[e] >> 16) : ev[e]; };
    auto sign_of = [&](int e) { return CACHED ? (int)sgn[e] : w1_sign(f[e]); };
    auto len_of = [&](int e) -> int64_t {
        if constexpr (!LEN) return 1;
        else return CACHED ? (int64_t)lens[e] : (int64_t)len[e];
    };
    // cost of crossing edge e (flow sign sg) from its first endpoint (fwd) or its second
    auto arc_cost = [&](int e, int sg, bool fwd) { return w1_cost(sg, fwd) * len_of(e); };
    if (tid == 0) s_stop = 0;
    __syncthreads();
    const long max_phases = 16L * ((long)n + m) + 16;
    const long max_tries = 3L * n + m + 8;                  // pushes and failed walks of one phase
    for (long phase = 0;; ++phase) {
        if (tid == 0) {
            s_any_src = 0;
            s_any_snk = 0;
        }
        __syncthreads();
        int src = 0, snk = 0;
        for (int v = tid; v < n; v += kW1Threads) {
            src |= ex[v] > 0.0;
            snk |= ex[v] < 0.0;
        }
        if (src) s_any_src = 1;
        if (snk) s_any_snk = 1;
        __syncthreads();
        if (!s_any_src || !s_any_snk) break;
        if (phase >= max_phases) {
            if (tid == 0) {
                atomicOr(err, 4);
                s_stop = 1;
            }
            break;
        }
        // labels from every node with surplus
        for (int v = tid; v < n; v += kW1Threads) {
            key[v] = ex[v] > 0.0 ? w1_label(0, 0) : kNoLabel;
            tried[v] = 0;
        }
        __syncthreads();
        for (int pass = 0;; ++pass) {
            if (tid == 0) s_changed = 0;
            __syncthreads();
            bool ch = false;
            for (int e = tid; e < m; e += kW1Threads) {
                const int a = end_a(e), b = end_b(e);
                const int sg = sign_of(e);
                const uint64_t ka = key[a], kb = key[b];
                if (ka != kNoLabel) {
                    const uint64_t c = w1_label(w1_dist(ka) + arc_cost(e, sg, true), (uint32_t)ka + 1u);
                    if (c < kb && atomicMin((unsigned long long *)&key[b], (unsigned long long)c) > c) ch = true;
                }
                if (kb != kNoLabel) {
                    const uint64_t c = w1_label(w1_dist(kb) + arc_cost(e, sg, false), (uint32_t)kb + 1u);
                    if (c < ka && atomicMin((unsigned long long *)&key[a], (unsigned long long)c) > c) ch = true;
                }
            }
            if (ch) s_changed = 1;
            __syncthreads();
            const int changed = s_changed;
            __syncthreads();   // every thread has read the flag before it is cleared again
            if (!changed) break;
            if (pass > n + 1) {
                if (tid == 0) {
                    atomicOr(err, 4);
                    s_stop = 1;
                }
                break;
            }
        }
        __syncthreads();
        if (s_stop) break;
        // D*: the smallest distance of a deficit node
        if (tid == 0) s_best = kNoLabel;
        __syncthreads();
        for (int v = tid; v < n; v += kW1Threads)
            if (ex[v] < 0.0 && key[v] != kNoLabel)
                atomicMin((unsigned long long *)&s_best, (unsigned long long)(key[v] | 0xFFFFFFFFull));
        __syncthreads();
        if (s_best == kNoLabel) {   // surplus that reaches no deficit: components out of balance
            if (tid == 0) {
                atomicOr(err, 4);
                s_stop = 1;
            }
            break;
        }
        const uint32_t dhi = (uint32_t)(s_best >> 32);
        // one label-realising arc into every labelled node (the smallest arc
        // code 2 e + dir), so that a path is followed by one thread
        uint32_t *pred = (uint32_t *)path;
        for (int v = tid; v < n; v += kW1Threads) pred[v] = 0xFFFFFFFFu;
        if (tid == 0) s_pushed = 0;
        __syncthreads();
        for (int e = tid; e < m; e += kW1Threads) {
            const int a = end_a(e), b = end_b(e);
            const int sg = sign_of(e);
            const uint64_t ka = key[a], kb = key[b];
            if (ka != kNoLabel && kb != kNoLabel) {
                if (w1_label(w1_dist(ka) + arc_cost(e, sg, true), (uint32_t)ka + 1u) == kb)
                    atomicMin(&pred[b], 2u * (uint32_t)e);
                if (w1_label(w1_dist(kb) + arc_cost(e, sg, false), (uint32_t)kb + 1u) == ka)
                    atomicMin(&pred[a], 2u * (uint32_t)e + 1u);
            }
        }
        __syncthreads();
        int pushes = 0;
        for (long attempt = 0;; ++attempt) {
            if (attempt >= max_tries) {
                if (tid == 0) {
                    atomicOr(err, 4);
                    s_stop = 1;
                }
                break;
            }
            // the next deficit node at distance D* (smallest index)
            if (tid == 0) s_sink = 0xFFFFFFFFu;
            __syncthreads();
            for (int v = tid; v < n; v += kW1Threads)
                if (ex[v] < 0.0 && !tried[v] && key[v] != kNoLabel && (uint32_t)(key[v] >> 32) == dhi)
                    atomicMin(&s_sink, (uint32_t)v);
            __syncthreads();
            const uint32_t tsel = s_sink;
            if (tsel == 0xFFFFFFFFu) break;
            const int t = (int)tsel;
            // thread 0 follows the predecessor arcs back to a node that had
            // surplus, checking each arc against the current flow, then pushes
            if (tid == 0) {
                bool ok = true;
                int x = t, steps = 0;
                double th = -ex[t];
                while ((uint32_t)key[x] != 0u) {                 // hop count 0: a node that had surplus
                    const uint32_t arc = pred[x];
                    if (arc == 0xFFFFFFFFu || ++steps > n) {
                        ok = false;
                        break;
                    }
                    const int e = (int)(arc >> 1);
                    const bool fwd = (arc & 1u) == 0u;           // eu -> ev arrives at x
                    const int y = fwd ? end_a(e) : end_b(e);
                    const uint64_t ky = key[y];
                    if (w1_label(w1_dist(ky) + arc_cost(e, sign_of(e), fwd), (uint32_t)ky + 1u) != key[x]) {
                        ok = false;                               // a push changed this arc's cost
                        break;
                    }
                    const double fe = f[e];
                    if (fwd && fe < 0.0 && -fe < th) th = -fe;
                    if (!fwd && fe > 0.0 && fe < th) th = fe;
                    x = y;
                }
                const int s = x;
                if (!ok || !(ex[s] > 0.0)) {
                    tried[t] = 1;                                 // left to the next phase
                } else {
                    if (ex[s] < th) th = ex[s];
                    for (int z = t; z != s;) {
                        const uint32_t arc = pred[z];
                        const int e = (int)(arc >> 1);
                        const bool fwd = (arc & 1u) == 0u;
                        f[e] += fwd ? th : -th;
                        if constexpr (CACHED) sgn[e] = (int8_t)w1_sign(f[e]);
                        z = fwd ? end_a(e) : end_b(e);
                    }
                    ex[s] -= th;
                    ex[t] += th;
                    s_pushed = 1;
                }
            }
            __syncthreads();
        }
        pushes = s_pushed;
        __syncthreads();
        if (s_stop) break;
        if (pushes == 0) {   // the first walk of a phase always succeeds
            if (tid == 0) {
                atomicOr(err, 4);
                s_stop = 1;
            }
            break;
        }
    }
    __syncthreads();
    double acc = 0.0;
    for (int e = tid; e < m; e += kW1Threads) acc += (double)len_of(e) * fabs(f[e]);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((tid & 63) == 0) s_part[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        double tot = 0.0;
        for (int w = 0; w < kW1Threads / 64; ++w) tot += s_part[w];
        w1[k] = s_stop ? NAN : tot;
    }
}

size_t w1_lds_bytes(int n) { return 20 * (size_t)n + (((size_t)n + 3) & ~(size_t)3); }

// The solver's LDS arrays may use the device's whole LDS (past the default
// 64 KB of dynamic LDS).
hipError_t set_w1_attrs(int max_lds) {
    const void *ks[] = {(const void *)k_w1<true, true>, (const void *)k_w1<true, false>,
                        (const void *)k_w1<false, true>, (const void *)k_w1<false, false>};
    for (const void *kf : ks) {
        const hipError_t e = hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t robust_w1(int n, int m, const int32_t *eu, const int32_t *ev, const uint32_t *len, const int32_t *rp,
                     const int32_t *inc, int batch, const double *P, const double *q, double *fscr, double *w1, int *err,
                     hipStream_t st) {
    // cached layout: ends u32[m] | signs i8[m] (rounded up to even) | lengths u16[m]
    const size_t cached = w1_lds_bytes(n) + 4 * (size_t)m + (((size_t)m + 1) & ~(size_t)1) + (len ? 2 * (size_t)m : 0);
    const bool c = cached <= 64000;
    const uint32_t lds = c ? (uint32_t)cached : w1_lds_bytes(n);
    auto kern = c ? (len ? k_w1<true, true> : k_w1<true, false>) : (len ? k_w1<false, true> : k_w1<false, false>);
    hipLaunchKernelGGL(kern, dim3(batch), dim3(kW1Threads), lds, st, n, m, eu, ev, len, rp, inc, P, q, fscr, w1, err);
    return hipGetLastError();
}

}  // namespace amc
