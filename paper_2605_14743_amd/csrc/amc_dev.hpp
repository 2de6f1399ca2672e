// amc_dev.hpp -- device-side building blocks shared by the sweep and tail
// kernels of the MI355X (gfx950) AFC engine.
//
// Paper: Bao, Kontou, Vogiatzis, "Betweenness-Central Nodes Under
// Uncertainty: An Absorbing Markov Chain Approach".
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amc {

// ---------------------------------------------------------------------------
// Counter-based generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
// Each round multiplies words 0 and 2 by the two Philox multipliers, xors the
// high halves with the other words and the round key; the key is advanced by
// the two Weyl increments between rounds.  The "one Philox call per (r, edge)"
// keying means no realized graph is ever stored: any (r, e) is recomputed.
// ---------------------------------------------------------------------------
struct u32x4 {
    uint32_t x, y, z, w;
};

__host__ __device__ __forceinline__ u32x4 philox10(u32x4 c, uint32_t k0, uint32_t k1) {
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t pa = (uint64_t)kMulA * c.x;
        const uint64_t pb = (uint64_t)kMulB * c.z;
        const u32x4 o = {(uint32_t)(pb >> 32) ^ c.y ^ k0, (uint32_t)pb, (uint32_t)(pa >> 32) ^ c.w ^ k1,
                         (uint32_t)pa};
        c = o;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return c;
}

// ---------------------------------------------------------------------------
// Parameters of one sweep launch (device pointers unless noted).
// ---------------------------------------------------------------------------
struct SweepParams {
    // base graph G(V,E) in CSR form (both directions of every edge)
    int32_t n;
    int64_t m;
    const int32_t *rp_base;     // n+1
    const uint16_t *col;        // 2m neighbour of each slot
    const int32_t *slot_edge;   // 2m edge id of each slot
    const int32_t *eu, *ev;     // m canonical endpoints (Philox counters)
    const uint32_t *w0;         // m fixed weights or nullptr
    // network-state law
    uint64_t t_fail;            // failure threshold floor(p 2^32) of every edge
    const uint64_t *t_fail_edge;// per-edge thresholds or nullptr
    int32_t weight_kind;        // 0 unit, 1 uniform integer, 2 fixed, 3 per-edge table
    uint32_t w_lo, w_span;      // uniform integer law: lo + ((x * span) >> 32); table: w_span = w_max
    const uint64_t *w_cdf;      // table law: m x w_max cumulative thresholds
    // query
    uint32_t key0, key1;        // Philox key = seed
    uint32_t r_begin;           // absolute index of realization 0 of this query
    uint64_t t_alpha;           // stop-coin threshold floor(alpha 2^32)
    uint32_t k_min;
    double tau;                 // tie band
    const uint8_t *pool;        // n membership of W or nullptr
    // work decomposition: item = (r_local, tile), r-major
    int32_t tile;               // sources per item
    int32_t tiles_per_r;
    // LDS carve-up (bytes), computed on the host
    uint32_t adj_cap;           // capacity of the realized adjacency in slots
    uint32_t wave_bytes;        // per-wavefront private region
    uint32_t shift;             // neighbour bits of a realized adjacency entry
    // outputs
    uint32_t *counts, *counts_w;
    int32_t *center_global, *next_table, *next_table_w;
    double *bsum;
    unsigned long long *stats;  // [units, sum_nK, sum_AK, sum_DK, near_band]
    int *err;                   // bit 0: sigma overflow
    // partial-B exchange when a realization spans several items; with
    // keep_rows every realization's B(H_r) and labels are left here for the
    // finite-k Top-k stage
    double *Bg;                 // R x n
    int32_t *compg, *sizeg;     // R x n
    unsigned int *done;         // R
    int32_t keep_rows;
    int32_t hop_radius;         // anchored r-hop neighbourhoods (0 = off)
    int32_t b_global;           // L2 mode: B(H_r) in the global scratch (1) or in LDS (0)
    // per-(r, s) dumps for the parity checks
    const uint32_t *dbg_pairs;  // n_dbg x (r, s)
    int32_t n_dbg;
    uint32_t *dbg_dist;
    unsigned long long *dbg_sigma;
    double *dbg_delta;
};

// Finite-k Top-k stage of one query (one workgroup per realization).
struct TopkArgs {
    int32_t n;
    uint32_t R, r_begin;
    uint32_t key0, key1;
    uint64_t t_alpha;
    uint32_t k_min;
    double tau;
    int32_t topk;
    const double *Bg;           // R x n: B(H_r)
    const int32_t *compg, *sizeg;
    const uint8_t *pool;        // n or nullptr
    const double *gamma;        // n or nullptr (unit values)
    double *psi, *psi_w;        // n: step-reward sums (psi_w nullptr without a pool)
    uint32_t *counts_w;         // n x (n+1) finite-k pool selector counts, or nullptr
    int32_t *next_table_w;      // R x n or nullptr
    unsigned char *gscr;        // per-workgroup arrays in global memory (graphs whose arrays exceed
    uint64_t gscr_bytes;        // the LDS), else nullptr; bytes per workgroup
};

// Trajectory simulator (one workgroup per episode).
struct TrajArgs {
    const SweepParams *desc;    // graph, law, key, k_min, tau, LDS carve-up (device)
    int32_t episodes;
    const int32_t *x0;          // episodes
    int32_t max_steps;
    const double *f;            // node reward (n) or nullptr
    int32_t *lengths;           // episodes
    int32_t *paths;             // episodes x max_steps or nullptr
    unsigned long long *visits; // n
    double *reward;             // sum of f(X_t)
    unsigned long long *ctr;    // switches, total steps, truncated, sources run, sources run by other workgroups
    unsigned int *work;         // [0] next episode, [1] episodes ended
    int *err;
    uint32_t *bscratch;         // L2 layout: per-workgroup scratch (realized graph), else nullptr
    uint64_t bscratch_words;    // 32-bit words per workgroup
    // shared steps (L2 layout): per workgroup a claim word (epoch << 32 |
    // |K| << 16 | next source) and a completion word (sources other
    // workgroups ran << 32 | sources done), the step's K(X_t;H) and the B(H)
    // contributions of the sources other workgroups ran
    unsigned long long *share;  // 2 per workgroup
    unsigned long long *open;   // bit b: workgroup b's step has unclaimed sources ((blocks + 63) / 64 words)
    int32_t *glist;             // n per workgroup
    double *hb;                 // n per workgroup
};

// One sweep launch serves one or several queries: the launch's work items are
// the concatenation of every query's (r, tile) items; item_start[q] is the
// first item of query q (item_start[nq] = total).
struct LaunchCtl {
    const SweepParams *descs;   // nq query descriptors (device)
    const uint32_t *item_start; // nq + 1 (device)
    int32_t nq;
    uint32_t n_items;           // items fetched by this launch
    uint32_t item_base;         // item index of fetch 0
    int32_t static_items;       // 1: block b takes item item_base + b; 0: work counter
    unsigned int *work_ctr;
    uint32_t *bscratch;         // workgroup-per-source and L2 modes: per-workgroup global scratch
    uint32_t bscratch_words;
    // nq entries or nullptr: the launch's items of query q are that query's own
    // items item_off[q] .. item_off[q] + (item_start[q+1] - item_start[q]) - 1
    // (a launch may carry any contiguous range of a query's items)
    const uint32_t *item_off;
};

// The query owning global item `item` (uniform scalar search).
__device__ __forceinline__ int item_query(const LaunchCtl &L, uint32_t item) {
    int q = 0;
    while (q + 1 < L.nq && item >= L.item_start[q + 1]) ++q;
    return q;
}

// Index of global item `item` among query q's own items.
__device__ __forceinline__ uint32_t item_local(const LaunchCtl &L, int q, uint32_t item) {
    return item - L.item_start[q] + (L.item_off ? L.item_off[q] : 0u);
}

constexpr uint32_t kInf = 0x3FFFFFFFu;   // "unreached"; d + w never wraps
// Weight given to an adjacency slot past a vertex's list: for every distance
// d <= kInf and every reached distance D < kInf, d + kNoEdge != D,
// D + kNoEdge > d and d != D + kNoEdge, and no sum exceeds 2^31.
constexpr uint32_t kNoEdge = kInf + 1u;
constexpr int kMaxWaves = 16;
constexpr uint32_t kAdjPad = 24;         // zero entries after the realized adjacency

// ---------------------------------------------------------------------------
// Wavefront helpers (wave64).
// ---------------------------------------------------------------------------
// Orders the LDS traffic of one wavefront: every LDS access issued before the
// call completes before any issued after it (LDS requests of one wavefront are
// serviced in order once they are all issued), and the compiler may not move
// memory operations across it.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// Number of set bits of m below the calling lane (its rank among the lanes of m).
__device__ __forceinline__ uint32_t rank_lt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    const uint32_t lo = __builtin_amdgcn_mbcnt_lo(~0u, 0u);
    const uint32_t lane = __builtin_amdgcn_mbcnt_hi(~0u, lo);
    return (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const uint32_t o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ int wave_min_i32(int v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const int o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ double wave_max_f64(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------------------
// DPP lane exchanges (VALU only, no LDS traffic).  All callers run with the
// whole wavefront active.
//   0xB1 quad_perm [1,0,3,2]  (lane ^ 1)      0x4E quad_perm [2,3,0,1] (lane ^ 2)
//   0x141 row_half_mirror (7 - lane in 8)     0x140 row_mirror (15 - lane in 16)
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp64(unsigned long long v) {
    const uint32_t lo = dpp32<CTRL>((uint32_t)v), hi = dpp32<CTRL>((uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// Sum over aligned groups of G lanes (G in 1, 4, 8, 16); every lane of a group
// receives the group total.  `ovf` records a wrap of the uint64 sum.
template <int G>
__device__ __forceinline__ unsigned long long group_sum_u64(unsigned long long x, bool &ovf) {
    unsigned long long y, t;
    if (G >= 2) { y = dpp64<0xB1>(x); t = x + y; ovf |= t < x; x = t; }
    if (G >= 4) { y = dpp64<0x4E>(x); t = x + y; ovf |= t < x; x = t; }
    if (G >= 8) { y = dpp64<0x141>(x); t = x + y; ovf |= t < x; x = t; }
    if (G >= 16) { y = dpp64<0x140>(x); t = x + y; ovf |= t < x; x = t; }
    return x;
}
template <int G>
__device__ __forceinline__ double group_sum_f64(double x) {
    if (G >= 2) x += __longlong_as_double((long long)dpp64<0xB1>((unsigned long long)__double_as_longlong(x)));
    if (G >= 4) x += __longlong_as_double((long long)dpp64<0x4E>((unsigned long long)__double_as_longlong(x)));
    if (G >= 8) x += __longlong_as_double((long long)dpp64<0x141>((unsigned long long)__double_as_longlong(x)));
    if (G >= 16) x += __longlong_as_double((long long)dpp64<0x140>((unsigned long long)__double_as_longlong(x)));
    return x;
}
// Minimum / maximum over the wavefront, returned uniformly.
__device__ __forceinline__ uint32_t wave_min_fast(uint32_t x) {
    uint32_t y;
    y = dpp32<0xB1>(x); x = y < x ? y : x;
    y = dpp32<0x4E>(x); x = y < x ? y : x;
    y = dpp32<0x141>(x); x = y < x ? y : x;
    y = dpp32<0x140>(x); x = y < x ? y : x;
    const uint32_t a = __builtin_amdgcn_readlane(x, 0), b = __builtin_amdgcn_readlane(x, 16);
    const uint32_t c = __builtin_amdgcn_readlane(x, 32), d = __builtin_amdgcn_readlane(x, 48);
    const uint32_t ab = a < b ? a : b, cd = c < d ? c : d;
    return ab < cd ? ab : cd;
}
__device__ __forceinline__ uint32_t wave_max_fast(uint32_t x) {
    uint32_t y;
    y = dpp32<0xB1>(x); x = y > x ? y : x;
    y = dpp32<0x4E>(x); x = y > x ? y : x;
    y = dpp32<0x141>(x); x = y > x ? y : x;
    y = dpp32<0x140>(x); x = y > x ? y : x;
    const uint32_t a = __builtin_amdgcn_readlane(x, 0), b = __builtin_amdgcn_readlane(x, 16);
    const uint32_t c = __builtin_amdgcn_readlane(x, 32), d = __builtin_amdgcn_readlane(x, 48);
    const uint32_t ab = a > b ? a : b, cd = c > d ? c : d;
    return ab > cd ? ab : cd;
}

// Appends the lanes with `pred` set to a queue whose tail is *ctr (LDS): one
// LDS atomic per wavefront; returns each appending lane's slot.  Called with
// the whole wavefront active.
__device__ __forceinline__ uint32_t wave_append(uint32_t *ctr, bool pred) {
    const uint64_t mask = __ballot(pred);
    uint32_t pos = 0;
    if (mask) {
        const int leader = __ffsll((unsigned long long)mask) - 1;
        uint32_t base = 0;
        if ((int)(threadIdx.x & 63) == leader) base = atomicAdd(ctr, (uint32_t)__popcll(mask));
        base = __builtin_amdgcn_readlane(base, leader);
        pos = base + (uint32_t)__popcll(mask & lanemask_lt());
    }
    return pos;
}

__device__ __forceinline__ double as_f64(unsigned long long b) { return __longlong_as_double((long long)b); }
__device__ __forceinline__ unsigned long long as_u64(double d) { return (unsigned long long)__double_as_longlong(d); }

// A pointer the compiler treats as global memory (addrspace 1), so loads and
// stores through it are global_* rather than flat instructions (flat accesses
// also count against the LDS wait counter and serialise with LDS traffic).
template <typename T>
__device__ __forceinline__ T *to_global(T *p) {
    return (T *)((__attribute__((address_space(1))) T *)p);
}

// Element idx of an array addressed by a 32-bit byte offset from its base: a
// global array is then read with the base in scalar registers and the offset
// in one vector register, without 64-bit address arithmetic per lane (the
// arrays read this way are far below 4 GiB).
template <typename T>
__device__ __forceinline__ T ld_off32(const T *base, uint32_t idx) {
    return *(const T *)((const char *)base + idx * (uint32_t)sizeof(T));
}

// Adds into a double in global memory with a global (not flat) atomic: a flat
// atomic would also hold the LDS wait counter of the issuing wavefront.
__device__ __forceinline__ void global_add_f64(double *p, double v) {
    (void)__builtin_amdgcn_global_atomic_fadd_f64((__attribute__((address_space(1))) double *)p, v);
}

// Plain store through a global (not flat) pointer.
template <typename T>
__device__ __forceinline__ void st_global(T *p, T v) {
    *(__attribute__((address_space(1))) T *)p = v;
}

// Where a wavefront adds delta_s(v) into B(H_r): an LDS array (lds), or,
// with glob set, an array in the workgroup's global scratch (gl).  Device
// atomics on a global B leave the XCD's L2 as one fabric write each, so B
// stays in LDS unless that costs a wavefront.  Both pointers keep their
// address space, so each add is a plain LDS or global atomic.
struct BAcc {
    double *lds, *gl;
    bool glob;
};
__device__ __forceinline__ void add_B(const BAcc &B, int v, double delta) {
    if (B.glob) global_add_f64(&B.gl[v], delta);
    else unsafeAtomicAdd(&B.lds[v], delta);
}

// Load that bypasses the CU's vector L1 when COH: values produced by device
// atomics (performed at L2) or by other workgroups.
template <bool COH, typename T>
__device__ __forceinline__ T ld_coh(const T *p) {
    if constexpr (COH) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *p;
}

}  // namespace amc
