// sweep_common.hpp -- pieces shared by the two sweep modes: the block scan,
// the staging of one realization, the per-realization reduction and the
// dump lookup.
//
// Paper: Bao, Kontou, Vogiatzis, "Betweenness-Central Nodes Under
// Uncertainty: An Absorbing Markov Chain Approach".
#pragma once

#include "amc_dev.hpp"

namespace amc {

struct ReduceScratch {
    unsigned long long *cmax, *wmax;   // per component: max B (bit pattern), max B over the pool
    int32_t *ccen, *wcen;              // per component: centre, pool-constrained centre
};

// ---------------------------------------------------------------------------
// Block-wide exclusive scan of one uint32 per thread.
// ---------------------------------------------------------------------------
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *tmp, uint32_t &total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) tmp[wave] = x;
    __syncthreads();
    if (wave == 0) {
        uint32_t t = lane < nwaves ? tmp[lane] : 0u;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(t, off, 64);
            if (lane >= off) t += y;
        }
        if (lane < nwaves) tmp[lane] = t;
    }
    __syncthreads();
    const uint32_t prefix = (wave > 0 ? tmp[wave - 1] : 0u) + x - v;
    total = tmp[nwaves - 1];
    __syncthreads();
    return prefix;
}

// Realizes every base edge of realization r (Section 3.1) and builds the
// compacted adjacency of H_r: rp[v] .. rp[v+1] index adj, each entry holds
// (weight << shift) | neighbour.  `ew` is scratch for the per-edge weights
// (0 = the edge failed).  Edge (u, v) draws from counter (r, u, v, stream):
// stream 0 for the row-wise sweep, 2 + step for a trajectory step.
template <typename RP, typename ADJ>
__device__ inline void stage_realization(const SweepParams &P, uint32_t r, RP *rp, ADJ *adj, uint32_t shift,
                                         uint16_t *ew, uint32_t *scan_tmp, uint32_t stream = 0u) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int n = P.n;
    for (int64_t e = tid; e < P.m; e += nthr) {
        const u32x4 x = philox10({r, (uint32_t)P.eu[e], (uint32_t)P.ev[e], stream}, P.key0, P.key1);
        const uint64_t t = P.t_fail_edge ? P.t_fail_edge[e] : P.t_fail;
        uint32_t w;
        if (P.weight_kind == 0) w = 1u;
        else if (P.weight_kind == 1) w = P.w_lo + __umulhi(x.y, P.w_span);
        else if (P.weight_kind == 3) {   // smallest v with x1 < T_e(v) (Section 9.2 resampling)
            const uint64_t *T = P.w_cdf + (size_t)e * P.w_span;
            w = 1u;
            while (w < P.w_span && (uint64_t)x.y >= T[w - 1]) ++w;
        }
        else w = P.w0[e];
        ew[e] = ((uint64_t)x.x >= t) ? (uint16_t)w : (uint16_t)0;
    }
    __syncthreads();
    // contiguous vertex chunk per thread: count, scan, scatter
    const int chunk = (n + nthr - 1) / nthr;
    const int v0 = min(n, tid * chunk), v1 = min(n, v0 + chunk);
    uint32_t cnt = 0;
    for (int v = v0; v < v1; ++v)
        for (int j = P.rp_base[v]; j < P.rp_base[v + 1]; ++j) cnt += ew[P.slot_edge[j]] != 0;
    uint32_t total;
    uint32_t pos = block_exclusive_scan(cnt, scan_tmp, total);
    for (int v = v0; v < v1; ++v) {
        rp[v] = (RP)pos;
        for (int j = P.rp_base[v]; j < P.rp_base[v + 1]; ++j) {
            const uint32_t w = ew[P.slot_edge[j]];
            if (w) adj[pos++] = (ADJ)((w << shift) | (uint32_t)P.col[j]);
        }
    }
    if (tid == 0) rp[n] = (RP)total;
    if (tid < (int)kAdjPad) adj[total + tid] = (ADJ)0;   // padding read by unpredicated loads
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Reduction of one realization (all sources done): centres, coins, counts.
// `comp`/`csize` give each vertex's component label (smallest index) and
// size; the scratch arrays hold n entries each (LDS or global memory).  With
// COH, B, comp and csize are global arrays written by device atomics or by
// other workgroups and are read past the vector L1.
// ---------------------------------------------------------------------------
template <typename RP, typename CT, bool COH = false>
__device__ inline void reduce_realization(const SweepParams &P, uint32_t r_local, uint32_t r, const RP *rp,
                                   const double *B, const CT *comp, const CT *csize, const ReduceScratch &S,
                                   double *red_f, int *red_i, unsigned long long *acc_stats, bool write_rows) {
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, wave = tid >> 6, nwaves = nthr >> 6;
    const int n = P.n;
    unsigned long long *cmax = S.cmax;   // B >= 0: max on the bit pattern
    unsigned long long *wmax = S.wmax;
    int32_t *ccen = S.ccen;
    int32_t *wcen = S.wcen;
    for (int v = tid; v < n; v += nthr) {
        cmax[v] = 0ull;
        wmax[v] = 0ull;
        ccen[v] = 0x7FFFFFFF;
        wcen[v] = 0x7FFFFFFF;
    }
    __syncthreads();
    // work counters: every anchor i counts the surviving and the base slots
    // of its component, i.e. vertex v's slots are counted once per member
    // of v's component (size csize[v])
    unsigned long long s_ak = 0, s_dk = 0;
    double gm = 0.0;
    for (int v = tid; v < n; v += nthr) {
        const int c = (int)ld_coh<COH>(&comp[v]);
        const double bv = ld_coh<COH>(&B[v]);
        const unsigned long long bb = as_u64(bv);
        atomicMax(&cmax[c], bb);
        if (P.pool && P.pool[v]) atomicMax(&wmax[c], bb);
        const unsigned long long sz = (unsigned long long)ld_coh<COH>(&csize[v]);
        s_ak += sz * ((uint32_t)rp[v + 1] - (uint32_t)rp[v]);
        s_dk += sz * (unsigned long long)(P.rp_base[v + 1] - P.rp_base[v]);
        gm = bv > gm ? bv : gm;
    }
    gm = wave_max_f64(gm);
    if (lane == 0) red_f[wave] = gm;
    __syncthreads();
    gm = red_f[0];
    for (int w = 1; w < nwaves; ++w) gm = red_f[w] > gm ? red_f[w] : gm;
    const double gband = P.tau * (gm > 1.0 ? gm : 1.0);
    int gbest = 0x7FFFFFFF;
    unsigned long long near = 0;
    for (int v = tid; v < n; v += nthr) {
        const int c = (int)ld_coh<COH>(&comp[v]);
        const double bv = ld_coh<COH>(&B[v]);
        const double mx = as_f64(cmax[c]);
        const double band = P.tau * (mx > 1.0 ? mx : 1.0);
        const double gap = mx - bv;
        if (gap <= band) atomicMin(&ccen[c], v);
        near += (band > 0.0 && gap >= 0.25 * band && gap <= 4.0 * band);
        if (P.pool && P.pool[v]) {
            const double mw = as_f64(wmax[c]);
            const double bw = P.tau * (mw > 1.0 ? mw : 1.0);
            const double gw = mw - bv;
            if (gw <= bw) atomicMin(&wcen[c], v);
            near += (bw > 0.0 && gw >= 0.25 * bw && gw <= 4.0 * bw);
        }
        const double gg = gm - bv;
        if (gg <= gband && v < gbest) gbest = v;
        near += (gband > 0.0 && gg >= 0.25 * gband && gg <= 4.0 * gband);
    }
    gbest = wave_min_i32(gbest);
    __syncthreads();   // red_f reads done before red_i reuse
    if (lane == 0) red_i[wave] = gbest;
    __syncthreads();
    if (tid == 0) {
        int b = red_i[0];
        for (int w = 1; w < nwaves; ++w) b = min(b, red_i[w]);
        if (P.center_global) P.center_global[r_local] = b;
    }
    // anchors: Alg. 1 for every i, counted as in Alg. 2
    unsigned long long s_nk = 0, units = 0;
    for (int i = tid; i < n; i += nthr) {
        const int c = (int)ld_coh<COH>(&comp[i]);
        const uint32_t sz = (uint32_t)ld_coh<COH>(&csize[i]);
        const u32x4 x = philox10({r, (uint32_t)i, 0xFFFFFFFFu, 1u}, P.key0, P.key1);
        const bool coin = (uint64_t)x.x < P.t_alpha;
        const bool valid = !coin && sz >= P.k_min;
        const int nx = valid ? ccen[c] : -1;
        atomicAdd(&P.counts[(size_t)i * (n + 1) + (nx >= 0 ? nx : n)], 1u);
        if (P.next_table) P.next_table[(size_t)r_local * n + i] = nx;
        if (P.counts_w) {
            const int nw = (valid && P.pool && wcen[c] != 0x7FFFFFFF) ? wcen[c] : -1;
            atomicAdd(&P.counts_w[(size_t)i * (n + 1) + (nw >= 0 ? nw : n)], 1u);
            if (P.next_table_w) P.next_table_w[(size_t)r_local * n + i] = nw;
        }
        units += 1;
        s_nk += (unsigned long long)sz;
    }
    if (P.bsum)
        for (int v = tid; v < n; v += nthr) unsafeAtomicAdd(&P.bsum[v], ld_coh<COH>(&B[v]));
    // B(H_r) and the labels for the finite-k Top-k stage (rows a split
    // realization has already assembled there are left as they are)
    if (P.keep_rows && write_rows)
        for (int v = tid; v < n; v += nthr) {
            P.Bg[(size_t)r_local * n + v] = ld_coh<COH>(&B[v]);
            P.compg[(size_t)r_local * n + v] = (int32_t)ld_coh<COH>(&comp[v]);
            P.sizeg[(size_t)r_local * n + v] = (int32_t)ld_coh<COH>(&csize[v]);
        }
    acc_stats[0] += units;
    acc_stats[1] += s_nk;
    acc_stats[2] += s_ak;
    acc_stats[3] += s_dk;
    acc_stats[4] += near;
    __syncthreads();
}

// Adds a workgroup's counters to its query's totals and clears them.
__device__ inline void flush_stats(const SweepParams &P, unsigned long long (&acc)[5], bool &ovf) {
    const int lane = threadIdx.x & 63;
    const bool any_ovf = __ballot(ovf) != 0ull;
    if (any_ovf && lane == 0) atomicOr(P.err, 1);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const unsigned long long v = wave_sum_u64(acc[k]);
        if (lane == 0 && v) atomicAdd(&P.stats[k], v);
        acc[k] = 0;
    }
    ovf = false;
}

// Lookup of a (r, s) pair in the dump list; -1 when absent.
__device__ __forceinline__ int debug_slot(const SweepParams &P, uint32_t r, int s) {
    for (int k = 0; k < P.n_dbg; ++k)
        if (P.dbg_pairs[2 * k] == r && (int)P.dbg_pairs[2 * k + 1] == s) return k;
    return -1;
}

}  // namespace amc
