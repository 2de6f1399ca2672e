// sweep_wave.hip -- realization x source sweep with the realized graph staged
// in LDS and one wavefront per (realization, source).
//
// Paper: Bao, Kontou, Vogiatzis, "Betweenness-Central Nodes Under
// Uncertainty: An Absorbing Markov Chain Approach".
//
// One workgroup takes a work item (realization r, source tile) at a time:
//   1. realize every base edge of r with one Philox call (Section 3.1) and
//      compact the surviving slots into an LDS adjacency (weight | neighbour);
//   2. each wavefront runs, for its sources s, the single-source shortest
//      paths with exact uint64 path counts (breadth-first levels for unit
//      weights, distance buckets for integer weights >= 1) and the reverse
//      dependency accumulation of the Section 3.1 betweenness, adding delta_s
//      into a workgroup-wide B(H_r) in LDS;
//   3. once every source of r is done, the workgroup reduces B(H_r) to the
//      global centre (eq. central-node), the component centres (eq.
//      local-center) and the pool-constrained centres (Section 7.1), draws
//      every anchor's stop coin, applies k_min and counts next(r, i)
//      (Alg. 1 for every anchor, tallied as in Alg. 2).
#include "amc_dev.hpp"
#include "amc_kernels.hpp"
#include "sweep_common.hpp"

namespace amc {

// ---------------------------------------------------------------------------
// One source on one wavefront.  State (LDS, private to the wavefront):
//   dist[n]  tentative / final distance (kInf = unreached)
//   sig[n]   exact path count sigma_s(v) (uint64); after v's dependency is
//            known the slot holds c_v = (1 + delta_v) / sigma_v as a double,
//            so a predecessor u gets delta_u = sigma_u * sum_{succ w} c_w
//   ord[n]   settled vertices in non-decreasing distance
//   aux[n]   front: unsettled reached vertices (integer weights only);
//            back:  start of each equal-distance segment of ord
// G lanes cooperate on one vertex's adjacency.
// ---------------------------------------------------------------------------
template <bool WEIGHTED, int G>
__device__ void wave_source(const SweepParams &P, const uint32_t *rp, const uint32_t *adj, double *B, uint32_t *dist,
                            unsigned long long *sig, uint16_t *ord, uint16_t *aux, uint32_t *ctr, int s,
                            int dbg_slot, int &comp_out, int &size_out, bool &ovf) {
    const int n = P.n;
    const int lane = threadIdx.x & 63;
    const int sub = lane % G;
    constexpr int VPI = 64 / G;   // vertices per wave iteration

    for (int v = lane; v < n; v += 64) dist[v] = kInf;
    wave_sync();
    if (lane == 0) {
        dist[s] = 0u;
        sig[s] = 1ull;
        ord[0] = (uint16_t)s;
        *ctr = WEIGHTED ? 0u : 1u;
    }
    wave_sync();

    int f_lo = 0, ord_end = 1, nseg = 0;
    uint32_t D = 0;
    // ------------------------------------------------------------ forward
    for (;;) {
        if (lane == 0) aux[n - 1 - nseg] = (uint16_t)f_lo;
        ++nseg;
        for (int base = f_lo; base < ord_end; base += VPI) {
            const int idx = base + lane / G;
            const bool mine = idx < ord_end;
            unsigned long long acc = 0ull;
            int v = 0;
            if (mine) {
                v = ord[idx];
                const uint32_t beg = rp[v], end = rp[v + 1];
                for (uint32_t j = beg + sub; j < end; j += G) {
                    const uint32_t a = adj[j];
                    const uint32_t u = a & 0xFFFFu;
                    const uint32_t w = WEIGHTED ? (a >> 16) : 1u;
                    const uint32_t du = dist[u];
                    if (du + w == D) {                       // u precedes v: pull sigma_u
                        const unsigned long long t = acc + sig[u];
                        ovf |= t < acc;
                        acc = t;
                    } else if (D + w < du) {                 // relax the edge v -> u
                        const uint32_t old = atomicMin(&dist[u], D + w);
                        if (old == kInf) {                   // first discovery of u
                            const uint32_t pos = atomicAdd(ctr, 1u);
                            if (WEIGHTED) aux[pos] = (uint16_t)u;
                            else ord[pos] = (uint16_t)u;
                        }
                    }
                }
            }
#pragma unroll
            for (int off = 1; off < G; off <<= 1) {
                const unsigned long long o = __shfl_xor(acc, off, 64);
                const unsigned long long t = acc + o;
                ovf |= t < acc;
                acc = t;
            }
            if (mine && sub == 0 && v != s) sig[v] = acc;
        }
        wave_sync();
        if (!WEIGHTED) {
            const int new_end = (int)*ctr;
            if (new_end == ord_end) break;
            f_lo = ord_end;
            ord_end = new_end;
            D += 1u;
        } else {
            const int fr = (int)*ctr;
            if (fr == 0) break;
            uint32_t mn = kInf;
            for (int k = lane; k < fr; k += 64) {
                const uint32_t dk = dist[aux[k]];
                mn = dk < mn ? dk : mn;
            }
            mn = wave_min_u32(mn);
            // move the vertices at the new minimum distance to ord, keep the
            // rest (compacted in place: writes never pass the read position)
            int settled = 0, kept = 0;
            const uint64_t lt = lanemask_lt();
            for (int k0 = 0; k0 < fr; k0 += 64) {
                const int k = k0 + lane;
                const bool valid = k < fr;
                const uint32_t x = valid ? aux[k] : 0u;
                const bool is_s = valid && dist[x] == mn;
                const bool is_k = valid && !is_s;
                const uint64_t ms = __ballot(is_s), mk = __ballot(is_k);
                if (is_s) ord[ord_end + settled + __popcll(ms & lt)] = (uint16_t)x;
                if (is_k) aux[kept + __popcll(mk & lt)] = (uint16_t)x;
                settled += __popcll(ms);
                kept += __popcll(mk);
            }
            if (lane == 0) *ctr = (uint32_t)kept;
            wave_sync();
            f_lo = ord_end;
            ord_end += settled;
            D = mn;
        }
    }

    // component of s: smallest reached index, and its size
    {
        int mn = n;
        for (int k = lane; k < ord_end; k += 64) mn = min(mn, (int)ord[k]);
        comp_out = wave_min_i32(mn);
        size_out = ord_end;
    }
    if (dbg_slot >= 0) {
        for (int v = lane; v < n; v += 64) {
            const uint32_t d = dist[v];
            P.dbg_dist[(size_t)dbg_slot * n + v] = d == kInf ? 0xFFFFFFFFu : d;
            P.dbg_sigma[(size_t)dbg_slot * n + v] = d == kInf ? 0ull : sig[v];
            P.dbg_delta[(size_t)dbg_slot * n + v] = 0.0;
        }
        wave_sync();
    }

    // ------------------------------------------------------------ backward
    for (int k = nseg - 1; k >= 0; --k) {
        const int lo = aux[n - 1 - k];
        const int hi = (k == nseg - 1) ? ord_end : (int)aux[n - 2 - k];
        for (int base = lo; base < hi; base += VPI) {
            const int idx = base + lane / G;
            const bool mine = idx < hi;
            double sum = 0.0;
            int v = 0;
            if (mine) {
                v = ord[idx];
                const uint32_t dv = dist[v];
                const uint32_t beg = rp[v], end = rp[v + 1];
                for (uint32_t j = beg + sub; j < end; j += G) {
                    const uint32_t a = adj[j];
                    const uint32_t u = a & 0xFFFFu;
                    const uint32_t w = WEIGHTED ? (a >> 16) : 1u;
                    if (dist[u] == dv + w) sum += as_f64(sig[u]);   // u succeeds v: c_u
                }
            }
#pragma unroll
            for (int off = 1; off < G; off <<= 1) sum += __shfl_xor(sum, off, 64);
            if (mine && sub == 0) {
                const double sv = (double)sig[v];
                const double delta = sv * sum;
                sig[v] = as_u64((1.0 + delta) / sv);
                if (v != s) atomicAdd(&B[v], delta);
                if (dbg_slot >= 0) P.dbg_delta[(size_t)dbg_slot * n + v] = delta;
            }
        }
        wave_sync();
    }
}

// Byte offsets of the LDS carve-up (mirrors lds_layout_wave on the host).
struct WaveLayout {
    uint32_t rp, adj, B, comp, csize, waves;
};
__device__ __forceinline__ WaveLayout wave_layout(int n, uint32_t adj_cap) {
    WaveLayout L;
    L.rp = 0;
    L.adj = L.rp + 4u * (uint32_t)(n + 1);
    L.B = (L.adj + 4u * adj_cap + 7u) & ~7u;
    L.comp = L.B + 8u * (uint32_t)n;
    L.csize = L.comp + 4u * (uint32_t)n;
    L.waves = (L.csize + 4u * (uint32_t)n + 15u) & ~15u;
    return L;
}

template <bool WEIGHTED, int G>
__global__ __launch_bounds__(1024) void sweep_wave_kernel(SweepParams P) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __shared__ uint32_t scan_tmp[kMaxWaves];
    __shared__ uint32_t wctr[kMaxWaves];
    __shared__ double red_f[kMaxWaves];
    __shared__ int red_i[kMaxWaves];
    __shared__ int item_sh;
    __shared__ int last_sh;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
    const int n = P.n;
    const WaveLayout L = wave_layout(n, P.adj_cap);
    uint32_t *rp = (uint32_t *)(smem + L.rp);
    uint32_t *adj = (uint32_t *)(smem + L.adj);
    double *B = (double *)(smem + L.B);
    int32_t *comp = (int32_t *)(smem + L.comp);
    int32_t *csize = (int32_t *)(smem + L.csize);
    unsigned char *wbase = smem + L.waves;
    uint32_t *dist = (uint32_t *)(wbase + (size_t)wave * P.wave_bytes);
    unsigned long long *sig = (unsigned long long *)(((uintptr_t)(dist + n) + 7u) & ~(uintptr_t)7u);
    uint16_t *ord = (uint16_t *)(sig + n);
    uint16_t *aux = ord + n;
    ReduceScratch RS;
    RS.cmax = (unsigned long long *)wbase;
    RS.wmax = RS.cmax + n;
    RS.ccen = (int32_t *)(RS.wmax + n);
    RS.wcen = RS.ccen + n;
    RS.kal = (uint32_t *)(RS.wcen + n);
    RS.kba = RS.kal + n;

    unsigned long long acc_stats[5] = {0, 0, 0, 0, 0};
    bool ovf = false;
    uint32_t local = 0;
    for (;;) {
        if (P.static_items) {
            if (local > 0) break;
            local = 1;
            item_sh = (int)blockIdx.x;
        } else {
            if (tid == 0) item_sh = (int)atomicAdd(P.work_ctr, 1u);
            __syncthreads();
        }
        const int it = item_sh;
        __syncthreads();
        if ((uint32_t)it >= P.n_items) break;
        const uint32_t item = P.item_base + (uint32_t)it;
        const uint32_t r_local = item / (uint32_t)P.tiles_per_r;
        const int t = (int)(item % (uint32_t)P.tiles_per_r);
        const uint32_t r = P.r_begin + r_local;

        stage_realization(P, r, rp, adj, (uint16_t *)wbase, scan_tmp);
        for (int v = tid; v < n; v += blockDim.x) B[v] = 0.0;
        __syncthreads();

        const int s_lo = t * P.tile, s_hi = min(n, s_lo + P.tile);
        for (int s = s_lo + wave; s < s_hi; s += nwaves) {
            int cs = 0, sz = 0;
            const int slot = P.n_dbg ? debug_slot(P, r, s) : -1;
            wave_source<WEIGHTED, G>(P, rp, adj, B, dist, sig, ord, aux, &wctr[wave], s, slot, cs, sz, ovf);
            if (lane == 0) {
                comp[s] = cs;
                csize[s] = sz;
            }
        }
        __syncthreads();

        if (P.tiles_per_r == 1) {
            reduce_realization(P, r_local, r, rp, B, comp, csize, RS, red_f, red_i, acc_stats);
        } else {
            // publish this tile's partial B and component labels; the last
            // tile of the realization to finish performs the reduction
            double *Bg = P.Bg + (size_t)r_local * n;
            for (int v = tid; v < n; v += blockDim.x)
                if (B[v] != 0.0) unsafeAtomicAdd(&Bg[v], B[v]);
            for (int s = s_lo + tid; s < s_hi; s += blockDim.x) {
                P.compg[(size_t)r_local * n + s] = comp[s];
                P.sizeg[(size_t)r_local * n + s] = csize[s];
            }
            __threadfence();
            __syncthreads();
            if (tid == 0) last_sh = (atomicAdd(&P.done[r_local], 1u) == (unsigned)(P.tiles_per_r - 1));
            __syncthreads();
            if (last_sh) {
                __threadfence();
                for (int v = tid; v < n; v += blockDim.x) {
                    B[v] = __hip_atomic_load(&Bg[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    comp[v] = __hip_atomic_load(&P.compg[(size_t)r_local * n + v], __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
                    csize[v] = __hip_atomic_load(&P.sizeg[(size_t)r_local * n + v], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
                }
                __syncthreads();
                reduce_realization(P, r_local, r, rp, B, comp, csize, RS, red_f, red_i, acc_stats);
            }
            __syncthreads();
        }
    }
    // flush counters
    if (ovf) atomicOr(P.err, 1);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const unsigned long long v = wave_sum_u64(acc_stats[k]);
        if (lane == 0 && v) atomicAdd(&P.stats[k], v);
    }
}

// ---------------------------------------------------------------------------
// Host-side launch (compiled into the same object).
// ---------------------------------------------------------------------------
uint32_t lds_bytes_wave(int n, uint32_t adj_cap, int waves, uint32_t *wave_bytes) {
    const uint32_t per_wave = ((4u * (uint32_t)n + 7u) & ~7u) + 8u * (uint32_t)n + 2u * (uint32_t)n + 2u * (uint32_t)n;
    const uint32_t wb = (per_wave + 15u) & ~15u;
    const uint32_t head = (((((4u * (uint32_t)(n + 1) + 4u * adj_cap) + 7u) & ~7u) + 16u * (uint32_t)n) + 15u) & ~15u;
    if (wave_bytes) *wave_bytes = wb;
    return head + wb * (uint32_t)waves;
}

template <bool W, int G>
static hipError_t launch_t(const SweepParams &P, int blocks, int waves, uint32_t lds, hipStream_t st) {
    auto k = sweep_wave_kernel<W, G>;
    hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(blocks), dim3(64 * waves), lds, st, P);
    return hipGetLastError();
}

hipError_t launch_sweep_wave(const SweepParams &P, bool weighted, int group, int blocks, int waves, uint32_t lds,
                             hipStream_t st) {
    if (weighted) {
        switch (group) {
            case 4: return launch_t<true, 4>(P, blocks, waves, lds, st);
            case 16: return launch_t<true, 16>(P, blocks, waves, lds, st);
            default: return launch_t<true, 8>(P, blocks, waves, lds, st);
        }
    }
    switch (group) {
        case 4: return launch_t<false, 4>(P, blocks, waves, lds, st);
        case 16: return launch_t<false, 16>(P, blocks, waves, lds, st);
        default: return launch_t<false, 8>(P, blocks, waves, lds, st);
    }
}

}  // namespace amc
