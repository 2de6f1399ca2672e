// sweep_wave.hip -- realization x source sweep with the realized graph staged
// in LDS and one wavefront per (realization, source).
//
// Paper: Bao, Kontou, Vogiatzis, "Betweenness-Central Nodes Under
// Uncertainty: An Absorbing Markov Chain Approach".
//
// One workgroup takes a work item (realization r, source tile) at a time:
//   1. realize every base edge of r with one Philox call (Section 3.1) and
//      compact the surviving slots into an adjacency (weight | neighbour) in
//      LDS (LDS mode) or in the workgroup's L2-resident scratch (L2 mode);
//   2. each wavefront takes sources s from a workgroup counter and runs the
//      single-source shortest paths with exact uint64 path counts
//      (breadth-first levels for unit weights; for integer weights >= 1 one
//      equal-distance segment per step, settled from the fringe by its
//      minimum) and the reverse dependency accumulation of the Section 3.1
//      betweenness, adding delta_s into a workgroup-wide B(H_r);
//   3. once every source of r is done, the workgroup reduces B(H_r) to the
//      global centre (eq. central-node), the component centres (eq.
//      local-center) and the pool-constrained centres (Section 7.1), draws
//      every anchor's stop coin, applies k_min and counts next(r, i)
//      (Alg. 1 for every anchor, tallied as in Alg. 2).
#include <type_traits>

#include "amc_dev.hpp"
#include "amc_kernels.hpp"
#include "sweep_common.hpp"
#include "wave_source.hpp"

namespace amc {

// Persistent sweep.  GL = false: LDS mode (realized graph, B(H_r) and the
// component labels in LDS next to the wavefronts' regions).  GL = true: L2
// mode (the realized graph and the labels in the workgroup's global scratch,
// B(H_r) alone in LDS), which leaves almost the whole LDS to per-source state
// and so keeps more sources in flight on graphs whose realized adjacency
// would crowd the LDS.
// The 8-slot lane mapping needs more than the 128 VGPRs a 1024-thread
// workgroup allows; it is limited to 8 wavefronts per workgroup.  D16: 16-bit
// distance entries in the wavefront regions.  SG (L2 mode, lane-per-vertex
// mappings): each wavefront's path counts live in the workgroup's global
// scratch, so a wavefront region holds only distances and the order (4 or 6
// n bytes instead of 12 or 14 n) and more sources fit in flight on large
// graphs.
template <bool WEIGHTED, int G, typename ADJ, bool GL, bool D16, bool SG>
__global__ __launch_bounds__(G == 3 ? 512 : 1024) void sweep_wave_kernel(LaunchCtl LC) {
    using DT = typename std::conditional<D16, uint16_t, uint32_t>::type;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __shared__ uint32_t scan_tmp[kMaxWaves];
    __shared__ uint32_t wctr[kMaxWaves];
    __shared__ double red_f[kMaxWaves];
    __shared__ int red_i[kMaxWaves];
    __shared__ int item_sh;
    __shared__ int last_sh;
    __shared__ uint32_t src_ctr;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    unsigned long long acc_stats[5] = {0, 0, 0, 0, 0};
    bool ovf = false;
    int q_prev = -1;
    uint32_t local = 0;
    for (;;) {
        if (LC.static_items) {
            if (local > 0) break;
            local = 1;
            item_sh = (int)blockIdx.x;
        } else {
            if (tid == 0) item_sh = (int)atomicAdd(LC.work_ctr, 1u);
            __syncthreads();
        }
        const int it = __builtin_amdgcn_readfirstlane(item_sh);
        __syncthreads();
        if ((uint32_t)it >= LC.n_items) break;
        const uint32_t item = LC.item_base + (uint32_t)it;
        const int q = item_query(LC, item);
        const SweepParams &P = LC.descs[q];
        if (q != q_prev) {   // counters belong to the query that produced them
            if (q_prev >= 0) flush_stats(LC.descs[q_prev], acc_stats, ovf);
            q_prev = q;
        }
        const uint32_t qitem = item_local(LC, q, item);
        const uint32_t r_local = qitem / (uint32_t)P.tiles_per_r;
        const int t = (int)(qitem % (uint32_t)P.tiles_per_r);
        const uint32_t r = P.r_begin + r_local;
        const uint32_t shift = P.shift;
        const int n = P.n;
        const bool split = P.tiles_per_r > 1;

        ADJ *rp, *adj;
        double *B;               // B(H_r) as the reduction reads it
        BAcc BA{nullptr, nullptr, false};
        unsigned char *wbase;
        // component labels / sizes of the sources: LDS u16 (LDS mode) or
        // global int32 (L2 mode)
        uint16_t *comp16 = nullptr, *csize16 = nullptr;
        int32_t *comp32 = nullptr, *csize32 = nullptr;
        if constexpr (GL) {
            const L2Layout L = l2_layout(n, P.adj_cap, (uint32_t)sizeof(ADJ));
            unsigned char *gs = (unsigned char *)(LC.bscratch + (size_t)blockIdx.x * LC.bscratch_words);
            rp = to_global((ADJ *)(gs + L.rp));
            adj = to_global((ADJ *)(gs + L.adj));
            BA.glob = P.b_global != 0;
            BA.lds = (double *)smem;
            BA.gl = to_global((double *)(gs + L.B));
            B = BA.glob ? BA.gl : BA.lds;
            // a split realization writes its labels straight into its exchange rows
            comp32 = to_global(split ? P.compg + (size_t)r_local * n : (int32_t *)(gs + L.comp));
            csize32 = to_global(split ? P.sizeg + (size_t)r_local * n : (int32_t *)(gs + L.csize));
            wbase = smem + (BA.glob ? 0u : l2_lds_b_bytes(n));
        } else {
            const WaveLayout L = wave_layout(n, P.adj_cap, (uint32_t)sizeof(ADJ));
            rp = (ADJ *)(smem + L.rp);
            adj = (ADJ *)(smem + L.adj);
            B = (double *)(smem + L.B);
            BA.lds = B;
            comp16 = (uint16_t *)(smem + L.comp);
            csize16 = (uint16_t *)(smem + L.csize);
            wbase = smem + L.waves;
        }
        // byte offsets from the LDS base keep every pointer in the LDS address space
        unsigned char *wmine = wbase + wave * P.wave_bytes;
        const uint32_t sig_off = wave_sig_offset(n, D16);
        DT *dist = (DT *)wmine;
        unsigned long long *sig;
        uint16_t *ord;
        if constexpr (SG) {
            const L2Layout L = l2_layout(n, P.adj_cap, (uint32_t)sizeof(ADJ));
            unsigned char *gs = (unsigned char *)(LC.bscratch + (size_t)blockIdx.x * LC.bscratch_words);
            sig = to_global((unsigned long long *)(gs + L.total + (uint32_t)wave * l2_sig_stride(n)));
            ord = (uint16_t *)(wmine + sig_off);
        } else {
            sig = (unsigned long long *)(wmine + sig_off);
            ord = (uint16_t *)(wmine + wave_ord_offset(n, D16));
        }
        ReduceScratch RS;
        RS.cmax = (unsigned long long *)wbase;
        RS.wmax = RS.cmax + n;
        RS.ccen = (int32_t *)(RS.wmax + n);
        RS.wcen = RS.ccen + n;

        if (tid == 0) src_ctr = 0u;
        stage_realization(P, r, rp, adj, shift, (uint16_t *)wbase, scan_tmp);
        if (BA.glob) {
            for (int v = tid; v < n; v += blockDim.x) st_global(&BA.gl[v], 0.0);
        } else {
            for (int v = tid; v < n; v += blockDim.x) BA.lds[v] = 0.0;
        }
        // L2 mode: the realized graph (and a global B) are complete at L2
        // before any wavefront reads them or adds into B
        if constexpr (GL) __threadfence();
        __syncthreads();

        // sources are taken from a workgroup counter: the wavefronts of a
        // workgroup need not spread evenly over the SIMDs
        const int s_lo = t * P.tile, s_hi = min(n, s_lo + P.tile);
        for (;;) {
            uint32_t k = 0;
            if (lane == 0) k = atomicAdd(&src_ctr, 1u);
            const int s = s_lo + (int)__builtin_amdgcn_readfirstlane(k);
            if (s >= s_hi) break;
            int cs = 0, sz = 0;
            const int slot = P.n_dbg ? debug_slot(P, r, s) : -1;
            run_source<WEIGHTED, G, ADJ, GL, DT, SG>(P, rp, adj, shift, BA, dist, sig, ord, &wctr[wave], s, slot, cs,
                                                     sz, ovf);
            if (lane == 0) {
                if constexpr (GL) {
                    st_global(&comp32[s], (int32_t)cs);
                    st_global(&csize32[s], (int32_t)sz);
                } else {
                    comp16[s] = (uint16_t)cs;
                    csize16[s] = (uint16_t)sz;
                }
            }
        }
        if constexpr (GL) {
            // every label store (and global B atomic) of this item has reached L2
            __threadfence();
            __syncthreads();
            if (!split) {
                reduce_realization<ADJ, int32_t, true>(P, r_local, r, rp, B, comp32, csize32, RS, red_f, red_i,
                                                       acc_stats, true);
            } else {
                // publish this tile's partial B; the last tile of the
                // realization to finish gathers the row and reduces
                double *Bg = P.Bg + (size_t)r_local * n;
                for (int v = tid; v < n; v += blockDim.x) {
                    const double b = ld_coh<true>(&B[v]);
                    if (b != 0.0) unsafeAtomicAdd(&Bg[v], b);
                }
                __threadfence();
                __syncthreads();
                if (tid == 0) last_sh = (atomicAdd(&P.done[r_local], 1u) == (unsigned)(P.tiles_per_r - 1));
                __syncthreads();
                if (last_sh) {
                    __threadfence();
                    reduce_realization<ADJ, int32_t, true>(P, r_local, r, rp, Bg, comp32, csize32, RS, red_f, red_i,
                                                           acc_stats, false);
                }
                __syncthreads();
            }
            continue;
        }
        __syncthreads();

        if (!split) {
            reduce_realization(P, r_local, r, rp, B, comp16, csize16, RS, red_f, red_i, acc_stats, true);
        } else {
            // publish this tile's partial B and component labels; the last
            // tile of the realization to finish performs the reduction
            double *Bg = P.Bg + (size_t)r_local * n;
            for (int v = tid; v < n; v += blockDim.x)
                if (B[v] != 0.0) unsafeAtomicAdd(&Bg[v], B[v]);
            for (int s = s_lo + tid; s < s_hi; s += blockDim.x) {
                P.compg[(size_t)r_local * n + s] = comp16[s];
                P.sizeg[(size_t)r_local * n + s] = csize16[s];
            }
            __threadfence();
            __syncthreads();
            if (tid == 0) last_sh = (atomicAdd(&P.done[r_local], 1u) == (unsigned)(P.tiles_per_r - 1));
            __syncthreads();
            if (last_sh) {
                __threadfence();
                for (int v = tid; v < n; v += blockDim.x) {
                    B[v] = __hip_atomic_load(&Bg[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    comp16[v] = (uint16_t)__hip_atomic_load(&P.compg[(size_t)r_local * n + v], __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT);
                    csize16[v] = (uint16_t)__hip_atomic_load(&P.sizeg[(size_t)r_local * n + v], __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
                }
                __syncthreads();
                reduce_realization(P, r_local, r, rp, B, comp16, csize16, RS, red_f, red_i, acc_stats, false);
            }
            __syncthreads();
        }
    }
    if (q_prev >= 0) flush_stats(LC.descs[q_prev], acc_stats, ovf);
}

// ---------------------------------------------------------------------------
// Host-side launch (compiled into the same object).
// ---------------------------------------------------------------------------
uint32_t lds_bytes_wave(int n, uint32_t adj_cap, uint32_t adj_bytes, int waves, bool dist16, uint32_t *wave_bytes) {
    const uint32_t wb = wave_private_bytes(n, dist16);
    if (wave_bytes) *wave_bytes = wb;
    return wave_layout(n, adj_cap, adj_bytes).waves + wb * (uint32_t)waves;
}

uint32_t lds_bytes_wave_l2(int n, int waves, bool dist16, bool b_global, bool sg, uint32_t *wave_bytes) {
    const uint32_t wb = wave_private_bytes(n, dist16, sg);
    if (wave_bytes) *wave_bytes = wb;
    return (b_global ? 0u : l2_lds_b_bytes(n)) + wb * (uint32_t)waves;
}

size_t l2_scratch_words(int n, uint32_t adj_cap, uint32_t adj_bytes, int sg_waves) {
    return (l2_layout(n, adj_cap, adj_bytes).total + (size_t)sg_waves * l2_sig_stride(n)) / 4u;
}

template <bool W, int G, typename ADJ, bool GL, bool D16, bool SG>
static hipError_t launch_t(const LaunchCtl &LC, int blocks, int waves, uint32_t lds, hipStream_t st) {
    hipLaunchKernelGGL((sweep_wave_kernel<W, G, ADJ, GL, D16, SG>), dim3(blocks), dim3(64 * waves), lds, st, LC);
    return hipGetLastError();
}

template <bool W, typename ADJ, bool GL, bool D16>
static hipError_t attrs_g(int max_lds) {
    const void *ks[] = {(const void *)sweep_wave_kernel<W, 1, ADJ, GL, D16, false>,
                        (const void *)sweep_wave_kernel<W, 2, ADJ, GL, D16, false>,
                        (const void *)sweep_wave_kernel<W, 3, ADJ, GL, D16, false>,
                        (const void *)sweep_wave_kernel<W, 4, ADJ, GL, D16, false>,
                        (const void *)sweep_wave_kernel<W, 8, ADJ, GL, D16, false>,
                        (const void *)sweep_wave_kernel<W, 16, ADJ, GL, D16, false>};
    for (const void *k : ks) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
        if (e != hipSuccess) return e;
    }
    if constexpr (GL) {
        const void *kg[] = {(const void *)sweep_wave_kernel<W, 1, ADJ, GL, D16, true>,
                            (const void *)sweep_wave_kernel<W, 2, ADJ, GL, D16, true>,
                            (const void *)sweep_wave_kernel<W, 3, ADJ, GL, D16, true>};
        for (const void *k : kg) {
            const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

template <bool GL, bool D16>
static hipError_t attrs_all(int max_lds) {
    hipError_t e;
    if ((e = attrs_g<true, uint16_t, GL, D16>(max_lds)) != hipSuccess) return e;
    if ((e = attrs_g<false, uint16_t, GL, D16>(max_lds)) != hipSuccess) return e;
    if ((e = attrs_g<true, uint32_t, GL, D16>(max_lds)) != hipSuccess) return e;
    return attrs_g<false, uint32_t, GL, D16>(max_lds);
}

// Allows every LDS-mode and L2-mode instantiation the device's dynamic LDS
// (set once per context, outside any stream capture).
hipError_t set_sweep_wave_attrs(int max_lds) {
    hipError_t e;
    if ((e = attrs_all<false, false>(max_lds)) != hipSuccess) return e;
    if ((e = attrs_all<true, false>(max_lds)) != hipSuccess) return e;
    if ((e = attrs_all<false, true>(max_lds)) != hipSuccess) return e;
    return attrs_all<true, true>(max_lds);
}

template <bool W, typename ADJ, bool GL, bool D16>
static hipError_t launch_g(const LaunchCtl &LC, int group, bool sg, int blocks, int waves, uint32_t lds,
                           hipStream_t st) {
    if constexpr (GL) {
        if (sg) {
            switch (group) {
                case 2: return launch_t<W, 2, ADJ, GL, D16, true>(LC, blocks, waves, lds, st);
                case 3: return launch_t<W, 3, ADJ, GL, D16, true>(LC, blocks, waves, lds, st);
                case 1: return launch_t<W, 1, ADJ, GL, D16, true>(LC, blocks, waves, lds, st);
                default: return hipErrorInvalidValue;
            }
        }
    }
    if (sg) return hipErrorInvalidValue;
    switch (group) {
        case 1: return launch_t<W, 1, ADJ, GL, D16, false>(LC, blocks, waves, lds, st);
        case 2: return launch_t<W, 2, ADJ, GL, D16, false>(LC, blocks, waves, lds, st);
        case 3: return launch_t<W, 3, ADJ, GL, D16, false>(LC, blocks, waves, lds, st);
        case 4: return launch_t<W, 4, ADJ, GL, D16, false>(LC, blocks, waves, lds, st);
        case 16: return launch_t<W, 16, ADJ, GL, D16, false>(LC, blocks, waves, lds, st);
        default: return launch_t<W, 8, ADJ, GL, D16, false>(LC, blocks, waves, lds, st);
    }
}

template <bool GL, bool D16>
static hipError_t launch_w(const LaunchCtl &LC, bool weighted, int group, bool sg, uint32_t adj_bytes, int blocks,
                           int waves, uint32_t lds, hipStream_t st) {
    if (adj_bytes == 2)
        return weighted ? launch_g<true, uint16_t, GL, D16>(LC, group, sg, blocks, waves, lds, st)
                        : launch_g<false, uint16_t, GL, D16>(LC, group, sg, blocks, waves, lds, st);
    return weighted ? launch_g<true, uint32_t, GL, D16>(LC, group, sg, blocks, waves, lds, st)
                    : launch_g<false, uint32_t, GL, D16>(LC, group, sg, blocks, waves, lds, st);
}

hipError_t launch_sweep_wave(const LaunchCtl &LC, bool weighted, bool l2, bool dist16, bool sg, int group,
                             uint32_t adj_bytes, int blocks, int waves, uint32_t lds, hipStream_t st) {
    if (dist16)
        return l2 ? launch_w<true, true>(LC, weighted, group, sg, adj_bytes, blocks, waves, lds, st)
                  : launch_w<false, true>(LC, weighted, group, sg, adj_bytes, blocks, waves, lds, st);
    return l2 ? launch_w<true, false>(LC, weighted, group, sg, adj_bytes, blocks, waves, lds, st)
              : launch_w<false, false>(LC, weighted, group, sg, adj_bytes, blocks, waves, lds, st);
}

}  // namespace amc
