// anchored.hip -- row-wise sweep with anchored r-hop neighbourhoods (Section
// 9.2): anchor i's step ranks the betweenness of the subgraph of H_r induced
// by S_r(i), the vertices within r surviving hops of i.
//
// Paper: Bao, Kontou, Vogiatzis, "Betweenness-Central Nodes Under
// Uncertainty: An Absorbing Markov Chain Approach".
//
// A work item is (realization r, tile of anchors).  The workgroup stages H_r
// in LDS once; each wavefront then takes anchors: a hop-limited breadth-first
// search from i gives S_r(i) (a vertex mask and a list), the wavefront runs
// every source of S_r(i) inside the mask and accumulates the betweenness of
// the induced subgraph in its own LDS array, reduces it to the tie-broken
// maximiser (and the pool-constrained one), draws the stop coin and counts.
#include "amc_dev.hpp"
#include "amc_kernels.hpp"
#include "sweep_common.hpp"
#include "wave_source.hpp"

namespace amc {

// Per-wavefront region: dist u32[n] | sig u64[n + 1] | ord u16[n] | B f64[n] |
// list u16[n] | mask u8[n] (sig[n] stays 0, as in the sweep kernels).
__host__ __device__ inline uint32_t anchored_b_offset(int n) {
    return (wave_ord_offset(n, false) + 2u * (uint32_t)n + 7u) & ~7u;
}
__host__ __device__ inline uint32_t anchored_private_bytes(int n) {
    const uint32_t un = (uint32_t)n;
    return (anchored_b_offset(n) + 8u * un + 2u * un + un + 15u) & ~15u;
}

template <bool WEIGHTED, typename ADJ>
__global__ __launch_bounds__(1024) void anchored_kernel(LaunchCtl LC) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __shared__ uint32_t scan_tmp[kMaxWaves];
    __shared__ uint32_t wctr[kMaxWaves];
    __shared__ int item_sh;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
    unsigned long long acc[5] = {0, 0, 0, 0, 0};
    bool ovf = false;
    int q_prev = -1;
    for (;;) {
        if (tid == 0) item_sh = (int)atomicAdd(LC.work_ctr, 1u);
        __syncthreads();
        const int it = item_sh;
        __syncthreads();
        if ((uint32_t)it >= LC.n_items) break;
        const uint32_t item = LC.item_base + (uint32_t)it;
        const int q = item_query(LC, item);
        const SweepParams &P = LC.descs[q];
        if (q != q_prev) {
            if (q_prev >= 0) flush_stats(LC.descs[q_prev], acc, ovf);
            q_prev = q;
        }
        const uint32_t qitem = item_local(LC, q, item);
        const uint32_t r_local = qitem / (uint32_t)P.tiles_per_r;
        const int t = (int)(qitem % (uint32_t)P.tiles_per_r);
        const uint32_t r = P.r_begin + r_local;
        const int n = P.n;
        const uint32_t shift = P.shift, nmask = (1u << shift) - 1u;
        const WaveLayout L = wave_layout(n, P.adj_cap, (uint32_t)sizeof(ADJ));
        ADJ *rp = (ADJ *)(smem + L.rp);
        ADJ *adj = (ADJ *)(smem + L.adj);
        unsigned char *wbase = smem + L.waves;
        unsigned char *wmine = wbase + wave * P.wave_bytes;
        const uint32_t sig_off = (4u * (uint32_t)n + 7u) & ~7u;
        const uint32_t b_off = anchored_b_offset(n);
        uint32_t *dist = (uint32_t *)wmine;
        unsigned long long *sig = (unsigned long long *)(wmine + sig_off);
        uint16_t *ord = (uint16_t *)(wmine + wave_ord_offset(n, false));
        double *Bw = (double *)(wmine + b_off);
        const BAcc BA{Bw, nullptr, false};
        uint16_t *list = (uint16_t *)(wmine + b_off + 8u * (uint32_t)n);
        uint8_t *mask = (uint8_t *)(list + n);

        stage_realization(P, r, rp, adj, shift, (uint16_t *)wbase, scan_tmp);

        const int a_lo = t * P.tile, a_hi = min(n, a_lo + P.tile);
        for (int i = a_lo + wave; i < a_hi; i += nwaves) {
            // S_r(i): breadth-first hops from i over the surviving edges
            for (int v = lane; v < n; v += 64) {
                dist[v] = kInf;
                mask[v] = 0;
            }
            wave_sync();
            if (lane == 0) {
                dist[i] = 0u;
                list[0] = (uint16_t)i;
                wctr[wave] = 1u;
            }
            wave_sync();
            int lo = 0, hi = 1;
            for (int level = 0; level < P.hop_radius && lo < hi; ++level) {
                for (int base = lo; base < hi; base += 64) {
                    const int idx = base + lane;
                    uint32_t beg = 0, len = 0;
                    if (idx < hi) {
                        const int v = list[idx];
                        beg = rp[v];
                        len = (uint32_t)rp[v + 1] - beg;
                    }
                    const uint32_t maxlen = wave_max_fast(len);
                    for (uint32_t off = 0; off < maxlen; ++off) {
                        bool found = false;
                        uint32_t u = 0;
                        if (off < len) {
                            u = (uint32_t)adj[beg + off] & nmask;
                            if (dist[u] == kInf) found = atomicCAS(&dist[u], kInf, (uint32_t)level + 1u) == kInf;
                        }
                        const uint32_t pos = wave_append(&wctr[wave], found);
                        if (found) list[pos] = (uint16_t)u;
                    }
                }
                wave_sync();
                lo = hi;
                hi = (int)wctr[wave];
            }
            const int sz = hi;
            for (int k = lane; k < sz; k += 64) mask[list[k]] = 1;
            for (int v = lane; v < n; v += 64) Bw[v] = 0.0;
            wave_sync();
            // surviving slots inside S and base slots of S's vertices (work counters)
            unsigned long long ak = 0, dk = 0;
            for (int k = lane; k < sz; k += 64) {
                const int v = list[k];
                for (uint32_t j = (uint32_t)rp[v]; j < (uint32_t)rp[v + 1]; ++j) ak += mask[(uint32_t)adj[j] & nmask];
                dk += (unsigned long long)(P.rp_base[v + 1] - P.rp_base[v]);
            }
            ak = wave_sum_u64(ak);
            dk = wave_sum_u64(dk);
            // betweenness of the induced subgraph, one source after another
            for (int k = 0; k < sz; ++k) {
                int cs = 0, zz = 0;
                wave_source_lane<WEIGHTED, 4, ADJ, false, uint32_t, true>(P, rp, adj, shift, BA, dist, sig, ord,
                                                                          &wctr[wave], (int)list[k], -1, cs, zz,
                                                                          ovf, mask);
            }
            // tie-broken maximiser over S_r(i), and over S_r(i) ∩ W
            double mx = 0.0, mw = -1.0;
            for (int k = lane; k < sz; k += 64) {
                const int v = list[k];
                mx = fmax(mx, Bw[v]);
                if (P.pool && P.pool[v]) mw = fmax(mw, Bw[v]);
            }
            mx = wave_max_f64(mx);
            mw = wave_max_f64(mw);
            const double band = P.tau * (mx > 1.0 ? mx : 1.0);
            const double bandw = P.tau * (mw > 1.0 ? mw : 1.0);
            int c = 0x7FFFFFFF, cw = 0x7FFFFFFF;
            for (int k = lane; k < sz; k += 64) {
                const int v = list[k];
                if (mx - Bw[v] <= band && v < c) c = v;
                if (P.pool && P.pool[v] && mw - Bw[v] <= bandw && v < cw) cw = v;
            }
            c = wave_min_i32(c);
            cw = wave_min_i32(cw);
            if (lane == 0) {
                const u32x4 x = philox10({r, (uint32_t)i, 0xFFFFFFFFu, 1u}, P.key0, P.key1);
                const bool coin = (uint64_t)x.x < P.t_alpha;
                const bool valid = !coin && (uint32_t)sz >= P.k_min;
                const int nx = valid ? c : -1;
                atomicAdd(&P.counts[(size_t)i * (n + 1) + (nx >= 0 ? nx : n)], 1u);
                if (P.next_table) P.next_table[(size_t)r_local * n + i] = nx;
                if (P.counts_w) {
                    const int nw = (valid && P.pool && cw != 0x7FFFFFFF) ? cw : -1;
                    atomicAdd(&P.counts_w[(size_t)i * (n + 1) + (nw >= 0 ? nw : n)], 1u);
                    if (P.next_table_w) P.next_table_w[(size_t)r_local * n + i] = nw;
                }
                acc[0] += (unsigned long long)sz;
                acc[1] += (unsigned long long)sz * (unsigned long long)sz;
                acc[2] += (unsigned long long)sz * ak;
                acc[3] += (unsigned long long)sz * dk;
            }
            wave_sync();
        }
        __syncthreads();
    }
    if (q_prev >= 0) flush_stats(LC.descs[q_prev], acc, ovf);
}

// ---------------------------------------------------------------------------
uint32_t lds_bytes_anchored(int n, uint32_t adj_cap, uint32_t adj_bytes, int waves, uint32_t *wave_bytes) {
    const uint32_t wb = anchored_private_bytes(n);
    if (wave_bytes) *wave_bytes = wb;
    return wave_layout(n, adj_cap, adj_bytes).waves + wb * (uint32_t)waves;
}

template <bool W, typename ADJ>
static hipError_t launch_a(const LaunchCtl &LC, int blocks, int waves, uint32_t lds, hipStream_t st) {
    hipLaunchKernelGGL((anchored_kernel<W, ADJ>), dim3(blocks), dim3(64 * waves), lds, st, LC);
    return hipGetLastError();
}

hipError_t set_anchored_attrs(int max_lds) {
    const void *ks[] = {(const void *)anchored_kernel<true, uint16_t>, (const void *)anchored_kernel<false, uint16_t>,
                        (const void *)anchored_kernel<true, uint32_t>, (const void *)anchored_kernel<false, uint32_t>};
    for (const void *k : ks) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_anchored(const LaunchCtl &LC, bool weighted, uint32_t adj_bytes, int blocks, int waves, uint32_t lds,
                           hipStream_t st) {
    if (adj_bytes == 2)
        return weighted ? launch_a<true, uint16_t>(LC, blocks, waves, lds, st)
                        : launch_a<false, uint16_t>(LC, blocks, waves, lds, st);
    return weighted ? launch_a<true, uint32_t>(LC, blocks, waves, lds, st)
                    : launch_a<false, uint32_t>(LC, blocks, waves, lds, st);
}

}  // namespace amc
