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
// G lanes cooperate on one vertex's adjacency; an adjacency entry holds the
// neighbour in its low `shift` bits and the weight above them.
// ---------------------------------------------------------------------------
template <bool WEIGHTED, int G, typename ADJ, bool GB>
__device__ void wave_source(const SweepParams &P, const ADJ *rp, const ADJ *adj, uint32_t shift, double *B,
                            uint32_t *dist, unsigned long long *sig, uint16_t *ord, uint16_t *aux, uint32_t *ctr,
                            int s, int dbg_slot, int &comp_out, int &size_out, bool &ovf) {
    const int n = P.n;
    const int lane = threadIdx.x & 63;
    const int sub = lane % G;
    constexpr int VPI = 64 / G;   // vertices per wave iteration
    const uint32_t nmask = (1u << shift) - 1u;

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
    uint32_t kmin = kInf;   // lane minimum over the fringe entries kept by the last partition
    // ------------------------------------------------------------ forward
    for (;;) {
        if (lane == 0) aux[n - 1 - nseg] = (uint16_t)f_lo;
        ++nseg;
        uint32_t lmin = kInf;  // lane minimum over successful relaxations
        for (int base = f_lo; base < ord_end; base += VPI) {
            const int idx = base + lane / G;
            const bool mine = idx < ord_end;
            int v = 0;
            uint32_t beg = 0, len = 0;
            if (mine) {
                v = ord[idx];
                beg = rp[v];
                len = rp[v + 1] - beg;
            }
            const uint32_t trips = len > (uint32_t)sub ? (len - (uint32_t)sub + G - 1) / G : 0u;
            const uint32_t maxtrips = wave_max_fast(trips);
            unsigned long long acc = 0ull;
            for (uint32_t t = 0; t < maxtrips; ++t) {
                bool found = false;
                uint32_t u = 0;
                if (t < trips) {
                    const uint32_t a = adj[beg + (uint32_t)sub + t * G];
                    u = a & nmask;
                    const uint32_t w = WEIGHTED ? (a >> shift) : 1u;
                    const uint32_t du = dist[u];
                    if (du + w == D) {                       // u precedes v: pull sigma_u
                        const unsigned long long x = acc + sig[u];
                        ovf |= x < acc;
                        acc = x;
                    } else if (D + w < du) {                 // relax the edge v -> u
                        const uint32_t old = atomicMin(&dist[u], D + w);
                        if (old > D + w) lmin = (D + w) < lmin ? (D + w) : lmin;
                        found = old == kInf;                 // first discovery of u
                    }
                }
                const uint32_t pos = wave_append(ctr, found);
                if (found) {
                    if (WEIGHTED) aux[pos] = (uint16_t)u;
                    else ord[pos] = (uint16_t)u;
                }
            }
            acc = group_sum_u64<G>(acc, ovf);
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
            // the fringe minimum: every current fringe distance is either a
            // value kept at the last partition or a successful relaxation
            const uint32_t mn = wave_min_fast(lmin < kmin ? lmin : kmin);
            // move the vertices at the new minimum distance to ord, keep the
            // rest (compacted in place: writes never pass the read position)
            int settled = 0, kept = 0;
            kmin = kInf;
            const uint64_t lt = lanemask_lt();
            for (int k0 = 0; k0 < fr; k0 += 64) {
                const int k = k0 + lane;
                const bool valid = k < fr;
                const uint32_t x = valid ? aux[k] : 0u;
                const uint32_t dx = valid ? dist[x] : kInf;
                const bool is_s = valid && dx == mn;
                const bool is_k = valid && !is_s;
                if (is_k) kmin = dx < kmin ? dx : kmin;
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
        uint32_t mn = (uint32_t)n;
        for (int k = lane; k < ord_end; k += 64) mn = min(mn, (uint32_t)ord[k]);
        comp_out = (int)wave_min_fast(mn);
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
                    const uint32_t u = a & nmask;
                    const uint32_t w = WEIGHTED ? (a >> shift) : 1u;
                    if (dist[u] == dv + w) sum += as_f64(sig[u]);   // u succeeds v: c_u
                }
            }
            sum = group_sum_f64<G>(sum);
            if (mine && sub == 0) {
                const double sv = (double)sig[v];
                const double delta = sv * sum;
                sig[v] = as_u64((1.0 + delta) / sv);
                if (v != s) add_B<GB>(B, v, delta);
                if (dbg_slot >= 0) P.dbg_delta[(size_t)dbg_slot * n + v] = delta;
            }
        }
        wave_sync();
    }
}

// ---------------------------------------------------------------------------
// Lane-per-vertex variant of wave_source: each lane owns one frontier vertex
// and walks its adjacency U slots at a time, issuing the U neighbour loads
// (and the U distance loads) back to back so that their LDS latencies
// overlap; the path count of the vertex accumulates in the lane itself.  The
// U appends of a block share one LDS atomic per wavefront.
// ---------------------------------------------------------------------------
template <int U>
__device__ __forceinline__ void append_block(uint32_t *ctr, const bool (&found)[U], uint32_t (&pos)[U]) {
    uint64_t m[U];
    uint32_t tot = 0;
#pragma unroll
    for (int k = 0; k < U; ++k) {
        m[k] = __ballot(found[k]);
        tot += (uint32_t)__popcll(m[k]);
    }
    if (tot == 0) return;
    uint32_t base = 0;
    if ((threadIdx.x & 63) == 0) base = atomicAdd(ctr, tot);
    base = __builtin_amdgcn_readfirstlane(base);
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int k = 0; k < U; ++k) {
        pos[k] = base + (uint32_t)__popcll(m[k] & lt);
        base += (uint32_t)__popcll(m[k]);
    }
}

template <bool WEIGHTED, int U, typename ADJ, bool GB>
__device__ void wave_source_lane(const SweepParams &P, const ADJ *rp, const ADJ *adj, uint32_t shift,
                                 double *B, uint32_t *dist, unsigned long long *sig, uint16_t *ord, uint16_t *aux,
                                 uint32_t *ctr, int s, int dbg_slot, int &comp_out, int &size_out, bool &ovf) {
    const int n = P.n;
    const int lane = threadIdx.x & 63;
    const uint32_t nmask = (1u << shift) - 1u;

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
    uint32_t kmin = kInf;
    // ------------------------------------------------------------ forward
    for (;;) {
        if (lane == 0) aux[n - 1 - nseg] = (uint16_t)f_lo;
        ++nseg;
        uint32_t lmin = kInf;
        for (int base = f_lo; base < ord_end; base += 64) {
            const int idx = base + lane;
            const bool mine = idx < ord_end;
            int v = 0;
            uint32_t beg = 0, len = 0;
            if (mine) {
                v = ord[idx];
                beg = rp[v];
                len = rp[v + 1] - beg;
            }
            const uint32_t maxlen = wave_max_fast(len);
            unsigned long long acc = 0ull;
            // the adjacency carries kAdjPad zero entries past its end (and, in
            // the L2 mode, the rest of the workgroup scratch), so these loads
            // need no predication; masked results are dropped.  In the L2
            // mode the next block of U entries is loaded while the current
            // one is used (global latency); LDS loads are issued in place.
            uint32_t nxt[U];
            if constexpr (GB) {
#pragma unroll
                for (int k = 0; k < U; ++k) nxt[k] = (uint32_t)adj[beg + k];
            }
            for (uint32_t off = 0; off < maxlen; off += U) {
                uint32_t u[U], w[U], du[U], cur[U];
                bool found[U];
                if constexpr (GB) {
#pragma unroll
                    for (int k = 0; k < U; ++k) cur[k] = nxt[k];
                    if (off + U < maxlen) {
#pragma unroll
                        for (int k = 0; k < U; ++k) nxt[k] = (uint32_t)adj[beg + off + U + k];
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < U; ++k) cur[k] = (uint32_t)adj[beg + off + k];
                }
                // a slot past the vertex's adjacency gets weight kNoEdge, which
                // fails both tests below (du + kNoEdge > D, D + kNoEdge > du)
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const uint32_t a = cur[k];
                    u[k] = a & nmask;
                    w[k] = (off + k < len) ? (WEIGHTED ? (a >> shift) : 1u) : kNoEdge;
                }
#pragma unroll
                for (int k = 0; k < U; ++k) du[k] = dist[u[k]];
                bool pred[U], rel[U];
                unsigned long long sg[U];
                uint32_t old[U];
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    pred[k] = du[k] + w[k] == D;                        // u precedes v: pull sigma_u
                    rel[k] = D + w[k] < du[k];                          // relax the edge v -> u
                }
#pragma unroll
                for (int k = 0; k < U; ++k) sg[k] = pred[k] ? sig[u[k]] : 0ull;
#pragma unroll
                for (int k = 0; k < U; ++k) old[k] = rel[k] ? atomicMin(&dist[u[k]], D + w[k]) : 0u;
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const unsigned long long x = acc + sg[k];
                    ovf |= x < acc;
                    acc = x;
                    const uint32_t cand = (rel[k] && old[k] > D + w[k]) ? D + w[k] : kInf;
                    lmin = cand < lmin ? cand : lmin;
                    found[k] = rel[k] && old[k] == kInf;                // first discovery of u
                }
                uint32_t pos[U];
                append_block<U>(ctr, found, pos);
#pragma unroll
                for (int k = 0; k < U; ++k)
                    if (found[k]) {
                        if (WEIGHTED) aux[pos[k]] = (uint16_t)u[k];
                        else ord[pos[k]] = (uint16_t)u[k];
                    }
            }
            if (mine && v != s) sig[v] = acc;
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
            const uint32_t mn = wave_min_fast(lmin < kmin ? lmin : kmin);
            int settled = 0, kept = 0;
            kmin = kInf;
            const uint64_t lt = lanemask_lt();
            for (int k0 = 0; k0 < fr; k0 += 64 * U) {
                uint32_t x[U], dx[U];
#pragma unroll
                for (int c = 0; c < U; ++c) {
                    const int k = k0 + 64 * c + lane;
                    x[c] = k < fr ? (uint32_t)aux[k] : 0xFFFFFFFFu;
                }
#pragma unroll
                for (int c = 0; c < U; ++c) dx[c] = x[c] != 0xFFFFFFFFu ? dist[x[c]] : kInf;
                // all reads of the U chunks precede their writes (positions
                // never pass the read positions)
                wave_sync();
#pragma unroll
                for (int c = 0; c < U; ++c) {
                    const bool valid = x[c] != 0xFFFFFFFFu;
                    const bool is_s = valid && dx[c] == mn;
                    const bool is_k = valid && !is_s;
                    if (is_k) kmin = dx[c] < kmin ? dx[c] : kmin;
                    const uint64_t ms = __ballot(is_s), mk = __ballot(is_k);
                    if (is_s) ord[ord_end + settled + __popcll(ms & lt)] = (uint16_t)x[c];
                    if (is_k) aux[kept + __popcll(mk & lt)] = (uint16_t)x[c];
                    settled += __popcll(ms);
                    kept += __popcll(mk);
                }
            }
            if (lane == 0) *ctr = (uint32_t)kept;
            wave_sync();
            f_lo = ord_end;
            ord_end += settled;
            D = mn;
        }
    }

    {
        uint32_t mn = (uint32_t)n;
        for (int k = lane; k < ord_end; k += 64) mn = min(mn, (uint32_t)ord[k]);
        comp_out = (int)wave_min_fast(mn);
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
        for (int base = lo; base < hi; base += 64) {
            const int idx = base + lane;
            const bool mine = idx < hi;
            int v = 0;
            uint32_t beg = 0, len = 0, dv = 0;
            if (mine) {
                v = ord[idx];
                beg = rp[v];
                len = rp[v + 1] - beg;
                dv = dist[v];
            }
            double sum = 0.0;
            uint32_t nxt[U];
            if constexpr (GB) {
#pragma unroll
                for (int k = 0; k < U; ++k) nxt[k] = (uint32_t)adj[beg + k];
            }
            for (uint32_t off = 0; off < len; off += U) {
                uint32_t u[U], w[U], du[U], cur[U];
                if constexpr (GB) {
#pragma unroll
                    for (int k = 0; k < U; ++k) cur[k] = nxt[k];
                    if (off + U < len) {
#pragma unroll
                        for (int k = 0; k < U; ++k) nxt[k] = (uint32_t)adj[beg + off + U + k];
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < U; ++k) cur[k] = (uint32_t)adj[beg + off + k];
                }
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const uint32_t a = cur[k];
                    u[k] = a & nmask;
                    w[k] = (off + k < len) ? (WEIGHTED ? (a >> shift) : 1u) : kNoEdge;
                }
#pragma unroll
                for (int k = 0; k < U; ++k) du[k] = dist[u[k]];
                double cu[U];
#pragma unroll
                for (int k = 0; k < U; ++k) cu[k] = (du[k] == dv + w[k]) ? as_f64(sig[u[k]]) : 0.0;
#pragma unroll
                for (int k = 0; k < U; ++k) sum += cu[k];                       // u succeeds v: c_u
            }
            if (mine) {
                const double sv = (double)sig[v];
                const double delta = sv * sum;
                sig[v] = as_u64((1.0 + delta) / sv);
                if (v != s) add_B<GB>(B, v, delta);
                if (dbg_slot >= 0) P.dbg_delta[(size_t)dbg_slot * n + v] = delta;
            }
        }
        wave_sync();
    }
}

// Byte offsets of the LDS carve-up (mirrors lds_bytes_wave on the host).
struct WaveLayout {
    uint32_t rp, adj, B, comp, csize, waves;
};
__host__ __device__ inline WaveLayout wave_layout(int n, uint32_t adj_cap, uint32_t adj_bytes) {
    WaveLayout L;
    const uint32_t un = (uint32_t)n;
    L.rp = 0;
    L.adj = (L.rp + adj_bytes * (un + 1u) + 3u) & ~3u;
    L.B = (L.adj + adj_bytes * adj_cap + 7u) & ~7u;
    L.comp = L.B + 8u * un;
    L.csize = L.comp + 2u * un;
    L.waves = (L.csize + 2u * un + 15u) & ~15u;
    return L;
}

// L2 mode: the realized graph, B(H_r) and the component labels of one
// workgroup live in its global scratch (small enough to stay in L2); the LDS
// holds only the wavefronts' private regions.
struct L2Layout {
    uint32_t rp, adj, B, comp, csize, total;
};
__host__ __device__ inline L2Layout l2_layout(int n, uint32_t adj_cap, uint32_t adj_bytes) {
    L2Layout L;
    const uint32_t un = (uint32_t)n;
    L.rp = 0;
    L.adj = (adj_bytes * (un + 1u) + 3u) & ~3u;
    L.B = (L.adj + adj_bytes * adj_cap + 7u) & ~7u;
    L.comp = L.B + 8u * un;
    L.csize = L.comp + 4u * un;
    L.total = (L.csize + 4u * un + 255u) & ~255u;
    return L;
}

// Persistent sweep.  GL = false: LDS mode (realized graph, B(H_r) and the
// component labels in LDS next to the wavefronts' regions).  GL = true: L2
// mode (those in the workgroup's global scratch, B accumulated with device
// atomics), which leaves the whole LDS to per-source state and so keeps more
// sources in flight on graphs whose realized adjacency would crowd the LDS.
// The 8-slot lane mapping needs more than the 128 VGPRs a 1024-thread
// workgroup allows; it is limited to 8 wavefronts per workgroup.
template <bool WEIGHTED, int G, typename ADJ, bool GL>
__global__ __launch_bounds__(G == 3 ? 512 : 1024) void sweep_wave_kernel(LaunchCtl LC) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __shared__ uint32_t scan_tmp[kMaxWaves];
    __shared__ uint32_t wctr[kMaxWaves];
    __shared__ double red_f[kMaxWaves];
    __shared__ int red_i[kMaxWaves];
    __shared__ int item_sh;
    __shared__ int last_sh;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
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
        const int it = item_sh;
        __syncthreads();
        if ((uint32_t)it >= LC.n_items) break;
        const uint32_t item = LC.item_base + (uint32_t)it;
        const int q = item_query(LC, item);
        const SweepParams &P = LC.descs[q];
        if (q != q_prev) {   // counters belong to the query that produced them
            if (q_prev >= 0) flush_stats(LC.descs[q_prev], acc_stats, ovf);
            q_prev = q;
        }
        const uint32_t qitem = item - LC.item_start[q];
        const uint32_t r_local = qitem / (uint32_t)P.tiles_per_r;
        const int t = (int)(qitem % (uint32_t)P.tiles_per_r);
        const uint32_t r = P.r_begin + r_local;
        const uint32_t shift = P.shift;
        const int n = P.n;
        const bool split = P.tiles_per_r > 1;

        ADJ *rp, *adj;
        double *B;
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
            // a split realization accumulates straight into its exchange rows
            B = to_global(split ? P.Bg + (size_t)r_local * n : (double *)(gs + L.B));
            comp32 = to_global(split ? P.compg + (size_t)r_local * n : (int32_t *)(gs + L.comp));
            csize32 = to_global(split ? P.sizeg + (size_t)r_local * n : (int32_t *)(gs + L.csize));
            wbase = smem;
        } else {
            const WaveLayout L = wave_layout(n, P.adj_cap, (uint32_t)sizeof(ADJ));
            rp = (ADJ *)(smem + L.rp);
            adj = (ADJ *)(smem + L.adj);
            B = (double *)(smem + L.B);
            comp16 = (uint16_t *)(smem + L.comp);
            csize16 = (uint16_t *)(smem + L.csize);
            wbase = smem + L.waves;
        }
        // byte offsets from the LDS base keep every pointer in the LDS address space
        unsigned char *wmine = wbase + wave * P.wave_bytes;
        const uint32_t sig_off = (4u * (uint32_t)n + 7u) & ~7u;
        uint32_t *dist = (uint32_t *)wmine;
        unsigned long long *sig = (unsigned long long *)(wmine + sig_off);
        uint16_t *ord = (uint16_t *)(wmine + sig_off + 8u * (uint32_t)n);
        uint16_t *aux = ord + n;
        ReduceScratch RS;
        RS.cmax = (unsigned long long *)wbase;
        RS.wmax = RS.cmax + n;
        RS.ccen = (int32_t *)(RS.wmax + n);
        RS.wcen = RS.ccen + n;
        RS.kal = (uint32_t *)(RS.wcen + n);
        RS.kba = RS.kal + n;

        stage_realization(P, r, rp, adj, shift, (uint16_t *)wbase, scan_tmp);
        if constexpr (GL) {
            if (!split)
                for (int v = tid; v < n; v += blockDim.x) B[v] = 0.0;
            // the realized graph and the cleared B are complete at L2 before
            // any wavefront reads them or adds into B
            __threadfence();
        } else {
            for (int v = tid; v < n; v += blockDim.x) B[v] = 0.0;
        }
        __syncthreads();

        const int s_lo = t * P.tile, s_hi = min(n, s_lo + P.tile);
        for (int s = s_lo + wave; s < s_hi; s += nwaves) {
            int cs = 0, sz = 0;
            const int slot = P.n_dbg ? debug_slot(P, r, s) : -1;
            if constexpr (G == 1 || G == 2 || G == 3)    // lane per vertex, unroll 4 / 2 / 8
                wave_source_lane<WEIGHTED, (G == 1 ? 4 : (G == 2 ? 2 : 8)), ADJ, GL>(
                    P, rp, adj, shift, B, dist, sig, ord, aux, &wctr[wave], s, slot, cs, sz, ovf);
            else
                wave_source<WEIGHTED, G, ADJ, GL>(P, rp, adj, shift, B, dist, sig, ord, aux, &wctr[wave], s, slot, cs,
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
            // every B atomic and label store of this item has reached L2
            __threadfence();
            __syncthreads();
            if (!split) {
                reduce_realization<ADJ, int32_t, true>(P, r_local, r, rp, B, comp32, csize32, RS, red_f, red_i,
                                                       acc_stats, true);
            } else {
                if (tid == 0) last_sh = (atomicAdd(&P.done[r_local], 1u) == (unsigned)(P.tiles_per_r - 1));
                __syncthreads();
                if (last_sh) {
                    __threadfence();
                    reduce_realization<ADJ, int32_t, true>(P, r_local, r, rp, B, comp32, csize32, RS, red_f, red_i,
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
static uint32_t wave_private_bytes(int n) {
    const uint32_t un = (uint32_t)n;
    const uint32_t per_wave = ((4u * un + 7u) & ~7u) + 8u * un + 2u * un + 2u * un;
    return (per_wave + 15u) & ~15u;
}

uint32_t lds_bytes_wave(int n, uint32_t adj_cap, uint32_t adj_bytes, int waves, uint32_t *wave_bytes) {
    const uint32_t wb = wave_private_bytes(n);
    if (wave_bytes) *wave_bytes = wb;
    return wave_layout(n, adj_cap, adj_bytes).waves + wb * (uint32_t)waves;
}

uint32_t lds_bytes_wave_l2(int n, int waves, uint32_t *wave_bytes) {
    const uint32_t wb = wave_private_bytes(n);
    if (wave_bytes) *wave_bytes = wb;
    return wb * (uint32_t)waves;
}

size_t l2_scratch_words(int n, uint32_t adj_cap, uint32_t adj_bytes) {
    return l2_layout(n, adj_cap, adj_bytes).total / 4u;
}

template <bool W, int G, typename ADJ, bool GL>
static hipError_t launch_t(const LaunchCtl &LC, int blocks, int waves, uint32_t lds, hipStream_t st) {
    hipLaunchKernelGGL((sweep_wave_kernel<W, G, ADJ, GL>), dim3(blocks), dim3(64 * waves), lds, st, LC);
    return hipGetLastError();
}

template <bool W, typename ADJ, bool GL>
static hipError_t attrs_g(int max_lds) {
    const void *ks[] = {(const void *)sweep_wave_kernel<W, 1, ADJ, GL>, (const void *)sweep_wave_kernel<W, 2, ADJ, GL>,
                        (const void *)sweep_wave_kernel<W, 3, ADJ, GL>, (const void *)sweep_wave_kernel<W, 4, ADJ, GL>,
                        (const void *)sweep_wave_kernel<W, 8, ADJ, GL>,
                        (const void *)sweep_wave_kernel<W, 16, ADJ, GL>};
    for (const void *k : ks) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <bool GL>
static hipError_t attrs_all(int max_lds) {
    hipError_t e;
    if ((e = attrs_g<true, uint16_t, GL>(max_lds)) != hipSuccess) return e;
    if ((e = attrs_g<false, uint16_t, GL>(max_lds)) != hipSuccess) return e;
    if ((e = attrs_g<true, uint32_t, GL>(max_lds)) != hipSuccess) return e;
    return attrs_g<false, uint32_t, GL>(max_lds);
}

// Allows every LDS-mode and L2-mode instantiation the device's dynamic LDS
// (set once per context, outside any stream capture).
hipError_t set_sweep_wave_attrs(int max_lds) {
    const hipError_t e = attrs_all<false>(max_lds);
    if (e != hipSuccess) return e;
    return attrs_all<true>(max_lds);
}

template <bool W, typename ADJ, bool GL>
static hipError_t launch_g(const LaunchCtl &LC, int group, int blocks, int waves, uint32_t lds, hipStream_t st) {
    switch (group) {
        case 1: return launch_t<W, 1, ADJ, GL>(LC, blocks, waves, lds, st);
        case 2: return launch_t<W, 2, ADJ, GL>(LC, blocks, waves, lds, st);
        case 3: return launch_t<W, 3, ADJ, GL>(LC, blocks, waves, lds, st);
        case 4: return launch_t<W, 4, ADJ, GL>(LC, blocks, waves, lds, st);
        case 16: return launch_t<W, 16, ADJ, GL>(LC, blocks, waves, lds, st);
        default: return launch_t<W, 8, ADJ, GL>(LC, blocks, waves, lds, st);
    }
}

template <bool GL>
static hipError_t launch_w(const LaunchCtl &LC, bool weighted, int group, uint32_t adj_bytes, int blocks, int waves,
                           uint32_t lds, hipStream_t st) {
    if (adj_bytes == 2)
        return weighted ? launch_g<true, uint16_t, GL>(LC, group, blocks, waves, lds, st)
                        : launch_g<false, uint16_t, GL>(LC, group, blocks, waves, lds, st);
    return weighted ? launch_g<true, uint32_t, GL>(LC, group, blocks, waves, lds, st)
                    : launch_g<false, uint32_t, GL>(LC, group, blocks, waves, lds, st);
}

hipError_t launch_sweep_wave(const LaunchCtl &LC, bool weighted, bool l2, int group, uint32_t adj_bytes, int blocks,
                             int waves, uint32_t lds, hipStream_t st) {
    return l2 ? launch_w<true>(LC, weighted, group, adj_bytes, blocks, waves, lds, st)
              : launch_w<false>(LC, weighted, group, adj_bytes, blocks, waves, lds, st);
}

}  // namespace amc
