// sweep_block.hip -- realization x source sweep for graphs beyond the LDS
// mode: one workgroup per (realization, source), frontier queues in LDS,
// the realized adjacency in a per-workgroup global scratch (L2-resident).
//
// Paper: Bao, Kontou, Vogiatzis, "Betweenness-Central Nodes Under
// Uncertainty: An Absorbing Markov Chain Approach".
//
// Per work item (realization r, tile of sources) the workgroup realizes the
// edges of r (Section 3.1) into its scratch, then runs the sources one after
// another.  A source is a level-synchronous traversal: the current frontier
// (vertices at the same distance, settled) is spread over groups of G lanes
// (one lane per vertex when the frontier fills the workgroup, else two or
// four); each group pulls the exact path count of its vertex from its
// predecessors and relaxes the vertex's edges; newly reached vertices are
// appended to the queue with one LDS atomic per wavefront and block of slots
// (ballot + prefix).  With unit weights a wide new level is ordered by degree
// so that a wavefront's lanes walk lists of about one length.  With integer
// weights the unsettled reached vertices wait in a fringe and the next
// distance is the fringe minimum (distance buckets).  The reverse pass walks
// the equal-distance segments backwards and accumulates the dependencies of
// the Section 3.1 betweenness into B(H_r) held in LDS; the reduction and the
// counting are the same as in the LDS mode.  Placement PL of that state:
// 0 in LDS; 2 in the workgroup's global scratch (graphs whose per-source
// state exceeds the LDS, up to 65535 vertices); 1 as 2 but with the
// distances and the realized row offsets (the most used arrays) in LDS.  All
// of the state is read and written by the one workgroup, whose global
// accesses a barrier orders as it does its LDS accesses, so the code is the
// same.  Levels are ordered by degree only while vertex ids fit the 13 bits
// that order packs them into.
#include <type_traits>

#include "amc_dev.hpp"
#include "amc_kernels.hpp"
#include "sweep_common.hpp"

namespace amc {

constexpr int kBU = 4;          // adjacency slots per lane and trip
constexpr int kSortMin = 512;    // unit weights: levels at least this large are ordered by degree
constexpr int kDegClasses = 4;   // degree classes of that order: 1-4, 5-8, 9-12, 13 or more
constexpr int kSortMaxN = 8191;  // the order packs vertex ids into 13 bits
static_assert(kDegClasses * 16 <= 64, "the class counters share one 64-bit word");

// LDS: dist u32[n] | sig u64[n] | ord u16[n] | aux u16[n] | B f64[n] | comp
// u16[n] | csize u16[n] | rp u32[n+1] (the realized row offsets: every
// frontier vertex reads its pair, so they stay on chip; the adjacency lives
// in the workgroup's global scratch)
struct BlockLayout {
    uint32_t dist, sig, ord, aux, B, comp, csize, rp, total;
};

__host__ __device__ inline BlockLayout block_layout(int n) {
    BlockLayout L;
    const uint32_t un = (uint32_t)n;
    L.dist = 0;
    L.sig = (4u * un + 7u) & ~7u;
    L.ord = L.sig + 8u * un;
    L.aux = L.ord + 2u * un;
    L.B = (L.aux + 2u * un + 7u) & ~7u;
    L.comp = L.B + 8u * un;
    L.csize = L.comp + 2u * un;
    L.rp = (L.csize + 2u * un + 3u) & ~3u;
    L.total = (L.rp + 4u * (un + 1u) + 15u) & ~15u;
    return L;
}

// 32-bit words of the realized adjacency (2m entries plus padding).
__host__ __device__ inline size_t block_adj_words(int64_t m, uint32_t adj_bytes) {
    return ((2 * (size_t)m + kAdjPad) * adj_bytes + 3) / 4;
}

// Appends the found[k] lanes of U slots to the queue whose tail is *ctr (LDS)
// with one atomic per wavefront; pos[k] is the position of slot k's entry.
template <int U>
__device__ __forceinline__ void block_append(uint32_t *ctr, const bool (&found)[U], uint32_t (&pos)[U]) {
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
#pragma unroll
    for (int k = 0; k < U; ++k) {
        pos[k] = base + rank_lt(m[k]);
        base += (uint32_t)__popcll(m[k]);
    }
}

// Reorders q[0, cnt) (one BFS level) by degree class min((deg - 1) / 4,
// kDegClasses - 1), buf[0, cnt) holding each entry with its class in bits
// 13-15 (the workgroup mode stages at most 5103 vertices, so ids fit in 13
// bits), so that the lanes of a wavefront walk adjacency lists of about one
// length.  cls[0] counts the classes and cls[1] hands out their positions,
// four 16-bit fields each (cnt < 2^13), so that a wavefront claims its share
// of every class with one atomic.  The order inside a class is arbitrary: a
// level's vertices are processed independently, so the traversal's results
// do not depend on it.  Every thread of the workgroup calls it.
__device__ void order_level_by_degree(uint16_t *q, uint16_t *buf, const uint32_t *rp, int cnt,
                                      unsigned long long *cls) {
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63;
    if (tid < 2) cls[tid] = 0ull;
    __syncthreads();
    for (int k0 = 0; k0 < cnt; k0 += nthr) {
        const int k = k0 + tid;
        int c = kDegClasses;   // none
        if (k < cnt) {
            const uint32_t v = q[k];
            const uint32_t deg = rp[v + 1] - rp[v];   // >= 1: v was reached over an edge
            c = min((int)((deg - 1u) >> 2), kDegClasses - 1);
            buf[k] = (uint16_t)(v | ((uint32_t)c << 13));
        }
        unsigned long long packed = 0ull;
#pragma unroll
        for (int j = 0; j < kDegClasses; ++j)
            packed |= (unsigned long long)__popcll(__ballot(c == j)) << (16 * j);
        if (lane == 0 && packed) atomicAdd(&cls[0], packed);
    }
    __syncthreads();
    const unsigned long long tot = cls[0];
    uint32_t start[kDegClasses];
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < kDegClasses; ++j) {
        start[j] = acc;
        acc += (uint32_t)(tot >> (16 * j)) & 0xFFFFu;
    }
    for (int k0 = 0; k0 < cnt; k0 += nthr) {
        const int k = k0 + tid;
        int c = kDegClasses;
        uint32_t v = 0;
        if (k < cnt) {
            const uint32_t e = buf[k];
            v = e & 0x1FFFu;
            c = (int)(e >> 13);
        }
        uint64_t m[kDegClasses];
        unsigned long long packed = 0ull;
#pragma unroll
        for (int j = 0; j < kDegClasses; ++j) {
            m[j] = __ballot(c == j);
            packed |= (unsigned long long)__popcll(m[j]) << (16 * j);
        }
        unsigned long long base = 0ull;
        if (lane == 0 && packed) base = atomicAdd(&cls[1], packed);
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
        base = ((unsigned long long)hi << 32) | lo;
        uint32_t pos = 0;
#pragma unroll
        for (int j = 0; j < kDegClasses; ++j)
            if (c == j) pos = start[j] + ((uint32_t)(base >> (16 * j)) & 0xFFFFu) + rank_lt(m[j]);
        if (k < cnt) q[pos] = (uint16_t)v;
    }
    __syncthreads();
}

// Lanes per vertex for a level (or segment) of k vertices: one when the
// level fills every lane of the workgroup, else two or four so that more
// wavefronts share it.
__device__ __forceinline__ int level_group(int k, int nthr) { return k >= nthr ? 1 : (k >= nthr / 2 ? 2 : 4); }

template <bool WEIGHTED, typename ADJ>
__device__ void block_source(const SweepParams &P, const uint32_t *rp, const ADJ *adj, double *B,
                             uint32_t *dist, unsigned long long *sig, uint16_t *ord, uint16_t *aux, uint32_t *ctl,
                             uint32_t *tmp, int s, int dbg_slot, int &comp_out, int &size_out, bool &ovf) {
    const int n = P.n;
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, wave = tid >> 6, nwaves = nthr >> 6;
    // ctl[0]: queue / fringe tail
    for (int v = tid; v < n; v += nthr) dist[v] = kInf;
    __syncthreads();
    if (tid == 0) {
        dist[s] = 0u;
        sig[s] = 1ull;
        ord[0] = (uint16_t)s;
        ctl[0] = WEIGHTED ? 0u : 1u;
    }
    __syncthreads();

    // one frontier sweep over ord[f_lo, f_hi) at distance D: groups of G
    // lanes per vertex, each lane taking kBU of its vertex's slots per trip
    // (loads issued together, the next trip's entries fetched while this one
    // is used); a vertex pulls its exact path count from its predecessors and
    // relaxes its edges, newly reached vertices are appended to the queue
    // (unit weights: ord, the next level) or the fringe (aux)
    auto relax_level = [&](auto gtag, int f_lo, int f_hi, uint32_t D) {
        constexpr int G = decltype(gtag)::value;
        const int sub = G == 1 ? 0 : tid % G, grp = tid / G, ngrp = nthr / G;
        for (int base = f_lo; base < f_hi; base += ngrp) {
            const int idx = base + grp;
            const bool mine = idx < f_hi;
            unsigned long long acc = 0ull;
            int v = 0;
            uint32_t beg = 0, end = 0;
            if (mine) {
                v = ord[idx];
                beg = rp[v];
                end = rp[v + 1];
            }
            const uint32_t len = end - beg;
            const uint32_t trips = G == 1 ? len : (len > (uint32_t)sub ? (len - (uint32_t)sub + G - 1) / G : 0u);
            const uint32_t maxtrips = wave_max_fast(trips);
            const uint32_t first = beg + (uint32_t)sub;
            uint32_t nxt[kBU];
#pragma unroll
            for (int k = 0; k < kBU; ++k) nxt[k] = (uint32_t)adj[first + G * k];
            for (uint32_t t = 0; t < maxtrips; t += kBU) {
                uint32_t cur[kBU], u[kBU], w[kBU], du[kBU], old[kBU], pos[kBU];
                bool pred[kBU], rel[kBU], found[kBU];
#pragma unroll
                for (int k = 0; k < kBU; ++k) cur[k] = nxt[k];
                if (t + kBU < maxtrips) {
#pragma unroll
                    for (int k = 0; k < kBU; ++k) nxt[k] = (uint32_t)adj[first + G * (t + kBU + k)];
                }
                // a slot past the vertex's list reads vertex 0 with weight
                // kNoEdge (fails both tests)
#pragma unroll
                for (int k = 0; k < kBU; ++k) {
                    const bool in = t + k < trips;
                    u[k] = in ? (cur[k] & 0xFFFFu) : 0u;
                    w[k] = in ? (WEIGHTED ? (cur[k] >> 16) : 1u) : kNoEdge;
                }
#pragma unroll
                for (int k = 0; k < kBU; ++k) du[k] = dist[u[k]];
#pragma unroll
                for (int k = 0; k < kBU; ++k) {
                    pred[k] = du[k] + w[k] == D;
                    rel[k] = D + w[k] < du[k];
                }
#pragma unroll
                for (int k = 0; k < kBU; ++k) {
                    // read from a vertex in range either way (no branch)
                    const unsigned long long val = sig[pred[k] ? u[k] : (uint32_t)s];
                    const unsigned long long x = acc + (pred[k] ? val : 0ull);
                    ovf |= x < acc;
                    acc = x;
                }
#pragma unroll
                for (int k = 0; k < kBU; ++k) old[k] = rel[k] ? atomicMin(&dist[u[k]], D + w[k]) : 0u;
#pragma unroll
                for (int k = 0; k < kBU; ++k) found[k] = old[k] == kInf;   // a lane that does not relax keeps 0
                block_append<kBU>(&ctl[0], found, pos);
#pragma unroll
                for (int k = 0; k < kBU; ++k)
                    if (found[k]) {
                        if (WEIGHTED) aux[pos[k]] = (uint16_t)u[k];
                        else ord[pos[k]] = (uint16_t)u[k];
                    }
            }
            if constexpr (G > 1) acc = group_sum_u64<G>(acc, ovf);
            if (mine && sub == 0 && v != s) sig[v] = acc;
        }
    };

    int f_lo = 0, ord_end = 1, nseg = 0;
    uint32_t D = 0;
    for (;;) {
        if (tid == 0) aux[n - 1 - nseg] = (uint16_t)f_lo;
        ++nseg;
        const int G = level_group(ord_end - f_lo, nthr);
        if (G == 1) relax_level(std::integral_constant<int, 1>{}, f_lo, ord_end, D);
        else if (G == 2) relax_level(std::integral_constant<int, 2>{}, f_lo, ord_end, D);
        else relax_level(std::integral_constant<int, 4>{}, f_lo, ord_end, D);
        __syncthreads();
        if (!WEIGHTED) {
            const int new_end = (int)ctl[0];
            __syncthreads();
            if (new_end == ord_end) break;
            // the new level occupies ord[ord_end, new_end) and aux[0, new_end -
            // ord_end) stays below the segment starts at aux[n - nseg, n)
            if (new_end - ord_end >= kSortMin && n <= kSortMaxN)
                order_level_by_degree(ord + ord_end, aux, rp, new_end - ord_end, (unsigned long long *)tmp);
            f_lo = ord_end;
            ord_end = new_end;
            D += 1u;
        } else {
            const int fr = (int)ctl[0];
            if (fr == 0) break;
            // next distance: minimum over the fringe
            uint32_t mn = kInf;
            for (int k = tid; k < fr; k += nthr) {
                const uint32_t dk = dist[aux[k]];
                mn = dk < mn ? dk : mn;
            }
            mn = wave_min_u32(mn);
            if (lane == 0) tmp[wave] = mn;
            __syncthreads();
            mn = tmp[0];
            for (int w = 1; w < nwaves; ++w) mn = tmp[w] < mn ? tmp[w] : mn;
            __syncthreads();
            // partition chunk by chunk: every read of a chunk precedes the
            // barrier, every write follows it, and writes land at or below
            // the read positions of this or earlier chunks
            int settled = 0, kept = 0;
            for (int k0 = 0; k0 < fr; k0 += nthr) {
                const int k = k0 + tid;
                const bool valid = k < fr;
                const uint32_t x = valid ? aux[k] : 0u;
                const bool is_s = valid && dist[x] == mn;
                const bool is_k = valid && !is_s;
                const uint64_t ms = __ballot(is_s), mk = __ballot(is_k);
                if (lane == 0) {
                    tmp[wave] = (uint32_t)__popcll(ms);
                    tmp[kMaxWaves + wave] = (uint32_t)__popcll(mk);
                }
                __syncthreads();
                int ps = settled, pk = kept, ts = 0, tk = 0;
                for (int w = 0; w < nwaves; ++w) {
                    if (w < wave) {
                        ps += (int)tmp[w];
                        pk += (int)tmp[kMaxWaves + w];
                    }
                    ts += (int)tmp[w];
                    tk += (int)tmp[kMaxWaves + w];
                }
                const uint64_t lt = lanemask_lt();
                if (is_s) ord[ord_end + ps + __popcll(ms & lt)] = (uint16_t)x;
                if (is_k) aux[pk + __popcll(mk & lt)] = (uint16_t)x;
                settled += ts;
                kept += tk;
                __syncthreads();
            }
            if (tid == 0) ctl[0] = (uint32_t)kept;
            __syncthreads();
            f_lo = ord_end;
            ord_end += settled;
            D = mn;
        }
    }
    // component of s and its size
    {
        int mn = n;
        for (int k = tid; k < ord_end; k += nthr) mn = min(mn, (int)ord[k]);
        mn = wave_min_i32(mn);
        if (lane == 0) tmp[wave] = (uint32_t)mn;
        __syncthreads();
        int c = (int)tmp[0];
        for (int w = 1; w < nwaves; ++w) c = min(c, (int)tmp[w]);
        comp_out = c;
        size_out = ord_end;
        __syncthreads();
    }
    if (dbg_slot >= 0) {
        for (int v = tid; v < n; v += nthr) {
            const uint32_t d = dist[v];
            P.dbg_dist[(size_t)dbg_slot * n + v] = d == kInf ? 0xFFFFFFFFu : d;
            P.dbg_sigma[(size_t)dbg_slot * n + v] = d == kInf ? 0ull : sig[v];
            P.dbg_delta[(size_t)dbg_slot * n + v] = 0.0;
        }
        __syncthreads();
    }
    // reverse pass over the equal-distance segments: a vertex sums c_u over
    // its successors u (G lanes per vertex, as in the forward sweep)
    auto accumulate_segment = [&](auto gtag, int lo, int hi) {
        constexpr int G = decltype(gtag)::value;
        const int sub = G == 1 ? 0 : tid % G, grp = tid / G, ngrp = nthr / G;
        for (int base = lo; base < hi; base += ngrp) {
            const int idx = base + grp;
            const bool mine = idx < hi;
            double sum = 0.0;
            int v = 0;
            if (mine) {
                v = ord[idx];
                const uint32_t dv = dist[v];
                const uint32_t beg = rp[v], end = rp[v + 1];
                const uint32_t len = end - beg;
                const uint32_t trips = G == 1 ? len : (len > (uint32_t)sub ? (len - (uint32_t)sub + G - 1) / G : 0u);
                const uint32_t first = beg + (uint32_t)sub;
                for (uint32_t t = 0; t < trips; t += kBU) {
                    uint32_t a[kBU], u[kBU], du[kBU];
#pragma unroll
                    for (int k = 0; k < kBU; ++k) a[k] = (uint32_t)adj[first + G * (t + k)];
#pragma unroll
                    for (int k = 0; k < kBU; ++k) u[k] = (t + k < trips) ? (a[k] & 0xFFFFu) : 0u;
#pragma unroll
                    for (int k = 0; k < kBU; ++k) du[k] = dist[u[k]];
#pragma unroll
                    for (int k = 0; k < kBU; ++k) {
                        const uint32_t w = (t + k < trips) ? (WEIGHTED ? (a[k] >> 16) : 1u) : kNoEdge;
                        if (du[k] == dv + w) sum += as_f64(sig[u[k]]);   // u succeeds v: c_u
                    }
                }
            }
            if constexpr (G > 1) sum = group_sum_f64<G>(sum);
            if (mine && sub == 0) {
                const double sv = (double)sig[v];
                const double delta = sv * sum;
                sig[v] = as_u64((1.0 + delta) / sv);
                if (v != s) B[v] += delta;
                if (dbg_slot >= 0) P.dbg_delta[(size_t)dbg_slot * n + v] = delta;
            }
        }
    };
    for (int k = nseg - 1; k >= 0; --k) {
        const int lo = aux[n - 1 - k];
        const int hi = (k == nseg - 1) ? ord_end : (int)aux[n - 2 - k];
        const int G = level_group(hi - lo, nthr);
        if (G == 1) accumulate_segment(std::integral_constant<int, 1>{}, lo, hi);
        else if (G == 2) accumulate_segment(std::integral_constant<int, 2>{}, lo, hi);
        else accumulate_segment(std::integral_constant<int, 4>{}, lo, hi);
        __syncthreads();
    }
}

// ADJ: the realized adjacency entry, uint32_t (weight << 16 | neighbour) or,
// with unit weights, uint16_t (the neighbour alone), which halves the
// per-workgroup scratch the traversal reads so that it stays in the L2.
// Words of the per-workgroup scratch before the global state region: the
// realized adjacency, then the component centres (2 n words) and 64 words of
// slack.
__host__ __device__ inline size_t block_gs_state_words(int n, int64_t m, uint32_t adj_bytes) {
    return (block_adj_words(m, adj_bytes) + 2 * (size_t)n + 64 + 3) & ~(size_t)3;
}
// Placement 1: LDS bytes of dist u32[n] | rp u32[n+1].
__host__ __device__ inline uint32_t block_hybrid_rp(int n) { return (4u * (uint32_t)n + 15u) & ~15u; }
__host__ __device__ inline uint32_t block_hybrid_lds(int n) {
    return (block_hybrid_rp(n) + 4u * ((uint32_t)n + 1u) + 15u) & ~15u;
}

template <bool WEIGHTED, typename ADJ, int PL>
__global__ __launch_bounds__(1024) void sweep_block_kernel(LaunchCtl LC) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __shared__ __attribute__((aligned(8))) uint32_t scan_tmp[2 * kMaxWaves];
    __shared__ uint32_t ctl[4];
    __shared__ double red_f[kMaxWaves];
    __shared__ int red_i[kMaxWaves];
    __shared__ int item_sh;
    __shared__ int last_sh;

    const int tid = threadIdx.x, lane = tid & 63, nthr = blockDim.x;
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
        if (q != q_prev) {
            if (q_prev >= 0) flush_stats(LC.descs[q_prev], acc_stats, ovf);
            q_prev = q;
        }
        const uint32_t qitem = item_local(LC, q, item);
        const uint32_t r_local = qitem / (uint32_t)P.tiles_per_r;
        const int t = (int)(qitem % (uint32_t)P.tiles_per_r);
        const uint32_t r = P.r_begin + r_local;

        const int n = P.n;
        const BlockLayout L = block_layout(n);
        // per-workgroup global scratch: the realized adjacency (2m plus
        // padding entries), then the component centres (2 n words), which
        // also absorb the reads past the last vertex's slots; with GS the
        // state region follows
        uint32_t *gs = LC.bscratch + (size_t)blockIdx.x * LC.bscratch_words;
        unsigned char *st;
        if constexpr (PL != 0) st = (unsigned char *)to_global(gs + block_gs_state_words(n, P.m, (uint32_t)sizeof(ADJ)));
        else st = smem;
        uint32_t *dist = PL == 1 ? (uint32_t *)smem : (uint32_t *)(st + L.dist);
        unsigned long long *sig = (unsigned long long *)(st + L.sig);
        uint16_t *ord = (uint16_t *)(st + L.ord);
        uint16_t *aux = (uint16_t *)(st + L.aux);
        double *B = (double *)(st + L.B);
        uint16_t *comp = (uint16_t *)(st + L.comp);
        uint16_t *csize = (uint16_t *)(st + L.csize);
        uint32_t *rp = PL == 1 ? (uint32_t *)(smem + block_hybrid_rp(n)) : (uint32_t *)(st + L.rp);
        ADJ *adj = to_global((ADJ *)gs);
        ReduceScratch RS;
        RS.cmax = (unsigned long long *)st;                // aliases dist/sig (free during the reduction)
        RS.wmax = RS.cmax + n;
        uint32_t *tail4 = gs + block_adj_words(P.m, (uint32_t)sizeof(ADJ));
        RS.ccen = (int32_t *)tail4;
        RS.wcen = RS.ccen + n;

        // entries (w << 16) | neighbour; a 16-bit entry keeps the neighbour
        stage_realization(P, r, rp, adj, 16u, (uint16_t *)st, scan_tmp);
        for (int v = tid; v < n; v += nthr) B[v] = 0.0;
        __syncthreads();

        const int s_lo = t * P.tile, s_hi = min(n, s_lo + P.tile);
        for (int s = s_lo; s < s_hi; ++s) {
            int cs = 0, sz = 0;
            const int slot = P.n_dbg ? debug_slot(P, r, s) : -1;
            block_source<WEIGHTED, ADJ>(P, rp, adj, B, dist, sig, ord, aux, ctl, scan_tmp, s, slot, cs, sz, ovf);
            if (tid == 0) {
                comp[s] = (uint16_t)cs;
                csize[s] = (uint16_t)(sz & 0xFFFF);
            }
        }
        __syncthreads();
        if (P.tiles_per_r == 1) {
            reduce_realization(P, r_local, r, rp, B, comp, csize, RS, red_f, red_i, acc_stats, true);
        } else {
            double *Bg = P.Bg + (size_t)r_local * n;
            for (int v = tid; v < n; v += nthr)
                if (B[v] != 0.0) unsafeAtomicAdd(&Bg[v], B[v]);
            for (int s = s_lo + tid; s < s_hi; s += nthr) {
                P.compg[(size_t)r_local * n + s] = comp[s];
                P.sizeg[(size_t)r_local * n + s] = csize[s];
            }
            __threadfence();
            __syncthreads();
            if (tid == 0) last_sh = (atomicAdd(&P.done[r_local], 1u) == (unsigned)(P.tiles_per_r - 1));
            __syncthreads();
            if (last_sh) {
                __threadfence();
                for (int v = tid; v < n; v += nthr) {
                    B[v] = __hip_atomic_load(&Bg[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    comp[v] = (uint16_t)__hip_atomic_load(&P.compg[(size_t)r_local * n + v], __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
                    csize[v] = (uint16_t)__hip_atomic_load(&P.sizeg[(size_t)r_local * n + v], __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
                }
                __syncthreads();
                reduce_realization(P, r_local, r, rp, B, comp, csize, RS, red_f, red_i, acc_stats, false);
            }
            __syncthreads();
        }
    }
    if (q_prev >= 0) flush_stats(LC.descs[q_prev], acc_stats, ovf);
    (void)lane;
}

uint32_t lds_bytes_block(int n, int threads) {
    (void)threads;
    return block_layout(n).total;
}

// Bytes at the start of the LDS that the per-edge staging may use (below rp).
uint32_t block_staging_bytes(int n) { return block_layout(n).rp; }

uint32_t lds_bytes_block_hybrid(int n) { return block_hybrid_lds(n); }

size_t block_scratch_words(int n, int64_t m, bool weighted, int state_place) {
    const uint32_t ab = weighted ? 4u : 2u;
    if (state_place == 0) return block_adj_words(m, ab) + 2 * (size_t)n + 64;
    return block_gs_state_words(n, m, ab) + block_layout(n).total / 4;
}

template <int PL>
static hipError_t launch_block_t(const LaunchCtl &LC, bool weighted, int blocks, int threads, uint32_t lds,
                                 hipStream_t st) {
    if (weighted)
        hipLaunchKernelGGL((sweep_block_kernel<true, uint32_t, PL>), dim3(blocks), dim3(threads), lds, st, LC);
    else
        hipLaunchKernelGGL((sweep_block_kernel<false, uint16_t, PL>), dim3(blocks), dim3(threads), lds, st, LC);
    return hipGetLastError();
}

hipError_t launch_sweep_block(const LaunchCtl &LC, bool weighted, int state_place, int blocks, int threads,
                              uint32_t lds, hipStream_t st) {
    if (state_place == 1) return launch_block_t<1>(LC, weighted, blocks, threads, lds, st);
    if (state_place == 2) return launch_block_t<2>(LC, weighted, blocks, threads, lds, st);
    return launch_block_t<0>(LC, weighted, blocks, threads, lds, st);
}

hipError_t set_sweep_block_attrs(int max_lds) {
    const void *ks[] = {(const void *)sweep_block_kernel<true, uint32_t, 0>,
                        (const void *)sweep_block_kernel<false, uint16_t, 0>,
                        (const void *)sweep_block_kernel<true, uint32_t, 1>,
                        (const void *)sweep_block_kernel<false, uint16_t, 1>,
                        (const void *)sweep_block_kernel<true, uint32_t, 2>,
                        (const void *)sweep_block_kernel<false, uint16_t, 2>};
    for (const void *k : ks) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace amc
