// wave_source.hpp -- one source of the realization x source sweep on one
// wavefront, and the LDS / L2 carve-ups of a workgroup; shared by the sweep
// kernel and the trajectory kernel.
//
// Paper: Bao, Kontou, Vogiatzis, "Betweenness-Central Nodes Under
// Uncertainty: An Absorbing Markov Chain Approach" (Section 3.1).
#pragma once

#include "amc_dev.hpp"

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

// With MASK the traversal stays inside the vertex set mask[v] != 0 (an induced
// subgraph): an edge into a vertex outside it is never relaxed, so such a
// vertex stays unreached and fails the predecessor and successor tests.
template <bool WEIGHTED, int U, typename ADJ, bool GB, bool MASK = false>
__device__ void wave_source_lane(const SweepParams &P, const ADJ *rp, const ADJ *adj, uint32_t shift,
                                 double *B, uint32_t *dist, unsigned long long *sig, uint16_t *ord, uint16_t *aux,
                                 uint32_t *ctr, int s, int dbg_slot, int &comp_out, int &size_out, bool &ovf,
                                 const uint8_t *mask = nullptr) {
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
                    if constexpr (MASK) rel[k] = rel[k] && mask[u[k]] != 0;
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

// One source with the vertex mapping G: 1 / 2 / 3 = lane per vertex with 4 /
// 2 / 8 adjacency slots in flight, otherwise G lanes per vertex.
template <bool WEIGHTED, int G, typename ADJ, bool GB>
__device__ __forceinline__ void run_source(const SweepParams &P, const ADJ *rp, const ADJ *adj, uint32_t shift,
                                           double *B, uint32_t *dist, unsigned long long *sig, uint16_t *ord,
                                           uint16_t *aux, uint32_t *ctr, int s, int dbg_slot, int &comp_out,
                                           int &size_out, bool &ovf) {
    if constexpr (G == 1 || G == 2 || G == 3)
        wave_source_lane<WEIGHTED, (G == 1 ? 4 : (G == 2 ? 2 : 8)), ADJ, GB>(P, rp, adj, shift, B, dist, sig, ord,
                                                                            aux, ctr, s, dbg_slot, comp_out,
                                                                            size_out, ovf);
    else
        wave_source<WEIGHTED, G, ADJ, GB>(P, rp, adj, shift, B, dist, sig, ord, aux, ctr, s, dbg_slot, comp_out,
                                          size_out, ovf);
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

}  // namespace amc
