// wave_source.hpp -- one source of the realization x source sweep on one
// wavefront, and the LDS / L2 carve-ups of a workgroup; shared by the sweep,
// trajectory and anchored-neighbourhood kernels.
//
// Paper: Bao, Kontou, Vogiatzis, "Betweenness-Central Nodes Under
// Uncertainty: An Absorbing Markov Chain Approach" (Section 3.1).
#pragma once

#include <type_traits>

#include "amc_dev.hpp"

namespace amc {

// ---------------------------------------------------------------------------
// One source on one wavefront.  State (LDS, private to the wavefront):
//   dist[n]  tentative / final distance (DistOps<DT>::unreached = unreached)
//   sig[n]   exact path count sigma_s(v) (uint64); after v's dependency is
//            known the slot holds c_v = (1 + delta_v) / sigma_v as a double,
//            so a predecessor u gets delta_u = sigma_u * sum_{succ w} c_w
//   ord[n]   ord[0, ord_end): settled vertices in non-decreasing distance,
//            the first vertex of each equal-distance segment tagged with
//            kSegMark; ord[ord_end, ord_end + fringe): the reached but
//            unsettled vertices (integer weights only).  Settled and
//            unsettled vertices are distinct, so the two parts fit in n.
// G lanes cooperate on one vertex's adjacency; an adjacency entry holds the
// neighbour in its low `shift` bits and the weight above them.
// ---------------------------------------------------------------------------
constexpr uint16_t kSegMark = 0x8000u;   // vertex ids stay below 2^15
constexpr uint16_t kVertexMask = 0x7FFFu;

// Distance entries: uint32_t, or uint16_t when every finite distance plus one
// edge weight stays below 0xFFFF (the host checks n * w_max < 0xFFFF), which
// halves the array.  A relaxation reads the 32-bit word holding d[u]
// (word / value), issues its atomic minimum (issue_min, returning the
// previous word) and resolves the previous value of d[u] (resolve): the
// lane-per-vertex code issues the minima of its U slots back to back before
// resolving any.  fetch_min does both at once.
template <typename DT>
struct DistOps;
template <>
struct DistOps<uint32_t> {
    static constexpr uint32_t unreached = kInf;
    __device__ static __forceinline__ uint32_t word(const uint32_t *d, uint32_t u) { return d[u]; }
    __device__ static __forceinline__ uint32_t value(uint32_t wd, uint32_t) { return wd; }
    __device__ static __forceinline__ uint32_t issue_min(uint32_t *d, uint32_t u, uint32_t val, uint32_t) {
        return atomicMin(&d[u], val);
    }
    __device__ static __forceinline__ uint32_t resolve(uint32_t *, uint32_t, uint32_t, uint32_t, uint32_t prev) {
        return prev;
    }
    __device__ static __forceinline__ uint32_t fetch_min(uint32_t *d, uint32_t u, uint32_t val) {
        return atomicMin(&d[u], val);
    }
};
template <>
struct DistOps<uint16_t> {
    static constexpr uint32_t unreached = 0xFFFFu;
    // the array starts 4-byte aligned and is padded to a whole word
    __device__ static __forceinline__ uint32_t *word_ptr(uint16_t *d, uint32_t u) {
        return reinterpret_cast<uint32_t *>(d) + (u >> 1);
    }
    __device__ static __forceinline__ uint32_t word(const uint16_t *d, uint32_t u) {
        return reinterpret_cast<const uint32_t *>(d)[u >> 1];
    }
    __device__ static __forceinline__ uint32_t value(uint32_t wd, uint32_t u) { return (wd >> ((u & 1u) * 16u)) & 0xFFFFu; }
    __device__ static __forceinline__ uint32_t with(uint32_t wd, uint32_t u, uint32_t val) {
        const uint32_t sh = (u & 1u) * 16u;
        return (wd & ~(0xFFFFu << sh)) | (val << sh);
    }
    // compare-and-swap against the word read before (val < value(wd, u))
    __device__ static __forceinline__ uint32_t issue_min(uint16_t *d, uint32_t u, uint32_t val, uint32_t wd) {
        return atomicCAS(word_ptr(d, u), wd, with(wd, u, val));
    }
    // the word changed in between (the other half, or d[u] itself): retry
    // from the word found until d[u] <= val or the swap goes in
    __device__ static __forceinline__ uint32_t resolve(uint16_t *d, uint32_t u, uint32_t val, uint32_t wd,
                                                       uint32_t prev) {
        if (prev == wd) return value(wd, u);
        uint32_t cur = prev;
        for (;;) {
            const uint32_t h = value(cur, u);
            if (h <= val) return h;
            const uint32_t p = atomicCAS(word_ptr(d, u), cur, with(cur, u, val));
            if (p == cur) return h;
            cur = p;
        }
    }
    __device__ static __forceinline__ uint32_t fetch_min(uint16_t *d, uint32_t u, uint32_t val) {
        const uint32_t wd = __hip_atomic_load(word_ptr(d, u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (value(wd, u) <= val) return value(wd, u);
        return resolve(d, u, val, wd, issue_min(d, u, val, wd));
    }
};

// In-place partition of the fringe ord[a, a + fr): the vertices at distance
// mn go to ord[a, a + settled) (returned; ord[a], the start of the new
// segment, carries kSegMark), the others to ord[a + settled, a + fr); kmin
// gets the lane minimum over the distances of the others.  The caller
// synchronises the wavefront after the last chunk's writes.
// Chunks of 64 U entries are taken in order.  The unsettled entries of the
// chunks already taken form one block right after the settled ones; the
// settled entries of a new chunk take that block's first slots and the
// entries they displace move to the slots the chunk itself was read from.
template <int U, typename DT>
__device__ __forceinline__ int fringe_partition(uint16_t *ord, const DT *dist, int a, int fr, uint32_t mn,
                                                uint32_t &kmin) {
    const int lane = threadIdx.x & 63;
    const int end = a + fr;
    int S = 0, K = 0;   // settled and kept entries so far
    kmin = kInf;
    for (int p = a; p < end; p += 64 * U) {   // p == a + S + K
        // sub-chunk c holds entries p + 64 c + lane; its valid lanes form a prefix of nv[c]
        int nv[U];
        uint32_t x[U], dx[U];
#pragma unroll
        for (int c = 0; c < U; ++c) {
            nv[c] = min(64, max(0, end - (p + 64 * c)));
            x[c] = lane < nv[c] ? (uint32_t)ord[p + 64 * c + lane] : 0u;
        }
#pragma unroll
        for (int c = 0; c < U; ++c) dx[c] = lane < nv[c] ? (uint32_t)dist[x[c]] : kInf;
        uint64_t ms[U];
        int s = 0, kk = 0;
#pragma unroll
        for (int c = 0; c < U; ++c) {
            const bool valid = lane < nv[c];
            const bool is_s = valid && dx[c] == mn;
            kmin = (valid && !is_s && dx[c] < kmin) ? dx[c] : kmin;
            ms[c] = __ballot(is_s);
            const int sc = __popcll(ms[c]);
            s += sc;
            kk += nv[c] - sc;
        }
        // entries of the kept block displaced by this chunk's settled ones
        const int d = s < K ? s : K;
        uint32_t y[U];
        if (d > 0) {
#pragma unroll
            for (int c = 0; c < U; ++c) {
                const int j = 64 * c + lane;
                y[c] = j < d ? (uint32_t)ord[a + S + j] : 0u;
            }
        }
        wave_sync();   // every read of this chunk precedes its writes
        // one store per entry: a settled one goes after the settled ones so
        // far, a kept one after this chunk's settled ones (its rank among the
        // kept lanes is its lane minus its rank among the settled ones)
        int so = 0, ko = 0;
#pragma unroll
        for (int c = 0; c < U; ++c) {
            const int rs = (int)rank_lt(ms[c]);
            const bool is_s = dx[c] == mn;
            const int dst = is_s ? a + S + so + rs : p + s + ko + (lane - rs);
            // the first settled entry lands at a (a kept one lands there only
            // when no entry of the first chunk settles, and is not tagged)
            if (lane < nv[c]) ord[dst] = (uint16_t)x[c] | ((is_s && dst == a) ? kSegMark : (uint16_t)0u);
            const int sc = __popcll(ms[c]);
            so += sc;
            ko += nv[c] - sc;
        }
        if (d > 0) {
            const int dst = a + S + (s > K ? s : K);
#pragma unroll
            for (int c = 0; c < U; ++c) {
                const int j = 64 * c + lane;
                if (j < d) ord[dst + j] = (uint16_t)y[c];
            }
        }
        S += s;
        K += kk;
        if (p + 64 * U < end) wave_sync();   // the next chunk reads the block written here
    }
    return S;
}

// Start of the backward batch that ends at ord index hi: the batch holds up
// to `width` entries of one equal-distance segment, ending at hi.  e is the
// entry at hi - width + slot (slot = lane / G), or 0 below index 0; every
// lane of the wavefront takes part.
__device__ __forceinline__ int batch_start(int hi, int width, uint32_t e, int G) {
    const uint64_t mk = __ballot((e & kSegMark) != 0u);
    if (mk == 0ull) return hi - width;
    const int top = 63 - (int)__builtin_clzll(mk);   // highest lane holding a segment start
    return hi - width + top / G;
}

template <bool WEIGHTED, int G, typename ADJ, bool GB, typename DT>
__device__ void wave_source(const SweepParams &P, const ADJ *rp, const ADJ *adj, uint32_t shift, const BAcc &BA,
                            DT *dist, unsigned long long *sig, uint16_t *ord, uint32_t *ctr, int s, int dbg_slot,
                            int &comp_out, int &size_out, bool &ovf) {
    using DO = DistOps<DT>;
    const int n = P.n;
    const int lane = threadIdx.x & 63;
    const int sub = lane % G;
    constexpr int VPI = 64 / G;   // vertices per wave iteration
    const uint32_t nmask = (1u << shift) - 1u;

    for (int v = lane; v < n; v += 64) dist[v] = (DT)DO::unreached;
    wave_sync();
    if (lane == 0) {
        dist[s] = (DT)0u;
        sig[s] = 1ull;
        ord[0] = (uint16_t)s | kSegMark;
        *ctr = WEIGHTED ? 0u : 1u;
    }
    wave_sync();

    int f_lo = 0, ord_end = 1;
    uint32_t D = 0;
    uint32_t kmin = kInf;   // lane minimum over the fringe entries kept by the last partition
    // ------------------------------------------------------------ forward
    for (;;) {
        uint32_t lmin = kInf;  // lane minimum over successful relaxations
        for (int base = f_lo; base < ord_end; base += VPI) {
            const int idx = base + lane / G;
            const bool mine = idx < ord_end;
            int v = 0;
            uint32_t beg = 0, len = 0;
            if (mine) {
                v = ord[idx] & kVertexMask;
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
                    const uint32_t du = (uint32_t)dist[u];
                    if (du + w == D) {                       // u precedes v: pull sigma_u
                        const unsigned long long x = acc + sig[u];
                        ovf |= x < acc;
                        acc = x;
                    } else if (D + w < du) {                 // relax the edge v -> u
                        const uint32_t old = DO::fetch_min(dist, u, D + w);
                        if (old > D + w) lmin = (D + w) < lmin ? (D + w) : lmin;
                        found = old == DO::unreached;        // first discovery of u
                    }
                }
                const uint32_t pos = wave_append(ctr, found);
                if (found) {
                    // unit weights: the next level starts at ord_end
                    if (WEIGHTED) ord[ord_end + (int)pos] = (uint16_t)u;
                    else ord[pos] = (uint16_t)u | ((int)pos == ord_end ? kSegMark : (uint16_t)0u);
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
            const int settled = fringe_partition<1>(ord, dist, ord_end, fr, mn, kmin);
            if (lane == 0) *ctr = (uint32_t)(fr - settled);
            wave_sync();
            f_lo = ord_end;
            ord_end += settled;
            D = mn;
        }
    }

    // component of s: smallest reached index, and its size
    {
        uint32_t mn = (uint32_t)n;
        for (int k = lane; k < ord_end; k += 64) mn = min(mn, (uint32_t)(ord[k] & kVertexMask));
        comp_out = (int)wave_min_fast(mn);
        size_out = ord_end;
    }
    if (dbg_slot >= 0) {
        for (int v = lane; v < n; v += 64) {
            const uint32_t d = (uint32_t)dist[v];
            P.dbg_dist[(size_t)dbg_slot * n + v] = d == DO::unreached ? 0xFFFFFFFFu : d;
            P.dbg_sigma[(size_t)dbg_slot * n + v] = d == DO::unreached ? 0ull : sig[v];
            P.dbg_delta[(size_t)dbg_slot * n + v] = 0.0;
        }
        wave_sync();
    }

    // ------------------------------------------------------------ backward
    // batches of one segment each, from the deepest vertices up
    for (int hi = ord_end; hi > 0;) {
        const int idx = hi - VPI + lane / G;
        const uint32_t e = idx >= 0 ? (uint32_t)ord[idx] : 0u;
        const int lo = batch_start(hi, VPI, e, G);
        const bool mine = idx >= lo;
        double sum = 0.0;
        int v = 0;
        if (mine) {
            v = (int)(e & kVertexMask);
            const uint32_t dv = (uint32_t)dist[v];
            const uint32_t beg = rp[v], end = rp[v + 1];
            for (uint32_t j = beg + sub; j < end; j += G) {
                const uint32_t a = adj[j];
                const uint32_t u = a & nmask;
                const uint32_t w = WEIGHTED ? (a >> shift) : 1u;
                if ((uint32_t)dist[u] == dv + w) sum += as_f64(sig[u]);   // u succeeds v: c_u
            }
        }
        sum = group_sum_f64<G>(sum);
        if (mine && sub == 0) {
            const double sv = (double)sig[v];
            const double delta = sv * sum;
            sig[v] = as_u64((1.0 + delta) / sv);
            if (v != s) add_B(BA, v, delta);
            if (dbg_slot >= 0) P.dbg_delta[(size_t)dbg_slot * n + v] = delta;
        }
        wave_sync();
        hi = lo;
    }
}

// ---------------------------------------------------------------------------
// Lane-per-vertex variant of wave_source: a lane owns one vertex of the batch
// and walks its adjacency U slots at a time, issuing the U neighbour loads
// (and the U distance loads) back to back so that their LDS latencies
// overlap; the path count of the vertex accumulates in the lane itself.  The
// U appends of a block share one LDS atomic per wavefront.  A batch of at
// most 32 (16) vertices gives each vertex 2 (4) lanes, which take every
// second (fourth) slot: small segments, common near the source and at the
// far end, then finish in half (a quarter) of the blocks.
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
#pragma unroll
    for (int k = 0; k < U; ++k) {
        pos[k] = base + rank_lt(m[k]);
        base += (uint32_t)__popcll(m[k]);
    }
}

// With MASK the traversal stays inside the vertex set mask[v] != 0 (an induced
// subgraph): an edge into a vertex outside it is never relaxed, so such a
// vertex stays unreached and fails the predecessor and successor tests.
//
// With SG the path counts sig[] live in global memory (the workgroup's
// scratch, L2 mode): a slot loads sigma_u / c_u only when u is a predecessor /
// successor, instead of the branch-free load from the source's entry that the
// LDS array affords.  Every access to sig[] is by the owning wavefront, and
// steps are separated by wave_sync(), whose workgroup-scope fence orders the
// global stores of one step before the loads of the next.
//
// Reads past a vertex's slots: a lane reads slots sub + G t for t below the
// wavefront's rounded-up trip count, i.e. at most max-degree + G (U + 1)
// entries past its vertex's first slot.  Past the last vertex these land in
// the kAdjPad zero entries and then in what follows the adjacency (LDS, or
// the rest of the workgroup's scratch in the L2 mode, 16 n + 64 bytes or more);
// their neighbour is masked and their weight replaced by kNoEdge, so they are
// never used.
template <bool WEIGHTED, int U, typename ADJ, bool GB, typename DT, bool MASK = false, bool SG = false>
__device__ void wave_source_lane(const SweepParams &P, const ADJ *rp, const ADJ *adj, uint32_t shift,
                                 const BAcc &BA, DT *dist, unsigned long long *sig, uint16_t *ord, uint32_t *ctr, int s,
                                 int dbg_slot, int &comp_out, int &size_out, bool &ovf,
                                 const uint8_t *mask = nullptr) {
    using DO = DistOps<DT>;
    const int n = P.n;
    const int lane = threadIdx.x & 63;
    const uint32_t nmask = (1u << shift) - 1u;

    for (int v = lane; v < n; v += 64) dist[v] = (DT)DO::unreached;
    wave_sync();
    if (lane == 0) {
        dist[s] = (DT)0u;
        sig[s] = 1ull;
        if constexpr (!SG) sig[n] = 0ull;
        ord[0] = (uint16_t)s | kSegMark;
        *ctr = WEIGHTED ? 0u : 1u;
    }
    wave_sync();

    int f_lo = 0, ord_end = 1;
    uint32_t D = 0;
    uint32_t kmin = kInf;
    uint32_t lmin = kInf;
    const uint32_t zero = (uint32_t)n;   // sig[n] == 0

    // relaxations out of the batch ord[base, min(base + 64 / G, ord_end))
    auto relax_batch = [&](auto gtag, int base) {
        constexpr int G = decltype(gtag)::value;
        const int sub = G == 1 ? 0 : lane % G;
        const int idx = base + lane / G;
        const bool mine = idx < ord_end;
        int v = 0;
        uint32_t beg = 0, len = 0;
        if (mine) {
            v = ord[idx] & kVertexMask;
            beg = ld_off32(rp, (uint32_t)v);
            len = ld_off32(rp, (uint32_t)v + 1u) - beg;
        }
        const uint32_t trips = G == 1 ? len : (len > (uint32_t)sub ? (len - (uint32_t)sub + G - 1) / G : 0u);
        const uint32_t maxtrips = wave_max_fast(trips);
        const uint32_t first = beg + (uint32_t)sub;
        unsigned long long acc = 0ull;
        // the L2 mode loads the next block of U slots while the current one
        // is used (global latency); LDS loads are issued in place
        uint32_t nxt[U];
        if constexpr (GB) {
#pragma unroll
            for (int k = 0; k < U; ++k) nxt[k] = (uint32_t)ld_off32(adj, first + G * k);
        }
        for (uint32_t off = 0; off < maxtrips; off += U) {
            uint32_t u[U], w[U], du[U], wd[U], cur[U];
            bool found[U];
            if constexpr (GB) {
#pragma unroll
                for (int k = 0; k < U; ++k) cur[k] = nxt[k];
                if (off + U < maxtrips) {
#pragma unroll
                    for (int k = 0; k < U; ++k) nxt[k] = (uint32_t)ld_off32(adj, first + G * (off + U + k));
                }
            } else {
#pragma unroll
                for (int k = 0; k < U; ++k) cur[k] = (uint32_t)ld_off32(adj, first + G * (off + k));
            }
            // a slot past the vertex's adjacency gets weight kNoEdge, which
            // fails both tests below (du + kNoEdge > D, D + kNoEdge > du)
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const uint32_t a = cur[k];
                u[k] = a & nmask;
                w[k] = (off + k < trips) ? (WEIGHTED ? (a >> shift) : 1u) : kNoEdge;
            }
#pragma unroll
            for (int k = 0; k < U; ++k) wd[k] = DO::word(dist, u[k]);
#pragma unroll
            for (int k = 0; k < U; ++k) du[k] = DO::value(wd[k], u[k]);
            bool pred[U], rel[U];
            unsigned long long sg[U];
            uint32_t old[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                pred[k] = du[k] + w[k] == D;                        // u precedes v: pull sigma_u
                rel[k] = D + w[k] < du[k];                          // relax the edge v -> u
                if constexpr (MASK) rel[k] = rel[k] && mask[u[k]] != 0;
            }
            if constexpr (SG) {
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    sg[k] = 0ull;
                    if (pred[k]) sg[k] = sig[u[k]];
                }
            } else {
#pragma unroll
                for (int k = 0; k < U; ++k) sg[k] = sig[pred[k] ? u[k] : zero];   // no branch: 0 unless u precedes v
            }
#pragma unroll
            for (int k = 0; k < U; ++k) old[k] = rel[k] ? DO::issue_min(dist, u[k], D + w[k], wd[k]) : 0u;
#pragma unroll
            for (int k = 0; k < U; ++k)
                if (rel[k]) old[k] = DO::resolve(dist, u[k], D + w[k], wd[k], old[k]);
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const unsigned long long x = acc + sg[k];
                ovf |= x < acc;
                acc = x;
                // a lane that does not relax keeps old = 0, which fails both
                // tests (written as selects, so no branch per slot)
                const uint32_t dw = D + w[k];
                const uint32_t cand = old[k] > dw ? dw : kInf;
                lmin = cand < lmin ? cand : lmin;
                found[k] = old[k] == DO::unreached;                 // first discovery of u
            }
            uint32_t pos[U];
            append_block<U>(ctr, found, pos);
#pragma unroll
            for (int k = 0; k < U; ++k)
                if (found[k]) {
                    // unit weights: the next level starts at ord_end
                    if (WEIGHTED) ord[ord_end + (int)pos[k]] = (uint16_t)u[k];
                    else ord[pos[k]] = (uint16_t)u[k] | ((int)pos[k] == ord_end ? kSegMark : (uint16_t)0u);
                }
        }
        if constexpr (G > 1) acc = group_sum_u64<G>(acc, ovf);
        if (mine && sub == 0 && v != s) sig[v] = acc;
    };

    // ------------------------------------------------------------ forward
    for (;;) {
        lmin = kInf;
        for (int base = f_lo; base < ord_end; base += 64) {
            const int k = ord_end - base;
            if (k > 32) relax_batch(std::integral_constant<int, 1>{}, base);
            else if (k > 16) relax_batch(std::integral_constant<int, 2>{}, base);
            else relax_batch(std::integral_constant<int, 4>{}, base);
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
            // chunks of 64, 128 or 64 U entries, by the fringe's length
            int settled;
            if (fr <= 64 || U == 1) settled = fringe_partition<1>(ord, dist, ord_end, fr, mn, kmin);
            else if (fr <= 128 || U == 2) settled = fringe_partition<2>(ord, dist, ord_end, fr, mn, kmin);
            else settled = fringe_partition<U>(ord, dist, ord_end, fr, mn, kmin);
            if (lane == 0) *ctr = (uint32_t)(fr - settled);
            wave_sync();
            f_lo = ord_end;
            ord_end += settled;
            D = mn;
        }
    }

    {
        uint32_t mn = (uint32_t)n;
        for (int k = lane; k < ord_end; k += 64) mn = min(mn, (uint32_t)(ord[k] & kVertexMask));
        comp_out = (int)wave_min_fast(mn);
        size_out = ord_end;
    }
    if (dbg_slot >= 0) {
        for (int v = lane; v < n; v += 64) {
            const uint32_t d = (uint32_t)dist[v];
            P.dbg_dist[(size_t)dbg_slot * n + v] = d == DO::unreached ? 0xFFFFFFFFu : d;
            P.dbg_sigma[(size_t)dbg_slot * n + v] = d == DO::unreached ? 0ull : sig[v];
            P.dbg_delta[(size_t)dbg_slot * n + v] = 0.0;
        }
        wave_sync();
    }

    // dependencies of the batch ord[lo, hi) (one equal-distance segment, k =
    // hi - lo vertices); e0 is ord[hi - 64 + lane] and, in the L2 mode, b0 /
    // l0 the row offset and length of its vertex (loaded one batch ahead)
    auto accumulate_batch = [&](auto gtag, int lo, int hi, uint32_t e0, uint32_t b0, uint32_t l0) {
        constexpr int G = decltype(gtag)::value;
        const int sub = G == 1 ? 0 : lane % G;
        bool mine;
        uint32_t e, eb = b0, el = l0;
        if constexpr (G == 1) {
            mine = hi - 64 + lane >= lo;
            e = e0;
        } else {
            const int slot = lane / G, k = hi - lo;
            mine = slot < k;
            const int src = mine ? 64 - k + slot : 63;
            e = (uint32_t)__shfl((int)e0, src, 64);
            if constexpr (GB) {
                eb = (uint32_t)__shfl((int)b0, src, 64);
                el = (uint32_t)__shfl((int)l0, src, 64);
            }
        }
        int v = 0;
        uint32_t beg = 0, len = 0, dv = 0;
        if (mine) {
            v = (int)(e & kVertexMask);
            if constexpr (GB) {
                beg = eb;
                len = el;
            } else {
                beg = ld_off32(rp, (uint32_t)v);
                len = ld_off32(rp, (uint32_t)v + 1u) - beg;
            }
            dv = (uint32_t)dist[v];
        }
        const uint32_t trips = G == 1 ? len : (len > (uint32_t)sub ? (len - (uint32_t)sub + G - 1) / G : 0u);
        const uint32_t first = beg + (uint32_t)sub;
        double sum = 0.0;
        uint32_t nxt[U];
        if constexpr (GB) {
#pragma unroll
            for (int k = 0; k < U; ++k) nxt[k] = (uint32_t)ld_off32(adj, first + G * k);
        }
        for (uint32_t off = 0; off < trips; off += U) {
            uint32_t u[U], w[U], du[U], cur[U];
            if constexpr (GB) {
#pragma unroll
                for (int k = 0; k < U; ++k) cur[k] = nxt[k];
                if (off + U < trips) {
#pragma unroll
                    for (int k = 0; k < U; ++k) nxt[k] = (uint32_t)ld_off32(adj, first + G * (off + U + k));
                }
            } else {
#pragma unroll
                for (int k = 0; k < U; ++k) cur[k] = (uint32_t)ld_off32(adj, first + G * (off + k));
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const uint32_t a = cur[k];
                u[k] = a & nmask;
                w[k] = (off + k < trips) ? (WEIGHTED ? (a >> shift) : 1u) : kNoEdge;
            }
#pragma unroll
            for (int k = 0; k < U; ++k) du[k] = (uint32_t)dist[u[k]];
            double cu[U];
            if constexpr (SG) {
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    cu[k] = 0.0;
                    if (du[k] == dv + w[k]) cu[k] = as_f64(sig[u[k]]);
                }
            } else {
#pragma unroll
                for (int k = 0; k < U; ++k) cu[k] = as_f64(sig[du[k] == dv + w[k] ? u[k] : zero]);   // 0.0 unless u succeeds v
            }
#pragma unroll
            for (int k = 0; k < U; ++k) sum += cu[k];                       // u succeeds v: c_u
        }
        if constexpr (G > 1) sum = group_sum_f64<G>(sum);
        if (mine && sub == 0) {
            const double sv = (double)sig[v];
            const double delta = sv * sum;
            sig[v] = as_u64((1.0 + delta) / sv);
            if (v != s) add_B(BA, v, delta);
            if (dbg_slot >= 0) P.dbg_delta[(size_t)dbg_slot * n + v] = delta;
        }
    };

    // ------------------------------------------------------------ backward
    // batches of one segment each, from the deepest vertices up.  The L2
    // mode loads the row offsets of the entries below the batch (the next
    // batch's candidates) before working on the batch, so that their global
    // latency overlaps it.
    uint32_t e_nx = 0, b_nx = 0, l_nx = 0;
    auto prefetch = [&](int hi) {
        const int idx = hi - 64 + lane;
        e_nx = idx >= 0 ? (uint32_t)ord[idx] : 0u;
        if constexpr (GB) {
            const uint32_t x = e_nx & kVertexMask;
            b_nx = ld_off32(rp, x);
            l_nx = ld_off32(rp, x + 1u) - b_nx;
        }
    };
    prefetch(ord_end);
    for (int hi = ord_end; hi > 0;) {
        const uint32_t e0 = e_nx, b0 = b_nx, l0 = l_nx;
        const int lo = batch_start(hi, 64, e0, 1);
        prefetch(lo);
        const int k = hi - lo;
        if (k > 32) accumulate_batch(std::integral_constant<int, 1>{}, lo, hi, e0, b0, l0);
        else if (k > 16) accumulate_batch(std::integral_constant<int, 2>{}, lo, hi, e0, b0, l0);
        else accumulate_batch(std::integral_constant<int, 4>{}, lo, hi, e0, b0, l0);
        wave_sync();
        hi = lo;
    }
}

// One source with the vertex mapping G: 1 / 2 / 3 = lane per vertex with 4 /
// 2 / 8 adjacency slots in flight, otherwise G lanes per vertex.  SG (path
// counts in global memory) exists for the lane-per-vertex mappings only.
template <bool WEIGHTED, int G, typename ADJ, bool GB, typename DT, bool SG = false>
__device__ __forceinline__ void run_source(const SweepParams &P, const ADJ *rp, const ADJ *adj, uint32_t shift,
                                           const BAcc &BA, DT *dist, unsigned long long *sig, uint16_t *ord,
                                           uint32_t *ctr, int s, int dbg_slot, int &comp_out, int &size_out,
                                           bool &ovf) {
    static_assert(!SG || G == 1 || G == 2 || G == 3, "path counts in global memory need a lane per vertex");
    if constexpr (G == 1 || G == 2 || G == 3)
        wave_source_lane<WEIGHTED, (G == 1 ? 4 : (G == 2 ? 2 : 8)), ADJ, GB, DT, false, SG>(
            P, rp, adj, shift, BA, dist, sig, ord, ctr, s, dbg_slot, comp_out, size_out, ovf);
    else
        wave_source<WEIGHTED, G, ADJ, GB, DT>(P, rp, adj, shift, BA, dist, sig, ord, ctr, s, dbg_slot, comp_out,
                                              size_out, ovf);
}

// Per-wavefront region of the sweep and trajectory kernels: dist DT[n] |
// sig u64[n + 1] | ord u16[n] (sig[n] stays 0: the slot a path-count load
// reads for a neighbour that is not a predecessor / successor); with the
// path counts in global memory (sg) just dist DT[n] | ord u16[n].
__host__ __device__ inline uint32_t wave_sig_offset(int n, bool dist16) {
    return ((dist16 ? 2u : 4u) * (uint32_t)n + 7u) & ~7u;
}
__host__ __device__ inline uint32_t wave_ord_offset(int n, bool dist16) {
    return wave_sig_offset(n, dist16) + 8u * ((uint32_t)n + 1u);
}
__host__ __device__ inline uint32_t wave_private_bytes(int n, bool dist16, bool sg = false) {
    return ((sg ? wave_sig_offset(n, dist16) : wave_ord_offset(n, dist16)) + 2u * (uint32_t)n + 15u) & ~15u;
}
// Bytes of one wavefront's path-count array in the workgroup's global scratch.
__host__ __device__ inline uint32_t l2_sig_stride(int n) { return (8u * (uint32_t)n + 255u) & ~255u; }

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

// L2 mode: the realized graph and the component labels of one workgroup live
// in its global scratch (small enough to stay in L2), and so does B(H_r) when
// the plan puts it there; otherwise the LDS holds B (l2_lds_b_bytes) before
// the wavefronts' private regions.  The 8 n + 64 bytes past the labels bound
// the adjacency reads past its padding (wave_source_lane).  With the path
// counts in global memory, wavefront w's array starts at total + w
// l2_sig_stride(n).
struct L2Layout {
    uint32_t rp, adj, comp, csize, B, total;
};
__host__ __device__ inline L2Layout l2_layout(int n, uint32_t adj_cap, uint32_t adj_bytes) {
    L2Layout L;
    const uint32_t un = (uint32_t)n;
    L.rp = 0;
    L.adj = (adj_bytes * (un + 1u) + 3u) & ~3u;
    L.comp = (L.adj + adj_bytes * adj_cap + 3u) & ~3u;
    L.csize = L.comp + 4u * un;
    L.B = (L.csize + 4u * un + 7u) & ~7u;
    L.total = (L.B + 8u * un + 64u + 255u) & ~255u;
    return L;
}
__host__ __device__ inline uint32_t l2_lds_b_bytes(int n) { return (8u * (uint32_t)n + 15u) & ~15u; }

}  // namespace amc
