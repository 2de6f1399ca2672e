// traj.hip -- trajectory simulator of the network process (Section 4.3).
//
// Paper: Bao, Kontou, Vogiatzis, "Betweenness-Central Nodes Under
// Uncertainty: An Absorbing Markov Chain Approach".
//
// A persistent kernel whose work items are episodes.  One workgroup runs an
// episode to absorption: at step t the anchor X_t draws its stop coin and a
// fresh network state (counters (e, X_t, 2^32-1, 2 + t) and (e, u, v, 2 + t)),
// the realized graph is staged in LDS, wavefront 0 runs the source X_t (which
// also yields the component K(X_t;H)), and when |K| >= k_min every wavefront
// takes further sources of K; the band maximiser of B over K is X_{t+1}.
// Visits, lengths, node rewards and switches feed the length-biased
// estimators of the uniform-step equivalence.  Placement PL: 0 stages the
// realized graph in LDS; 1 and 2 keep it in a per-workgroup global scratch
// (L2-resident, as in the sweep's L2 mode), which leaves room for more
// wavefronts, with B(H) in LDS (1) or in that scratch as well (2).  In the L2
// placements a step's sources after X_t are shared: the owner publishes the
// step (epoch, |K|) in a claim word, its wavefronts and those of workgroups
// that have run out of episodes claim sources from it by atomic adds (a
// claim is the add's old value: step and source), the latter read the
// owner's realized graph from its scratch and add their B(H) terms into a
// per-owner global array that the owner merges before the maximiser.  The
// owner waits only for claimed sources, so every wait ends without any
// assumption on which workgroups are resident.
#include <type_traits>

#include "amc_dev.hpp"
#include "amc_kernels.hpp"
#include "sweep_common.hpp"
#include "wave_source.hpp"

namespace amc {

// Polls of the owner's wait for claimed sources (about 4 s at 2.4 GHz) after
// which the step is abandoned with error bit 2: claimed sources always end,
// so reaching it means the completion word was not seen.
constexpr uint32_t kShareSpinLimit = 1u << 26;

// LDS bytes before the wavefront regions in the L2 placements: B (unless it
// is global) and the component list u16[n]
__host__ __device__ inline uint32_t traj_l2_base(int n, bool b_global) {
    return ((b_global ? 0u : l2_lds_b_bytes(n)) + 2u * (uint32_t)n + 15u) & ~15u;
}

template <bool WEIGHTED, int G, typename ADJ, bool D16, int PL>
__global__ __launch_bounds__(G == 3 ? 512 : 1024) void traj_kernel(TrajArgs T) {
    using DT = typename std::conditional<D16, uint16_t, uint32_t>::type;
    constexpr bool GL = PL != 0, BG = PL == 2;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __shared__ uint32_t scan_tmp[kMaxWaves];
    __shared__ uint32_t wctr[kMaxWaves];
    __shared__ double red_f[kMaxWaves];
    __shared__ int red_i[kMaxWaves];
    __shared__ int ep_sh, size_sh, nx_sh, helped_sh;

    const SweepParams &P = *T.desc;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6, nt = blockDim.x;
    const int n = P.n;
    ADJ *rp, *adj;
    double *B;
    uint16_t *list;                                      // K(X_t;H), in wavefront 0's visit order
    unsigned char *wbase;
    if constexpr (GL) {
        const L2Layout L = l2_layout(n, P.adj_cap, (uint32_t)sizeof(ADJ));
        unsigned char *gs = (unsigned char *)(T.bscratch + (size_t)blockIdx.x * T.bscratch_words);
        rp = to_global((ADJ *)(gs + L.rp));
        adj = to_global((ADJ *)(gs + L.adj));
        B = BG ? to_global((double *)(gs + L.B)) : (double *)smem;
        list = (uint16_t *)(smem + (BG ? 0u : l2_lds_b_bytes(n)));
        wbase = smem + traj_l2_base(n, BG);
    } else {
        const WaveLayout L = wave_layout(n, P.adj_cap, (uint32_t)sizeof(ADJ));
        rp = (ADJ *)(smem + L.rp);
        adj = (ADJ *)(smem + L.adj);
        B = (double *)(smem + L.B);
        list = (uint16_t *)(smem + L.comp);
        wbase = smem + L.waves;
    }
    // with B in global memory the wavefronts add with device atomics (at L2)
    // and the maximiser reads past the vector L1
    const BAcc BA{BG ? nullptr : B, BG ? B : nullptr, BG};
    unsigned char *wmine = wbase + wave * P.wave_bytes;
    const uint32_t sig_off = wave_sig_offset(n, D16);
    DT *dist = (DT *)wmine;
    unsigned long long *sig = (unsigned long long *)(wmine + sig_off);
    uint16_t *ord = (uint16_t *)(wmine + wave_ord_offset(n, D16));

    bool ovf = false;
    double rew = 0.0;
    unsigned long long sw = 0, tot = 0, trunc = 0, units = 0, shared = 0;
    uint32_t epoch = 1;                                  // this workgroup's next published step
    for (;;) {
        if (tid == 0) ep_sh = (int)atomicAdd(T.work, 1u);
        __syncthreads();
        const int e = ep_sh;
        __syncthreads();
        if (e >= T.episodes) break;
        int x = T.x0[e];
        int t = 0;
        for (;;) {
            if (tid == 0) {                                  // X_t is a pre-absorption state
                atomicAdd(&T.visits[x], 1ull);
                if (T.f) rew += T.f[x];
                if (T.paths) T.paths[(size_t)e * T.max_steps + t] = x;
            }
            ++t;
            const uint32_t stream = 2u + (uint32_t)(t - 1);
            const u32x4 c = philox10({(uint32_t)e, (uint32_t)x, 0xFFFFFFFFu, stream}, P.key0, P.key1);
            int nx = -1;
            if ((uint64_t)c.x >= P.t_alpha) {                // no stop: a fresh network state
                stage_realization(P, (uint32_t)e, rp, adj, P.shift, (uint16_t *)wbase, scan_tmp, stream);
                for (int v = tid; v < n; v += nt) {
                    if constexpr (BG) st_global(&B[v], 0.0);
                    else B[v] = 0.0;
                }
                // L2 placements: the realized graph (and a global B) are
                // complete at L2 before any wavefront reads them or adds into B
                if constexpr (GL) __threadfence();
                __syncthreads();
                if (wave == 0) {
                    int cs = 0, sz = 0;
                    run_source<WEIGHTED, G, ADJ, GL, DT>(P, rp, adj, P.shift, BA, dist, sig, ord, &wctr[0], x, -1, cs,
                                                         sz, ovf);
                    for (int k = lane; k < sz; k += 64) {
                        const uint16_t v = ord[k] & kVertexMask;
                        list[k] = v;
                        if constexpr (GL) T.glist[(size_t)blockIdx.x * n + k] = (int32_t)v;
                    }
                    if (lane == 0) size_sh = sz;
                }
                if constexpr (GL) __threadfence();               // K(X_t;H) in memory before the step opens
                __syncthreads();
                const int sz = size_sh;
                if ((uint32_t)sz >= P.k_min) {
                    if constexpr (GL) {
                        unsigned long long *claim = T.share + 2 * blockIdx.x, *done = claim + 1;
                        unsigned long long *open_w = T.open + (blockIdx.x >> 6);
                        const unsigned long long open_bit = 1ull << (blockIdx.x & 63u);
                        if (tid == 0) {
                            __hip_atomic_store(done, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            __threadfence();                 // graph, K and cleared sums before the claims open
                            __hip_atomic_store(claim,
                                               ((unsigned long long)epoch << 32) |
                                                   ((unsigned long long)sz << 16) | 1ull,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            if (sz > 1) atomicOr(open_w, open_bit);   // a hint for the helpers
                        }
                        __syncthreads();
                        // the next claim is issued before a source runs, so its
                        // latency hides behind the source's first loads
                        auto claim_k = [&]() -> unsigned int {
                            unsigned int v = 0;
                            if (lane == 0) v = (unsigned int)(atomicAdd(claim, 1ull) & 0xFFFFull);
                            return v;
                        };
                        unsigned int k = __builtin_amdgcn_readfirstlane(claim_k());
                        while (k < (unsigned int)sz) {
                            const unsigned int kn = claim_k();
                            int cs = 0, zz = 0;
                            run_source<WEIGHTED, G, ADJ, GL, DT>(P, rp, adj, P.shift, BA, dist, sig, ord,
                                                                 &wctr[wave], (int)list[k], -1, cs, zz, ovf);
                            if (lane == 0) atomicAdd(done, 1ull);
                            k = __builtin_amdgcn_readfirstlane(kn);
                        }
                        // every source is claimed: withdraw the hint (complete
                        // with the fence, before the next step sets it again)
                        if (lane == 0 && k == (unsigned int)sz) atomicAnd(open_w, ~open_bit);
                        __threadfence();                     // this workgroup's global B atomics are complete
                        __syncthreads();
                        if (tid == 0) {                      // sources other workgroups claimed
                            unsigned long long d;
                            uint32_t spins = 0;
                            while (((d = __hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) &
                                    0xFFFFFFFFull) < (unsigned long long)(sz - 1)) {
                                if (++spins == kShareSpinLimit) {
                                    atomicOr(T.err, 2);
                                    break;
                                }
                                __builtin_amdgcn_s_sleep(2);
                            }
                            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                            helped_sh = (int)(d >> 32);
                            shared += d >> 32;
                        }
                        __syncthreads();
                        if (helped_sh > 0) {
                            double *hb = T.hb + (size_t)blockIdx.x * n;
                            for (int v = tid; v < n; v += nt) {
                                const double h = ld_coh<true>(&hb[v]);
                                if (h != 0.0) {
                                    if constexpr (BG) st_global(&B[v], ld_coh<true>(&B[v]) + h);
                                    else B[v] += h;
                                    st_global(&hb[v], 0.0);
                                }
                            }
                            __threadfence();
                        }
                        ++epoch;
                    } else {
                        for (int k = 1 + wave; k < sz; k += nwaves) {
                            int cs = 0, zz = 0;
                            run_source<WEIGHTED, G, ADJ, GL, DT>(P, rp, adj, P.shift, BA, dist, sig, ord,
                                                                 &wctr[wave], (int)list[k], -1, cs, zz, ovf);
                        }
                    }
                    __syncthreads();
                    // tie-broken maximiser of B over K(X_t;H) (eq. local-center)
                    double mx = 0.0;
                    for (int k = tid; k < sz; k += nt) mx = fmax(mx, ld_coh<BG>(&B[list[k]]));
                    mx = wave_max_f64(mx);
                    if (lane == 0) red_f[wave] = mx;
                    __syncthreads();
                    mx = red_f[0];
                    for (int w = 1; w < nwaves; ++w) mx = fmax(mx, red_f[w]);
                    const double band = P.tau * (mx > 1.0 ? mx : 1.0);
                    int best = 0x7FFFFFFF;
                    for (int k = tid; k < sz; k += nt) {
                        const int v = list[k];
                        if (mx - ld_coh<BG>(&B[v]) <= band && v < best) best = v;
                    }
                    best = wave_min_i32(best);
                    if (lane == 0) red_i[wave] = best;
                    __syncthreads();
                    if (tid == 0) {
                        int b = red_i[0];
                        for (int w = 1; w < nwaves; ++w) b = min(b, red_i[w]);
                        nx_sh = b;
                    }
                    __syncthreads();
                    nx = nx_sh;
                    units += (unsigned long long)sz;
                } else {
                    units += 1ull;
                }
            }
            if (tid == 0 && nx >= 0 && nx != x) sw += 1;
            if (nx < 0) break;
            if (t == T.max_steps) {
                trunc += 1;
                break;
            }
            x = nx;
        }
        if (tid == 0) {
            T.lengths[e] = t;
            tot += (unsigned long long)t;
        }
        if (T.paths)
            for (int k = t + tid; k < T.max_steps; k += nt) T.paths[(size_t)e * T.max_steps + k] = -1;
        if (tid == 0) atomicAdd(&T.work[1], 1u);
        __syncthreads();
    }
    if constexpr (GL) {
        // out of episodes: every wavefront runs sources of other workgroups'
        // open steps until all episodes have ended
        const int nb = (int)gridDim.x;
        const L2Layout L = l2_layout(n, P.adj_cap, (uint32_t)sizeof(ADJ));
        const int nwords = (nb + 63) >> 6;
        int start = (int)((blockIdx.x * 7u + (uint32_t)wave * 131u) % (uint32_t)nb);
        int idle = 0;
        int last_b = -1;
        unsigned int last_ep = 0;
        for (;;) {
            unsigned int ended = 0;
            if (lane == 0) ended = __hip_atomic_load(&T.work[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__builtin_amdgcn_readfirstlane(ended) >= (unsigned int)T.episodes) break;
            // an owner with unclaimed sources, from the hint words: the first
            // set bit at or after `start`, else the first set bit
            int found = -1;
            for (int j = 0; j < nwords && found < 0; j += 64) {
                unsigned long long w = 0;
                if (j + lane < nwords)
                    w = __hip_atomic_load(T.open + j + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const int base = (j + lane) << 6;
                int after = 0x7FFFFFFF, first = 0x7FFFFFFF;
                if (w) {
                    first = base + (int)__builtin_ctzll(w);
                    const int sh = start - base;
                    const unsigned long long hi = sh <= 0 ? w : (sh >= 64 ? 0ull : (w >> sh) << sh);
                    if (hi) after = base + (int)__builtin_ctzll(hi);
                }
                after = wave_min_i32(after);
                first = wave_min_i32(first);
                if (after != 0x7FFFFFFF) found = after;
                else if (first != 0x7FFFFFFF) found = first;
            }
            if (found < 0 || found >= nb) {
                if (idle < 8) ++idle;
                for (int z = 0; z < idle; ++z) __builtin_amdgcn_s_sleep(16);   // back off while nothing is open
                continue;
            }
            idle = 0;
            unsigned long long *claim = T.share + 2 * found;
            unsigned int got = 0, kk = 0, ep_w = 0;
            if (lane == 0) {
                // a plain add after a check: the old value names the step and
                // the source this wavefront now owns (a later step of the same
                // owner is as good); an add that lands past |K| is lost, at
                // most one per wavefront and step, so `next` stays below 2^16
                const unsigned long long w = __hip_atomic_load(claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((w & 0xFFFFull) < ((w >> 16) & 0xFFFFull)) {
                    const unsigned long long old = atomicAdd(claim, 1ull);
                    if ((old & 0xFFFFull) < ((old >> 16) & 0xFFFFull)) {
                        got = 1;
                        kk = (unsigned int)(old & 0xFFFFull);
                        ep_w = (unsigned int)(old >> 32);
                    }
                }
            }
            const bool ok = __builtin_amdgcn_readfirstlane(got) != 0;
            start = ok ? found : (found + 1) % nb;           // an exhausted step: look past it
            if (!ok) continue;
            const int k = (int)__builtin_amdgcn_readfirstlane(kk);
            const unsigned int ep = __builtin_amdgcn_readfirstlane(ep_w);
            if (found != last_b || ep != last_ep) {          // first source of this step: see its graph and K
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                last_b = found;
                last_ep = ep;
            }
            const int s = (int)ld_coh<true>(&T.glist[(size_t)found * n + k]);
            unsigned char *gs = (unsigned char *)(T.bscratch + (size_t)found * T.bscratch_words);
            const ADJ *orp = to_global((ADJ *)(gs + L.rp));
            const ADJ *oadj = to_global((ADJ *)(gs + L.adj));
            const BAcc HB{nullptr, T.hb + (size_t)found * n, true};
            int cs = 0, zz = 0;
            run_source<WEIGHTED, G, ADJ, GL, DT>(P, orp, oadj, P.shift, HB, dist, sig, ord, &wctr[wave], s, -1, cs,
                                                 zz, ovf);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (lane == 0) atomicAdd(claim + 1, (1ull << 32) | 1ull);
        }
    }
    const bool any_ovf = __ballot(ovf) != 0ull;
    if (lane == 0 && any_ovf) atomicOr(T.err, 1);
    if (tid == 0) {
        if (T.f) global_add_f64(T.reward, rew);
        atomicAdd(&T.ctr[0], sw);
        atomicAdd(&T.ctr[1], tot);
        atomicAdd(&T.ctr[2], trunc);
        atomicAdd(&T.ctr[3], units);
        if (shared) atomicAdd(&T.ctr[4], shared);
    }
}

// Length-biased estimators (Definition of the length-biased uniform step and
// its corollary): b_v = visits_v / sum T, w_t = #{e : T_e > t} / sum T.
__global__ void k_traj_hist(int episodes, const int32_t *lengths, uint32_t *hist) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < episodes) atomicAdd(&hist[lengths[e]], 1u);
}

__global__ void k_traj_estimates(int n, int max_steps, const unsigned long long *visits,
                                 const unsigned long long *ctr, const uint32_t *hist, double *b_hat,
                                 double *survival) {
    const double tot = (double)ctr[1];
    for (int v = threadIdx.x; v < n; v += blockDim.x) b_hat[v] = tot > 0.0 ? (double)visits[v] / tot : 0.0;
    if (threadIdx.x == 0) {
        // #{T_e > t} by a suffix sum of the length histogram (lengths <= max_steps)
        unsigned long long above = 0;
        for (int t = max_steps; t >= 1; --t) {
            above += hist[t];
            survival[t - 1] = tot > 0.0 ? (double)above / tot : 0.0;
        }
    }
}

// ---------------------------------------------------------------------------
uint32_t traj_l2_lds_base(int n, bool b_global) { return traj_l2_base(n, b_global); }

template <bool W, int G, typename ADJ, bool D16, int PL>
static hipError_t launch_tt(const TrajArgs &T, int blocks, int waves, uint32_t lds, hipStream_t st) {
    hipLaunchKernelGGL((traj_kernel<W, G, ADJ, D16, PL>), dim3(blocks), dim3(64 * waves), lds, st, T);
    return hipGetLastError();
}

template <bool W, typename ADJ, bool D16, int PL>
static hipError_t launch_l2(const TrajArgs &T, int group, int blocks, int waves, uint32_t lds, hipStream_t st) {
    switch (group) {
        case 1: return launch_tt<W, 1, ADJ, D16, PL>(T, blocks, waves, lds, st);
        case 2: return launch_tt<W, 2, ADJ, D16, PL>(T, blocks, waves, lds, st);
        case 3: return launch_tt<W, 3, ADJ, D16, PL>(T, blocks, waves, lds, st);
        default: return hipErrorInvalidValue;
    }
}

// the L2 placements exist for the lane-per-vertex mappings (1, 2, 3)
template <bool W, typename ADJ, bool D16>
static hipError_t launch_tg(const TrajArgs &T, int place, int group, int blocks, int waves, uint32_t lds,
                            hipStream_t st) {
    if (place == 1) return launch_l2<W, ADJ, D16, 1>(T, group, blocks, waves, lds, st);
    if (place == 2) return launch_l2<W, ADJ, D16, 2>(T, group, blocks, waves, lds, st);
    switch (group) {
        case 1: return launch_tt<W, 1, ADJ, D16, 0>(T, blocks, waves, lds, st);
        case 2: return launch_tt<W, 2, ADJ, D16, 0>(T, blocks, waves, lds, st);
        case 3: return launch_tt<W, 3, ADJ, D16, 0>(T, blocks, waves, lds, st);
        case 4: return launch_tt<W, 4, ADJ, D16, 0>(T, blocks, waves, lds, st);
        case 16: return launch_tt<W, 16, ADJ, D16, 0>(T, blocks, waves, lds, st);
        default: return launch_tt<W, 8, ADJ, D16, 0>(T, blocks, waves, lds, st);
    }
}

template <bool W, typename ADJ, bool D16>
static hipError_t attrs_t(int max_lds) {
    const void *ks[] = {(const void *)traj_kernel<W, 1, ADJ, D16, 0>, (const void *)traj_kernel<W, 2, ADJ, D16, 0>,
                        (const void *)traj_kernel<W, 3, ADJ, D16, 0>, (const void *)traj_kernel<W, 4, ADJ, D16, 0>,
                        (const void *)traj_kernel<W, 8, ADJ, D16, 0>, (const void *)traj_kernel<W, 16, ADJ, D16, 0>,
                        (const void *)traj_kernel<W, 1, ADJ, D16, 1>, (const void *)traj_kernel<W, 2, ADJ, D16, 1>,
                        (const void *)traj_kernel<W, 3, ADJ, D16, 1>, (const void *)traj_kernel<W, 1, ADJ, D16, 2>,
                        (const void *)traj_kernel<W, 2, ADJ, D16, 2>, (const void *)traj_kernel<W, 3, ADJ, D16, 2>};
    for (const void *k : ks) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <bool D16>
static hipError_t attrs_td(int max_lds) {
    hipError_t e;
    if ((e = attrs_t<true, uint16_t, D16>(max_lds)) != hipSuccess) return e;
    if ((e = attrs_t<false, uint16_t, D16>(max_lds)) != hipSuccess) return e;
    if ((e = attrs_t<true, uint32_t, D16>(max_lds)) != hipSuccess) return e;
    return attrs_t<false, uint32_t, D16>(max_lds);
}

hipError_t set_traj_attrs(int max_lds) {
    const hipError_t e = attrs_td<false>(max_lds);
    if (e != hipSuccess) return e;
    return attrs_td<true>(max_lds);
}

template <bool D16>
static hipError_t launch_td(const TrajArgs &T, bool weighted, int place, int group, uint32_t adj_bytes, int blocks,
                            int waves, uint32_t lds, hipStream_t st) {
    if (adj_bytes == 2)
        return weighted ? launch_tg<true, uint16_t, D16>(T, place, group, blocks, waves, lds, st)
                        : launch_tg<false, uint16_t, D16>(T, place, group, blocks, waves, lds, st);
    return weighted ? launch_tg<true, uint32_t, D16>(T, place, group, blocks, waves, lds, st)
                    : launch_tg<false, uint32_t, D16>(T, place, group, blocks, waves, lds, st);
}

hipError_t launch_traj(const TrajArgs &T, bool weighted, bool dist16, int place, int group, uint32_t adj_bytes,
                       int blocks, int waves, uint32_t lds, hipStream_t st) {
    return dist16 ? launch_td<true>(T, weighted, place, group, adj_bytes, blocks, waves, lds, st)
                  : launch_td<false>(T, weighted, place, group, adj_bytes, blocks, waves, lds, st);
}

hipError_t traj_estimates(int n, int episodes, int max_steps, const int32_t *lengths,
                          const unsigned long long *visits, const unsigned long long *ctr, uint32_t *hist,
                          double *b_hat, double *survival, hipStream_t st) {
    hipLaunchKernelGGL(k_traj_hist, dim3((episodes + 255) / 256), dim3(256), 0, st, episodes, lengths, hist);
    hipLaunchKernelGGL(k_traj_estimates, dim3(1), dim3(256), 0, st, n, max_steps, visits, ctr, hist, b_hat,
                       survival);
    return hipGetLastError();
}

}  // namespace amc
