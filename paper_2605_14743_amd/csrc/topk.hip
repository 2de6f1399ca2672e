// topk.hip -- finite-k local Top-k stage and its tail pieces.
//
// Paper: Bao, Kontou, Vogiatzis, "Betweenness-Central Nodes Under
// Uncertainty: An Absorbing Markov Chain Approach" (Section 3.3, Sections
// 6.2-6.3, Section 7.1, Sections 7.3-7.4).
//
// The sweep leaves every realization's B(H_r) and component labels in HBM
// (R x n rows).  One workgroup per realization then ranks each component by
// applying the tie rule repeatedly (the band maximiser, then the band
// maximiser of the rest, ...) up to k vertices, and for every anchor i with a
// valid draw adds the gamma mass of C_k(i) (eq. realized-topk-set) and of
// C_k(i) ∩ W to the step-reward sums, and counts the finite-k pool selector
// (the highest-ranked pool member of C_k(i), bottom when there is none).
#include "amc_dev.hpp"
#include "amc_kernels.hpp"

namespace amc {

constexpr uint32_t kNone = 0xFFFFFFFFu;

// LDS carve-up for n vertices: [8n] per-component maximum (bit pattern) and
// later the gamma mass of the Top-k set | [8n] gamma mass of its pool part |
// [4n] per-component band minimum index, later the best-ranked pool member
// (rank << 16 | v) | [n] rank of each vertex (0 = not ranked yet).
__host__ __device__ inline uint32_t topk_lds_bytes(int n) {
    return (uint32_t)(8 * n + 8 * n + 4 * n + ((n + 15) & ~15));
}
// With ACC the workgroup also sums its realizations' step rewards per anchor
// in LDS ([8n] psi | [8n] psi_w after the carve-up above) and adds them to
// the global sums once at the end, instead of one global atomic per anchor
// and realization (R atomics on each of n addresses); used while the
// carve-up stays small enough for several workgroups per CU.
constexpr int kTopkAccMaxN = 4000;
__host__ __device__ inline uint32_t topk_acc_offset(int n) { return (topk_lds_bytes(n) + 15u) & ~15u; }
__host__ __device__ inline uint32_t topk_lds_total(int n) {
    return n <= kTopkAccMaxN ? topk_acc_offset(n) + 16u * (uint32_t)n : topk_lds_bytes(n);
}

// Anchors per thread whose selector counts are kept as runs in registers.
constexpr int kRunSlots = 4;

// GM: the carve-up lives in a per-workgroup global array instead of LDS
// (graphs whose arrays exceed the LDS); the workgroup alone reads and writes
// it, and a barrier orders its global accesses as it does its LDS ones.
template <bool ACC, bool GM>
__global__ __launch_bounds__(256) void k_topk_reduce(TopkArgs A) {
    static_assert(!(ACC && GM), "the LDS step-reward sums go with the LDS carve-up");
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_base[];
    unsigned char *smem = lds_base;
    if constexpr (GM) smem = (unsigned char *)to_global(A.gscr + (size_t)blockIdx.x * A.gscr_bytes);
    const int n = A.n, tid = threadIdx.x, nt = blockDim.x;
    double *lpsi = ACC ? (double *)(smem + topk_acc_offset(n)) : nullptr;
    double *lpsiw = ACC ? lpsi + n : nullptr;
    if constexpr (ACC) {
        for (int v = tid; v < n; v += nt) {
            lpsi[v] = 0.0;
            lpsiw[v] = 0.0;
        }
    }
    unsigned long long *cmax = (unsigned long long *)smem;
    double *gsum = (double *)smem;                        // aliases cmax after the ranking
    double *gsumw = (double *)(smem + 8 * (size_t)n);
    uint32_t *cband = (uint32_t *)(smem + 16 * (size_t)n);
    uint32_t *wsel = cband;                               // aliases cband after the ranking
    uint8_t *rank = smem + 20 * (size_t)n;

    // selector counts of the thread's first kRunSlots anchors, as runs of
    // equal selections over the workgroup's realizations (one atomic per run)
    uint32_t run_col[kRunSlots], run_len[kRunSlots];
#pragma unroll
    for (int q = 0; q < kRunSlots; ++q) {
        run_col[q] = 0u;
        run_len[q] = 0u;
    }
    for (uint32_t rl = blockIdx.x; rl < A.R; rl += gridDim.x) {
        const double *B = A.Bg + (size_t)rl * n;
        const int32_t *comp = A.compg + (size_t)rl * n;
        const int32_t *csize = A.sizeg + (size_t)rl * n;
        const uint32_t r = A.r_begin + rl;
        for (int v = tid; v < n; v += nt) rank[v] = 0;
        __syncthreads();
        for (int t = 1; t <= A.topk; ++t) {
            for (int v = tid; v < n; v += nt) {
                cmax[v] = 0ull;
                cband[v] = kNone;
            }
            __syncthreads();
            for (int v = tid; v < n; v += nt)
                if (!rank[v]) atomicMax(&cmax[comp[v]], as_u64(B[v]));   // B >= 0: bit order = value order
            __syncthreads();
            for (int v = tid; v < n; v += nt) {
                if (rank[v]) continue;
                const int c = comp[v];
                const double mx = as_f64(cmax[c]);
                const double band = A.tau * (mx > 1.0 ? mx : 1.0);
                if (mx - B[v] <= band) atomicMin(&cband[c], (uint32_t)v);
            }
            __syncthreads();
            int any = 0;
            for (int c = tid; c < n; c += nt)
                if (cband[c] != kNone) {
                    rank[cband[c]] = (uint8_t)t;
                    any = 1;
                }
            if (!__syncthreads_or(any)) break;   // every component fully ranked
        }
        for (int c = tid; c < n; c += nt) {
            gsum[c] = 0.0;
            gsumw[c] = 0.0;
            wsel[c] = kNone;
        }
        __syncthreads();
        for (int v = tid; v < n; v += nt) {
            if (!rank[v]) continue;
            const int c = comp[v];
            const double g = A.gamma ? A.gamma[v] : 1.0;
            atomicAdd(&gsum[c], g);
            if (A.pool && A.pool[v]) {
                atomicAdd(&gsumw[c], g);
                atomicMin(&wsel[c], ((uint32_t)rank[v] << 16) | (uint32_t)v);
            }
        }
        __syncthreads();
        // anchor i is always this thread's (a fixed stride over the anchors):
        // the LDS sums need no atomics, and the first kRunSlots anchors of
        // the thread keep their selector count as a run in registers
        auto anchor = [&](int i, uint32_t *run_col, uint32_t *run_len) {
            const int c = comp[i];
            const u32x4 x = philox10({r, (uint32_t)i, 0xFFFFFFFFu, 1u}, A.key0, A.key1);
            const bool coin = (uint64_t)x.x < A.t_alpha;
            const bool valid = !coin && (uint32_t)csize[i] >= A.k_min;
            if (valid) {
                if constexpr (ACC) {
                    lpsi[i] += gsum[c];
                    lpsiw[i] += gsumw[c];
                } else {
                    global_add_f64(&A.psi[i], gsum[c]);
                    if (A.psi_w) global_add_f64(&A.psi_w[i], gsumw[c]);
                }
            }
            if (A.counts_w) {
                const int nw = (valid && wsel[c] != kNone) ? (int)(wsel[c] & 0xFFFFu) : -1;
                const uint32_t col = nw >= 0 ? (uint32_t)nw : (uint32_t)n;
                if (run_col) {
                    if (*run_len > 0u && *run_col != col)
                        atomicAdd(&A.counts_w[(size_t)i * (n + 1) + *run_col], *run_len);
                    *run_len = *run_col == col ? *run_len + 1u : 1u;
                    *run_col = col;
                } else {
                    atomicAdd(&A.counts_w[(size_t)i * (n + 1) + col], 1u);
                }
                if (A.next_table_w) A.next_table_w[(size_t)rl * n + i] = nw;
            }
        };
#pragma unroll
        for (int q = 0; q < kRunSlots; ++q)
            if (tid + q * nt < n) anchor(tid + q * nt, &run_col[q], &run_len[q]);
        for (int i = tid + kRunSlots * nt; i < n; i += nt) anchor(i, nullptr, nullptr);
        __syncthreads();
    }
    if (A.counts_w) {
#pragma unroll
        for (int q = 0; q < kRunSlots; ++q) {
            const int i = tid + q * nt;
            if (i < n && run_len[q] > 0u) atomicAdd(&A.counts_w[(size_t)i * (n + 1) + run_col[q]], run_len[q]);
        }
    }
    if constexpr (ACC) {
        for (int i = tid; i < n; i += nt) {
            if (lpsi[i] != 0.0) global_add_f64(&A.psi[i], lpsi[i]);
            if (A.psi_w && lpsiw[i] != 0.0) global_add_f64(&A.psi_w[i], lpsiw[i]);
        }
    }
}

// y = x / d (the step-reward sums over R draws -> their averages).
__global__ void k_div(int n, const double *x, double d, double *y) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) y[j] = x[j] / d;
}

// Reward-AFC of a step reward (Proposition on reward-AFC):
// b_l = s N psi / s N 1 = mu . psi / E_s[T].
__global__ void k_reward_afc(int n, const double *mu, const double *scal, const double *psi, double *out) {
    __shared__ double red[256];
    const int tid = threadIdx.x;
    double acc = 0.0;
    for (int j = tid; j < n; j += blockDim.x) acc += mu[j] * psi[j];
    red[tid] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) *out = red[0] / scal[0];
}

// Counts of the fallback selector (Section 7.3): row i keeps the pool
// selections, moves its valid-but-empty draws (C^W_i,bottom - C_i,bottom) to
// v_fb and absorbs only the invalid draws (C_i,bottom).
__global__ void k_fb_counts(int n, const uint32_t *counts, const uint32_t *counts_w, int fb, uint32_t *cf) {
    const int i = blockIdx.x;
    const uint32_t *cw = counts_w + (size_t)i * (n + 1);
    uint32_t *row = cf + (size_t)i * (n + 1);
    for (int j = threadIdx.x; j < n; j += blockDim.x) row[j] = cw[j];
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t inval = counts[(size_t)i * (n + 1) + n];
        row[fb] += cw[n] - inval;
        row[n] = inval;
    }
}

// Censored profile (Section 7.4): c_fb = sum of b^{W,fb} off V_fb and
// b~_v = b^{W,fb}_v / c_fb off V_fb (0 on V_fb).
__global__ void k_censor(int n, const double *b, const uint8_t *fb_mask, double *b_cens, double *c_out) {
    __shared__ double red[256];
    const int tid = threadIdx.x;
    double acc = 0.0;
    for (int j = tid; j < n; j += blockDim.x)
        if (!fb_mask[j]) acc += b[j];
    red[tid] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    const double c = red[0];
    for (int j = tid; j < n; j += blockDim.x) b_cens[j] = (!fb_mask[j] && c > 0.0) ? b[j] / c : 0.0;
    if (tid == 0) *c_out = c;
}

// ---------------------------------------------------------------------------
hipError_t set_topk_attrs(int max_lds) {
    const void *ks[] = {(const void *)k_topk_reduce<true, false>, (const void *)k_topk_reduce<false, false>,
                        (const void *)k_topk_reduce<false, true>};
    for (const void *k : ks) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

uint32_t topk_lds(int n) { return topk_lds_total(n); }

uint64_t topk_global_bytes(int n) { return ((uint64_t)topk_lds_bytes(n) + 255u) & ~255ull; }

hipError_t launch_topk_reduce(const TopkArgs &A, int blocks, hipStream_t st) {
    if (A.gscr)
        hipLaunchKernelGGL((k_topk_reduce<false, true>), dim3(blocks), dim3(256), 0, st, A);
    else if (A.n <= kTopkAccMaxN)
        hipLaunchKernelGGL((k_topk_reduce<true, false>), dim3(blocks), dim3(256), topk_lds_total(A.n), st, A);
    else
        hipLaunchKernelGGL((k_topk_reduce<false, false>), dim3(blocks), dim3(256), topk_lds_total(A.n), st, A);
    return hipGetLastError();
}

hipError_t tail_div(int n, const double *x, double d, double *y, hipStream_t st) {
    hipLaunchKernelGGL(k_div, dim3((n + 255) / 256), dim3(256), 0, st, n, x, d, y);
    return hipGetLastError();
}

hipError_t tail_reward_afc(int n, const double *mu, const double *scal, const double *psi, double *out,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_reward_afc, dim3(1), dim3(256), 0, st, n, mu, scal, psi, out);
    return hipGetLastError();
}

hipError_t tail_fb_counts(int n, const uint32_t *counts, const uint32_t *counts_w, int fb, uint32_t *cf,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_fb_counts, dim3(n), dim3(256), 0, st, n, counts, counts_w, fb, cf);
    return hipGetLastError();
}

hipError_t tail_censor(int n, const double *b, const uint8_t *fb_mask, double *b_cens, double *c_out,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_censor, dim3(1), dim3(256), 0, st, n, b, fb_mask, b_cens, c_out);
    return hipGetLastError();
}

}  // namespace amc
