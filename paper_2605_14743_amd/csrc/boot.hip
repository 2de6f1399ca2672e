// boot.hip -- nonparametric bootstrap of the AFC profile: resampled
// transition counts written straight into I - Q*, and per-node summaries of
// the replicates.
//
// Paper: Bao, Kontou, Vogiatzis, "Betweenness-Central Nodes Under
// Uncertainty: An Absorbing Markov Chain Approach" (Section 8.4: resample each
// row's M draws with replacement and recompute b; Section 8.2: the floor on a
// row that never absorbed).
//
// Draw t of row i in replicate beta is the index
//     j = (x * R) >> 32,  x = word (t mod 4) of Philox4x32-10 at counter
//     (beta, i, t / 4, 0x80000004) under the seed,
// and the replicate's count of row i goes to the outcome the original draw j
// of row i had.  The draws of one row are independent of every other row's,
// so a workgroup owns one (row, replicate) pair and counts in LDS.
#include "amc_dev.hpp"
#include "amc_kernels.hpp"

namespace amc {

constexpr uint32_t kBootStream = 0x80000004u;

// u32 words before the staged row in k_boot_rows' LDS (the counts, n + 1,
// rounded up to 16 bytes), and the largest LDS it stages within (the default
// dynamic LDS of a launch).
__host__ __device__ inline uint32_t boot_stage_offset(int n) { return ((uint32_t)n + 1u + 3u) & ~3u; }
constexpr size_t kBootStageMaxLds = 65536;

// next table R x n (int32, -1 = bottom) -> row-major n x R (uint16, next + 1,
// 0 = bottom), so that every row's R outcomes are contiguous.  32 x 32 tiles
// through LDS keep both sides coalesced.
__global__ void k_boot_transpose(int n, uint32_t R, const int32_t *nt, uint16_t *tr) {
    __shared__ uint16_t tile[32][33];
    const uint32_t t0 = blockIdx.x * 32u, i0 = blockIdx.y * 32u;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: 8 rows of 32
    for (int k = ty; k < 32; k += 8) {
        const uint32_t t = t0 + k, i = i0 + tx;
        if (t < R && i < (uint32_t)n) tile[k][tx] = (uint16_t)(nt[(size_t)t * n + i] + 1);
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const uint32_t i = i0 + k, t = t0 + tx;
        if (t < R && i < (uint32_t)n) tr[(size_t)i * R + t] = tile[tx][k];
    }
}

// Workgroup (i, z): counts of row i in replicate beta0 + z (or of the draws
// themselves when ident), then row i of A_z = I - Q* with the floor rule of the
// estimated kernel (a row that never absorbed gets P_i,bottom = eta and its
// transient part scaled by 1 - eta, when eta > 0).  STAGE: the row's R
// outcomes are first copied to LDS (coalesced), so that the random draws
// gather from LDS instead of touching a cache line per lane.
template <bool STAGE>
__global__ __launch_bounds__(256) void k_boot_rows(int n, uint32_t R, const uint16_t *tr, uint64_t seed,
                                                   uint32_t beta0, int ident, double eta, double *A,
                                                   size_t stride) {
    extern __shared__ uint32_t cnt[];   // n + 1 (index n = bottom), then (STAGE) the row's R outcomes
    const int i = blockIdx.x;
    const uint32_t beta = beta0 + blockIdx.y;
    A += (size_t)blockIdx.y * stride + (size_t)i * n;
    for (int j = threadIdx.x; j <= n; j += blockDim.x) cnt[j] = 0u;
    const uint16_t *row = tr + (size_t)i * R;
    if constexpr (STAGE) {
        uint16_t *lrow = (uint16_t *)(cnt + boot_stage_offset(n));
        for (uint32_t t = threadIdx.x; t < R; t += blockDim.x) lrow[t] = row[t];
        row = lrow;
    }
    __syncthreads();
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    if (ident) {
        for (uint32_t t = threadIdx.x; t < R; t += blockDim.x) {
            const uint32_t v = row[t];
            atomicAdd(&cnt[v ? v - 1u : (uint32_t)n], 1u);
        }
    } else {
        const uint32_t quads = (R + 3u) >> 2;
        for (uint32_t q = threadIdx.x; q < quads; q += blockDim.x) {
            const u32x4 x = philox10({beta, (uint32_t)i, q, kBootStream}, k0, k1);
            const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (4u * q + k < R) {
                    const uint32_t j = (uint32_t)(((uint64_t)w[k] * R) >> 32);
                    const uint32_t v = row[j];
                    atomicAdd(&cnt[v ? v - 1u : (uint32_t)n], 1u);
                }
            }
        }
    }
    __syncthreads();
    const bool fl = cnt[n] == 0u && eta > 0.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double q = (double)cnt[j] / (double)R;
        const double v = fl ? (1.0 - eta) * q : q;
        A[j] = (i == j ? 1.0 : 0.0) - v;
    }
}

// Per node v: mean, sample standard deviation (B - 1) and the order statistics
// klo, khi of the B replicate values b_rep[beta][v].  Values are sorted in LDS
// by a bitonic network over the next power of two (padding +inf).
__global__ __launch_bounds__(256) void k_boot_stats(int n, int B, const double *b_rep, int klo, int khi,
                                                    double *mean, double *sd, double *lo, double *hi) {
    extern __shared__ double vals[];    // P >= B, a power of two
    __shared__ double red[256];
    const int v = blockIdx.x, tid = threadIdx.x;
    int P = 1;
    while (P < B) P <<= 1;
    double acc = 0.0;
    for (int b = tid; b < P; b += blockDim.x) {
        const double x = b < B ? b_rep[(size_t)b * n + v] : INFINITY;
        vals[b] = x;
        if (b < B) acc += x;
    }
    red[tid] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    const double m = red[0] / (double)B;
    __syncthreads();
    acc = 0.0;
    for (int b = tid; b < B; b += blockDim.x) acc += (vals[b] - m) * (vals[b] - m);
    red[tid] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    const double ss = red[0];
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int a = tid; a < P; a += blockDim.x) {
                const int c = a ^ j;
                if (c > a) {
                    const double x = vals[a], y = vals[c];
                    const bool up = (a & k) == 0;
                    if (up ? x > y : x < y) {
                        vals[a] = y;
                        vals[c] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (tid == 0) {
        mean[v] = m;
        sd[v] = B > 1 ? sqrt(ss / (double)(B - 1)) : 0.0;
        lo[v] = vals[klo];
        hi[v] = vals[khi];
    }
}

hipError_t boot_transpose(int n, uint32_t R, const int32_t *nt, uint16_t *tr, hipStream_t st) {
    const dim3 grid((R + 31u) / 32u, (uint32_t)(n + 31) / 32u);
    hipLaunchKernelGGL(k_boot_transpose, grid, dim3(256), 0, st, n, R, nt, tr);
    return hipGetLastError();
}

hipError_t boot_rows(int n, uint32_t R, const uint16_t *tr, uint64_t seed, uint32_t beta0, int batch, bool ident,
                     double eta, double *A, size_t stride, hipStream_t st) {
    const size_t staged = 4 * (size_t)boot_stage_offset(n) + 2 * (size_t)R;
    if (!ident && staged <= kBootStageMaxLds)
        hipLaunchKernelGGL(k_boot_rows<true>, dim3(n, batch), dim3(256), staged, st, n, R, tr, seed, beta0, 0, eta, A,
                           stride);
    else
        hipLaunchKernelGGL(k_boot_rows<false>, dim3(n, batch), dim3(256), 4 * ((size_t)n + 1), st, n, R, tr, seed,
                           beta0, ident ? 1 : 0, eta, A, stride);
    return hipGetLastError();
}

size_t boot_stats_lds(int B) {
    size_t P = 1;
    while (P < (size_t)B) P <<= 1;
    return 8 * P;
}

hipError_t boot_stats(int n, int B, const double *b_rep, int klo, int khi, double *mean, double *sd, double *lo,
                      double *hi, hipStream_t st) {
    hipLaunchKernelGGL(k_boot_stats, dim3(n), dim3(256), boot_stats_lds(B), st, n, B, b_rep, klo, khi, mean, sd, lo,
                       hi);
    return hipGetLastError();
}

}  // namespace amc
