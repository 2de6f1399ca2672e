// robust.hip -- robust tail on a given transient block Q0 (Sections 5.1, 5.4,
// 6.4 and the robust experiment of Section 9.1), FP64 on the device.
//
// Paper: Bao, Kontou, Vogiatzis, "Betweenness-Central Nodes Under
// Uncertainty: An Absorbing Markov Chain Approach".
//
//  - sampled admissible kernels: Q_ij = clip(Q0_ij (1 + delta (2u - 1)), 0, 1)
//    with u the 53-bit fraction of the Philox block of counter (sample, i, j,
//    3), each row scaled to 1 - r_min when its sum exceeds that;
//  - KL(b(P) || b0) and total variation for each sample, and their maximisers;
//  - first-order sensitivity for E = Q* - Q0 (the KL maximiser): b_lin, the
//    infinity norms |N0 E|, |N0| and |N* - N0 - N0 E N0|;
//  - transition rewards: switching (j != i) and improvement ((f_j - f_i)_+).
// The multiplier is formed with explicitly rounded operations so that no
// fused multiply-add changes it.
#include "amc_dev.hpp"
#include "amc_kernels.hpp"

namespace amc {

__device__ __forceinline__ double u53(uint32_t a, uint32_t b, uint32_t c, uint32_t k0, uint32_t k1) {
    const u32x4 x = philox10({a, b, c, 3u}, k0, k1);
    const uint64_t bits = (((uint64_t)x.x) << 21) ^ (((uint64_t)x.y) >> 11);
    return (double)bits * (1.0 / 9007199254740992.0);
}

// One workgroup per row: the sampled row of Q and the row of A = I - Q.  The
// sample index is read from `sample_ptr` when given (the KL maximiser).
__global__ void k_perturb(int n, const double *Q0, uint32_t k0, uint32_t k1, int sample, const int *sample_ptr,
                          double delta, double r_min, double *Q, double *A, size_t stride) {
    // batch y: sample + y (or *sample_ptr) into A + y * stride; the rows of A
    // hold the clipped q first, then I - Q; Q (optional) gets Q itself
    __shared__ double red[256];
    const int i = blockIdx.x, tid = threadIdx.x;
    const uint32_t smp = (uint32_t)(sample_ptr ? *sample_ptr : sample + (int)blockIdx.y);
    A += (size_t)blockIdx.y * stride;
    double tot = 0.0;
    for (int j = tid; j < n; j += blockDim.x) {
        const double u = u53(smp, (uint32_t)i, (uint32_t)j, k0, k1);
        const double f = __dadd_rn(1.0, __dmul_rn(delta, __dadd_rn(__dmul_rn(2.0, u), -1.0)));
        double q = __dmul_rn(Q0[(size_t)i * n + j], f);
        q = q < 0.0 ? 0.0 : (q > 1.0 ? 1.0 : q);
        A[(size_t)i * n + j] = q;
        tot += q;
    }
    red[tid] = tot;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    const double cap = 1.0 - r_min;
    const double sc = red[0] > cap ? cap / red[0] : 1.0;
    for (int j = tid; j < n; j += blockDim.x) {
        const double q = red[0] > cap ? A[(size_t)i * n + j] * sc : A[(size_t)i * n + j];
        if (Q) Q[(size_t)i * n + j] = q;
        A[(size_t)i * n + j] = (i == j ? 1.0 : 0.0) - q;
    }
}
// one block per sampled profile x: b + x * n against b0 into kl[x], tv[x]
__global__ void k_divergence(int n, const double *b, const double *b0, double *kl, double *tv) {
    __shared__ double r1[256], r2[256];
    const int tid = threadIdx.x;
    b += (size_t)blockIdx.x * n;
    kl += blockIdx.x;
    tv += blockIdx.x;
    double a = 0.0, t = 0.0;
    for (int j = tid; j < n; j += blockDim.x) {
        if (b[j] > 0.0) a += b[j] * log(b[j] / b0[j]);
        t += fabs(b[j] - b0[j]);
    }
    r1[tid] = a;
    r2[tid] = t;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) {
            r1[tid] += r1[tid + s];
            r2[tid] += r2[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        *kl = r1[0];
        *tv = 0.5 * r2[0];
    }
}

// First index of the maximum of x[0..m) (single workgroup).

// b = mu / (mu 1) for the rows of a batch (one block per row)
__global__ void k_normalize_rows(int n, const double *mu, double *b) {
    __shared__ double red[256];
    const int tid = threadIdx.x;
    mu += (size_t)blockIdx.x * n;
    b += (size_t)blockIdx.x * n;
    double t = 0.0;
    for (int j = tid; j < n; j += blockDim.x) t += mu[j];
    red[tid] = t;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    const double tot = red[0];
    for (int j = tid; j < n; j += blockDim.x) b[j] = mu[j] / tot;
}

__global__ void k_argmax(int m, const double *x, int *out) {
    __shared__ double rv[256];
    __shared__ int ri[256];
    const int tid = threadIdx.x;
    double best = -INFINITY;
    int bi = 0x7FFFFFFF;
    for (int k = tid; k < m; k += blockDim.x)
        if (x[k] > best || (x[k] == best && k < bi)) {
            best = x[k];
            bi = k;
        }
    rv[tid] = best;
    ri[tid] = bi;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s && (rv[tid + s] > rv[tid] || (rv[tid + s] == rv[tid] && ri[tid + s] < ri[tid]))) {
            rv[tid] = rv[tid + s];
            ri[tid] = ri[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) *out = ri[0];
}

// dst = rows[*idx] (n entries).
__global__ void k_gather_row(int n, const double *rows, const int *idx, double *dst) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) dst[j] = rows[(size_t)(*idx) * n + j];
}

// y = x M (row vector times matrix).  A workgroup per 64 columns, lane = column: each of its kVecWaves
// wavefronts sums every kVecWaves-th row in order and the partial sums are
// added in wavefront order.
constexpr int kVecWaves = 16;
__global__ __launch_bounds__(64 * kVecWaves) void k_vecmat(int n, const double *x, const double *M, double *y) {
    __shared__ double part[kVecWaves][64];
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + lane;
    double acc = 0.0;
    if (j < n)
        for (int i = wave; i < n; i += kVecWaves) acc += x[i] * M[(size_t)i * n + j];
    part[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && j < n) {
        double t = 0.0;
        for (int w = 0; w < kVecWaves; ++w) t += part[w][lane];
        y[j] = t;
    }
}

// b_lin = b0 + v / (mu0 1) - b0 (v 1) / (mu0 1)  (single workgroup).
__global__ void k_blin(int n, const double *b0, const double *mu0, const double *v, double *b_lin) {
    __shared__ double r1[256], r2[256];
    const int tid = threadIdx.x;
    double a = 0.0, t = 0.0;
    for (int j = tid; j < n; j += blockDim.x) {
        a += mu0[j];
        t += v[j];
    }
    r1[tid] = a;
    r2[tid] = t;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) {
            r1[tid] += r1[tid + s];
            r2[tid] += r2[tid + s];
        }
        __syncthreads();
    }
    const double tot = r1[0], vs = r2[0];
    for (int j = tid; j < n; j += blockDim.x) b_lin[j] = b0[j] + v[j] / tot - b0[j] * vs / tot;
}

// C = A + alpha B + beta D (elementwise; D may be null).
__global__ void k_axpy(size_t count, const double *A, double alpha, const double *B, double beta, const double *D,
                       double *C) {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < count; k += (size_t)gridDim.x * blockDim.x)
        C[k] = A[k] + alpha * B[k] + (D ? beta * D[k] : 0.0);
}

// Infinity norm (largest absolute row sum): one workgroup per row, atomic max
// on the bit pattern (non-negative doubles order like their bits).
__global__ void k_rowabs(int n, const double *A, unsigned long long *out) {
    __shared__ double red[256];
    const int i = blockIdx.x, tid = threadIdx.x;
    double acc = 0.0;
    for (int j = tid; j < n; j += blockDim.x) acc += fabs(A[(size_t)i * n + j]);
    red[tid] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) atomicMax(out, as_u64(red[0]));
}

// C = A B for n x n row-major FP64 matrices on the FP64 matrix cores: a
// 64 x 64 output tile per workgroup of 256 threads, each wavefront a 32 x 32
// quadrant as 2 x 2 blocks of v_mfma_f64_16x16x4 (lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] of a 16 x 4 by 4 x 16 product and
// holds D[4 r + l / 16][l % 16] in item r), K staged 32 at a time through LDS
// (zero past n, so a partial last step is exact).
typedef double gemm_f64x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_gemm(int n, const double *A, const double *B, double *C) {
    constexpr int GT = 64, GK = 32;
    __shared__ double As[GT][GK + 1];
    __shared__ double Bs[GK][GT + 1];
    const int i0 = blockIdx.y * GT, j0 = blockIdx.x * GT;
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    const int rw = (wave >> 1) * 32, cw = (wave & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    gemm_f64x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = gemm_f64x4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < n; k0 += GK) {
        if (k0 > 0) __syncthreads();   // the previous slice is consumed
        for (int t = threadIdx.x; t < GT * GK; t += blockDim.x) {
            const int r = t / GK, c = t % GK;
            As[r][c] = (i0 + r < n && k0 + c < n) ? A[(size_t)(i0 + r) * n + k0 + c] : 0.0;
            const int r2 = t / GT, c2 = t % GT;
            Bs[r2][c2] = (k0 + r2 < n && j0 + c2 < n) ? B[(size_t)(k0 + r2) * n + j0 + c2] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < GK; p += 4) {
            double af[2], bf[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) af[a] = As[rw + 16 * a + li][p + lk];
#pragma unroll
            for (int b = 0; b < 2; ++b) bf[b] = Bs[p + lk][cw + 16 * b + li];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + rw + 16 * a + 4 * r + lk, j = j0 + cw + 16 * b + li;
                if (i < n && j < n) C[(size_t)i * n + j] = acc[a][b][r];
            }
}

// Transition rewards per row: switching sum_{j != i} Q_ij, improvement
// sum_j Q_ij (f_j - f_i)_+.
__global__ void k_trans_rewards(int n, const double *Q, const double *f, double *psw, double *pimp) {
    __shared__ double r1[256], r2[256];
    const int i = blockIdx.x, tid = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int j = tid; j < n; j += blockDim.x) {
        const double q = Q[(size_t)i * n + j];
        if (j != i) a += q;
        const double d = f[j] - f[i];
        if (d > 0.0) b += q * d;
    }
    r1[tid] = a;
    r2[tid] = b;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) {
            r1[tid] += r1[tid + s];
            r2[tid] += r2[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        psw[i] = r1[0];
        pimp[i] = r2[0];
    }
}

// Remainder bound of Section 5.4 from the norms [|N0 E|, |N0|]:
// |N0 E|^2 |N0| / (1 - |N0 E|), infinite when |N0 E| >= 1.
__global__ void k_rem_bound(const unsigned long long *norms, double *out) {
    const double a = as_f64(norms[0]), b = as_f64(norms[1]);
    *out = a < 1.0 ? a * a * b / (1.0 - a) : INFINITY;
}

// ---------------------------------------------------------------------------
hipError_t robust_rem_bound(const unsigned long long *norms, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_rem_bound, dim3(1), dim3(1), 0, st, norms, out);
    return hipGetLastError();
}

hipError_t robust_perturb(int n, const double *Q0, uint64_t seed, int sample, const int *sample_ptr, double delta,
                          double r_min, double *Q, double *A, hipStream_t st) {
    hipLaunchKernelGGL(k_perturb, dim3(n), dim3(256), 0, st, n, Q0, (uint32_t)seed, (uint32_t)(seed >> 32), sample,
                       sample_ptr, delta, r_min, Q, A, (size_t)0);
    return hipGetLastError();
}

hipError_t robust_perturb_batch(int n, const double *Q0, uint64_t seed, int sample0, int batch, double delta,
                                double r_min, double *A, size_t stride, hipStream_t st) {
    hipLaunchKernelGGL(k_perturb, dim3(n, batch), dim3(256), 0, st, n, Q0, (uint32_t)seed, (uint32_t)(seed >> 32),
                       sample0, (const int *)nullptr, delta, r_min, (double *)nullptr, A, stride);
    return hipGetLastError();
}

hipError_t robust_divergence(int n, int batch, const double *b, const double *b0, double *kl, double *tv,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_divergence, dim3(batch), dim3(256), 0, st, n, b, b0, kl, tv);
    return hipGetLastError();
}

hipError_t robust_normalize_rows(int n, int batch, const double *mu, double *b, hipStream_t st) {
    hipLaunchKernelGGL(k_normalize_rows, dim3(batch), dim3(256), 0, st, n, mu, b);
    return hipGetLastError();
}

hipError_t robust_argmax(int m, const double *x, int *out, hipStream_t st) {
    hipLaunchKernelGGL(k_argmax, dim3(1), dim3(256), 0, st, m, x, out);
    return hipGetLastError();
}

hipError_t robust_gather_row(int n, const double *rows, const int *idx, double *dst, hipStream_t st) {
    hipLaunchKernelGGL(k_gather_row, dim3((n + 255) / 256), dim3(256), 0, st, n, rows, idx, dst);
    return hipGetLastError();
}

hipError_t robust_vecmat(int n, const double *x, const double *M, double *y, hipStream_t st) {
    hipLaunchKernelGGL(k_vecmat, dim3((n + 63) / 64), dim3(64 * kVecWaves), 0, st, n, x, M, y);
    return hipGetLastError();
}

hipError_t robust_blin(int n, const double *b0, const double *mu0, const double *v, double *b_lin, hipStream_t st) {
    hipLaunchKernelGGL(k_blin, dim3(1), dim3(256), 0, st, n, b0, mu0, v, b_lin);
    return hipGetLastError();
}

hipError_t robust_axpy(size_t count, const double *A, double alpha, const double *B, double beta, const double *D,
                       double *C, hipStream_t st) {
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_axpy, dim3((unsigned)blocks), dim3(256), 0, st, count, A, alpha, B, beta, D, C);
    return hipGetLastError();
}

hipError_t robust_infnorm(int n, const double *A, unsigned long long *out, hipStream_t st) {
    hipLaunchKernelGGL(k_rowabs, dim3(n), dim3(256), 0, st, n, A, out);
    return hipGetLastError();
}

hipError_t robust_gemm(int n, const double *A, const double *B, double *C, hipStream_t st) {
    const unsigned t = (unsigned)((n + 63) / 64);
    hipLaunchKernelGGL(k_gemm, dim3(t, t), dim3(256), 0, st, n, A, B, C);
    return hipGetLastError();
}

hipError_t robust_trans_rewards(int n, const double *Q, const double *f, double *psw, double *pimp, hipStream_t st) {
    hipLaunchKernelGGL(k_trans_rewards, dim3(n), dim3(256), 0, st, n, Q, f, psw, pimp);
    return hipGetLastError();
}

}  // namespace amc
