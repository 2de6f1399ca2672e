// tail.hip -- FP64 chain algebra on the device: the estimated kernel, the
// fundamental matrix N = (I - Q)^{-1}, visits, AFC, rewards, the
// pool-constrained kernel and the visit-gap certificates.
//
// Paper: Bao, Kontou, Vogiatzis, "Betweenness-Central Nodes Under
// Uncertainty: An Absorbing Markov Chain Approach" (Section 4, Section 5.5,
// Section 6.4, Section 7, Section 8.2).
//
// I - Q is strictly diagonally dominant by rows whenever every row absorbs
// (row i: (1 - Q_ii) - sum_{j != i} Q_ij = r_i > 0), so the inverse is taken
// by blocked Gauss-Jordan elimination without pivoting (growth factor at most
// 2 for such matrices).
#include <algorithm>

#include "amc_dev.hpp"
#include "amc_kernels.hpp"

namespace amc {

constexpr int NB = 64;      // Gauss-Jordan panel width
constexpr int TT = 64;      // trailing-update tile edge
constexpr int PT = 32;      // panel-kernel tile edge (keeps their LDS under 64 KB)
constexpr int KC = 32;      // panel columns staged per pass of the trailing update
constexpr int kDiagThreads = 1024;  // threads of the diagonal-block inversion

// Empirical kernel of Alg. 2 plus the floor of Section 8.2: when row i never
// absorbed and eta > 0, P_i,bottom := eta and the transient part is scaled by
// (1 - eta).  Also writes A = I - Q.
__global__ void k_counts_to_kernel(int n, const uint32_t *counts, uint32_t R, double eta, double *Q, double *r,
                                   double *A) {
    const int i = blockIdx.x;
    const uint32_t *row = counts + (size_t)i * (n + 1);
    const bool fl = row[n] == 0u && eta > 0.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double q = (double)row[j] / (double)R;
        const double v = fl ? (1.0 - eta) * q : q;
        Q[(size_t)i * n + j] = v;
        A[(size_t)i * n + j] = (i == j ? 1.0 : 0.0) - v;
    }
    if (threadIdx.x == 0) r[i] = fl ? eta : (double)row[n] / (double)R;
}

// A = I - Q for a given Q; r = 1 - Q 1.
__global__ void k_from_Q(int n, const double *Q, double *r, double *A) {
    const int i = blockIdx.x;
    __shared__ double part[256];
    double acc = 0.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double v = Q[(size_t)i * n + j];
        A[(size_t)i * n + j] = (i == j ? 1.0 : 0.0) - v;
        acc += v;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) r[i] = 1.0 - part[0];
}

// The four steps take a batch of matrices A + z * stride, z = blockIdx.z.
// (a) invert the diagonal block A[k0:k1, k0:k1] in place (unblocked
// Gauss-Jordan without pivoting); flags a zero pivot.  Each thread holds
// NB * NB / kDiagThreads entries of the block (padded with the identity,
// which every pivot step leaves unchanged) in registers across the pivots.
__device__ __forceinline__ void gj_diag_body(int n, double *A, int k0, int *err, double (*M)[NB + 1]) {
    constexpr int PER = NB * NB / kDiagThreads;
    const int kb = min(NB, n - k0);
    int ii[PER], jj[PER];
    double x[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int t = (int)threadIdx.x + r * kDiagThreads;
        ii[r] = t / NB;
        jj[r] = t % NB;
        const bool in = ii[r] < kb && jj[r] < kb;
        x[r] = in ? A[(size_t)(k0 + ii[r]) * n + k0 + jj[r]] : (ii[r] == jj[r] ? 1.0 : 0.0);
        M[ii[r]][jj[r]] = x[r];
    }
    __syncthreads();
    // a thread's entries share one column (kDiagThreads is a multiple of NB),
    // so the pivot row is read and scaled once per step
    static_assert(kDiagThreads % NB == 0, "one column per thread");
    const int jc = jj[0];
    for (int p = 0; p < kb; ++p) {
        const double piv = M[p][p];
        const double rowv = M[p][jc];
        double col[PER];
#pragma unroll
        for (int r = 0; r < PER; ++r) col[r] = M[ii[r]][p];
        __syncthreads();   // every read of step p is done before its writes
        if (piv == 0.0) {
            if (threadIdx.x == 0) atomicOr(err, 2);
            return;
        }
        const double d = 1.0 / piv;
        const double rowd = rowv * d;
        const bool pc = jc == p;
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            if (ii[r] == p) x[r] = pc ? d : rowd;    // pivot row scaled, pivot replaced by its inverse
            else if (pc) x[r] = -col[r] * d;         // pivot column
            else x[r] -= col[r] * rowd;              // the rest, against the scaled pivot row
            M[ii[r]][jc] = x[r];
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < PER; ++r)
        if (ii[r] < kb && jj[r] < kb) A[(size_t)(k0 + ii[r]) * n + k0 + jj[r]] = x[r];
}
__global__ __launch_bounds__(kDiagThreads) void k_gj_diag(int n, double *A, size_t stride, int k0, int *err) {
    __shared__ double M[NB][NB + 1];
    gj_diag_body(n, A + (size_t)blockIdx.z * stride, k0, err, M);
}

// (b) row panel: A[k, j] <- Dinv A[k, j] for columns j outside the block
// (PT columns per workgroup).
__global__ void k_gj_rowpanel(int n, double *A, size_t stride, int k0) {
    A += (size_t)blockIdx.z * stride;
    __shared__ double Dv[NB][NB + 1];
    __shared__ double X[NB][PT + 1];
    const int kb = min(NB, n - k0);
    const int j0 = blockIdx.x * PT;
    for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) {
        const int i = t / NB, j = t % NB;
        Dv[i][j] = (i < kb && j < kb) ? A[(size_t)(k0 + i) * n + k0 + j] : 0.0;
    }
    for (int t = threadIdx.x; t < NB * PT; t += blockDim.x) {
        const int i = t / PT, j = t % PT;
        const int c = j0 + j;
        X[i][j] = (i < kb && c < n) ? A[(size_t)(k0 + i) * n + c] : 0.0;
    }
    __syncthreads();
    // thread (ty, tx): column tx, rows ty + RS q; X[p][tx] read once per p
    constexpr int RS = 256 / PT, RQ = NB / RS;
    const int tx = (int)threadIdx.x % PT, ty = (int)threadIdx.x / PT;
    double acc[RQ];
#pragma unroll
    for (int q = 0; q < RQ; ++q) acc[q] = 0.0;
    for (int p = 0; p < kb; ++p) {
        const double xv = X[p][tx];
#pragma unroll
        for (int q = 0; q < RQ; ++q) acc[q] += Dv[ty + RS * q][p] * xv;
    }
    const int c = j0 + tx;
    if (c >= n || (c >= k0 && c < k0 + kb)) return;
#pragma unroll
    for (int q = 0; q < RQ; ++q)
        if (ty + RS * q < kb) A[(size_t)(k0 + ty + RS * q) * n + c] = acc[q];
}

// (c) trailing update A[i, j] -= A[i, k] A[k, j] for i, j outside the block
// (A[k, j] already holds the row panel of step (b)), on the FP64 matrix
// cores: a 64 x 64 tile per workgroup, each wavefront a 32 x 32 quadrant as
// 2 x 2 blocks of v_mfma_f64_16x16x4 (lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] of a 16 x 4 by 4 x 16 product and holds
// D[4 r + l / 16][l % 16] in item r), the panel staged KC columns at a time.
typedef double mfma_f64x4 __attribute__((ext_vector_type(4)));
// Workgroups are dispatched to the XCDs in turn (linear id mod 8): for the
// first batch - batch % 8 matrices every tile of a matrix goes to one XCD, so
// that its panels are fetched into one L2 only; the rest follow in order.
__global__ __launch_bounds__(256) void k_gj_update_mfma(int n, double *A, size_t stride, int k0, int batch) {
    const uint32_t tiles = (uint32_t)(n + TT - 1) / TT, T = tiles * tiles, L = blockIdx.x;
    const uint32_t grouped = T * ((uint32_t)batch & ~7u);
    uint32_t z, t;
    if (L < grouped) {
        const uint32_t slot = L >> 3;
        z = (slot / T) * 8u + (L & 7u);
        t = slot % T;
    } else {
        z = ((uint32_t)batch & ~7u) + (L - grouped) / T;
        t = (L - grouped) % T;
    }
    A += (size_t)z * stride;
    __shared__ double Ap[TT][KC + 1];
    __shared__ double Bp[KC][TT + 1];
    const int kb = min(NB, n - k0);
    const int i0 = (int)(t / tiles) * TT, j0 = (int)(t % tiles) * TT;
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    const int rw = (wave >> 1) * 32, cw = (wave & 1) * 32;     // the wavefront's quadrant
    const int li = lane & 15, lk = lane >> 4;
    mfma_f64x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma_f64x4{0.0, 0.0, 0.0, 0.0};
    // the lane's entries of the output tile are loaded first, so that their
    // latency overlaps the panel staging and the products
    double old[2][2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + rw + 16 * a + 4 * r + lk, j = j0 + cw + 16 * b + li;
                old[a][b][r] = (i < n && j < n) ? A[(size_t)i * n + j] : 0.0;
            }
    for (int c0 = 0; c0 < kb; c0 += KC) {
        const int kc = min(KC, kb - c0);
        if (c0 > 0) __syncthreads();   // the previous slice is consumed
        for (int t = threadIdx.x; t < TT * KC; t += blockDim.x) {
            const int i = t / KC, p = t % KC;
            Ap[i][p] = (i0 + i < n && p < kc) ? A[(size_t)(i0 + i) * n + k0 + c0 + p] : 0.0;
        }
        for (int t = threadIdx.x; t < KC * TT; t += blockDim.x) {
            const int p = t / TT, j = t % TT;
            Bp[p][j] = (p < kc && j0 + j < n) ? A[(size_t)(k0 + c0 + p) * n + j0 + j] : 0.0;
        }
        __syncthreads();
        // zero padding past kc makes the last partial group of 4 exact
        for (int p = 0; p < kc; p += 4) {
            double af[2], bf[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) af[a] = Ap[rw + 16 * a + li][p + lk];
#pragma unroll
            for (int b = 0; b < 2; ++b) bf[b] = Bp[p + lk][cw + 16 * b + li];
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
                if (i >= n || j >= n || (i >= k0 && i < k0 + kb) || (j >= k0 && j < k0 + kb)) continue;
                A[(size_t)i * n + j] = old[a][b][r] - acc[a][b][r];
            }
}

// (d) column panel: A[i, k] <- -A[i, k] Dinv for rows i outside the block
// (PT rows per workgroup of THREADS threads).
template <int THREADS>
__device__ __forceinline__ void gj_colpanel_body(int n, double *A, int k0, int tile, double (*Dv)[NB + 1],
                                                 double (*X)[NB + 1]) {
    const int kb = min(NB, n - k0);
    const int i0 = tile * PT;
    for (int t = threadIdx.x; t < NB * NB; t += THREADS) {
        const int i = t / NB, j = t % NB;
        Dv[i][j] = (i < kb && j < kb) ? A[(size_t)(k0 + i) * n + k0 + j] : 0.0;
    }
    for (int t = threadIdx.x; t < PT * NB; t += THREADS) {
        const int i = t / NB, p = t % NB;
        X[i][p] = (i0 + i < n && p < kb) ? A[(size_t)(i0 + i) * n + k0 + p] : 0.0;
    }
    __syncthreads();
    // thread (ty, tx): column tx, rows ty + RS q; Dv[p][tx] read once per p
    constexpr int RS = THREADS / NB, RQ = PT / RS;
    static_assert(THREADS % NB == 0 && PT % RS == 0, "whole rows per thread");
    const int tx = (int)threadIdx.x % NB, ty = (int)threadIdx.x / NB;
    double acc[RQ];
#pragma unroll
    for (int q = 0; q < RQ; ++q) acc[q] = 0.0;
    for (int p = 0; p < kb; ++p) {
        const double dv = Dv[p][tx];
#pragma unroll
        for (int q = 0; q < RQ; ++q) acc[q] += X[ty + RS * q][p] * dv;
    }
    if (tx >= kb) return;
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
        const int row = i0 + ty + RS * q;
        if (row < n && (row < k0 || row >= k0 + kb)) A[(size_t)row * n + k0 + tx] = -acc[q];
    }
}
__global__ __launch_bounds__(256) void k_gj_colpanel(int n, double *A, size_t stride, int k0) {
    __shared__ double Dv[NB][NB + 1];
    __shared__ double X[PT][NB + 1];
    gj_colpanel_body<256>(n, A + (size_t)blockIdx.z * stride, k0, blockIdx.x, Dv, X);
}

// (d) of step k0 together with (a) of step k0 + NB, in one launch: the column
// panel writes columns k0 .. k0 + NB - 1 and the next diagonal block lies in
// columns from k0 + NB on, so the two are independent, and the panel's
// workgroups run beside the latency-bound block inversion (the last
// workgroup of each matrix).
__global__ __launch_bounds__(kDiagThreads) void k_gj_colpanel_diag(int n, double *A, size_t stride, int k0,
                                                                   int *err) {
    __shared__ double S[(NB + PT) * (NB + 1)];
    A += (size_t)blockIdx.z * stride;
    if (blockIdx.x == gridDim.x - 1)
        gj_diag_body(n, A, k0 + NB, err, (double (*)[NB + 1])S);
    else
        gj_colpanel_body<kDiagThreads>(n, A, k0, blockIdx.x, (double (*)[NB + 1])S,
                                       (double (*)[NB + 1])(S + NB * (NB + 1)));
}

// mu = s N (eq. visits): a workgroup per 64 columns, lane = column; its
// kVisitWaves wavefronts each sum every kVisitWaves-th row in order, and the
// partial sums are added in wavefront order (a fixed summation order); a
// batch of matrices N + y * stride gives mu + y * n, y = blockIdx.y.
constexpr int kVisitWaves = 16;
__global__ __launch_bounds__(64 * kVisitWaves) void k_visits(int n, const double *N, const double *s, double *mu,
                                                            size_t stride) {
    __shared__ double part[kVisitWaves][64];
    N += (size_t)blockIdx.y * stride;
    mu += (size_t)blockIdx.y * n;
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + lane;
    double acc = 0.0;
    if (j < n)
        for (int i = wave; i < n; i += kVisitWaves) acc += s[i] * N[(size_t)i * n + j];
    part[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && j < n) {
        double t = 0.0;
        for (int w = 0; w < kVisitWaves; ++w) t += part[w][lane];
        mu[j] = t;
    }
}

// Single-workgroup reductions: E_s[T] = mu 1, b = mu / E_s[T], b . f, pool mass,
// within-pool profile, Top-k of b (ties to the smaller index), admissibility.
// scal: [0] E_T, [1] b_f, [2] m_w, [3] admissible
__global__ void k_afc(int n, const double *mu, double *b, const double *f, const uint8_t *pool, double *b_bar,
                      const double *r, double r_lower, int topk, int32_t *top, double *scal) {
    __shared__ double red[1024];
    __shared__ int redi[1024];
    const int tid = threadIdx.x, nt = blockDim.x;
    double acc = 0.0;
    for (int j = tid; j < n; j += nt) acc += mu[j];
    red[tid] = acc;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    const double ET = red[0];
    __syncthreads();
    double bf = 0.0, mw = 0.0;
    int adm = 1;
    for (int j = tid; j < n; j += nt) {
        const double bj = mu[j] / ET;
        b[j] = bj;
        if (f) bf += bj * f[j];
        if (pool && pool[j]) mw += bj;
        if (r && r[j] < r_lower) adm = 0;
    }
    red[tid] = bf;
    redi[tid] = adm;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
        if (tid < s) {
            red[tid] += red[tid + s];
            redi[tid] = min(redi[tid], redi[tid + s]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        scal[0] = ET;
        scal[1] = red[0];
        scal[3] = (double)redi[0];
    }
    __syncthreads();
    red[tid] = mw;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    const double mtot = red[0];
    if (tid == 0) scal[2] = mtot;
    if (pool && b_bar)
        for (int j = tid; j < n; j += nt) b_bar[j] = (pool[j] && mtot > 0.0) ? b[j] / mtot : 0.0;
    __syncthreads();
    // Top-k by repeated selection
    for (int t = 0; t < topk; ++t) {
        double best = -1.0;
        int bi = 0x7FFFFFFF;
        for (int j = tid; j < n; j += nt) {
            bool taken = false;
            for (int q = 0; q < t; ++q) taken |= (top[q] == j);
            if (taken) continue;
            const double bj = b[j];
            if (bj > best || (bj == best && j < bi)) {
                best = bj;
                bi = j;
            }
        }
        red[tid] = best;
        redi[tid] = bi;
        __syncthreads();
        for (int s = nt / 2; s > 0; s >>= 1) {
            if (tid < s) {
                const double o = red[tid + s];
                const int oi = redi[tid + s];
                if (o > red[tid] || (o == red[tid] && oi < redi[tid])) {
                    red[tid] = o;
                    redi[tid] = oi;
                }
            }
            __syncthreads();
        }
        if (tid == 0) top[t] = redi[0];
        __syncthreads();
    }
}

// Complement of the Top-k in increasing index order (single workgroup).
__global__ void k_complement(int n, int topk, const int32_t *top, int32_t *cv) {
    // v keeps its place among the vertices outside the Top-k: v minus the
    // members below it (members are distinct)
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    bool in = false;
    int below = 0;
    for (int q = 0; q < topk; ++q) {
        in |= top[q] == v;
        below += top[q] < v;
    }
    if (!in) cv[v - below] = v;
}

// Largest row support max_i #{j : Q_ij > 0} (support-restricted radii).
__global__ void k_support(int n, const double *Q, int *out) {
    __shared__ int part[256];
    const int i = blockIdx.x;
    int c = 0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) c += Q[(size_t)i * n + j] > 0.0;
    part[threadIdx.x] = c;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, part[0]);
}

// Visit-gap certificates (eq. pm-gap, eq. sharp-gap) for every boundary pair
// (u in Top-k, v outside): one thread per v.  Dense radii eps_ij = eps give
// epsbar = n eps; the support-restricted radii eps 1{Q_ij > 0} give
// epsbar_supp = eps max_i |supp Q_i|.
// Column maxima max_i |N_{i,top[a]} - N_{i,v}| over a slice of the rows,
// combined across slices by an integer maximum on the bit patterns
// (non-negative doubles order like their bits); mx starts at zero.
__global__ void k_cert_colmax(int n, int topk, const double *N, const int32_t *top, const int32_t *cv,
                              unsigned long long *mx) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int nc = n - topk;
    if (c >= nc) return;
    const int rows = (n + (int)gridDim.y - 1) / (int)gridDim.y;
    const int i0 = (int)blockIdx.y * rows, i1 = min(n, i0 + rows);
    const int v = cv[c];
    double m[16];
    for (int a = 0; a < topk; ++a) m[a] = 0.0;
    for (int i = i0; i < i1; ++i) {
        const double nv = N[(size_t)i * n + v];
        for (int a = 0; a < topk; ++a) {
            const double d = fabs(N[(size_t)i * n + top[a]] - nv);
            m[a] = d > m[a] ? d : m[a];
        }
    }
    for (int a = 0; a < topk; ++a)
        if (m[a] > 0.0) atomicMax(&mx[(size_t)a * nc + c], as_u64(m[a]));
}

// gap G_uv = mu_u - mu_v (eq. pm-gap) and the sharp thresholds (eq.
// sharp-gap) from the column maxima held in `sharp`.
// ok: bit 0 gap above the sharp threshold, bit 1 above the support-restricted
// one, bit 2 above the crude threshold 2 n eps / r_lower^2 (strict: a gap
// equal to its threshold certifies nothing)
__global__ void k_certificates(int n, int topk, const double *mu, const int32_t *top, const int32_t *cv, double eps,
                               double r_lower, const int *support, double *gap, double *sharp, double *sharp_supp,
                               uint8_t *ok) {
    const int nc = n - topk;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)topk * nc) return;
    const int a = (int)(idx / nc), c = (int)(idx % nc);
    const double coef = (double)n * eps / r_lower;
    const double coef_supp = (double)(*support) * eps / r_lower;
    const double crude = 2.0 * ((double)n * eps) / (r_lower * r_lower);
    const double mx = as_f64(((const unsigned long long *)sharp)[idx]);
    const double g = mu[top[a]] - mu[cv[c]];
    const double sh = coef * mx, shs = coef_supp * mx;
    gap[idx] = g;
    sharp[idx] = sh;
    if (sharp_supp) sharp_supp[idx] = shs;
    if (ok) ok[idx] = (uint8_t)((g > sh ? 1u : 0u) | (g > shs ? 2u : 0u) | (g > crude ? 4u : 0u));
}

__global__ void k_xi(int n, const uint32_t *counts_w, uint32_t R, double *xi) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) xi[i] = 1.0 - (double)counts_w[(size_t)i * (n + 1) + n] / (double)R;
}

__global__ void k_fill_u32(uint32_t *p, size_t count, uint32_t v) {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < count; k += (size_t)gridDim.x * blockDim.x)
        p[k] = v;
}

// ---------------------------------------------------------------------------
hipError_t fill_u32(void *p, size_t count, uint32_t v, hipStream_t st) {
    if (count == 0) return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, (uint32_t *)p, count, v);
    return hipGetLastError();
}

hipError_t tail_kernel_from_counts(int n, const uint32_t *counts, uint32_t R, double eta, double *Q, double *r,
                                   double *A, hipStream_t st) {
    hipLaunchKernelGGL(k_counts_to_kernel, dim3(n), dim3(256), 0, st, n, counts, R, eta, Q, r, A);
    return hipGetLastError();
}

hipError_t tail_kernel_from_Q(int n, const double *Q, double *r, double *A, hipStream_t st) {
    hipLaunchKernelGGL(k_from_Q, dim3(n), dim3(256), 0, st, n, Q, r, A);
    return hipGetLastError();
}

hipError_t tail_invert_batched(int n, double *A, size_t stride, int batch, int *err, hipStream_t st) {
    const int tiles = (n + TT - 1) / TT, ptiles = (n + PT - 1) / PT;
    hipLaunchKernelGGL(k_gj_diag, dim3(1, 1, batch), dim3(kDiagThreads), 0, st, n, A, stride, 0, err);
    for (int k0 = 0; k0 < n; k0 += NB) {
        hipLaunchKernelGGL(k_gj_rowpanel, dim3(ptiles, 1, batch), dim3(256), 0, st, n, A, stride, k0);
        hipLaunchKernelGGL(k_gj_update_mfma, dim3((unsigned)((size_t)tiles * tiles * batch)), dim3(256), 0, st, n, A,
                           stride, k0, batch);
        if (k0 + NB < n)
            hipLaunchKernelGGL(k_gj_colpanel_diag, dim3(ptiles + 1, 1, batch), dim3(kDiagThreads), 0, st, n, A,
                               stride, k0, err);
        else
            hipLaunchKernelGGL(k_gj_colpanel, dim3(ptiles, 1, batch), dim3(256), 0, st, n, A, stride, k0);
    }
    return hipGetLastError();
}

hipError_t tail_invert(int n, double *A, int *err, hipStream_t st) {
    return tail_invert_batched(n, A, (size_t)n * n, 1, err, st);
}

hipError_t tail_visits_batched(int n, const double *N, size_t stride, int batch, const double *s, double *mu,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_visits, dim3((n + 63) / 64, batch), dim3(64 * kVisitWaves), 0, st, n, N, s, mu, stride);
    return hipGetLastError();
}

hipError_t tail_visits(int n, const double *N, const double *s, double *mu, double *b, const double *f,
                       const uint8_t *pool, double *b_bar, const double *r, double r_lower, int topk, int32_t *top,
                       double *scal, hipStream_t st) {
    hipLaunchKernelGGL(k_visits, dim3((n + 63) / 64), dim3(64 * kVisitWaves), 0, st, n, N, s, mu, (size_t)0);
    hipLaunchKernelGGL(k_afc, dim3(1), dim3(1024), 0, st, n, mu, b, f, pool, b_bar, r, r_lower, topk, top, scal);
    return hipGetLastError();
}

hipError_t tail_certificates(int n, int topk, const double *Q, const double *N, const double *mu,
                             const int32_t *top, int32_t *cv, double eps, double r_lower, double *gap,
                             double *sharp, double *sharp_supp, uint8_t *ok, int *support, hipStream_t st) {
    hipLaunchKernelGGL(k_support, dim3(n), dim3(256), 0, st, n, Q, support);
    if (topk > 0 && topk < n) {
        const int nc = n - topk;
        const size_t pairs = (size_t)topk * nc;
        hipLaunchKernelGGL(k_complement, dim3((n + 255) / 256), dim3(256), 0, st, n, topk, top, cv);
        const hipError_t e = fill_u32(sharp, 2 * pairs, 0u, st);
        if (e != hipSuccess) return e;
        // enough row slices to give every CU a few workgroups
        const int cols = (nc + 63) / 64, slices = std::max(1, std::min(n / 8, 1024 / std::max(cols, 1)));
        hipLaunchKernelGGL(k_cert_colmax, dim3(cols, slices), dim3(64), 0, st, n, topk, N, top, cv,
                           (unsigned long long *)sharp);
        hipLaunchKernelGGL(k_certificates, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, st, n, topk, mu,
                           top, cv, eps, r_lower, support, gap, sharp, sharp_supp, ok);
    }
    return hipGetLastError();
}

hipError_t tail_xi(int n, const uint32_t *counts_w, uint32_t R, double *xi, hipStream_t st) {
    hipLaunchKernelGGL(k_xi, dim3((n + 255) / 256), dim3(256), 0, st, n, counts_w, R, xi);
    return hipGetLastError();
}

}  // namespace amc
