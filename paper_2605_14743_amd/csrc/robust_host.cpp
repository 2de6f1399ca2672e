// robust_host.cpp -- host side of the robust tail (amc_robust): checks,
// device buffers, the sequence of sample inversions and the sensitivity.
//
// Paper: Bao, Kontou, Vogiatzis, "Betweenness-Central Nodes Under
// Uncertainty: An Absorbing Markov Chain Approach" (Sections 5.1, 5.4, 6.4).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "amc_kernels.hpp"
#include "query.hpp"

using namespace amc;

namespace amc {
hipError_t set_w1_attrs(int max_lds);   // w1.hip
}

#define HIPCHK(expr)                          \
    do {                                      \
        if ((expr) != hipSuccess) {           \
            (void)hipGetLastError();          \
            return AMC_E_HIP;                 \
        }                                     \
    } while (0)
#define RCHK(expr)                            \
    do {                                      \
        int rc_ = (expr);                     \
        if (rc_ != AMC_OK) return rc_;        \
    } while (0)

extern "C" int amc_robust(amc_ctx *ctx, int32_t n, const double *Q0, const amc_robust_query *q,
                          amc_robust_result *out) {
    if (!ctx || !Q0 || !q || !out || n < 1) return AMC_E_INVALID_ARG;
    if (q->samples < 0 || q->samples > 4096 || !(q->delta >= 0.0) || !std::isfinite(q->delta)) return AMC_E_INVALID_ARG;
    if (!(q->r_min > 0.0 && q->r_min <= 1.0)) return AMC_E_INVALID_ARG;
    for (size_t k = 0; k < (size_t)n * n; ++k)
        if (!(Q0[k] >= 0.0 && Q0[k] <= 1.0)) return AMC_E_INVALID_ARG;
    for (int i = 0; i < n; ++i) {
        double t = 0.0;
        for (int j = 0; j < n; ++j) t += Q0[(size_t)i * n + j];
        if (!(t < 1.0)) return AMC_E_INVALID_ARG;
    }
    std::vector<double> s_uni;
    const double *s = q->s;
    if (s) {
        double t = 0.0;
        for (int i = 0; i < n; ++i) {
            if (!(s[i] >= 0.0)) return AMC_E_INVALID_ARG;
            t += s[i];
        }
        if (std::fabs(t - 1.0) > 1e-9) return AMC_E_INVALID_ARG;
    } else {
        s_uni.assign((size_t)n, 1.0 / n);
        s = s_uni.data();
    }
    if (q->f)
        for (int i = 0; i < n; ++i)
            if (!(q->f[i] >= 0.0) || !std::isfinite(q->f[i])) return AMC_E_INVALID_ARG;
    // base topology for W1: canonical, connected; CSR of incident edges
    const bool want_w1 = q->m > 0;
    const int64_t m = want_w1 ? q->m : 0;
    std::vector<int32_t> rp, inc;
    if (q->m < 0 || (want_w1 && (!q->eu || !q->ev || m > 0x7FFFFFFF))) return AMC_E_INVALID_ARG;
    if (want_w1) {
        if (n > AMC_MAX_W1_N || w1_lds_bytes(n) > (size_t)ctx->max_lds) return AMC_E_UNSUPPORTED;
        for (int64_t e = 0; e < m; ++e) {
            const int32_t a = q->eu[e], b = q->ev[e];
            if (a < 0 || b >= n || a >= b) return AMC_E_INVALID_ARG;
            if (e > 0 && (q->eu[e - 1] > a || (q->eu[e - 1] == a && q->ev[e - 1] >= b))) return AMC_E_INVALID_ARG;
            if (q->w && (q->w[e] < 1u || q->w[e] > 65535u)) return AMC_E_INVALID_ARG;
        }
        rp.assign((size_t)n + 1, 0);
        for (int64_t e = 0; e < m; ++e) {
            ++rp[(size_t)q->eu[e] + 1];
            ++rp[(size_t)q->ev[e] + 1];
        }
        for (int v = 0; v < n; ++v) rp[(size_t)v + 1] += rp[(size_t)v];
        inc.assign((size_t)2 * m, 0);
        std::vector<int32_t> fill(rp.begin(), rp.end() - 1);
        for (int64_t e = 0; e < m; ++e) {
            inc[(size_t)fill[(size_t)q->eu[e]]++] = (int32_t)e;
            inc[(size_t)fill[(size_t)q->ev[e]]++] = (int32_t)e;
        }
        // connected: a search from vertex 0 reaches every vertex
        std::vector<int32_t> stack{0};
        std::vector<uint8_t> seen((size_t)n, 0);
        seen[0] = 1;
        int reached = 1;
        while (!stack.empty()) {
            const int32_t x = stack.back();
            stack.pop_back();
            for (int32_t j = rp[(size_t)x]; j < rp[(size_t)x + 1]; ++j) {
                const int32_t e = inc[(size_t)j];
                const int32_t y = q->eu[e] == x ? q->ev[e] : q->eu[e];
                if (!seen[(size_t)y]) {
                    seen[(size_t)y] = 1;
                    ++reached;
                    stack.push_back(y);
                }
            }
        }
        if (reached != n) return AMC_E_INVALID_ARG;
    }

    std::lock_guard<std::mutex> lk(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return AMC_E_HIP;
    hipStream_t st = ctx->stream;
    DevArena A;
    A.stream = st;
    A.async = ctx->async_alloc;
    struct Guard {
        DevArena &a;
        hipStream_t s;
        ~Guard() {
            (void)hipStreamSynchronize(s);
            a.release();
        }
    } guard{A, st};
    const size_t nn = (size_t)n * n;
    const int S = q->samples;
    void *p;
    auto alloc = [&](size_t bytes) -> void * { return A.alloc(bytes, &p) == AMC_OK ? p : nullptr; };
    double *dQ0 = (double *)alloc(8 * nn), *N0 = (double *)alloc(8 * nn), *W = (double *)alloc(8 * nn);
    double *M1 = (double *)alloc(8 * nn), *M2 = (double *)alloc(8 * nn), *Qs = (double *)alloc(8 * nn);
    double *ds = (double *)alloc(8 * (size_t)n), *mu0 = (double *)alloc(8 * (size_t)n), *b0 = (double *)alloc(8 * (size_t)n);
    double *v = (double *)alloc(8 * (size_t)n), *w = (double *)alloc(8 * (size_t)n);
    double *blin = (double *)alloc(8 * (size_t)n), *bkl = (double *)alloc(8 * (size_t)n), *btv = (double *)alloc(8 * (size_t)n);
    double *scal = (double *)alloc(8 * 8), *rsc = (double *)alloc(8 * 8);
    double *brows = (double *)alloc(8 * (size_t)std::max(S, 1) * n);
    // sampled kernels are inverted in groups of up to 128 (at most 1 GiB of matrices)
    int Bt = std::max(1, std::min(S, 128));
    while (Bt > 1 && (size_t)Bt * nn * 8 > (size_t(1) << 30)) Bt /= 2;
    double *Wb = S > 0 ? (double *)alloc(8 * nn * (size_t)Bt) : nullptr;
    double *mub = S > 0 ? (double *)alloc(8 * (size_t)n * Bt) : nullptr;
    double *kl = (double *)alloc(8 * (size_t)std::max(S, 1)), *tv = (double *)alloc(8 * (size_t)std::max(S, 1));
    double *dr = (double *)alloc(8 * (size_t)n), *psw = (double *)alloc(8 * (size_t)n), *pimp = (double *)alloc(8 * (size_t)n);
    double *df = q->f ? (double *)alloc(8 * (size_t)n) : nullptr;
    const bool w1_on = want_w1 && S > 0;
    double *w1 = w1_on ? (double *)alloc(8 * (size_t)S) : nullptr;
    double *bw1 = w1_on ? (double *)alloc(8 * (size_t)n) : nullptr;
    // every sample's transshipment runs in one launch (a workgroup each), in
    // chunks of at most 1024 samples
    const int Wt = std::min(S, 1024);
    double *fscr = w1_on && m > 0 ? (double *)alloc(8 * (size_t)m * Wt) : nullptr;
    int32_t *deu = w1_on && m > 0 ? (int32_t *)alloc(4 * (size_t)m) : nullptr;
    int32_t *dev_ = w1_on && m > 0 ? (int32_t *)alloc(4 * (size_t)m) : nullptr;
    int32_t *drp = w1_on ? (int32_t *)alloc(4 * ((size_t)n + 1)) : nullptr;
    int32_t *dinc = w1_on && m > 0 ? (int32_t *)alloc(8 * (size_t)m) : nullptr;
    uint32_t *dlen = w1_on && m > 0 && q->w ? (uint32_t *)alloc(4 * (size_t)m) : nullptr;
    if (w1_on && (!w1 || !bw1 || !drp || (m > 0 && (!fscr || !deu || !dev_ || !dinc || (q->w && !dlen)))))
        return AMC_E_OOM;
    int32_t *top = (int32_t *)alloc(4 * 16);
    int *args = (int *)alloc(16), *err = (int *)alloc(16);
    unsigned long long *norms = (unsigned long long *)alloc(8 * 4);
    if ((S > 0 && (!Wb || !mub)) || !dQ0 || !N0 || !W || !M1 || !M2 || !Qs || !ds || !mu0 || !b0 || !v || !w ||
        !blin || !bkl || !btv || !scal || !rsc || !brows || !kl || !tv || !dr || !psw || !pimp || (q->f && !df) ||
        !top || !args || !err || !norms)
        return AMC_E_OOM;
    HIPCHK(hipMemcpyAsync(dQ0, Q0, 8 * nn, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(ds, s, 8 * (size_t)n, hipMemcpyHostToDevice, st));
    if (df) HIPCHK(hipMemcpyAsync(df, q->f, 8 * (size_t)n, hipMemcpyHostToDevice, st));
    if (w1_on) {
        HIPCHK(hipMemcpyAsync(drp, rp.data(), 4 * ((size_t)n + 1), hipMemcpyHostToDevice, st));
        if (m > 0) {
            HIPCHK(hipMemcpyAsync(deu, q->eu, 4 * (size_t)m, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(dev_, q->ev, 4 * (size_t)m, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(dinc, inc.data(), 8 * (size_t)m, hipMemcpyHostToDevice, st));
            if (dlen) HIPCHK(hipMemcpyAsync(dlen, q->w, 4 * (size_t)m, hipMemcpyHostToDevice, st));
        }
    }
    HIPCHK(fill_u32(err, 4, 0u, st));
    HIPCHK(fill_u32(norms, 8, 0u, st));
    HIPCHK(fill_u32(rsc, 16, 0u, st));
    hipEvent_t ev[2];
    for (auto &e : ev) HIPCHK(hipEventCreate(&e));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() {
            (void)hipEventDestroy(e[0]);
            (void)hipEventDestroy(e[1]);
        }
    } evg{ev};
    HIPCHK(hipEventRecord(ev[0], st));
    // nominal chain: N0, mu0, b0
    HIPCHK(tail_kernel_from_Q(n, dQ0, dr, N0, st));
    HIPCHK(tail_invert(n, N0, err, st));
    HIPCHK(tail_visits(n, N0, ds, mu0, b0, nullptr, nullptr, nullptr, nullptr, 0.0, 0, top, scal, st));
    // transition rewards (Section 6.4)
    if (df) {
        HIPCHK(robust_trans_rewards(n, dQ0, df, psw, pimp, st));
        HIPCHK(tail_reward_afc(n, mu0, scal, psw, &rsc[0], st));
        HIPCHK(tail_reward_afc(n, mu0, scal, pimp, &rsc[1], st));
    }
    // sampled admissible kernels, a group at a time: I - Q_k, its inverse,
    // mu_k = s N_k, b_k, and the divergences from b0
    for (int k0 = 0; k0 < S; k0 += Bt) {
        const int nb = std::min(Bt, S - k0);
        HIPCHK(robust_perturb_batch(n, dQ0, q->seed, k0, nb, q->delta, q->r_min, Wb, nn, st));
        HIPCHK(tail_invert_batched(n, Wb, nn, nb, err, st));
        HIPCHK(tail_visits_batched(n, Wb, nn, nb, ds, mub, st));
        HIPCHK(robust_normalize_rows(n, nb, mub, brows + (size_t)k0 * n, st));
        HIPCHK(robust_divergence(n, nb, brows + (size_t)k0 * n, b0, kl + k0, tv + k0, st));
    }
    if (w1_on) HIPCHK(set_w1_attrs(ctx->max_lds));
    for (int k0 = 0; w1_on && k0 < S; k0 += Wt) {
        const int nb = std::min(Wt, S - k0);
        HIPCHK(robust_w1(n, (int)m, deu, dev_, dlen, drp, dinc, nb, brows + (size_t)k0 * n, b0, fscr, w1 + k0, err,
                         st));
    }
    if (S > 0) {
        HIPCHK(robust_argmax(S, kl, args, st));
        HIPCHK(robust_argmax(S, tv, args + 1, st));
        HIPCHK(robust_gather_row(n, brows, args, bkl, st));
        HIPCHK(robust_gather_row(n, brows, args + 1, btv, st));
        if (w1_on) {
            HIPCHK(robust_argmax(S, w1, args + 2, st));
            HIPCHK(robust_gather_row(n, brows, args + 2, bw1, st));
        }
        // first-order sensitivity for E = Q* - Q0 (Section 5.4)
        HIPCHK(robust_perturb(n, dQ0, q->seed, 0, args, q->delta, q->r_min, Qs, W, st));
        HIPCHK(robust_axpy(nn, Qs, -1.0, dQ0, 0.0, nullptr, M2, st));          // M2 = E
        HIPCHK(robust_vecmat(n, mu0, M2, w, st));                              // w = mu0 E
        HIPCHK(robust_vecmat(n, w, N0, v, st));                                // v = mu0 E N0
        HIPCHK(robust_blin(n, b0, mu0, v, blin, st));
        HIPCHK(robust_gemm(n, N0, M2, M1, st));                                // M1 = N0 E
        HIPCHK(robust_infnorm(n, M1, &norms[0], st));
        HIPCHK(robust_infnorm(n, N0, &norms[1], st));
        HIPCHK(robust_gemm(n, M1, N0, M2, st));                                // M2 = N0 E N0
        HIPCHK(tail_invert(n, W, err, st));                                    // W = N*
        HIPCHK(robust_axpy(nn, W, -1.0, N0, -1.0, M2, M1, st));                // N* - N0 - N0 E N0
        HIPCHK(robust_infnorm(n, M1, &norms[2], st));
        HIPCHK(robust_rem_bound(norms, &rsc[2], st));
    }
    HIPCHK(hipEventRecord(ev[1], st));
    int herr = 0;
    unsigned long long hn[4] = {0, 0, 0, 0};
    double hr[3] = {0.0, 0.0, 0.0};
    int ha[3] = {-1, -1, -1};
    HIPCHK(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hn, norms, 8 * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hr, rsc, 24, hipMemcpyDeviceToHost, st));
    if (out->b0) HIPCHK(hipMemcpyAsync(out->b0, b0, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
    if (S > 0) {
        HIPCHK(hipMemcpyAsync(ha, args, 12, hipMemcpyDeviceToHost, st));
        if (out->kl) HIPCHK(hipMemcpyAsync(out->kl, kl, 8 * (size_t)S, hipMemcpyDeviceToHost, st));
        if (out->tv) HIPCHK(hipMemcpyAsync(out->tv, tv, 8 * (size_t)S, hipMemcpyDeviceToHost, st));
        if (out->b_kl) HIPCHK(hipMemcpyAsync(out->b_kl, bkl, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
        if (out->b_tv) HIPCHK(hipMemcpyAsync(out->b_tv, btv, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
        if (out->b_lin) HIPCHK(hipMemcpyAsync(out->b_lin, blin, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
        if (w1_on && out->w1) HIPCHK(hipMemcpyAsync(out->w1, w1, 8 * (size_t)S, hipMemcpyDeviceToHost, st));
        if (w1_on && out->b_w1) HIPCHK(hipMemcpyAsync(out->b_w1, bw1, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    if (herr & 2) return AMC_E_SINGULAR;
    if (herr & 4) return AMC_E_UNSUPPORTED;
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ev[0], ev[1]));
    auto f64 = [](unsigned long long b) {
        double d;
        std::memcpy(&d, &b, 8);
        return d;
    };
    out->b_sw = q->f ? hr[0] : 0.0;
    out->b_imp = q->f ? hr[1] : 0.0;
    out->kl_arg = S > 0 ? ha[0] : -1;
    out->tv_arg = S > 0 ? ha[1] : -1;
    out->w1_arg = w1_on ? ha[2] : -1;
    out->norm_N0E = S > 0 ? f64(hn[0]) : 0.0;
    out->norm_N0 = S > 0 ? f64(hn[1]) : 0.0;
    out->rem_actual = S > 0 ? f64(hn[2]) : 0.0;
    out->rem_bound = S > 0 ? hr[2] : 0.0;
    out->tail_ms = ms;
    return AMC_OK;
}
