// boot_host.cpp -- host side of the bootstrap of b (amc_bootstrap): checks,
// device buffers, the replicate groups and the per-node summaries.
//
// Paper: Bao, Kontou, Vogiatzis, "Betweenness-Central Nodes Under
// Uncertainty: An Absorbing Markov Chain Approach" (Section 8.4; the floor of
// Section 8.2; N, mu and b of Section 4).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <vector>

#include "amc_kernels.hpp"
#include "query.hpp"

using namespace amc;

#define HIPCHK(expr)                          \
    do {                                      \
        if ((expr) != hipSuccess) {           \
            (void)hipGetLastError();          \
            return AMC_E_HIP;                 \
        }                                     \
    } while (0)

extern "C" int amc_bootstrap(amc_ctx *ctx, int32_t n, uint32_t R, const int32_t *next_table,
                             const amc_boot_query *q, amc_boot_result *out) {
    if (!ctx || !next_table || !q || !out || n < 1 || R < 1) return AMC_E_INVALID_ARG;
    if (q->replicates < 1 || q->replicates > AMC_MAX_BOOT_REPLICATES) return AMC_E_INVALID_ARG;
    if (!(q->level > 0.0 && q->level < 1.0)) return AMC_E_INVALID_ARG;
    if (!(q->floor_eta < 1.0) || std::isnan(q->floor_eta)) return AMC_E_INVALID_ARG;
    if (n > AMC_MAX_BOOT_N) return AMC_E_UNSUPPORTED;
    const size_t RN = (size_t)R * (size_t)n;
    for (size_t k = 0; k < RN; ++k)
        if (next_table[k] < -1 || next_table[k] >= n) return AMC_E_INVALID_ARG;
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
    const double eta = q->floor_eta < 0.0 ? 0.1 / std::sqrt((double)R) : q->floor_eta;
    const int B = q->replicates;
    // nearest-rank order statistics of the two tails
    int klo = (int)std::ceil(0.5 * (1.0 - q->level) * (double)B) - 1;
    int khi = (int)std::ceil(0.5 * (1.0 + q->level) * (double)B) - 1;
    if (klo < 0) klo = 0;
    if (khi > B - 1) khi = B - 1;

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
    // replicates are inverted in groups of up to 128 (at most 1 GiB of matrices)
    int Bt = std::min(B, 128);
    while (Bt > 1 && (size_t)Bt * nn * 8 > (size_t(1) << 30)) Bt /= 2;
    void *p;
    auto alloc = [&](size_t bytes) -> void * { return A.alloc(bytes, &p) == AMC_OK ? p : nullptr; };
    int32_t *dnt = (int32_t *)alloc(4 * RN);
    uint16_t *tr = (uint16_t *)alloc(2 * RN);
    double *Wb = (double *)alloc(8 * nn * (size_t)Bt), *mub = (double *)alloc(8 * (size_t)n * Bt);
    double *ds = (double *)alloc(8 * (size_t)n), *b0 = (double *)alloc(8 * (size_t)n);
    double *brep = (double *)alloc(8 * (size_t)n * B), *stats = (double *)alloc(8 * 4 * (size_t)n);
    int *err = (int *)alloc(16);
    if (!dnt || !tr || !Wb || !mub || !ds || !b0 || !brep || !stats || !err) return AMC_E_OOM;
    HIPCHK(hipMemcpyAsync(dnt, next_table, 4 * RN, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(ds, s, 8 * (size_t)n, hipMemcpyHostToDevice, st));
    HIPCHK(fill_u32(err, 4, 0u, st));
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
    HIPCHK(boot_transpose(n, R, dnt, tr, st));
    // the estimate of the given draws
    HIPCHK(boot_rows(n, R, tr, q->seed, 0u, 1, true, eta, Wb, nn, st));
    HIPCHK(tail_invert_batched(n, Wb, nn, 1, err, st));
    HIPCHK(tail_visits_batched(n, Wb, nn, 1, ds, mub, st));
    HIPCHK(robust_normalize_rows(n, 1, mub, b0, st));
    // replicates, a group at a time: I - Q*, its inverse, mu* = s N*, b*
    for (int k0 = 0; k0 < B; k0 += Bt) {
        const int nb = std::min(Bt, B - k0);
        HIPCHK(boot_rows(n, R, tr, q->seed, (uint32_t)k0, nb, false, eta, Wb, nn, st));
        HIPCHK(tail_invert_batched(n, Wb, nn, nb, err, st));
        HIPCHK(tail_visits_batched(n, Wb, nn, nb, ds, mub, st));
        HIPCHK(robust_normalize_rows(n, nb, mub, brep + (size_t)k0 * n, st));
    }
    double *mean = stats, *sd = stats + n, *lo = stats + 2 * (size_t)n, *hi = stats + 3 * (size_t)n;
    HIPCHK(boot_stats(n, B, brep, klo, khi, mean, sd, lo, hi, st));
    HIPCHK(hipEventRecord(ev[1], st));
    int herr = 0;
    HIPCHK(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, st));
    if (out->b0) HIPCHK(hipMemcpyAsync(out->b0, b0, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
    if (out->mean) HIPCHK(hipMemcpyAsync(out->mean, mean, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
    if (out->sd) HIPCHK(hipMemcpyAsync(out->sd, sd, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
    if (out->lo) HIPCHK(hipMemcpyAsync(out->lo, lo, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
    if (out->hi) HIPCHK(hipMemcpyAsync(out->hi, hi, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
    if (out->b_rep) HIPCHK(hipMemcpyAsync(out->b_rep, brep, 8 * (size_t)n * B, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (herr & 2) return AMC_E_SINGULAR;
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ev[0], ev[1]));
    out->ms = ms;
    return AMC_OK;
}
