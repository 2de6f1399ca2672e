// stability.cpp -- the rank-stability check of Section 8.4 (amc_stability):
// the estimate at M realizations and at 2M, and whether the Top-k set by b
// moved.
//
// Paper: Bao, Kontou, Vogiatzis, "Betweenness-Central Nodes Under
// Uncertainty: An Absorbing Markov Chain Approach" (Section 8.4; Alg. 2 for
// the counts, Section 4 for b).
//
// The 2M estimate extends the M one: realizations r_begin .. r_begin + M - 1
// are swept once, their counts seed the second query, which sweeps
// r_begin + M .. r_begin + 2M - 1 on top of them and runs the tail at 2M.
// With counter-based realizations this is the same estimate a fresh run at
// 2M from r_begin gives, at the cost of 2M sweeps instead of 3M.
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
#define RCHK(expr)                            \
    do {                                      \
        int rc_ = (expr);                     \
        if (rc_ != AMC_OK) return rc_;        \
    } while (0)

namespace {

int stability(amc_ctx *ctx, const amc_graph *g, const amc_model *md, const amc_query *q, int32_t k,
              amc_stability_result *out, hipStream_t st) {
    const int n = g->n;
    const uint32_t M = q->R;
    // the M estimate: execution choices of the caller, no side outputs, the
    // tail's Top-k by b (ties to the smaller index)
    amc_query qa = *q;
    qa.flags = q->flags & (AMC_DIST16 | AMC_DIST32 | AMC_PLAIN_LAUNCH);
    qa.cert_topk = k;
    qa.eps = 0.0;
    qa.r_lower = 1.0;
    qa.reward = nullptr;
    qa.n_debug = 0;
    qa.debug_pairs = nullptr;
    std::vector<uint32_t> counts((size_t)n * (n + 1));
    std::vector<int32_t> top_a((size_t)k), top_b((size_t)k);
    std::vector<double> b_a((size_t)n), b_b((size_t)n);
    amc_result ra{};
    ra.counts = counts.data();
    ra.b = b_a.data();
    ra.top = top_a.data();
    RCHK(run_query(ctx, g, md, &qa, &ra, st));

    // the 2M estimate: a query over the next M realizations whose counts
    // start from the first M's
    amc_query qb = qa;
    qb.r_begin = q->r_begin + M;
    QueryRun R;
    RCHK(qr_init(R, ctx, g, md, &qb));
    struct Guard {
        QueryRun &r;
        hipStream_t s;
        ~Guard() { qr_release(r, s); }
    } guard{R, st};
    RCHK(qr_alloc(R, st));
    hipEvent_t ev[2];
    for (auto &e : ev) HIPCHK(hipEventCreate(&e));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() {
            (void)hipEventDestroy(e[0]);
            (void)hipEventDestroy(e[1]);
        }
    } evg{ev};
    RCHK(qr_enqueue_reset(R, st));
    HIPCHK(hipMemcpyAsync(R.P.counts, counts.data(), 4 * counts.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(ev[0], st));
    RCHK(qr_enqueue_sweep(R, st));
    HIPCHK(hipEventRecord(ev[1], st));
    R.q.R = 2 * M;
    R.eta = q->floor_eta < 0.0 ? 0.1 / std::sqrt(2.0 * (double)M) : q->floor_eta;
    RCHK(qr_enqueue_tail(R, st, false));
    amc_result rb{};
    rb.counts = out->counts_2M ? out->counts_2M : counts.data();
    rb.b = b_b.data();
    rb.top = top_b.data();
    RCHK(qr_finish(R, &rb, st));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ev[0], ev[1]));

    int overlap = 0;
    for (int a = 0; a < k; ++a)
        for (int c = 0; c < k; ++c) overlap += top_a[(size_t)a] == top_b[(size_t)c];
    double diff = 0.0;
    for (int v = 0; v < n; ++v) diff = std::fmax(diff, std::fabs(b_b[(size_t)v] - b_a[(size_t)v]));
    if (out->b_M) std::copy(b_a.begin(), b_a.end(), out->b_M);
    if (out->b_2M) std::copy(b_b.begin(), b_b.end(), out->b_2M);
    if (out->top_M) std::copy(top_a.begin(), top_a.end(), out->top_M);
    if (out->top_2M) std::copy(top_b.begin(), top_b.end(), out->top_2M);
    out->overlap = overlap;
    out->same_set = overlap == k ? 1 : 0;
    out->max_abs_diff = diff;
    out->sweep_ms = ra.stats.sweep_ms + ms;
    return AMC_OK;
}

}  // namespace

extern "C" int amc_stability(amc_ctx *ctx, const amc_graph *g, const amc_model *model, const amc_query *q,
                             int32_t k, amc_stability_result *out) {
    if (!ctx || !g || g->ctx != ctx || !model || !q || !out) return AMC_E_INVALID_ARG;
    if (k < 1 || k > 16 || k >= g->n) return AMC_E_INVALID_ARG;
    if (q->R < 1 || q->R > 0x7FFFFFFFu || (uint64_t)q->r_begin + 2ull * q->R > 0x100000000ull)
        return AMC_E_INVALID_ARG;
    if (q->topk != 0 || q->pool_size != 0 || q->pool || (q->flags & AMC_FALLBACK)) return AMC_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return AMC_E_HIP;
    return stability(ctx, g, model, q, k, out, ctx->stream);
}
