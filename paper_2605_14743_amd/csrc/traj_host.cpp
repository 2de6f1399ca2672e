// traj_host.cpp -- host side of the trajectory simulator (Section 4.3): argument
// checks, the layout plan (realized graph in LDS or in a per-workgroup L2
// scratch), device buffers, one persistent launch and the length-biased
// estimators.
//
// Paper: Bao, Kontou, Vogiatzis, "Betweenness-Central Nodes Under
// Uncertainty: An Absorbing Markov Chain Approach".
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

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

extern "C" int amc_trajectories(amc_ctx *ctx, const amc_graph *g, const amc_model *model, const amc_traj_query *tq,
                                amc_traj_result *out) {
    if (!ctx || !g || g->ctx != ctx || !model || !tq || !out || !out->lengths || !out->visits)
        return AMC_E_INVALID_ARG;
    const int n = g->n;
    const uint32_t known = AMC_WANT_PATHS | AMC_DIST16 | AMC_DIST32 | AMC_TRAJ_B_LDS | AMC_TRAJ_B_GLOBAL;
    if (tq->episodes < 1 || !tq->x0 || tq->max_steps < 1 || (tq->flags & ~known)) return AMC_E_INVALID_ARG;
    if ((tq->flags & AMC_DIST16) && (tq->flags & AMC_DIST32)) return AMC_E_INVALID_ARG;
    if ((tq->flags & AMC_TRAJ_B_LDS) && (tq->flags & AMC_TRAJ_B_GLOBAL)) return AMC_E_INVALID_ARG;
    if (tq->mode != AMC_MODE_AUTO && tq->mode != AMC_MODE_WAVE && tq->mode != AMC_MODE_WAVE_L2)
        return AMC_E_INVALID_ARG;
    const bool b_forced = (tq->flags & (AMC_TRAJ_B_LDS | AMC_TRAJ_B_GLOBAL)) != 0;
    if (b_forced && tq->mode == AMC_MODE_WAVE) return AMC_E_INVALID_ARG;
    for (int e = 0; e < tq->episodes; ++e)
        if (tq->x0[e] < 0 || tq->x0[e] >= n) return AMC_E_INVALID_ARG;
    if (tq->f)
        for (int v = 0; v < n; ++v)
            if (!(tq->f[v] >= 0.0) || !std::isfinite(tq->f[v])) return AMC_E_INVALID_ARG;
    // the anchor rules and the sweep configuration go through the query checks
    amc_query q;
    std::memset(&q, 0, sizeof(q));
    q.seed = tq->seed;
    q.R = 1;
    q.alpha = tq->alpha;
    q.k_min = tq->k_min;
    q.tie_tau = tq->tie_tau;
    q.floor_eta = -1.0;
    q.r_lower = 0.05;
    q.flags = AMC_SKIP_TAIL | (tq->flags & (AMC_DIST16 | AMC_DIST32));
    q.mode = AMC_MODE_WAVE;
    // the L2 layout exists for one lane per vertex (1 / 2 / 3): a request for
    // it without a mapping takes one lane per vertex
    q.group = tq->group == 0 && tq->mode == AMC_MODE_WAVE_L2 ? 1 : tq->group;
    q.waves = tq->mode == AMC_MODE_WAVE_L2 || b_forced ? 0 : tq->waves;

    std::lock_guard<std::mutex> lk(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return AMC_E_HIP;
    hipStream_t st = ctx->stream;
    QueryRun R;
    // the sweep planner's LDS mode gives the graph encoding (adjacency entry,
    // vertex mapping) and the LDS layout; a graph beyond it takes the
    // encoding of the L2 mode
    bool lds_ok = true;
    int rc = qr_init(R, ctx, g, model, &q);
    if (rc == AMC_E_UNSUPPORTED && tq->mode != AMC_MODE_WAVE) {
        q.mode = AMC_MODE_WAVE_L2;
        q.waves = 0;
        rc = qr_init(R, ctx, g, model, &q);
        lds_ok = false;
    }
    if (rc != AMC_OK) return rc;
    int place = 0;
    {
        // L2 placements: the realized graph in the workgroup's global
        // scratch, K(X_t;H) and (place 1) B(H) in LDS; the wavefront regions
        // stage the edge weights (2 m bytes).  Lane-per-vertex mappings only.
        // Rate of a wavefront relative to one of the LDS layout with 32-bit
        // distances (measured on MI355X, ws1000, 5000 episodes): 0.98 with B
        // in LDS, 0.86 with B in the scratch (the maximiser reads it past the
        // vector L1 every step), 0.77 for 16-bit distances.
        Plan &pl = R.pl;
        const bool lane_map = pl.group == 1 || pl.group == 2 || pl.group == 3;
        const int max_w = pl.group == 3 ? 8 : kMaxWaves;
        const bool d16_ok = (uint64_t)n * model_wmax(g, &R.md) < 0xFFFFull && !(tq->flags & AMC_DIST32);
        int l2_w = 0, l2_place = 0;
        bool l2_d16 = false;
        uint32_t l2_lds = 0, l2_wb = 0;
        double e_l2 = 0.0;
        if (tq->mode != AMC_MODE_WAVE && lane_map && tq->waves <= max_w) {
            for (int bg = 0; bg < 2; ++bg) {
                if ((bg && (tq->flags & AMC_TRAJ_B_LDS)) || (!bg && (tq->flags & AMC_TRAJ_B_GLOBAL))) continue;
                for (int d = 0; d < 2; ++d) {
                    if ((d && !d16_ok) || (!d && (tq->flags & AMC_DIST16))) continue;
                    uint32_t wb = 0;
                    (void)lds_bytes_wave_l2(n, 1, d != 0, true, false, &wb);   // one wavefront's region
                    const uint32_t base = traj_l2_lds_base(n, bg != 0);
                    int fw = 0;
                    for (int w = 2; w <= (tq->waves > 0 ? tq->waves : max_w); ++w) {
                        if (base + wb * (uint32_t)w > (uint32_t)ctx->max_lds) break;
                        if ((uint64_t)wb * (uint64_t)w < 2ull * (uint64_t)g->m) continue;
                        fw = w;
                    }
                    if (tq->waves > 0 && fw != tq->waves) fw = 0;
                    const double e = fw * (bg ? 0.86 : 0.98) * (d ? 0.77 : 1.0);
                    if (fw >= 2 && e > e_l2) {
                        e_l2 = e;
                        l2_w = fw;
                        l2_place = bg ? 2 : 1;
                        l2_d16 = d != 0;
                        l2_lds = base + wb * (uint32_t)fw;
                        l2_wb = wb;
                    }
                }
            }
        }
        const double e_lds = lds_ok ? pl.waves * (pl.dist16 ? 0.77 : 1.0) : 0.0;
        const bool use_l2 = l2_w > 0 && (tq->mode == AMC_MODE_WAVE_L2 || b_forced || e_l2 > e_lds);
        if (!use_l2 && (!lds_ok || tq->mode == AMC_MODE_WAVE_L2 || b_forced)) return AMC_E_UNSUPPORTED;
        if (use_l2) {
            place = l2_place;
            pl.mode = AMC_MODE_WAVE_L2;
            pl.waves = l2_w;
            pl.threads = 64 * l2_w;
            pl.dist16 = l2_d16;
            pl.lds = l2_lds;
            pl.wave_bytes = l2_wb;
            pl.b_global = place == 2;
            pl.sig_global = false;
            pl.scratch_words = (uint32_t)l2_scratch_words(n, pl.adj_cap, pl.adj_bytes, 0);
        } else {
            pl.mode = AMC_MODE_WAVE;
        }
    }
    struct Guard {
        QueryRun &r;
        hipStream_t s;
        ~Guard() { qr_release(r, s); }
    } guard{R, st};
    RCHK(qr_fill_desc(R, st));
    DevArena &A = R.A;
    const int E = tq->episodes, S = tq->max_steps;
    void *p;
    TrajArgs T;
    std::memset(&T, 0, sizeof(T));
    RCHK(A.alloc(sizeof(SweepParams), &p));
    HIPCHK(hipMemcpyAsync(p, &R.P, sizeof(SweepParams), hipMemcpyHostToDevice, st));
    T.desc = (const SweepParams *)p;
    T.episodes = E;
    T.max_steps = S;
    RCHK(A.alloc(4 * (size_t)E, &p));
    HIPCHK(hipMemcpyAsync(p, tq->x0, 4 * (size_t)E, hipMemcpyHostToDevice, st));
    T.x0 = (const int32_t *)p;
    if (tq->f) {
        RCHK(A.alloc(8 * (size_t)n, &p));
        HIPCHK(hipMemcpyAsync(p, tq->f, 8 * (size_t)n, hipMemcpyHostToDevice, st));
        T.f = (const double *)p;
    }
    RCHK(A.alloc(4 * (size_t)E, &p)); T.lengths = (int32_t *)p;
    if (tq->flags & AMC_WANT_PATHS) {
        RCHK(A.alloc(4 * (size_t)E * S, &p));
        T.paths = (int32_t *)p;
    }
    RCHK(A.alloc(8 * (size_t)n, &p)); T.visits = (unsigned long long *)p;
    RCHK(A.alloc(8, &p)); T.reward = (double *)p;
    RCHK(A.alloc(8 * 5, &p)); T.ctr = (unsigned long long *)p;
    RCHK(A.alloc(16, &p)); T.work = (unsigned int *)p;
    RCHK(A.alloc(16, &p)); T.err = (int *)p;
    uint32_t *hist;
    double *b_hat, *surv;
    RCHK(A.alloc(4 * ((size_t)S + 1), &p)); hist = (uint32_t *)p;
    RCHK(A.alloc(8 * (size_t)n, &p)); b_hat = (double *)p;
    RCHK(A.alloc(8 * (size_t)S, &p)); surv = (double *)p;
    HIPCHK(fill_u32(T.visits, 2 * (size_t)n, 0u, st));
    HIPCHK(fill_u32(T.reward, 2, 0u, st));
    HIPCHK(fill_u32(T.ctr, 10, 0u, st));
    HIPCHK(fill_u32(T.work, 4, 0u, st));
    HIPCHK(fill_u32(T.err, 4, 0u, st));
    HIPCHK(fill_u32(hist, (size_t)S + 1, 0u, st));

    const Plan &pl = R.pl;
    const uint32_t per_cu = std::max<uint32_t>(1u, (uint32_t)ctx->max_lds / std::max<uint32_t>(pl.lds, 1u));
    const int blocks = (int)std::min<uint64_t>((uint64_t)E, (uint64_t)ctx->cu_count * std::min<uint32_t>(per_cu, 8u));
    if (place) {
        // the claim word's 16-bit source field holds |K| plus at most one lost
        // add per wavefront of the launch
        if ((uint64_t)blocks * (uint64_t)pl.waves + (uint64_t)n + kMaxWaves >= 0x10000ull) return AMC_E_UNSUPPORTED;
        T.bscratch_words = pl.scratch_words;
        RCHK(A.alloc(4 * (size_t)pl.scratch_words * (size_t)blocks, &p));
        T.bscratch = (uint32_t *)p;
        // shared steps: claim and completion words, K and the helpers' B sums
        RCHK(A.alloc(16 * (size_t)blocks, &p));
        T.share = (unsigned long long *)p;
        const size_t open_words = ((size_t)blocks + 63) / 64;
        RCHK(A.alloc(8 * open_words, &p));
        T.open = (unsigned long long *)p;
        HIPCHK(fill_u32(T.open, 2 * open_words, 0u, st));
        RCHK(A.alloc(4 * (size_t)n * blocks, &p));
        T.glist = (int32_t *)p;
        RCHK(A.alloc(8 * (size_t)n * blocks, &p));
        T.hb = (double *)p;
        HIPCHK(fill_u32(T.share, 4 * (size_t)blocks, 0u, st));
        HIPCHK(fill_u32(T.hb, 2 * (size_t)n * blocks, 0u, st));
    }
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
    HIPCHK(launch_traj(T, pl.weighted, pl.dist16, place, pl.group, pl.adj_bytes, blocks, pl.waves, pl.lds, st));
    HIPCHK(hipEventRecord(ev[1], st));
    HIPCHK(traj_estimates(n, E, S, T.lengths, T.visits, T.ctr, hist, b_hat, surv, st));

    int herr = 0;
    unsigned long long hc[5] = {0, 0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(&herr, T.err, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hc, T.ctr, 8 * 5, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&out->reward_f, T.reward, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(out->lengths, T.lengths, 4 * (size_t)E, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(out->visits, T.visits, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
    if (T.paths) HIPCHK(hipMemcpyAsync(out->paths, T.paths, 4 * (size_t)E * S, hipMemcpyDeviceToHost, st));
    if (out->b_hat) HIPCHK(hipMemcpyAsync(out->b_hat, b_hat, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
    if (out->survival) HIPCHK(hipMemcpyAsync(out->survival, surv, 8 * (size_t)S, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (herr & 1) return AMC_E_SIGMA_OVERFLOW;
    if (herr & 2) return AMC_E_HIP;   // a shared step's completion was not seen in time
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ev[0], ev[1]));
    if (!tq->f) out->reward_f = 0.0;
    out->switches = hc[0];
    out->total_steps = hc[1];
    out->truncated = (int32_t)hc[2];
    out->sources = hc[3];
    out->shared_sources = hc[4];
    out->sweep_ms = ms;
    out->mode = pl.mode;
    out->waves = pl.waves;
    out->dist16 = pl.dist16 ? 1 : 0;
    out->b_global = place == 2 ? 1 : 0;
    return AMC_OK;
}
