// tune.cpp -- autotuner of the sweep configuration.
//
// For one graph and query it times every feasible configuration on a few
// realizations (counts only) and keeps the fastest for the graph's shape.
// The per-context cache is consulted by the planner whenever a query leaves
// mode, vertex mapping and wavefront count open; AMC_TUNE_CACHE names an
// optional text file ("n m weight_kind w_max mode group waves rate" per line)
// that is read at context creation and appended to after each tuning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "amc.h"
#include "amc_runtime.hpp"

namespace amc {

TuneKey tune_key(const amc_graph *g, const amc_model *md) {
    const uint32_t wmax = (uint32_t)model_wmax(g, md);
    return TuneKey{g->n, g->m, md->weight_kind == AMC_WEIGHT_UNIT ? 0 : 1, wmax};
}

void tune_load(amc_ctx *ctx) {
    const char *path = std::getenv("AMC_TUNE_CACHE");
    if (!path || !*path) return;
    ctx->tune_path = path;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    int n, wk, mode, group, waves;
    long long m;
    unsigned wmax;
    double rate;
    while (std::fscanf(f, "%d %lld %d %u %d %d %d %lf", &n, &m, &wk, &wmax, &mode, &group, &waves, &rate) == 8) {
        // entries the planner could not honour are ignored
        const bool mode_ok = mode == AMC_MODE_WAVE || mode == AMC_MODE_BLOCK || mode == AMC_MODE_WAVE_L2;
        const bool group_ok = group == 0 || group == 1 || group == 2 || group == 3 || group == 4 || group == 8 ||
                              group == 16;
        if (mode_ok && group_ok && waves >= 0 && waves <= 16)
            ctx->tune[TuneKey{n, (int64_t)m, wk, wmax}] = TuneChoice{mode, group, waves, rate};
    }
    std::fclose(f);
}

}  // namespace amc

using namespace amc;

extern "C" int amc_tune(amc_ctx *ctx, const amc_graph *g, const amc_model *model, const amc_query *q,
                        uint32_t probe_R, amc_tune_result *out) {
    if (!ctx || !g || !model || !q || !out || g->ctx != ctx || probe_R == 0) return AMC_E_INVALID_ARG;
    struct Cand {
        int mode, group;
    };
    const Cand cands[] = {{AMC_MODE_WAVE, 1},    {AMC_MODE_WAVE, 2},    {AMC_MODE_WAVE, 3},
                          {AMC_MODE_WAVE, 8},    {AMC_MODE_WAVE, 16},   {AMC_MODE_WAVE_L2, 1},
                          {AMC_MODE_WAVE_L2, 3}, {AMC_MODE_WAVE_L2, 8}, {AMC_MODE_BLOCK, 0}};
    amc_query pq = *q;
    pq.R = probe_R;
    pq.flags = AMC_SKIP_TAIL;
    pq.n_debug = 0;
    pq.debug_pairs = nullptr;
    pq.tile = 0;
    pq.waves = 0;
    std::vector<uint32_t> counts((size_t)g->n * (g->n + 1)), counts_w;
    if (q->pool_size > 0) counts_w.resize(counts.size());
    TuneChoice best{0, 0, 0, -1.0};
    int tried = 0;
    for (const Cand &c : cands) {
        pq.mode = c.mode;
        pq.group = c.group;
        amc_result res{};
        res.counts = counts.data();
        res.counts_w = counts_w.empty() ? nullptr : counts_w.data();
        int rc;
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            if (hipSetDevice(ctx->device) != hipSuccess) return AMC_E_HIP;
            rc = run_query(ctx, g, model, &pq, &res, ctx->stream);
        }
        if (rc == AMC_E_UNSUPPORTED) continue;
        if (rc != AMC_OK) return rc;
        ++tried;
        const double rate = (double)probe_R * g->n / (res.stats.sweep_ms * 1e-3);
        if (rate > best.units_per_s) best = TuneChoice{c.mode, c.mode == AMC_MODE_BLOCK ? 0 : c.group,
                                                       res.stats.waves, rate};
    }
    if (tried == 0) return AMC_E_UNSUPPORTED;
    {
        std::lock_guard<std::mutex> lk(ctx->tune_mu);
        const TuneKey key = tune_key(g, model);
        ctx->tune[key] = best;
        if (!ctx->tune_path.empty()) {
            FILE *f = std::fopen(ctx->tune_path.c_str(), "a");
            if (f) {
                std::fprintf(f, "%d %lld %d %u %d %d %d %.6g\n", std::get<0>(key), (long long)std::get<1>(key),
                             std::get<2>(key), std::get<3>(key), best.mode, best.group, best.waves, best.units_per_s);
                std::fclose(f);
            }
        }
    }
    out->mode = best.mode;
    out->group = best.group;
    out->waves = best.waves;
    out->units_per_s = best.units_per_s;
    out->candidates = tried;
    return AMC_OK;
}
