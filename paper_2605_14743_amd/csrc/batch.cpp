// batch.cpp -- persistent fused launches over a batch of queries, captured
// once into a hipGraph and replayed.
//
// The queries of a batch are grouped by kernel variant (sweep mode, weight
// law, vertex mapping, 16/32-bit adjacency and, in the LDS mode, a wavefront
// count every member fits).  Each group is one persistent launch whose work
// queue is the concatenation of its members' (realization, tile) items,
// largest queries first, so graphs of different sizes and realizations of
// uneven surviving-edge counts share the device without a launch per graph.
// Groups run on separate streams (default priority); every member's tail
// follows its group's sweep on the same stream.  The whole device sequence
// -- counter resets (fill kernels), sweeps, tails -- is recorded by stream
// capture into one graph; amc_batch_run replays it and copies the results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "amc.h"
#include "amc_kernels.hpp"
#include "query.hpp"

namespace amc {

struct BatchGroup {
    Plan pl;
    std::vector<int> members;
    SweepParams *d_descs = nullptr;
    uint32_t *d_item_start = nullptr;
    unsigned int *work_ctr = nullptr;
    uint32_t *bscratch = nullptr;
    uint32_t bscratch_words = 0;
    uint32_t items = 0;
    int blocks = 0;
    int stream = 0;
};

}  // namespace amc

struct amc_batch {
    amc_ctx *ctx = nullptr;
    std::vector<std::unique_ptr<amc::QueryRun>> runs;
    std::vector<amc::BatchGroup> groups;
    amc::DevArena A;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

using namespace amc;

namespace {

int wave_bucket(int w) { return w >= 12 ? 12 : (w >= 8 ? 8 : (w >= 6 ? 6 : (w >= 4 ? 4 : 2))); }

void batch_free(amc_batch *b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (auto &r : b->runs)
        if (r) qr_release(*r, b->streams.empty() ? nullptr : b->streams[0]);
    if (!b->streams.empty()) (void)hipStreamSynchronize(b->streams[0]);
    b->A.release();
    for (auto e : b->events) (void)hipEventDestroy(e);
    if (b->t0) (void)hipEventDestroy(b->t0);
    if (b->t1) (void)hipEventDestroy(b->t1);
    for (auto s : b->streams) (void)hipStreamDestroy(s);
    delete b;
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

int build(amc_batch *b, int32_t count, const amc_graph *const *graphs, const amc_model *models,
          const amc_query *queries) {
    amc_ctx *ctx = b->ctx;
    const int nstreams = 4;
    for (int k = 0; k < nstreams; ++k) {
        hipStream_t s;
        HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        b->streams.push_back(s);
    }
    hipStream_t s0 = b->streams[0];
    b->A.stream = s0;
    b->A.async = ctx->async_alloc;
    HIPCHK(hipEventCreateWithFlags(&b->t0, hipEventDefault));
    HIPCHK(hipEventCreateWithFlags(&b->t1, hipEventDefault));
    // plan and allocate every member (whole realizations per work item)
    for (int i = 0; i < count; ++i) {
        if (!graphs[i] || graphs[i]->ctx != ctx) return AMC_E_INVALID_ARG;
        amc_query q = queries[i];
        if (q.flags & AMC_PLAIN_LAUNCH) return AMC_E_INVALID_ARG;
        if (q.tile <= 0) q.tile = graphs[i]->n;
        b->runs.emplace_back(new (std::nothrow) QueryRun());
        if (!b->runs.back()) return AMC_E_OOM;
        RCHK(qr_init(*b->runs.back(), ctx, graphs[i], &models[i], &q));
    }
    // group by kernel variant
    // every member of a group runs the group's kernel instantiation: the
    // per-source placement (distance width, path counts in LDS or scratch)
    // is part of the key
    struct Key {
        int mode, weighted, group, adj_bytes, waves, anchored, dist16, sig_global, state_place;
        bool operator==(const Key &o) const {
            return mode == o.mode && weighted == o.weighted && group == o.group && adj_bytes == o.adj_bytes &&
                   waves == o.waves && anchored == o.anchored && dist16 == o.dist16 && sig_global == o.sig_global &&
                   state_place == o.state_place;
        }
    };
    std::vector<Key> keys;
    for (int i = 0; i < count; ++i) {
        const Plan &pl = b->runs[i]->pl;
        const bool per_wave = pl.mode != AMC_MODE_BLOCK;
        // a member may run with fewer wavefronts than planned as long as the
        // wavefront regions still hold the staging and reduction scratch
        int w = pl.threads / 64;
        if (per_wave && !pl.anchored) {
            w = wave_bucket(pl.waves);
            const uint64_t need = std::max<uint64_t>(2ull * (uint64_t)b->runs[i]->g->m,
                                                     kReduceBytesPerVertex * (uint64_t)b->runs[i]->g->n);
            if ((uint64_t)pl.wave_bytes * (uint64_t)w < need) w = pl.waves;
        }
        if (pl.anchored) w = pl.waves;
        Key k{pl.mode, pl.weighted ? 1 : 0, per_wave ? pl.group : 0, (int)pl.adj_bytes, w,
              pl.anchored ? 1 : 0, pl.dist16 ? 1 : 0, pl.sig_global ? 1 : 0, pl.state_place};
        size_t gi = 0;
        while (gi < keys.size() && !(keys[gi] == k)) ++gi;
        if (gi == keys.size()) {
            keys.push_back(k);
            b->groups.emplace_back();
            BatchGroup &G = b->groups.back();
            G.pl = pl;
            G.pl.waves = k.waves;
            G.pl.threads = 64 * k.waves;
            G.pl.lds = 0;
        }
        b->groups[gi].members.push_back(i);
    }
    // per member: the plan's waves/lds become the group's; allocate
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        BatchGroup &G = b->groups[gi];
        uint64_t cost_total = 0;
        std::sort(G.members.begin(), G.members.end(), [&](int x, int y) {
            const QueryRun &a = *b->runs[x], &c = *b->runs[y];
            const double ca = (double)a.q.R * a.g->n * (double)(a.g->m + a.g->n);
            const double cc = (double)c.q.R * c.g->n * (double)(c.g->m + c.g->n);
            return ca > cc;
        });
        for (int i : G.members) {
            QueryRun &R = *b->runs[i];
            if (G.pl.anchored) {
                R.pl.lds = lds_bytes_anchored(R.g->n, R.pl.adj_cap, R.pl.adj_bytes, G.pl.waves, &R.pl.wave_bytes);
            } else if (G.pl.mode == AMC_MODE_WAVE || G.pl.mode == AMC_MODE_WAVE_L2) {
                R.pl.waves = G.pl.waves;
                R.pl.threads = G.pl.threads;
                R.pl.lds = G.pl.mode == AMC_MODE_WAVE
                               ? lds_bytes_wave(R.g->n, R.pl.adj_cap, R.pl.adj_bytes, G.pl.waves, R.pl.dist16,
                                                &R.pl.wave_bytes)
                               : lds_bytes_wave_l2(R.g->n, G.pl.waves, R.pl.dist16, R.pl.b_global, R.pl.sig_global,
                                                   &R.pl.wave_bytes);
            }
            G.pl.lds = std::max(G.pl.lds, R.pl.lds);
            G.bscratch_words = std::max<uint32_t>(G.bscratch_words, R.pl.scratch_words);
            R.pl.blocks = 0;   // the group launch owns the workgroups
            RCHK(qr_alloc(R, s0));
            cost_total += R.pl.items;
        }
        if (cost_total > 0xFFFFFFFFull) return AMC_E_UNSUPPORTED;
        std::vector<SweepParams> descs;
        std::vector<uint32_t> starts{0u};
        for (int i : G.members) {
            descs.push_back(b->runs[i]->P);
            starts.push_back(starts.back() + (uint32_t)b->runs[i]->pl.items);
        }
        G.items = starts.back();
        void *p;
        RCHK(b->A.alloc(sizeof(SweepParams) * descs.size(), &p));
        G.d_descs = (SweepParams *)p;
        HIPCHK(hipMemcpyAsync(p, descs.data(), sizeof(SweepParams) * descs.size(), hipMemcpyHostToDevice, s0));
        RCHK(b->A.alloc(4 * starts.size(), &p));
        G.d_item_start = (uint32_t *)p;
        HIPCHK(hipMemcpyAsync(p, starts.data(), 4 * starts.size(), hipMemcpyHostToDevice, s0));
        RCHK(b->A.alloc(16, &p));
        G.work_ctr = (unsigned int *)p;
        const uint32_t per_cu = std::max<uint32_t>(1u, (uint32_t)ctx->max_lds / std::max<uint32_t>(G.pl.lds, 1u));
        const uint32_t cap = G.bscratch_words > 0 ? kMaxScratchBlocksPerCu : 8u;
        G.blocks = (int)std::min<uint64_t>(G.items, (uint64_t)ctx->cu_count * std::min<uint32_t>(per_cu, cap));
        if (G.bscratch_words > 0) {
            RCHK(b->A.alloc(4 * (size_t)G.bscratch_words * G.blocks, &p));
            G.bscratch = (uint32_t *)p;
        }
        G.stream = (int)(gi % b->streams.size());
        HIPCHK(hipStreamSynchronize(s0));
    }
    // record the device sequence
    const int ns = (int)std::min<size_t>(b->streams.size(), b->groups.size());
    for (int k = 0; k < 1 + 2 * ns; ++k) {
        hipEvent_t e;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        b->events.push_back(e);
    }
    HIPCHK(hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal));
    int rc = AMC_OK;
    for (auto &R : b->runs)
        if (rc == AMC_OK) rc = qr_enqueue_reset(*R, s0);
    for (auto &G : b->groups)
        if (rc == AMC_OK && fill_u32(G.work_ctr, 4, 0u, s0) != hipSuccess) rc = AMC_E_HIP;
    if (rc == AMC_OK && hipEventRecord(b->events[0], s0) != hipSuccess) rc = AMC_E_HIP;
    for (int k = 1; k < ns && rc == AMC_OK; ++k)
        if (hipStreamWaitEvent(b->streams[k], b->events[0], 0) != hipSuccess) rc = AMC_E_HIP;
    for (auto &G : b->groups) {
        if (rc != AMC_OK) break;
        hipStream_t st = b->streams[G.stream];
        LaunchCtl LC;
        std::memset(&LC, 0, sizeof(LC));
        LC.descs = G.d_descs;
        LC.item_start = G.d_item_start;
        LC.nq = (int32_t)G.members.size();
        LC.n_items = G.items;
        LC.work_ctr = G.work_ctr;
        LC.bscratch = G.bscratch;
        LC.bscratch_words = G.bscratch_words;
        hipError_t e = G.pl.anchored
                           ? launch_anchored(LC, G.pl.weighted, G.pl.adj_bytes, G.blocks, G.pl.waves, G.pl.lds, st)
                       : G.pl.mode == AMC_MODE_BLOCK
                           ? launch_sweep_block(LC, G.pl.weighted, G.pl.state_place, G.blocks, G.pl.threads,
                                                G.pl.lds, st)
                           : launch_sweep_wave(LC, G.pl.weighted, G.pl.mode == AMC_MODE_WAVE_L2, G.pl.dist16, G.pl.sig_global,
                                               G.pl.group, G.pl.adj_bytes, G.blocks, G.pl.waves, G.pl.lds, st);
        if (e != hipSuccess) {
            rc = AMC_E_HIP;
            break;
        }
        for (int i : G.members) {
            b->runs[i]->launches = 1;
            if (rc == AMC_OK) rc = qr_enqueue_post(*b->runs[i], st);
            if (rc == AMC_OK) rc = qr_enqueue_tail(*b->runs[i], st, false);
        }
    }
    for (int k = 1; k < ns && rc == AMC_OK; ++k) {
        if (hipEventRecord(b->events[k], b->streams[k]) != hipSuccess ||
            hipStreamWaitEvent(s0, b->events[k], 0) != hipSuccess)
            rc = AMC_E_HIP;
    }
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(s0, &graph);
    if (rc != AMC_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return rc;
    }
    if (ec != hipSuccess || !graph) {
        (void)hipGetLastError();
        return AMC_E_HIP;
    }
    b->graph = graph;
    HIPCHK(hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0));
    return AMC_OK;
}

}  // namespace

extern "C" int amc_batch_create(amc_ctx *ctx, int32_t count, const amc_graph *const *graphs,
                                const amc_model *models, const amc_query *queries, amc_batch **out) {
    if (!ctx || count < 1 || !graphs || !models || !queries || !out) return AMC_E_INVALID_ARG;
    *out = nullptr;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return AMC_E_HIP;
    amc_batch *b = new (std::nothrow) amc_batch();
    if (!b) return AMC_E_OOM;
    b->ctx = ctx;
    const int rc = build(b, count, graphs, models, queries);
    if (rc != AMC_OK) {
        batch_free(b);
        return rc;
    }
    *out = b;
    return AMC_OK;
}

extern "C" int amc_batch_run(amc_batch *b, amc_result *results) {
    if (!b || !results) return AMC_E_INVALID_ARG;
    for (size_t i = 0; i < b->runs.size(); ++i) {
        if (!results[i].counts) return AMC_E_INVALID_ARG;
        if (b->runs[i]->q.pool_size > 0 && !results[i].counts_w) return AMC_E_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lk(b->ctx->mu);
    if (hipSetDevice(b->ctx->device) != hipSuccess) return AMC_E_HIP;
    hipStream_t s0 = b->streams[0];
    HIPCHK(hipEventRecord(b->t0, s0));
    HIPCHK(hipGraphLaunch(b->exec, s0));
    HIPCHK(hipEventRecord(b->t1, s0));
    HIPCHK(hipStreamSynchronize(s0));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, b->t0, b->t1));
    int first = AMC_OK;
    for (size_t i = 0; i < b->runs.size(); ++i) {
        const int rc = qr_finish(*b->runs[i], &results[i], s0);
        results[i].stats.sweep_ms = ms;   // the whole batch graph (sweeps and tails)
        results[i].stats.tail_ms = 0.0;
        if (rc != AMC_OK && first == AMC_OK) first = rc;
    }
    return first;
}

extern "C" int amc_batch_info(amc_batch *b, int32_t *n_groups, int32_t *items) {
    if (!b) return AMC_E_INVALID_ARG;
    if (n_groups) *n_groups = (int32_t)b->groups.size();
    if (items) {
        uint64_t t = 0;
        for (auto &G : b->groups) t += G.items;
        *items = (int32_t)std::min<uint64_t>(t, 0x7FFFFFFF);
    }
    return AMC_OK;
}

extern "C" void amc_batch_destroy(amc_batch *b) {
    if (!b) return;
    std::lock_guard<std::mutex> lk(b->ctx->mu);
    (void)hipSetDevice(b->ctx->device);
    batch_free(b);
}
