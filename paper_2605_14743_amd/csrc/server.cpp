// server.cpp -- serving loop behind amc_submit / amc_poll / amc_wait:
// continuous batching of queries into shared persistent sweep launches.
//
// Queries wait in a FIFO and are admitted when their device footprint fits
// the context budget minus what admitted queries hold (first fit in arrival
// order; a query passed over kMaxBypass times blocks later arrivals until it
// fits).  Admission allocates the query's buffers (counts, exchange rows,
// chain state) and plans its work items (realization, source tile), with
// tiles small enough that one item stays short.
//
// One scheduler thread runs the device through kLanes lanes (a stream and a
// per-workgroup scratch each).  Admitted queries are grouped by kernel
// variant (sweep mode, weight law, vertex mapping, adjacency and distance
// widths, anchored or not, planned wavefronts per workgroup).  Whenever a
// lane is idle the scheduler launches an epoch on it: one persistent sweep
// over a contiguous range of items of each of several admitted queries of one
// variant -- the query with the least remaining work, then others of its
// variant in the same order -- up to a work budget of about kEpochMs.  A
// query that arrives while others run is admitted and joins the next epoch,
// so the items of several queries run inside one launch, and the lanes
// overlap so that one epoch's last items share the device with the next
// epoch's first.  A query whose last items have finished gets its Top-k
// stage and tail on a side stream; a finisher thread copies its results out,
// frees its buffers and completes the request.  Counts and chain state stay
// on the device until then.  The lanes are few on purpose: the device has
// four hardware queues per process, and streams beyond them would queue
// epochs behind one another.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>

#include "amc.h"
#include "amc_kernels.hpp"
#include "query.hpp"

namespace amc {

namespace {
double now_s() {
    using namespace std::chrono;
    return duration_cast<duration<double>>(steady_clock::now().time_since_epoch()).count();
}
constexpr int kMaxBypass = 8;
constexpr int kMaxMembers = 64;        // queries in one epoch launch
constexpr int kLanes = 3;              // epochs in flight at once
constexpr double kEpochMs = 30.0;       // work budget of one epoch
constexpr double kItemMs = 10.0;        // target duration of one work item on one workgroup
// rate of one wavefront in work units (sources x (surviving slots +
// vertices)) per millisecond, measured on MI355X in the L2 mode (ws1000: 1e7
// sources of 10.5 k units in 400 ms on 256 x 11 wavefronts); a
// workgroup-per-source workgroup counts as kBlockWaves wavefronts (er5000:
// 3.0 M sources/s of 41 k units on 256 workgroups)
constexpr double kWaveRate = 9.0e4;
constexpr double kBlockWaves = 5.0;
// a variant's starting rate in the same units for the whole chip is
// kWaveRate x wavefronts x CUs; it is refined from each epoch's events
constexpr double kRate0 = 2.0e8;
}  // namespace

struct Request {
    amc_ctx *ctx = nullptr;
    const amc_graph *g = nullptr;
    amc_model model{};
    ModelInputs min;
    amc_query q{};
    QueryInputs in;
    amc_result *out = nullptr;
    uint64_t footprint = 0;
    int status = AMC_E_NOT_READY;
    bool done = false;
    int bypassed = 0;
    double t_submit = 0, t_admit = 0, t_finish = 0;
    std::mutex mu;
    std::condition_variable cv;
};

// An admitted query.
struct Member {
    std::shared_ptr<Request> req;
    std::unique_ptr<QueryRun> run;
    int variant = -1;
    uint32_t items = 0, next = 0;   // items in total, first one not yet launched
    int inflight = 0;               // epochs in flight carrying its items
    double work_per_item = 1.0;
    int launches = 0;
    bool failed = false;
    int fail_rc = AMC_OK;
    hipEvent_t tail_done = nullptr;
    double t_sweep_done = 0;
};

struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t start = nullptr, end = nullptr;
    uint32_t *bscratch = nullptr;
    size_t bscratch_bytes = 0;
    SweepParams *h_descs = nullptr, *d_descs = nullptr;   // pinned staging / device table
    uint32_t *h_start = nullptr, *d_start = nullptr;      // nq + 1
    uint32_t *h_off = nullptr, *d_off = nullptr;          // nq
    unsigned int *d_ctr = nullptr;
    bool busy = false;
    double work = 0.0;
    int variant = -1;
    std::vector<Member *> members;
};

struct Variant {
    // dist16: bit 0 = 16-bit distances, bit 1 = path counts in the scratch,
    // bit 2 = workgroup-mode state in the scratch
    int mode = 0, weighted = 0, group = 0, adj_bytes = 0, dist16 = 0, anchored = 0, waves = 0;
    double rate = kRate0, rate0 = kRate0;   // estimated and modelled chip-wide work units per ms
};

struct Server {
    amc_ctx *ctx = nullptr;
    std::mutex mu;                  // pending, in_use, stop, st
    std::condition_variable cv;
    std::deque<std::shared_ptr<Request>> pending;
    uint64_t in_use = 0;
    bool stop = false;
    amc_server_stats st{};
    // scheduler-thread state
    std::vector<std::unique_ptr<Member>> active;
    std::vector<std::unique_ptr<Variant>> variants;
    Lane lanes[kLanes];
    hipStream_t alloc_stream = nullptr, tail_stream = nullptr;
    std::thread scheduler, finisher;
    // finisher hand-off
    std::mutex fin_mu;
    std::condition_variable fin_cv;
    std::deque<std::unique_ptr<Member>> finished;
    bool fin_stop = false;
    hipStream_t fin_stream = nullptr;

    // Picks the next admissible request (caller holds mu); null if none fits.
    std::shared_ptr<Request> pick() {
        for (size_t k = 0; k < pending.size(); ++k) {
            auto &r = pending[k];
            if (in_use + r->footprint <= ctx->budget) {
                auto got = r;
                for (size_t j = 0; j < k; ++j) pending[j]->bypassed++;
                pending.erase(pending.begin() + (long)k);
                return got;
            }
            if (r->bypassed >= kMaxBypass) break;   // starving head: nothing behind it may pass
        }
        return nullptr;
    }

    void complete(const std::shared_ptr<Request> &r, int rc) {
        {
            std::lock_guard<std::mutex> lk(r->mu);
            r->status = rc;
            r->t_finish = now_s();
            r->done = true;
        }
        r->cv.notify_all();
    }

    void release_budget(uint64_t fp) {
        {
            std::lock_guard<std::mutex> lk(mu);
            in_use -= fp;
            st.completed++;
        }
        cv.notify_all();
    }

    // Work units one workgroup of this plan processes per millisecond.
    static double wg_rate(const Plan &pl) {
        return kWaveRate * (pl.mode == AMC_MODE_BLOCK ? kBlockWaves : (double)std::max(1, pl.waves));
    }

    int variant_of(const Plan &pl) {
        const int key[7] = {pl.mode, pl.weighted ? 1 : 0, pl.mode == AMC_MODE_BLOCK ? 0 : pl.group,
                            (int)pl.adj_bytes,
                            (pl.dist16 ? 1 : 0) | (pl.sig_global ? 2 : 0) | (pl.state_place << 2),
                            pl.anchored ? 1 : 0,
                            pl.mode == AMC_MODE_BLOCK ? pl.threads / 64 : pl.waves};
        for (size_t i = 0; i < variants.size(); ++i) {
            const Variant &v = *variants[i];
            if (v.mode == key[0] && v.weighted == key[1] && v.group == key[2] && v.adj_bytes == key[3] &&
                v.dist16 == key[4] && v.anchored == key[5] && v.waves == key[6])
                return (int)i;
        }
        auto v = std::make_unique<Variant>();
        v->mode = key[0];
        v->weighted = key[1];
        v->group = key[2];
        v->adj_bytes = key[3];
        v->dist16 = key[4];
        v->anchored = key[5];
        v->waves = key[6];
        v->rate = v->rate0 = wg_rate(pl) * std::max(1, ctx->cu_count);
        variants.push_back(std::move(v));
        return (int)variants.size() - 1;
    }

    int make_lanes() {
        for (Lane &L : lanes) {
            bool ok = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) == hipSuccess &&
                      hipEventCreate(&L.start) == hipSuccess && hipEventCreate(&L.end) == hipSuccess &&
                      hipHostMalloc((void **)&L.h_descs, sizeof(SweepParams) * kMaxMembers) == hipSuccess &&
                      hipHostMalloc((void **)&L.h_start, 4 * (kMaxMembers + 1)) == hipSuccess &&
                      hipHostMalloc((void **)&L.h_off, 4 * kMaxMembers) == hipSuccess &&
                      hipMalloc((void **)&L.d_descs, sizeof(SweepParams) * kMaxMembers) == hipSuccess &&
                      hipMalloc((void **)&L.d_start, 4 * (kMaxMembers + 1)) == hipSuccess &&
                      hipMalloc((void **)&L.d_off, 4 * kMaxMembers) == hipSuccess &&
                      hipMalloc((void **)&L.d_ctr, 16) == hipSuccess;
            if (!ok) {
                (void)hipGetLastError();
                return AMC_E_HIP;
            }
        }
        return AMC_OK;
    }

    void free_lanes() {
        for (Lane &L : lanes) {
            if (L.stream) (void)hipStreamSynchronize(L.stream);
            if (L.bscratch) (void)hipFree(L.bscratch);
            if (L.d_descs) (void)hipFree(L.d_descs);
            if (L.d_start) (void)hipFree(L.d_start);
            if (L.d_off) (void)hipFree(L.d_off);
            if (L.d_ctr) (void)hipFree(L.d_ctr);
            if (L.h_descs) (void)hipHostFree(L.h_descs);
            if (L.h_start) (void)hipHostFree(L.h_start);
            if (L.h_off) (void)hipHostFree(L.h_off);
            if (L.start) (void)hipEventDestroy(L.start);
            if (L.end) (void)hipEventDestroy(L.end);
            if (L.stream) (void)hipStreamDestroy(L.stream);
            L = Lane();
        }
        variants.clear();
    }

    // Admission of one request: plan with short items, allocate, clear.
    int admit(const std::shared_ptr<Request> &r, std::unique_ptr<Member> &out) {
        auto m = std::make_unique<Member>();
        m->req = r;
        m->run.reset(new (std::nothrow) QueryRun());
        if (!m->run) return AMC_E_OOM;
        QueryRun &R = *m->run;
        amc_query q = r->q;
        q.flags &= ~(uint32_t)AMC_PLAIN_LAUNCH;     // the loop decides the launches
        const amc_graph *g = r->g;
        // work of one source: its surviving slots and vertices (expected)
        const double wps = 2.0 * (double)g->m * (1.0 - std::min(1.0, std::max(0.0, r->model.p_fail))) + g->n;
        if (q.tile <= 0) {
            // items short enough that a query arriving later waits for at
            // most about one item per workgroup before its own epoch starts
            Plan p0;
            int rc = validate(g, &r->model, &q);
            if (rc == AMC_OK) rc = plan(ctx, g, &r->model, &q, &p0);
            if (rc != AMC_OK) return rc;
            const int cap = (int)std::max(1.0, std::floor(kItemMs * wg_rate(p0) / std::max(wps, 1.0)));
            q.tile = std::max(1, std::min(p0.tile, std::max(cap, p0.mode == AMC_MODE_BLOCK ? 1 : p0.waves)));
        }
        int rc = qr_init(R, ctx, g, &r->model, &q);
        if (rc != AMC_OK) return rc;
        R.pl.blocks = 0;                 // the lanes own the per-workgroup scratch
        rc = qr_alloc(R, alloc_stream);
        if (rc == AMC_OK) rc = qr_enqueue_reset(R, alloc_stream);
        if (rc == AMC_OK && hipStreamSynchronize(alloc_stream) != hipSuccess) rc = AMC_E_HIP;
        if (rc == AMC_OK && hipEventCreateWithFlags(&m->tail_done, hipEventDisableTiming) != hipSuccess)
            rc = AMC_E_HIP;
        if (rc != AMC_OK) {
            (void)hipGetLastError();
            qr_release(R, alloc_stream);
            return rc;
        }
        m->variant = variant_of(R.pl);
        m->items = (uint32_t)R.pl.items;
        m->work_per_item = std::max(1.0, (double)R.pl.tile * wps);
        out = std::move(m);
        return AMC_OK;
    }

    // Launches one epoch on lane L; false if nothing to run.  The epoch
    // serves the query with the least remaining work and, up to the budget,
    // other queries of its variant in the same order.
    bool launch_epoch(Lane &L) {
        std::vector<Member *> cand;
        for (auto &m : active)
            if (!m->failed && m->next < m->items) cand.push_back(m.get());
        if (cand.empty()) return false;
        std::stable_sort(cand.begin(), cand.end(), [](const Member *a, const Member *b) {
            return (double)(a->items - a->next) * a->work_per_item < (double)(b->items - b->next) * b->work_per_item;
        });
        Variant &V = *variants[cand[0]->variant];
        const double budget = V.rate * kEpochMs;
        const int cu = std::max(1, ctx->cu_count);
        const int waves = V.waves;
        std::vector<Member *> pick;
        std::vector<uint32_t> take;
        double work = 0.0;
        for (Member *m : cand) {
            if ((int)pick.size() == kMaxMembers || work >= budget) break;
            if (&*variants[m->variant] != &V) continue;
            const double left = budget - work;
            uint32_t k = (uint32_t)std::ceil(left / m->work_per_item);
            // at least one round of the grid's workgroups, never past the query's end
            k = std::max<uint32_t>(k, (uint32_t)cu);
            k = std::min<uint32_t>(k, m->items - m->next);
            pick.push_back(m);
            take.push_back(k);
            work += k * m->work_per_item;
        }
        if (pick.empty()) return false;
        // launch shape: the most LDS any member needs at `waves` wavefronts
        uint32_t lds = 0;
        size_t words = 0;
        for (Member *m : pick) {
            const QueryRun &R = *m->run;
            const Plan &pl = R.pl;
            uint32_t wb = 0;
            uint32_t l = pl.anchored ? lds_bytes_anchored(R.g->n, pl.adj_cap, pl.adj_bytes, waves, &wb)
                         : pl.mode == AMC_MODE_WAVE ? lds_bytes_wave(R.g->n, pl.adj_cap, pl.adj_bytes, waves,
                                                                     pl.dist16, &wb)
                         : pl.mode == AMC_MODE_WAVE_L2 ? lds_bytes_wave_l2(R.g->n, waves, pl.dist16, pl.b_global, pl.sig_global,
                                                                           &wb)
                                                       : pl.lds;
            lds = std::max(lds, l);
            words = std::max<size_t>(words, pl.scratch_words);
        }
        const Plan &p0 = pick[0]->run->pl;
        const int threads = p0.mode == AMC_MODE_BLOCK ? p0.threads : 64 * waves;
        const uint32_t per_cu = std::max<uint32_t>(1u, (uint32_t)ctx->max_lds / std::max<uint32_t>(lds, 1u));
        const uint32_t capcu = words > 0 ? kMaxScratchBlocksPerCu : 8u;
        uint32_t total = 0;
        for (uint32_t k : take) total += k;
        const int blocks = (int)std::min<uint64_t>(total, (uint64_t)cu * std::min(per_cu, capcu));
        if (words > 0 && 4 * words * (size_t)blocks > L.bscratch_bytes) {
            (void)hipStreamSynchronize(L.stream);
            if (L.bscratch) (void)hipFree(L.bscratch);
            L.bscratch = nullptr;
            L.bscratch_bytes = 0;
            if (hipMalloc((void **)&L.bscratch, 4 * words * (size_t)blocks) != hipSuccess) {
                (void)hipGetLastError();
                for (Member *m : pick) fail(*m, AMC_E_OOM);
                return true;
            }
            L.bscratch_bytes = 4 * words * (size_t)blocks;
        }
        // the epoch's table: descriptors, item ranges and offsets
        L.h_start[0] = 0;
        for (size_t i = 0; i < pick.size(); ++i) {
            L.h_descs[i] = pick[i]->run->P;
            L.h_off[i] = pick[i]->next;
            L.h_start[i + 1] = L.h_start[i] + take[i];
        }
        const size_t nq = pick.size();
        bool ok = hipMemcpyAsync(L.d_descs, L.h_descs, sizeof(SweepParams) * nq, hipMemcpyHostToDevice,
                                 L.stream) == hipSuccess &&
                  hipMemcpyAsync(L.d_start, L.h_start, 4 * (nq + 1), hipMemcpyHostToDevice, L.stream) == hipSuccess &&
                  hipMemcpyAsync(L.d_off, L.h_off, 4 * nq, hipMemcpyHostToDevice, L.stream) == hipSuccess &&
                  fill_u32(L.d_ctr, 4, 0u, L.stream) == hipSuccess &&
                  hipEventRecord(L.start, L.stream) == hipSuccess;
        if (ok) {
            LaunchCtl LC;
            std::memset(&LC, 0, sizeof(LC));
            LC.descs = L.d_descs;
            LC.item_start = L.d_start;
            LC.item_off = L.d_off;
            LC.nq = (int32_t)nq;
            LC.n_items = total;
            LC.work_ctr = L.d_ctr;
            LC.bscratch = L.bscratch;
            LC.bscratch_words = (uint32_t)words;
            const hipError_t e =
                p0.anchored ? launch_anchored(LC, p0.weighted, p0.adj_bytes, blocks, waves, lds, L.stream)
                : p0.mode == AMC_MODE_BLOCK
                    ? launch_sweep_block(LC, p0.weighted, p0.state_place, blocks, threads, lds, L.stream)
                    : launch_sweep_wave(LC, p0.weighted, p0.mode == AMC_MODE_WAVE_L2, p0.dist16, p0.sig_global, p0.group,
                                        p0.adj_bytes, blocks, waves, lds, L.stream);
            ok = e == hipSuccess && hipEventRecord(L.end, L.stream) == hipSuccess;
        }
        if (!ok) {
            (void)hipGetLastError();
            for (Member *m : pick) fail(*m, AMC_E_HIP);
            return true;
        }
        L.busy = true;
        L.work = work;
        L.variant = cand[0]->variant;
        L.members = pick;
        for (size_t i = 0; i < pick.size(); ++i) {
            pick[i]->next += take[i];
            pick[i]->inflight++;
            pick[i]->launches++;
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            st.launches++;
            if (nq >= 2) st.shared_launches++;
            st.max_members = std::max(st.max_members, (int32_t)nq);
        }
        return true;
    }

    void fail(Member &m, int rc) {
        if (!m.failed) {
            m.failed = true;
            m.fail_rc = rc;
        }
    }

    // An epoch on lane L has finished: account it, start the tails of the
    // members whose last items it carried.
    void epoch_done(Lane &L) {
        float ms = 0.f;
        if (L.variant >= 0 && hipEventElapsedTime(&ms, L.start, L.end) == hipSuccess && ms > 0.f && L.work > 0.0) {
            // an epoch's rate while it shares the chip with other lanes is a
            // lower bound of the variant's; the estimate moves a third of the
            // way and stays within a factor of 4 of the model
            Variant &V = *variants[L.variant];
            const double model = V.rate0;
            const double r = std::min(4.0 * model, std::max(model / 4.0, L.work / ms));
            V.rate = 0.67 * V.rate + 0.33 * r;
        }
        (void)hipGetLastError();
        L.busy = false;
        for (Member *m : L.members) {
            m->inflight--;
            if (m->inflight == 0 && (m->next >= m->items || m->failed)) start_tail(*m, L);
        }
        L.members.clear();
    }

    void start_tail(Member &m, Lane &L) {
        m.t_sweep_done = now_s();
        QueryRun &R = *m.run;
        int rc = m.failed ? m.fail_rc : AMC_OK;
        if (rc == AMC_OK && hipStreamWaitEvent(tail_stream, L.end, 0) != hipSuccess) rc = AMC_E_HIP;
        if (rc == AMC_OK) rc = qr_enqueue_post(R, tail_stream);
        if (rc == AMC_OK) rc = qr_enqueue_tail(R, tail_stream, false);
        if (rc == AMC_OK && hipEventRecord(m.tail_done, tail_stream) != hipSuccess) rc = AMC_E_HIP;
        if (rc != AMC_OK) {
            (void)hipGetLastError();
            fail(m, rc);
            (void)hipStreamSynchronize(tail_stream);
            (void)hipEventRecord(m.tail_done, tail_stream);
        }
        m.next = m.items;                // nothing more to launch
        m.inflight = -1;                 // marks "tail enqueued"
    }

    void scheduler_loop() {
        (void)hipSetDevice(ctx->device);
        for (;;) {
            bool progress = false;
            // admissions
            for (;;) {
                std::shared_ptr<Request> r;
                {
                    std::lock_guard<std::mutex> lk(mu);
                    if (stop && pending.empty() && active.empty()) {
                        finish_all();
                        return;
                    }
                    r = pick();
                    if (r) {
                        in_use += r->footprint;
                        st.admitted++;
                        st.peak_in_use = std::max(st.peak_in_use, in_use);
                    }
                }
                if (!r) break;
                progress = true;
                r->t_admit = now_s();
                std::unique_ptr<Member> m;
                const int rc = admit(r, m);
                if (rc != AMC_OK) {
                    release_budget(r->footprint);
                    complete(r, rc);
                    continue;
                }
                active.push_back(std::move(m));
                std::lock_guard<std::mutex> lk(mu);
                st.peak_active = std::max(st.peak_active, (int32_t)active.size());
            }
            // finished epochs
            for (Lane &L : lanes)
                if (L.busy && hipEventQuery(L.end) == hipSuccess) {
                    epoch_done(L);
                    progress = true;
                }
            (void)hipGetLastError();
            // a member that failed with no epoch in flight skips its tail
            for (auto &m : active)
                if (m->failed && m->inflight == 0) {
                    m->t_sweep_done = now_s();
                    if (hipEventRecord(m->tail_done, tail_stream) != hipSuccess) {
                        (void)hipGetLastError();
                        (void)hipStreamSynchronize(tail_stream);
                    }
                    m->next = m->items;
                    m->inflight = -1;
                    progress = true;
                }
            // new epochs on idle lanes
            for (Lane &L : lanes)
                if (!L.busy && launch_epoch(L)) progress = true;
            // members whose tail has finished go to the finisher
            for (size_t i = 0; i < active.size();) {
                Member &m = *active[i];
                if (m.inflight == -1 && hipEventQuery(m.tail_done) == hipSuccess) {
                    {
                        std::lock_guard<std::mutex> lk(fin_mu);
                        finished.push_back(std::move(active[i]));
                    }
                    fin_cv.notify_all();
                    active.erase(active.begin() + (long)i);
                    progress = true;
                } else {
                    ++i;
                }
            }
            (void)hipGetLastError();
            if (!progress) {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait_for(lk, std::chrono::microseconds(200));
            }
        }
    }

    void finish_all() {
        {
            std::lock_guard<std::mutex> lk(fin_mu);
            fin_stop = true;
        }
        fin_cv.notify_all();
    }

    void finisher_loop() {
        (void)hipSetDevice(ctx->device);
        for (;;) {
            std::unique_ptr<Member> m;
            {
                std::unique_lock<std::mutex> lk(fin_mu);
                fin_cv.wait(lk, [&] { return fin_stop || !finished.empty(); });
                if (finished.empty()) return;
                m = std::move(finished.front());
                finished.pop_front();
            }
            QueryRun &R = *m->run;
            int rc = m->failed ? m->fail_rc : qr_finish(R, m->req->out, fin_stream);
            if (rc == AMC_OK) {
                amc_stats &s = m->req->out->stats;
                s.sweep_ms = (m->t_sweep_done - m->req->t_admit) * 1e3;
                s.tail_ms = 0.0;
                s.launches = m->launches;
                s.blocks = 0;
            }
            qr_release(R, alloc_stream);
            if (m->tail_done) (void)hipEventDestroy(m->tail_done);
            const uint64_t fp = m->req->footprint;
            auto req = m->req;
            m.reset();
            release_budget(fp);
            complete(req, rc);
        }
    }
};

void server_stop(amc_ctx *ctx) {
    Server *s = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->server_mu);
        s = ctx->server;
        ctx->server = nullptr;
    }
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->scheduler.joinable()) s->scheduler.join();
    if (s->finisher.joinable()) s->finisher.join();
    (void)hipSetDevice(ctx->device);
    s->free_lanes();
    for (hipStream_t x : {s->alloc_stream, s->tail_stream, s->fin_stream})
        if (x) (void)hipStreamDestroy(x);
    delete s;
}

static Server *server_get(amc_ctx *ctx, int *rc) {
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    *rc = AMC_OK;
    if (ctx->server) return ctx->server;
    Server *s = new (std::nothrow) Server();
    if (!s) {
        *rc = AMC_E_OOM;
        return nullptr;
    }
    s->ctx = ctx;
    (void)hipSetDevice(ctx->device);
    if (hipStreamCreateWithFlags(&s->alloc_stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->tail_stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->fin_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        for (hipStream_t x : {s->alloc_stream, s->tail_stream, s->fin_stream})
            if (x) (void)hipStreamDestroy(x);
        delete s;
        *rc = AMC_E_HIP;
        return nullptr;
    }
    if (s->make_lanes() != AMC_OK) {
        s->free_lanes();
        for (hipStream_t x : {s->alloc_stream, s->tail_stream, s->fin_stream})
            if (x) (void)hipStreamDestroy(x);
        delete s;
        *rc = AMC_E_HIP;
        return nullptr;
    }
    s->st.budget = ctx->budget;
    s->scheduler = std::thread([s] { s->scheduler_loop(); });
    s->finisher = std::thread([s] { s->finisher_loop(); });
    ctx->server = s;
    return s;
}

}  // namespace amc

struct amc_request {
    std::shared_ptr<amc::Request> r;
};

using namespace amc;

extern "C" int amc_submit(amc_ctx *ctx, const amc_graph *g, const amc_model *model, const amc_query *q,
                          amc_result *out, amc_request **req) {
    if (!ctx || !g || !model || !q || !out || !req || g->ctx != ctx) return AMC_E_INVALID_ARG;
    *req = nullptr;
    int rc = validate(g, model, q);
    if (rc != AMC_OK) return rc;
    if (!out->counts || (q->pool_size > 0 && !out->counts_w)) return AMC_E_INVALID_ARG;
    if (q->topk > 0 && (!out->psi || (q->pool_size > 0 && !out->psi_w))) return AMC_E_INVALID_ARG;
    auto r = std::make_shared<Request>();
    r->ctx = ctx;
    r->g = g;
    r->model = *model;
    r->min.capture(r->model, g->m);
    r->q = *q;
    r->in.capture(r->q, g->n);
    r->out = out;
    rc = amc_footprint(g, q, &r->footprint);
    if (rc != AMC_OK) return rc;
    if (r->footprint > ctx->budget) return AMC_E_ADMISSION;
    Server *s = server_get(ctx, &rc);
    if (!s) return rc;
    amc_request *h = new (std::nothrow) amc_request();
    if (!h) return AMC_E_OOM;
    h->r = r;
    r->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->pending.push_back(r);
    }
    s->cv.notify_all();
    *req = h;
    return AMC_OK;
}

extern "C" int amc_poll(amc_request *req) {
    if (!req || !req->r) return AMC_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(req->r->mu);
    return req->r->done ? req->r->status : AMC_E_NOT_READY;
}

extern "C" int amc_wait(amc_request *req) {
    if (!req || !req->r) return AMC_E_INVALID_ARG;
    std::unique_lock<std::mutex> lk(req->r->mu);
    req->r->cv.wait(lk, [&] { return req->r->done; });
    return req->r->status;
}

extern "C" void amc_request_destroy(amc_request *req) {
    if (!req) return;
    if (req->r) (void)amc_wait(req);
    delete req;
}

extern "C" int amc_request_times(amc_request *req, double t[3]) {
    if (!req || !req->r || !t) return AMC_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(req->r->mu);
    if (!req->r->done) return AMC_E_NOT_READY;
    t[0] = req->r->t_submit;
    t[1] = req->r->t_admit;
    t[2] = req->r->t_finish;
    return AMC_OK;
}

extern "C" int amc_server_info(amc_ctx *ctx, amc_server_stats *out) {
    if (!ctx || !out) return AMC_E_INVALID_ARG;
    std::memset(out, 0, sizeof(*out));
    out->budget = ctx->budget;
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    if (ctx->server) {
        std::lock_guard<std::mutex> lk2(ctx->server->mu);
        *out = ctx->server->st;
        out->budget = ctx->budget;
    }
    return AMC_OK;
}
