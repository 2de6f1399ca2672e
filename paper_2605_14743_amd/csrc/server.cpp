// server.cpp -- serving loop behind amc_submit / amc_poll / amc_wait.
//
// Queries wait in a FIFO; a query is admitted when a slot is free and its
// device footprint fits in the context budget minus what admitted queries
// hold (first fit in arrival order; a query that has been passed over
// kMaxBypass times blocks later arrivals until it fits).  Every slot owns a
// HIP stream (default priority) and a worker thread, so admitted queries run
// overlapped on the device; each keeps its counts and chain state in device
// memory until its tail has finished and its results are copied out.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>
#include <new>

#include "amc.h"
#include "amc_runtime.hpp"

namespace amc {

namespace {
double now_s() {
    using namespace std::chrono;
    return duration_cast<duration<double>>(steady_clock::now().time_since_epoch()).count();
}
constexpr int kSlots = 4;
constexpr int kMaxBypass = 8;
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

struct Server {
    amc_ctx *ctx = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::shared_ptr<Request>> pending;
    uint64_t in_use = 0;
    int active = 0;
    bool stop = false;
    amc_server_stats st{};

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

    void worker(int slot) {
        (void)hipSetDevice(ctx->device);
        for (;;) {
            std::shared_ptr<Request> r;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return (stop && pending.empty()) || (r = pick()) != nullptr; });
                if (!r) return;
                in_use += r->footprint;
                ++active;
                st.admitted++;
                st.launches++;
                st.peak_in_use = std::max(st.peak_in_use, in_use);
                st.peak_active = std::max(st.peak_active, active);
                st.max_members = std::max(st.max_members, 1);
            }
            r->t_admit = now_s();
            const int rc = run_query(ctx, r->g, &r->model, &r->q, r->out, streams[slot]);
            {
                std::lock_guard<std::mutex> lk(mu);
                in_use -= r->footprint;
                --active;
                st.completed++;
            }
            cv.notify_all();
            {
                std::lock_guard<std::mutex> lk(r->mu);
                r->status = rc;
                r->t_finish = now_s();
                r->done = true;
            }
            r->cv.notify_all();
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
    for (auto &t : s->workers) t.join();
    for (auto st : s->streams) (void)hipStreamDestroy(st);
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
    for (int k = 0; k < kSlots; ++k) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (auto x : s->streams) (void)hipStreamDestroy(x);
            delete s;
            *rc = AMC_E_HIP;
            return nullptr;
        }
        s->streams.push_back(st);
    }
    for (int k = 0; k < kSlots; ++k) s->workers.emplace_back([s, k] { s->worker(k); });
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
