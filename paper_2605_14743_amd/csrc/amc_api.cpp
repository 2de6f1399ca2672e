// amc_api.cpp -- host runtime behind the C-ABI of amc.h: contexts, staged
// graphs, argument checking, launch configuration, the device tail and the
// copy-back of results.
//
// Paper: Bao, Kontou, Vogiatzis, "Betweenness-Central Nodes Under
// Uncertainty: An Absorbing Markov Chain Approach".
#include "amc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "amc_kernels.hpp"
#include "amc_runtime.hpp"

using namespace amc;

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------
namespace amc {

int DevArena::alloc(size_t bytes, void **out) {
    *out = nullptr;
    if (bytes == 0) return AMC_OK;
    void *p = nullptr;
    const size_t sz = (bytes + 255) & ~(size_t)255;
    const hipError_t e = (stream && async) ? hipMallocAsync(&p, sz, stream) : hipMalloc(&p, sz);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return AMC_E_OOM;
    }
    ptrs.push_back(p);
    *out = p;
    return AMC_OK;
}

void DevArena::release() {
    for (void *p : ptrs) {
        if (stream && async) (void)hipFreeAsync(p, stream);
        else (void)hipFree(p);
    }
    ptrs.clear();
}

}  // namespace amc

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

// ---------------------------------------------------------------------------
// context and graph
// ---------------------------------------------------------------------------
extern "C" int amc_ctx_create(int device, uint64_t hbm_budget_bytes, amc_ctx **out) {
    if (!out) return AMC_E_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return AMC_E_HIP;
    }
    if (device < 0 || device >= count) return AMC_E_INVALID_ARG;
    HIPCHK(hipSetDevice(device));
    amc_ctx *c = new (std::nothrow) amc_ctx();
    if (!c) return AMC_E_OOM;
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete c;
        return AMC_E_HIP;
    }
    c->cu_count = prop.multiProcessorCount;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) lds = 65536;
    c->max_lds = lds - 512;    // headroom for the kernels' static LDS
    int pools = 0;
    if (hipDeviceGetAttribute(&pools, hipDeviceAttributeMemoryPoolsSupported, device) != hipSuccess) pools = 0;
    c->async_alloc = pools != 0;
    size_t free_b = 0, total_b = 0;
    (void)hipMemGetInfo(&free_b, &total_b);
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(free_b * 0.9);
    if (hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return AMC_E_HIP;
    }
    c->stream = c->own;
    *out = c;
    return AMC_OK;
}

extern "C" void amc_ctx_destroy(amc_ctx *ctx) {
    if (!ctx) return;
    server_stop(ctx);
    (void)hipSetDevice(ctx->device);
    if (ctx->own) (void)hipStreamDestroy(ctx->own);
    delete ctx;
}

extern "C" int amc_ctx_set_stream(amc_ctx *ctx, void *hip_stream) {
    if (!ctx) return AMC_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->stream = hip_stream ? (hipStream_t)hip_stream : ctx->own;
    return AMC_OK;
}

extern "C" void *amc_ctx_stream(amc_ctx *ctx) { return ctx ? (void *)ctx->stream : nullptr; }

extern "C" int amc_graph_create(amc_ctx *ctx, int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                                const uint32_t *w0, amc_graph **out) {
    if (!ctx || !out || n < 1 || m < 0 || (m > 0 && (!eu || !ev))) return AMC_E_INVALID_ARG;
    *out = nullptr;
    if (n > 65535 || m > (int64_t)1 << 30) return AMC_E_UNSUPPORTED;
    for (int64_t e = 0; e < m; ++e) {
        if (eu[e] < 0 || ev[e] >= n || eu[e] >= ev[e]) return AMC_E_INVALID_ARG;
        if (e > 0 && (eu[e - 1] > eu[e] || (eu[e - 1] == eu[e] && ev[e - 1] >= ev[e]))) return AMC_E_INVALID_ARG;
        if (w0 && (w0[e] < 1u || w0[e] > 65535u)) return AMC_E_INVALID_ARG;
    }
    amc_graph *g = new (std::nothrow) amc_graph();
    if (!g) return AMC_E_OOM;
    g->ctx = ctx;
    g->n = n;
    g->m = m;
    g->eu.assign(eu, eu + m);
    g->ev.assign(ev, ev + m);
    if (w0) g->w0.assign(w0, w0 + m);
    // CSR of both directions, neighbours in increasing order
    g->rp.assign((size_t)n + 1, 0);
    for (int64_t e = 0; e < m; ++e) {
        g->rp[eu[e] + 1]++;
        g->rp[ev[e] + 1]++;
    }
    for (int v = 0; v < n; ++v) g->rp[v + 1] += g->rp[v];
    std::vector<int32_t> fill(g->rp.begin(), g->rp.end() - 1);
    std::vector<uint16_t> col((size_t)2 * m + 1);
    std::vector<int32_t> sedge((size_t)2 * m + 1);
    // edges are sorted by (u, v): for u the v's come in increasing order; the
    // reverse slots are filled in increasing u as well
    for (int64_t e = 0; e < m; ++e) {
        const int a = eu[e], b = ev[e];
        col[fill[b]] = (uint16_t)a;
        sedge[fill[b]++] = (int32_t)e;
    }
    for (int64_t e = 0; e < m; ++e) {
        const int a = eu[e], b = ev[e];
        col[fill[a]] = (uint16_t)b;
        sedge[fill[a]++] = (int32_t)e;
    }
    for (int v = 0; v < n; ++v) {   // merge to increasing neighbour order
        std::vector<std::pair<uint16_t, int32_t>> tmp;
        for (int j = g->rp[v]; j < g->rp[v + 1]; ++j) tmp.push_back({col[j], sedge[j]});
        std::sort(tmp.begin(), tmp.end());
        for (size_t k = 0; k < tmp.size(); ++k) {
            col[g->rp[v] + k] = tmp[k].first;
            sedge[g->rp[v] + k] = tmp[k].second;
        }
        g->max_deg = std::max<int32_t>(g->max_deg, g->rp[v + 1] - g->rp[v]);
    }
    int rc = AMC_OK;
    (void)hipSetDevice(ctx->device);
    void *p;
    if ((rc = g->arena.alloc(sizeof(int32_t) * ((size_t)n + 1), &p)) == AMC_OK) g->d_rp = (int32_t *)p;
    if (rc == AMC_OK && (rc = g->arena.alloc(sizeof(uint16_t) * (2 * (size_t)m + 1), &p)) == AMC_OK)
        g->d_col = (uint16_t *)p;
    if (rc == AMC_OK && (rc = g->arena.alloc(sizeof(int32_t) * (2 * (size_t)m + 1), &p)) == AMC_OK)
        g->d_sedge = (int32_t *)p;
    if (rc == AMC_OK && (rc = g->arena.alloc(sizeof(int32_t) * ((size_t)m + 1), &p)) == AMC_OK) g->d_eu = (int32_t *)p;
    if (rc == AMC_OK && (rc = g->arena.alloc(sizeof(int32_t) * ((size_t)m + 1), &p)) == AMC_OK) g->d_ev = (int32_t *)p;
    if (rc == AMC_OK && w0 && (rc = g->arena.alloc(sizeof(uint32_t) * ((size_t)m + 1), &p)) == AMC_OK)
        g->d_w0 = (uint32_t *)p;
    if (rc == AMC_OK) {
        bool ok = hipMemcpy(g->d_rp, g->rp.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice) == hipSuccess;
        if (m > 0) {
            ok = ok && hipMemcpy(g->d_col, col.data(), sizeof(uint16_t) * 2 * m, hipMemcpyHostToDevice) == hipSuccess;
            ok = ok && hipMemcpy(g->d_sedge, sedge.data(), sizeof(int32_t) * 2 * m, hipMemcpyHostToDevice) == hipSuccess;
            ok = ok && hipMemcpy(g->d_eu, eu, sizeof(int32_t) * m, hipMemcpyHostToDevice) == hipSuccess;
            ok = ok && hipMemcpy(g->d_ev, ev, sizeof(int32_t) * m, hipMemcpyHostToDevice) == hipSuccess;
            if (w0) ok = ok && hipMemcpy(g->d_w0, w0, sizeof(uint32_t) * m, hipMemcpyHostToDevice) == hipSuccess;
        }
        if (!ok) {
            (void)hipGetLastError();
            rc = AMC_E_HIP;
        }
    }
    if (rc != AMC_OK) {
        g->arena.release();
        delete g;
        return rc;
    }
    *out = g;
    return AMC_OK;
}

extern "C" void amc_graph_destroy(amc_graph *g) {
    if (!g) return;
    (void)hipSetDevice(g->ctx->device);
    g->arena.release();
    delete g;
}

extern "C" const char *amc_strerror(int status) {
    switch (status) {
        case AMC_OK: return "ok";
        case AMC_E_INVALID_ARG: return "invalid argument";
        case AMC_E_OOM: return "out of memory";
        case AMC_E_HIP: return "HIP runtime error";
        case AMC_E_SIGMA_OVERFLOW: return "shortest-path count overflow (sigma > 2^64-1)";
        case AMC_E_SINGULAR: return "I - Q is singular (a row never absorbs and the floor is disabled)";
        case AMC_E_ADMISSION: return "query footprint exceeds the context budget";
        case AMC_E_NOT_READY: return "request not finished";
        case AMC_E_UNSUPPORTED: return "shape exceeds an engine limit";
        default: return "unknown status";
    }
}

extern "C" int amc_version(void) { return 100; }

// ---------------------------------------------------------------------------
// validation and planning
// ---------------------------------------------------------------------------
namespace amc {

int validate(const amc_graph *g, const amc_model *md, const amc_query *q) {
    if (!g || !md || !q) return AMC_E_INVALID_ARG;
    const int n = g->n;
    if (q->R == 0 || (uint64_t)q->r_begin + q->R > 0xFFFFFFFFull) return AMC_E_INVALID_ARG;
    if (!(q->alpha > 0.0 && q->alpha <= 1.0)) return AMC_E_INVALID_ARG;
    if (!(md->p_fail >= 0.0 && md->p_fail <= 1.0)) return AMC_E_INVALID_ARG;
    if (md->p_fail_edge)
        for (int64_t e = 0; e < g->m; ++e)
            if (!(md->p_fail_edge[e] >= 0.0 && md->p_fail_edge[e] <= 1.0)) return AMC_E_INVALID_ARG;
    if (md->weight_kind == AMC_WEIGHT_UNIFORM_INT) {
        if (md->w_lo < 1u || md->w_hi < md->w_lo || md->w_hi > 65535u) return AMC_E_INVALID_ARG;
    } else if (md->weight_kind == AMC_WEIGHT_FIXED) {
        if (g->w0.empty() && g->m > 0) return AMC_E_INVALID_ARG;
    } else if (md->weight_kind != AMC_WEIGHT_UNIT) {
        return AMC_E_INVALID_ARG;
    }
    if (q->s) {
        double tot = 0.0;
        for (int i = 0; i < n; ++i) {
            if (!(q->s[i] >= 0.0)) return AMC_E_INVALID_ARG;
            tot += q->s[i];
        }
        if (std::fabs(tot - 1.0) > 1e-9) return AMC_E_INVALID_ARG;
    }
    if (q->pool_size < 0 || (q->pool_size > 0 && !q->pool)) return AMC_E_INVALID_ARG;
    for (int k = 0; k < q->pool_size; ++k)
        if (q->pool[k] < 0 || q->pool[k] >= n) return AMC_E_INVALID_ARG;
    if (q->reward)
        for (int i = 0; i < n; ++i)
            if (!(q->reward[i] >= 0.0) || !std::isfinite(q->reward[i])) return AMC_E_INVALID_ARG;
    if (q->cert_topk < 0 || q->cert_topk > 16 || (q->cert_topk > 0 && q->cert_topk >= n)) return AMC_E_INVALID_ARG;
    if (q->cert_topk > 0 && !(q->r_lower > 0.0 && q->r_lower <= 1.0)) return AMC_E_INVALID_ARG;
    if (!(q->eps >= 0.0) || !std::isfinite(q->eps)) return AMC_E_INVALID_ARG;
    if (q->n_debug < 0 || q->n_debug > 64 || (q->n_debug > 0 && !q->debug_pairs)) return AMC_E_INVALID_ARG;
    for (int k = 0; k < q->n_debug; ++k)
        if (q->debug_pairs[2 * k + 1] >= (uint32_t)n) return AMC_E_INVALID_ARG;
    if (q->mode < AMC_MODE_AUTO || q->mode > AMC_MODE_BLOCK) return AMC_E_INVALID_ARG;
    if (q->waves < 0 || q->waves > kMaxWaves || q->tile < 0) return AMC_E_INVALID_ARG;
    if (q->group < 0 || q->group > 16 || (q->group > 4 && q->group != 8 && q->group != 16)) return AMC_E_INVALID_ARG;
    // longest possible distance must stay below the "unreached" sentinel
    const uint64_t wmax = md->weight_kind == AMC_WEIGHT_UNIT ? 1u
                          : md->weight_kind == AMC_WEIGHT_UNIFORM_INT
                              ? md->w_hi
                              : (g->w0.empty() ? 1u : *std::max_element(g->w0.begin(), g->w0.end()));
    if ((uint64_t)(n - 1) * wmax >= (uint64_t)kInf - 65536u) return AMC_E_UNSUPPORTED;
    return AMC_OK;
}

uint64_t prob_threshold(double p) {
    if (!(p > 0.0)) return 0;
    if (p >= 1.0) return 4294967296ull;
    return (uint64_t)std::floor(p * 4294967296.0);
}

// Launch configuration.  The LDS mode needs the realized adjacency, B and
// at least two wavefront states in one workgroup; otherwise the workgroup-
// per-source mode is used.
int plan(const amc_ctx *ctx, const amc_graph *g, const amc_model *md, const amc_query *q, Plan *pl) {
    const int n = g->n;
    const uint32_t adj_cap = (uint32_t)(2 * g->m) + kAdjPad;
    pl->weighted = md->weight_kind != AMC_WEIGHT_UNIT;
    const double avg_deg = n > 0 ? 2.0 * (double)g->m / n : 0.0;
    (void)avg_deg;
    pl->group = q->group > 0 ? q->group : 1;
    // adjacency entry: neighbour in the low bits, weight above; 16 bits when both fit
    uint32_t nbits = 1;
    while ((1u << nbits) < (uint32_t)n) ++nbits;
    const uint64_t wmax = md->weight_kind == AMC_WEIGHT_UNIT ? 1u
                          : md->weight_kind == AMC_WEIGHT_UNIFORM_INT
                              ? md->w_hi
                              : (g->w0.empty() ? 1u : *std::max_element(g->w0.begin(), g->w0.end()));
    if (nbits < 16 && wmax < (1ull << (16 - nbits)) && adj_cap <= 65535u) {
        pl->adj_bytes = 2;
        pl->shift = nbits;
    } else {
        pl->adj_bytes = 4;
        pl->shift = 16;
    }
    int best_w = 0;
    uint32_t best_lds = 0, best_wb = 0;
    const int want_w = q->waves > 0 ? q->waves : kMaxWaves;
    for (int w = 2; w <= want_w; ++w) {
        uint32_t wb = 0;
        const uint32_t lds = lds_bytes_wave(n, adj_cap, pl->adj_bytes, w, &wb);
        if (lds > (uint32_t)ctx->max_lds) break;
        if ((uint64_t)wb * w < std::max<uint64_t>(2ull * (uint64_t)g->m, 32ull * (uint64_t)n)) continue;
        best_w = w;
        best_lds = lds;
        best_wb = wb;
    }
    const bool wave_ok = best_w >= 2 && (q->waves == 0 || best_w == q->waves);
    int mode = q->mode;
    if (mode == AMC_MODE_AUTO) mode = wave_ok ? AMC_MODE_WAVE : AMC_MODE_BLOCK;
    if (mode == AMC_MODE_WAVE && !wave_ok) return AMC_E_UNSUPPORTED;
    pl->mode = mode;
    if (mode == AMC_MODE_WAVE) {
        pl->waves = best_w;
        pl->lds = best_lds;
        pl->wave_bytes = best_wb;
        pl->threads = 64 * best_w;
        pl->adj_cap = adj_cap;
    } else {
        pl->threads = q->waves > 0 ? 64 * q->waves : 1024;
        pl->lds = lds_bytes_block(n, pl->threads);
        if (pl->lds > (uint32_t)ctx->max_lds) return AMC_E_UNSUPPORTED;
        if (2ull * (uint64_t)g->m > pl->lds) return AMC_E_UNSUPPORTED;   // per-edge staging fits the LDS
        pl->waves = pl->threads / 64;
        pl->wave_bytes = 0;
        pl->adj_cap = adj_cap;
    }
    // sources per work item: whole realizations when there are enough of
    // them to fill the device, otherwise split the sources
    const uint32_t blocks_per_cu = std::max<uint32_t>(1u, (uint32_t)ctx->max_lds / std::max<uint32_t>(pl->lds, 1u));
    const uint64_t slots = (uint64_t)ctx->cu_count * blocks_per_cu;
    int tile = q->tile;
    if (q->flags & AMC_PLAIN_LAUNCH) tile = mode == AMC_MODE_WAVE ? pl->waves : 1;
    if (tile <= 0) {
        if ((uint64_t)q->R >= 2 * slots || mode == AMC_MODE_BLOCK) {
            tile = n;
        } else {
            const uint64_t want_items = 2 * slots;
            const uint64_t per_r = std::min<uint64_t>((uint64_t)n, (want_items + q->R - 1) / q->R);
            tile = (int)((n + per_r - 1) / per_r);
            if (mode == AMC_MODE_WAVE) tile = std::max(tile, pl->waves);
        }
    }
    tile = std::min(tile, n);
    pl->tile = tile;
    pl->tiles_per_r = (n + tile - 1) / tile;
    pl->items = (uint64_t)q->R * pl->tiles_per_r;
    if (pl->items > 0xFFFFFFFFull) return AMC_E_UNSUPPORTED;
    pl->blocks = (int)std::min<uint64_t>(pl->items, slots);
    return AMC_OK;
}

}  // namespace amc

// ---------------------------------------------------------------------------
// footprint
// ---------------------------------------------------------------------------
extern "C" int amc_footprint(const amc_graph *g, const amc_query *q, uint64_t *bytes) {
    if (!g || !q || !bytes) return AMC_E_INVALID_ARG;
    const uint64_t n = (uint64_t)g->n, R = q->R;
    uint64_t b = 4 * n * (n + 1);                        // counts
    if (q->pool_size > 0) b += 4 * n * (n + 1);          // pool counts
    if (q->flags & AMC_WANT_CENTER) b += 4 * R;
    if (q->flags & AMC_WANT_NEXT_TABLE) b += 4 * R * n * (q->pool_size > 0 ? 2 : 1);
    b += 8 * n * 8 + 8 * (uint64_t)g->m + 4096;          // bsum, vectors, thresholds, control
    // partial-B exchange when realizations are split (upper bound)
    b += (8 + 4 + 4) * R * n + 4 * R;
    if (!(q->flags & AMC_SKIP_TAIL)) b += 2 * 8 * n * n + 3 * 8 * 16 * n;
    if (q->n_debug > 0) b += (uint64_t)q->n_debug * n * 20;
    *bytes = b;
    return AMC_OK;
}

// ---------------------------------------------------------------------------
// one query on one stream
// ---------------------------------------------------------------------------
namespace amc {

static int dev_copy_in(DevArena &A, const void *src, size_t bytes, hipStream_t st, void **out) {
    RCHK(A.alloc(bytes, out));
    if (bytes) HIPCHK(hipMemcpyAsync(*out, src, bytes, hipMemcpyHostToDevice, st));
    return AMC_OK;
}

static int copy_out(void *dst, const void *src, size_t bytes, hipStream_t st) {
    if (dst && bytes) HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
    return AMC_OK;
}

// Tail on device: kernel, N, visits, AFC, rewards, certificates; then, with a
// pool, the constrained kernel P^W.  `counts` may be null when Qh is given.
static int run_tail(int n, const uint32_t *d_counts, const uint32_t *d_counts_w, const double *Qh, uint32_t R,
                    double eta, const amc_query *q, const uint8_t *d_pool, const double *s_host, amc_result *out,
                    hipStream_t st, DevArena &A, int *d_err) {
    const size_t nn = (size_t)n * n;
    void *p;
    double *Q, *Nm, *r, *mu, *b, *scal, *s_dev, *f_dev = nullptr, *bbar = nullptr;
    int32_t *top, *cv;
    int *support;
    RCHK(A.alloc(8 * nn, &p)); Q = (double *)p;
    RCHK(A.alloc(8 * nn, &p)); Nm = (double *)p;
    RCHK(A.alloc(8 * (size_t)n, &p)); r = (double *)p;
    RCHK(A.alloc(8 * (size_t)n, &p)); mu = (double *)p;
    RCHK(A.alloc(8 * (size_t)n, &p)); b = (double *)p;
    RCHK(A.alloc(8 * 8, &p)); scal = (double *)p;
    RCHK(A.alloc(4 * 16, &p)); top = (int32_t *)p;
    RCHK(A.alloc(4 * (size_t)n, &p)); cv = (int32_t *)p;
    RCHK(A.alloc(4 * 4, &p)); support = (int *)p;
    std::vector<double> s_uni;
    if (!s_host) {
        s_uni.assign((size_t)n, 1.0 / n);
        s_host = s_uni.data();
    }
    RCHK(dev_copy_in(A, s_host, 8 * (size_t)n, st, &p)); s_dev = (double *)p;
    if (q->reward) {
        RCHK(dev_copy_in(A, q->reward, 8 * (size_t)n, st, &p));
        f_dev = (double *)p;
    }
    HIPCHK(fill_u32(support, 1, 0u, st));
    const int k = q->cert_topk;
    double *gap = nullptr, *sharp = nullptr, *sharp_supp = nullptr;
    if (k > 0) {
        const size_t pairs = (size_t)k * (n - k);
        RCHK(A.alloc(8 * pairs, &p)); gap = (double *)p;
        RCHK(A.alloc(8 * pairs, &p)); sharp = (double *)p;
        RCHK(A.alloc(8 * pairs, &p)); sharp_supp = (double *)p;
    }
    if (Qh) {
        HIPCHK(hipMemcpyAsync(Q, Qh, 8 * nn, hipMemcpyHostToDevice, st));
        HIPCHK(tail_kernel_from_Q(n, Q, r, Nm, st));
    } else {
        HIPCHK(tail_kernel_from_counts(n, d_counts, R, eta, Q, r, Nm, st));
    }
    HIPCHK(tail_invert(n, Nm, d_err, st));
    HIPCHK(tail_visits(n, Nm, s_dev, mu, b, f_dev, nullptr, nullptr, r, q->r_lower, k, top, scal, st));
    HIPCHK(tail_certificates(n, k, Q, Nm, mu, top, cv, q->eps, q->r_lower, gap, sharp, sharp_supp, support, st));
    double hs[8] = {0};
    int hsupport = 0;
    RCHK(copy_out(out->Q, Q, 8 * nn, st));
    RCHK(copy_out(out->r, r, 8 * (size_t)n, st));
    if (q->flags & AMC_WANT_N) RCHK(copy_out(out->N, Nm, 8 * nn, st));
    RCHK(copy_out(out->mu, mu, 8 * (size_t)n, st));
    RCHK(copy_out(out->b, b, 8 * (size_t)n, st));
    RCHK(copy_out(hs, scal, 8 * 4, st));
    RCHK(copy_out(&hsupport, support, 4, st));
    if (k > 0) {
        const size_t pairs = (size_t)k * (n - k);
        RCHK(copy_out(out->top, top, 4 * (size_t)k, st));
        RCHK(copy_out(out->cert_v, cv, 4 * (size_t)(n - k), st));
        RCHK(copy_out(out->cert_gap, gap, 8 * pairs, st));
        RCHK(copy_out(out->cert_sharp, sharp, 8 * pairs, st));
        RCHK(copy_out(out->cert_sharp_supp, sharp_supp, 8 * pairs, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    out->E_T = hs[0];
    out->b_f = q->reward ? hs[1] : 0.0;
    out->admissible = hs[3] > 0.5 ? 1 : 0;
    out->epsbar = (double)n * q->eps;
    out->epsbar_supp = (double)hsupport * q->eps;
    out->cert_crude = q->r_lower > 0 ? 2.0 * out->epsbar / (q->r_lower * q->r_lower) : 0.0;
    out->cert_crude_supp = q->r_lower > 0 ? 2.0 * out->epsbar_supp / (q->r_lower * q->r_lower) : 0.0;

    if (d_counts_w && d_pool) {   // constrained kernel P^W (Section 7), same pipeline
        double *bw = b, *muw = mu;
        RCHK(A.alloc(8 * (size_t)n, &p)); bbar = (double *)p;
        double *xi;
        RCHK(A.alloc(8 * (size_t)n, &p)); xi = (double *)p;
        HIPCHK(tail_xi(n, d_counts_w, R, xi, st));
        HIPCHK(tail_kernel_from_counts(n, d_counts_w, R, eta, Q, r, Nm, st));
        HIPCHK(tail_invert(n, Nm, d_err, st));
        HIPCHK(tail_visits(n, Nm, s_dev, muw, bw, f_dev, d_pool, bbar, nullptr, 0.0, 0, top, scal, st));
        RCHK(copy_out(out->b_w, bw, 8 * (size_t)n, st));
        RCHK(copy_out(out->b_w_bar, bbar, 8 * (size_t)n, st));
        RCHK(copy_out(out->xi, xi, 8 * (size_t)n, st));
        RCHK(copy_out(hs, scal, 8 * 4, st));
        HIPCHK(hipStreamSynchronize(st));
        out->E_T_w = hs[0];
        out->b_w_f = q->reward ? hs[1] : 0.0;
        out->m_w = hs[2];
    }
    return AMC_OK;
}

int run_query(amc_ctx *ctx, const amc_graph *g, const amc_model *md, const amc_query *q, amc_result *out,
              hipStream_t st) {
    RCHK(validate(g, md, q));
    if (!out || !out->counts) return AMC_E_INVALID_ARG;
    if (q->pool_size > 0 && !out->counts_w) return AMC_E_INVALID_ARG;
    Plan pl;
    RCHK(plan(ctx, g, md, q, &pl));
    const int n = g->n;
    const uint32_t R = q->R;
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
    void *p;
    SweepParams P;
    std::memset(&P, 0, sizeof(P));
    P.n = n;
    P.m = g->m;
    P.rp_base = g->d_rp;
    P.col = g->d_col;
    P.slot_edge = g->d_sedge;
    P.eu = g->d_eu;
    P.ev = g->d_ev;
    P.w0 = g->d_w0;
    P.t_fail = prob_threshold(md->p_fail);
    if (md->p_fail_edge && g->m > 0) {
        std::vector<uint64_t> th((size_t)g->m);
        for (int64_t e = 0; e < g->m; ++e) th[e] = prob_threshold(md->p_fail_edge[e]);
        RCHK(dev_copy_in(A, th.data(), 8 * (size_t)g->m, st, &p));
        P.t_fail_edge = (const uint64_t *)p;
        HIPCHK(hipStreamSynchronize(st));
    }
    P.weight_kind = md->weight_kind;
    P.w_lo = md->w_lo;
    P.w_span = md->weight_kind == AMC_WEIGHT_UNIFORM_INT ? md->w_hi - md->w_lo + 1u : 1u;
    P.key0 = (uint32_t)q->seed;
    P.key1 = (uint32_t)(q->seed >> 32);
    P.r_begin = q->r_begin;
    P.t_alpha = prob_threshold(q->alpha);
    P.k_min = q->k_min;
    P.tau = q->tie_tau < 0.0 ? 1e-9 : q->tie_tau;
    std::vector<uint8_t> mask;
    if (q->pool_size > 0) {
        mask.assign((size_t)n, 0);
        for (int k = 0; k < q->pool_size; ++k) mask[q->pool[k]] = 1;
        RCHK(dev_copy_in(A, mask.data(), (size_t)n, st, &p));
        P.pool = (const uint8_t *)p;
    }
    P.tile = pl.tile;
    P.tiles_per_r = pl.tiles_per_r;
    P.adj_cap = pl.adj_cap;
    P.wave_bytes = pl.wave_bytes;
    const size_t cnt_elems = (size_t)n * (n + 1);
    RCHK(A.alloc(4 * cnt_elems, &p)); P.counts = (uint32_t *)p;
    HIPCHK(fill_u32(P.counts, cnt_elems, 0u, st));
    if (q->pool_size > 0) {
        RCHK(A.alloc(4 * cnt_elems, &p)); P.counts_w = (uint32_t *)p;
        HIPCHK(fill_u32(P.counts_w, cnt_elems, 0u, st));
    }
    if (q->flags & AMC_WANT_CENTER) {
        RCHK(A.alloc(4 * (size_t)R, &p));
        P.center_global = (int32_t *)p;
    }
    if (q->flags & AMC_WANT_NEXT_TABLE) {
        RCHK(A.alloc(4 * (size_t)R * n, &p));
        P.next_table = (int32_t *)p;
        if (q->pool_size > 0) {
            RCHK(A.alloc(4 * (size_t)R * n, &p));
            P.next_table_w = (int32_t *)p;
        }
    }
    if (q->flags & AMC_WANT_BSUM) {
        RCHK(A.alloc(8 * (size_t)n, &p)); P.bsum = (double *)p;
        HIPCHK(fill_u32(P.bsum, 2 * (size_t)n, 0u, st));
    }
    RCHK(A.alloc(8 * 8, &p)); P.stats = (unsigned long long *)p;
    HIPCHK(fill_u32(P.stats, 16, 0u, st));
    int *d_err;
    RCHK(A.alloc(16, &p)); d_err = (int *)p;
    P.err = d_err;
    HIPCHK(fill_u32(d_err, 4, 0u, st));
    RCHK(A.alloc(16, &p)); P.work_ctr = (unsigned int *)p;
    HIPCHK(fill_u32(P.work_ctr, 4, 0u, st));
    if (pl.tiles_per_r > 1) {
        RCHK(A.alloc(8 * (size_t)R * n, &p)); P.Bg = (double *)p;
        HIPCHK(fill_u32(P.Bg, 2 * (size_t)R * n, 0u, st));
        RCHK(A.alloc(4 * (size_t)R * n, &p)); P.compg = (int32_t *)p;
        RCHK(A.alloc(4 * (size_t)R * n, &p)); P.sizeg = (int32_t *)p;
        RCHK(A.alloc(4 * (size_t)R, &p)); P.done = (unsigned int *)p;
        HIPCHK(fill_u32(P.done, R, 0u, st));
    }
    if ((q->flags & AMC_WANT_DEBUG) && q->n_debug > 0) {
        RCHK(dev_copy_in(A, q->debug_pairs, 8 * (size_t)q->n_debug, st, &p));
        P.dbg_pairs = (const uint32_t *)p;
        P.n_dbg = q->n_debug;
        RCHK(A.alloc(4 * (size_t)q->n_debug * n, &p)); P.dbg_dist = (uint32_t *)p;
        RCHK(A.alloc(8 * (size_t)q->n_debug * n, &p)); P.dbg_sigma = (unsigned long long *)p;
        RCHK(A.alloc(8 * (size_t)q->n_debug * n, &p)); P.dbg_delta = (double *)p;
        HIPCHK(fill_u32(P.dbg_dist, (size_t)q->n_debug * n, 0xFFFFFFFFu, st));
        HIPCHK(fill_u32(P.dbg_sigma, 2 * (size_t)q->n_debug * n, 0u, st));
        HIPCHK(fill_u32(P.dbg_delta, 2 * (size_t)q->n_debug * n, 0u, st));
    }

    uint32_t *bscratch = nullptr;
    if (pl.mode == AMC_MODE_BLOCK) {
        const int nb = (q->flags & AMC_PLAIN_LAUNCH) ? pl.tiles_per_r : pl.blocks;
        RCHK(A.alloc(4 * block_scratch_words(n, g->m) * (size_t)nb, &p));
        bscratch = (uint32_t *)p;
    }

    hipEvent_t e0, e1, e2;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventCreate(&e2));
    struct EvGuard {
        hipEvent_t a, b, c;
        ~EvGuard() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            (void)hipEventDestroy(c);
        }
    } evg{e0, e1, e2};
    HIPCHK(hipEventRecord(e0, st));
    int launches = 0;
    if (q->flags & AMC_PLAIN_LAUNCH) {
        P.static_items = 1;
        P.n_items = (uint32_t)pl.tiles_per_r;
        for (uint32_t rl = 0; rl < R; ++rl) {
            P.item_base = rl * (uint32_t)pl.tiles_per_r;
            if (pl.mode == AMC_MODE_WAVE)
                HIPCHK(launch_sweep_wave(P, pl.weighted, pl.group, pl.adj_bytes, pl.shift, pl.tiles_per_r, pl.waves, pl.lds, st));
            else
                HIPCHK(launch_sweep_block(P, pl.weighted, pl.tiles_per_r, pl.threads, pl.lds, bscratch, st));
            ++launches;
        }
    } else {
        P.static_items = 0;
        P.n_items = (uint32_t)pl.items;
        P.item_base = 0;
        if (pl.mode == AMC_MODE_WAVE)
            HIPCHK(launch_sweep_wave(P, pl.weighted, pl.group, pl.adj_bytes, pl.shift, pl.blocks, pl.waves, pl.lds, st));
        else
            HIPCHK(launch_sweep_block(P, pl.weighted, pl.blocks, pl.threads, pl.lds, bscratch, st));
        launches = 1;
    }
    HIPCHK(hipEventRecord(e1, st));
    unsigned long long hstats[8] = {0};
    int herr = 0;
    RCHK(copy_out(hstats, P.stats, 8 * 5, st));
    RCHK(copy_out(&herr, d_err, 4, st));
    HIPCHK(hipStreamSynchronize(st));
    if (herr & 1) return AMC_E_SIGMA_OVERFLOW;
    RCHK(copy_out(out->counts, P.counts, 4 * cnt_elems, st));
    if (P.counts_w) RCHK(copy_out(out->counts_w, P.counts_w, 4 * cnt_elems, st));
    if (P.center_global) RCHK(copy_out(out->center_global, P.center_global, 4 * (size_t)R, st));
    if (P.next_table) RCHK(copy_out(out->next_table, P.next_table, 4 * (size_t)R * n, st));
    if (P.next_table_w) RCHK(copy_out(out->next_table_w, P.next_table_w, 4 * (size_t)R * n, st));
    if (P.bsum) RCHK(copy_out(out->bsum, P.bsum, 8 * (size_t)n, st));
    if (P.dbg_dist) {
        RCHK(copy_out(out->dbg_dist, P.dbg_dist, 4 * (size_t)q->n_debug * n, st));
        RCHK(copy_out(out->dbg_sigma, P.dbg_sigma, 8 * (size_t)q->n_debug * n, st));
        RCHK(copy_out(out->dbg_delta, P.dbg_delta, 8 * (size_t)q->n_debug * n, st));
    }
    float ms_sweep = 0.f;
    HIPCHK(hipEventElapsedTime(&ms_sweep, e0, e1));
    out->stats.units = hstats[0];
    out->stats.sum_nK = hstats[1];
    out->stats.sum_AK = hstats[2];
    out->stats.sum_DK = hstats[3];
    out->stats.near_band = hstats[4];
    out->stats.sweep_ms = ms_sweep;
    out->stats.mode = pl.mode;
    out->stats.waves = pl.waves;
    out->stats.tile = pl.tile;
    out->stats.blocks = (q->flags & AMC_PLAIN_LAUNCH) ? pl.tiles_per_r : pl.blocks;
    out->stats.lds_bytes = (int32_t)pl.lds;
    out->stats.launches = launches;
    out->stats.group = pl.group;
    out->stats.adj_bytes = (int32_t)pl.adj_bytes;
    out->stats.tail_ms = 0.0;
    if (!(q->flags & AMC_SKIP_TAIL)) {
        const double eta = q->floor_eta < 0.0 ? 0.1 / std::sqrt((double)R) : q->floor_eta;
        HIPCHK(hipEventRecord(e1, st));
        RCHK(run_tail(n, P.counts, P.counts_w, nullptr, R, eta, q, P.pool, q->s, out, st, A, d_err));
        HIPCHK(hipEventRecord(e2, st));
        RCHK(copy_out(&herr, d_err, 4, st));
        HIPCHK(hipStreamSynchronize(st));
        float ms_tail = 0.f;
        HIPCHK(hipEventElapsedTime(&ms_tail, e1, e2));
        out->stats.tail_ms = ms_tail;
        if (herr & 2) return AMC_E_SINGULAR;
    }
    HIPCHK(hipStreamSynchronize(st));
    return AMC_OK;
}

}  // namespace amc

extern "C" int amc_run(amc_ctx *ctx, const amc_graph *g, const amc_model *model, const amc_query *q,
                       amc_result *out) {
    if (!ctx || !g || g->ctx != ctx) return AMC_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return AMC_E_HIP;
    return run_query(ctx, g, model, q, out, ctx->stream);
}

extern "C" int amc_chain(amc_ctx *ctx, int32_t n, const double *Q, const amc_query *q, amc_result *out) {
    if (!ctx || !Q || !q || !out || n < 1) return AMC_E_INVALID_ARG;
    if (q->cert_topk < 0 || q->cert_topk > 16 || (q->cert_topk > 0 && q->cert_topk >= n)) return AMC_E_INVALID_ARG;
    if (q->cert_topk > 0 && !(q->r_lower > 0.0)) return AMC_E_INVALID_ARG;
    for (size_t k = 0; k < (size_t)n * n; ++k)
        if (!(Q[k] >= 0.0 && Q[k] <= 1.0)) return AMC_E_INVALID_ARG;
    for (int i = 0; i < n; ++i) {
        double t = 0.0;
        for (int j = 0; j < n; ++j) t += Q[(size_t)i * n + j];
        if (t > 1.0 + 1e-12) return AMC_E_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return AMC_E_HIP;
    hipStream_t st = ctx->stream;
    DevArena A;
    A.stream = st;
    A.async = ctx->async_alloc;
    int rc;
    {
        void *p;
        rc = A.alloc(16, &p);
        if (rc == AMC_OK) {
            int *d_err = (int *)p;
            if (fill_u32(d_err, 4, 0u, st) != hipSuccess) rc = AMC_E_HIP;
            if (rc == AMC_OK) rc = run_tail(n, nullptr, nullptr, Q, 1, 0.0, q, nullptr, q->s, out, st, A, d_err);
            int herr = 0;
            if (rc == AMC_OK && (hipMemcpy(&herr, d_err, 4, hipMemcpyDeviceToHost) != hipSuccess)) rc = AMC_E_HIP;
            if (rc == AMC_OK && (herr & 2)) rc = AMC_E_SINGULAR;
        }
    }
    (void)hipStreamSynchronize(st);
    A.release();
    return rc;
}
