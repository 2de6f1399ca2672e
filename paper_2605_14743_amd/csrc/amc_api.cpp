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
    if (fixed) {
        if (sz > fixed_cap - fixed_used) return AMC_E_SCRATCH;
        *out = fixed + fixed_used;
        fixed_used += sz;
        return AMC_OK;
    }
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
    if (fixed) {
        fixed_used = 0;
        return;
    }
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
    if (set_sweep_wave_attrs(c->max_lds) != hipSuccess || set_sweep_block_attrs(c->max_lds) != hipSuccess ||
        set_topk_attrs(c->max_lds) != hipSuccess || set_traj_attrs(c->max_lds) != hipSuccess ||
        set_anchored_attrs(c->max_lds) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return AMC_E_HIP;
    }
    if (hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return AMC_E_HIP;
    }
    c->stream = c->own;
    if (hipEventCreate(&c->static_ev[0]) != hipSuccess || hipEventCreate(&c->static_ev[1]) != hipSuccess) {
        (void)hipGetLastError();
        if (c->static_ev[0]) (void)hipEventDestroy(c->static_ev[0]);
        (void)hipStreamDestroy(c->own);
        delete c;
        return AMC_E_HIP;
    }
    // the no-allocation entry point's scratch: its address on this device
    // (a failure only disables amc_sweep_static, which then reports it)
    (void)static_scratch_init(device);
    tune_load(c);
    *out = c;
    return AMC_OK;
}

extern "C" void amc_ctx_destroy(amc_ctx *ctx) {
    if (!ctx) return;
    server_stop(ctx);
    (void)hipSetDevice(ctx->device);
    if (ctx->own) (void)hipStreamDestroy(ctx->own);
    for (hipEvent_t e : ctx->static_ev)
        if (e) (void)hipEventDestroy(e);
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
        case AMC_E_SCRATCH: return "the no-allocation scratch array is too small for this query";
        default: return "unknown status";
    }
}

extern "C" int amc_version(void) { return 100; }

// ---------------------------------------------------------------------------
// validation and planning
// ---------------------------------------------------------------------------
namespace amc {

void ModelInputs::capture(amc_model &md, int64_t m) {
    if (md.p_fail_edge) {
        p_fail_edge.assign(md.p_fail_edge, md.p_fail_edge + m);
        md.p_fail_edge = p_fail_edge.data();
    }
    if (md.weight_kind == AMC_WEIGHT_TABLE && md.w_cdf) {
        w_cdf.assign(md.w_cdf, md.w_cdf + (size_t)m * md.w_hi);
        md.w_cdf = w_cdf.data();
    }
}

void QueryInputs::capture(amc_query &q, int n) {
    if (q.s) {
        s.assign(q.s, q.s + n);
        q.s = s.data();
    }
    if (q.reward) {
        reward.assign(q.reward, q.reward + n);
        q.reward = reward.data();
    }
    if (q.gamma) {
        gamma.assign(q.gamma, q.gamma + n);
        q.gamma = gamma.data();
    }
    if (q.pool_size > 0) {
        pool.assign(q.pool, q.pool + q.pool_size);
        q.pool = pool.data();
    }
    if (q.fb_set_size > 0) {
        fb_set.assign(q.fb_set, q.fb_set + q.fb_set_size);
        q.fb_set = fb_set.data();
    }
    if (q.n_debug > 0) {
        dbg.assign(q.debug_pairs, q.debug_pairs + 2 * q.n_debug);
        q.debug_pairs = dbg.data();
    }
}

// Largest edge weight a realization can draw.
uint64_t model_wmax(const amc_graph *g, const amc_model *md) {
    switch (md->weight_kind) {
        case AMC_WEIGHT_UNIT: return 1u;
        case AMC_WEIGHT_UNIFORM_INT:
        case AMC_WEIGHT_TABLE: return md->w_hi;
        default: return g->w0.empty() ? 1u : *std::max_element(g->w0.begin(), g->w0.end());
    }
}

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
    } else if (md->weight_kind == AMC_WEIGHT_TABLE) {
        if (md->w_hi < 1u || md->w_hi > 255u || (g->m > 0 && !md->w_cdf)) return AMC_E_INVALID_ARG;
        for (int64_t e = 0; e < g->m; ++e) {
            const uint64_t *T = md->w_cdf + (size_t)e * md->w_hi;
            for (uint32_t v = 1; v < md->w_hi; ++v)
                if (T[v] < T[v - 1]) return AMC_E_INVALID_ARG;
            if (T[md->w_hi - 1] != (1ull << 32)) return AMC_E_INVALID_ARG;
        }
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
    if (q->topk < 0 || q->topk > AMC_MAX_TOPK) return AMC_E_INVALID_ARG;
    if (q->topk > 0 && n > AMC_MAX_TOPK_N) return AMC_E_UNSUPPORTED;
    if (q->gamma)
        for (int i = 0; i < n; ++i)
            if (!(q->gamma[i] >= 0.0) || !std::isfinite(q->gamma[i])) return AMC_E_INVALID_ARG;
    if (q->flags & AMC_FALLBACK) {
        if (q->fb_node < 0 || q->fb_node >= n) return AMC_E_INVALID_ARG;
        // a fallback needs a pool; an explicit V_fb holds v_fb and no pool
        // member, while V_fb = {v_fb} may sit inside the pool (Section 9)
        if (q->pool_size <= 0) return AMC_E_INVALID_ARG;
        if (q->fb_set_size < 0 || (q->fb_set_size > 0 && !q->fb_set)) return AMC_E_INVALID_ARG;
        std::vector<uint8_t> inW((size_t)n, 0), inF((size_t)n, 0);
        for (int k = 0; k < q->pool_size; ++k) inW[q->pool[k]] = 1;
        inF[q->fb_node] = 1;
        for (int k = 0; k < q->fb_set_size; ++k) {
            if (q->fb_set[k] < 0 || q->fb_set[k] >= n) return AMC_E_INVALID_ARG;
            inF[q->fb_set[k]] = 1;
        }
        bool has_node = q->fb_set_size == 0;
        for (int k = 0; k < q->fb_set_size; ++k) has_node |= q->fb_set[k] == q->fb_node;
        if (!has_node) return AMC_E_INVALID_ARG;
        if (q->fb_set_size > 0)
            for (int v = 0; v < n; ++v)
                if (inW[v] && inF[v]) return AMC_E_INVALID_ARG;
    }
    if (q->hop_radius < 0) return AMC_E_INVALID_ARG;
    if ((q->flags & AMC_DIST32) && (q->flags & AMC_DIST16)) return AMC_E_INVALID_ARG;
    if ((q->flags & AMC_STATE_GLOBAL) &&
        ((q->flags & AMC_SIGMA_GLOBAL) || q->hop_radius > 0 || (q->mode != AMC_MODE_AUTO && q->mode != AMC_MODE_BLOCK)))
        return AMC_E_INVALID_ARG;
    if (q->hop_radius > 0) {
        if (q->topk > 0 || (q->flags & (AMC_WANT_CENTER | AMC_WANT_BSUM | AMC_WANT_DEBUG | AMC_PLAIN_LAUNCH)) ||
            (q->mode != AMC_MODE_AUTO && q->mode != AMC_MODE_WAVE))
            return AMC_E_INVALID_ARG;
    }
    if (q->mode < AMC_MODE_AUTO || q->mode > AMC_MODE_WAVE_L2) return AMC_E_INVALID_ARG;
    if (q->waves < 0 || q->waves > kMaxWaves || q->tile < 0) return AMC_E_INVALID_ARG;
    if (q->group < 0 || q->group > 16 || (q->group > 4 && q->group != 8 && q->group != 16)) return AMC_E_INVALID_ARG;
    // longest possible distance must stay below the "unreached" sentinel
    const uint64_t wmax = model_wmax(g, md);
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
int plan(const amc_ctx *ctx, const amc_graph *g, const amc_model *md, const amc_query *q_in, Plan *pl) {
    const int n = g->n;
    // a tuned choice for this graph shape fills the fields the caller left open
    amc_query qt = *q_in;
    const amc_query *q = &qt;
    if (qt.mode == AMC_MODE_AUTO && qt.group == 0 && qt.waves == 0) {
        amc_ctx *mc = const_cast<amc_ctx *>(ctx);
        std::lock_guard<std::mutex> lk(mc->tune_mu);
        auto it = mc->tune.find(tune_key(g, md));
        if (it != mc->tune.end()) {
            qt.mode = it->second.mode;
            qt.group = it->second.group;
            qt.waves = it->second.waves;
        }
    }
    const uint32_t adj_cap = (uint32_t)(2 * g->m) + kAdjPad;
    pl->weighted = md->weight_kind != AMC_WEIGHT_UNIT;
    const double avg_deg = n > 0 ? 2.0 * (double)g->m / n : 0.0;
    // default mapping (measured on MI355X): several lanes per vertex pay off
    // only for small graphs, where many sources share the LDS
    (void)avg_deg;
    pl->group = q->group > 0 ? q->group : (n <= 400 && !(q->flags & AMC_SIGMA_GLOBAL) ? 8 : 1);
    // adjacency entry: neighbour in the low bits, weight above; 16 bits when both fit
    uint32_t nbits = 1;
    while ((1u << nbits) < (uint32_t)n) ++nbits;
    const uint64_t wmax = model_wmax(g, md);
    if (nbits < 16 && wmax < (1ull << (16 - nbits)) && adj_cap <= 65535u) {
        pl->adj_bytes = 2;
        pl->shift = nbits;
    } else {
        pl->adj_bytes = 4;
        pl->shift = 16;
    }
    pl->anchored = false;
    // 16-bit distances are possible when every finite distance plus one
    // weight stays below 0xFFFF; the mode choice below decides
    pl->dist16 = (uint64_t)n * wmax < 0xFFFFull && !(q->flags & AMC_DIST32);
    if ((q->flags & AMC_DIST16) && !pl->dist16) return AMC_E_UNSUPPORTED;
    if (q->hop_radius > 0) {
        // anchored neighbourhoods: one wavefront per anchor, lane per vertex
        if (n > kMaxWaveVertices) return AMC_E_UNSUPPORTED;
        int aw = 0;
        uint32_t alds = 0, awb = 0;
        const int cap = q->waves > 0 ? q->waves : kMaxWaves;
        for (int w = 1; w <= cap; ++w) {
            uint32_t wb = 0;
            const uint32_t lds = lds_bytes_anchored(n, adj_cap, pl->adj_bytes, w, &wb);
            if (lds > (uint32_t)ctx->max_lds) break;
            if ((uint64_t)wb * w < 2ull * (uint64_t)g->m) continue;   // per-edge staging
            aw = w;
            alds = lds;
            awb = wb;
        }
        if (aw == 0 || (q->waves > 0 && aw != q->waves)) return AMC_E_UNSUPPORTED;
        pl->anchored = true;
        pl->dist16 = false;
        pl->mode = AMC_MODE_WAVE;
        pl->group = 1;
        pl->waves = aw;
        pl->threads = 64 * aw;
        pl->lds = alds;
        pl->wave_bytes = awb;
        pl->adj_cap = adj_cap;
        pl->scratch_words = 0;
        const uint32_t bpc = std::max<uint32_t>(1u, (uint32_t)ctx->max_lds / alds);
        const uint64_t slots = (uint64_t)ctx->cu_count * bpc;
        int tile = q->tile;
        if (tile <= 0) {
            if ((uint64_t)q->R >= 2 * slots) tile = n;
            else {
                const uint64_t per_r = std::min<uint64_t>((uint64_t)n, (2 * slots + q->R - 1) / q->R);
                tile = std::max((int)((n + per_r - 1) / per_r), aw);
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
    // the 8-slot lane mapping is built for at most 8 wavefronts per workgroup
    const int max_w = pl->group == 3 ? 8 : kMaxWaves;
    if (q->waves > max_w && q->mode != AMC_MODE_BLOCK) return AMC_E_UNSUPPORTED;
    const int want_w = n > kMaxWaveVertices ? 0 : (q->waves > 0 ? q->waves : max_w);
    const uint64_t need = std::max<uint64_t>(2ull * (uint64_t)g->m, kReduceBytesPerVertex * (uint64_t)n);
    // per-wavefront configurations [placement][16-bit distances]: the most
    // wavefronts that fit (or exactly the requested number).  Placement 0:
    // LDS mode; 1: L2 mode with B(H_r) in LDS; 2: L2 mode with B in the
    // global scratch; 3 / 4: as 1 / 2 with every wavefront's path counts in
    // the global scratch as well (lane-per-vertex mappings only)
    constexpr int kPlaces = 5;
    struct Fit {
        int w = 0;
        uint32_t lds = 0, wb = 0;
    } fits[kPlaces][2];
    const bool lane_map = pl->group == 1 || pl->group == 2 || pl->group == 3;
    const bool force_sg = (q->flags & AMC_SIGMA_GLOBAL) != 0;
    if (force_sg && (!lane_map || (q->mode != AMC_MODE_AUTO && q->mode != AMC_MODE_WAVE_L2))) return AMC_E_INVALID_ARG;
    for (int pc = 0; pc < kPlaces; ++pc)
        for (int d16 = 0; d16 < 2; ++d16) {
            if (d16 && !pl->dist16) continue;
            const bool sg = pc >= 3;
            if (sg && !lane_map) continue;
            // the automatic planner does not take these placements: a run
            // that let it choose them left the GPU faulted without a cause
            // found; they run when the caller asks (AMC_SIGMA_GLOBAL)
            if (force_sg != sg) continue;
            Fit &f = fits[pc][d16];
            for (int w = 2; w <= want_w; ++w) {
                uint32_t wb = 0;
                const uint32_t lds = pc ? lds_bytes_wave_l2(n, w, d16 != 0, pc == 2 || pc == 4, sg, &wb)
                                        : lds_bytes_wave(n, adj_cap, pl->adj_bytes, w, d16 != 0, &wb);
                if (lds > (uint32_t)ctx->max_lds) break;
                if ((uint64_t)wb * w < need) continue;   // staging and reduction scratch
                f = Fit{w, lds, wb};
            }
            if (q->waves > 0 && f.w != q->waves) f = Fit{};
        }
    // throughput of one wavefront relative to an LDS-mode wavefront with
    // 32-bit distances (measured on MI355X, ER degree 8, n = 1000 .. 5000):
    // L2 mode 0.92 with B in LDS (adjacency reads at L2), 0.87 with B in the
    // global scratch (B atomics leave the L2); path counts in the global
    // scratch 0.45 / 0.43 on weighted graphs and 0.25 / 0.24 with unit
    // weights (their loads and stores leave the LDS; they pay where many
    // short distance segments leave a few wavefronts latency-bound, i.e. on
    // weighted graphs of n >= 1800, and lose to the workgroup-per-source mode
    // on breadth-first levels); 16-bit distances 0.83 (compare-and-swap
    // minima); per-source rates grow close to linearly with the wavefronts a
    // CU holds up to about 11, more slowly beyond
    const double sg_eff = pl->weighted ? 0.45 : 0.25;
    const double place_eff[kPlaces] = {1.0, 0.92, 0.87, sg_eff, sg_eff * 0.955};
    auto eff = [&](int pc, int d16) { return fits[pc][d16].w * place_eff[pc] * (d16 ? 0.83 : 1.0); };
    auto width = [&](int pc) {
        if (q->flags & AMC_DIST16) return 1;
        return eff(pc, 1) > eff(pc, 0) ? 1 : 0;
    };
    int l2_pc = 1;
    for (int pc = 2; pc < kPlaces; ++pc)
        if (eff(pc, width(pc)) > eff(l2_pc, width(l2_pc))) l2_pc = pc;
    int mode = q->mode;
    const bool force_gs = (q->flags & AMC_STATE_GLOBAL) != 0;
    if (mode == AMC_MODE_AUTO && force_gs) mode = AMC_MODE_BLOCK;
    if (mode == AMC_MODE_AUTO) {
        const double e_lds = eff(0, width(0)), e_l2 = eff(l2_pc, width(l2_pc));
        const double e_best = std::max(e_lds, e_l2);
        // the workgroup-per-source mode, where it fits, wins once few
        // sources stay in flight (measured on MI355X, ER degree 8: unit
        // weights n = 2400, 5 L2 wavefronts 6.6 vs 6.8 M/s, n = 4000, 3 L2
        // wavefronts 2.3 vs 4.8 M/s; weighted n = 5000, 2 L2 wavefronts 1.05
        // vs 1.14 M/s)
        // with unit weights the mode also counts as fitting with its state in
        // the global scratch but distances and row offsets in LDS (measured on
        // MI355X, ER degree 8: n = 5400 1.99 vs 1.39 M/s for two L2
        // wavefronts, n = 6000 1.68 vs 1.12; weighted graphs gain little or
        // lose: n = 5400 0.86 vs 0.99, n = 6000 0.80 vs 0.77)
        const uint32_t block_lds = lds_bytes_block(n, 1024);
        const uint32_t mx = (uint32_t)ctx->max_lds;
        const bool block_fits = !force_sg && 2ull * (uint64_t)g->m <= block_staging_bytes(n) &&
            (block_lds <= mx || (!pl->weighted && lds_bytes_block_hybrid(n) <= mx));
        const double block_below = pl->weighted ? 1.8 : 4.0;
        if (e_best > 0.0 && (!block_fits || e_best >= block_below))
            mode = e_lds >= e_l2 ? AMC_MODE_WAVE : AMC_MODE_WAVE_L2;
        else mode = AMC_MODE_BLOCK;
    }
    pl->mode = mode;
    pl->scratch_words = 0;
    pl->b_global = false;
    pl->sig_global = false;
    pl->state_place = 0;
    if (mode == AMC_MODE_WAVE || mode == AMC_MODE_WAVE_L2) {
        const int pc = mode == AMC_MODE_WAVE_L2 ? l2_pc : 0;
        const int d16 = width(pc);
        const Fit &f = fits[pc][d16];
        if (f.w < 2) return AMC_E_UNSUPPORTED;
        pl->dist16 = d16 != 0;
        pl->b_global = pc == 2 || pc == 4;
        pl->sig_global = pc >= 3;
        pl->waves = f.w;
        pl->lds = f.lds;
        pl->wave_bytes = f.wb;
        pl->threads = 64 * f.w;
        pl->adj_cap = adj_cap;
        if (pc) pl->scratch_words = (uint32_t)l2_scratch_words(n, adj_cap, pl->adj_bytes, pl->sig_global ? f.w : 0);
    } else {
        pl->dist16 = false;
        pl->threads = q->waves > 0 ? 64 * q->waves : 1024;
        // the per-source state stays in LDS where it fits; otherwise it moves
        // to the workgroup's global scratch, keeping the distances and row
        // offsets (the most used arrays) in LDS where those fit; all of it
        // when the caller asks
        const uint32_t mx = (uint32_t)ctx->max_lds;
        pl->state_place = force_gs ? 2 : lds_bytes_block(n, pl->threads) <= mx ? 0
                                   : lds_bytes_block_hybrid(n) <= mx      ? 1
                                                                            : 2;
        pl->lds = pl->state_place == 0   ? lds_bytes_block(n, pl->threads)
                  : pl->state_place == 1 ? lds_bytes_block_hybrid(n)
                                         : 0u;
        // per-edge staging below the row offsets, in either placement
        if (2ull * (uint64_t)g->m > block_staging_bytes(n)) return AMC_E_UNSUPPORTED;
        pl->waves = pl->threads / 64;
        pl->wave_bytes = 0;
        pl->adj_cap = adj_cap;
        const size_t words = block_scratch_words(n, g->m, pl->weighted, pl->state_place);
        if (words > 0xFFFFFFFFull) return AMC_E_UNSUPPORTED;
        pl->scratch_words = (uint32_t)words;
    }
    // sources per work item: whole realizations when there are enough of
    // them to fill the device, otherwise split the sources
    uint32_t blocks_per_cu = std::max<uint32_t>(1u, (uint32_t)ctx->max_lds / std::max<uint32_t>(pl->lds, 1u));
    if (mode != AMC_MODE_WAVE) blocks_per_cu = std::min(blocks_per_cu, kMaxScratchBlocksPerCu);
    // workgroups of 16 wavefronts: two per CU are resident at most
    if (pl->state_place) blocks_per_cu = std::min(blocks_per_cu, 2u);
    const uint64_t slots = (uint64_t)ctx->cu_count * blocks_per_cu;
    int tile = q->tile;
    if (q->flags & AMC_PLAIN_LAUNCH) tile = mode == AMC_MODE_BLOCK ? 1 : pl->waves;
    if (tile <= 0) {
        if ((uint64_t)q->R >= 2 * slots) {
            tile = n;
        } else {
            const uint64_t want_items = 2 * slots;
            const uint64_t per_r = std::min<uint64_t>((uint64_t)n, (want_items + q->R - 1) / q->R);
            tile = (int)((n + per_r - 1) / per_r);
            if (mode != AMC_MODE_BLOCK) tile = std::max(tile, pl->waves);
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
    if (!(q->flags & AMC_SKIP_TAIL)) b += (q->pool_size > 0 ? 4 : 2) * 8 * n * n + (3 * 8 + 1) * 16 * n + 1024;
    // per-workgroup scratch of the block and L2 modes (4-byte entries, upper bound)
    const bool gs = (q->flags & AMC_STATE_GLOBAL) || lds_bytes_block((int)n, 1024) > (uint32_t)g->ctx->max_lds;
    const uint64_t sw = std::max<uint64_t>(block_scratch_words((int)n, g->m, true, gs ? 2 : 0),
                                           l2_scratch_words((int)n, (uint32_t)(2 * g->m) + kAdjPad, 4u, kMaxWaves));
    b += 4 * (uint64_t)g->ctx->cu_count * kMaxScratchBlocksPerCu * sw;
    if (q->n_debug > 0) b += (uint64_t)q->n_debug * n * 20;
    if (q->topk > 0) b += 32 * n + 8 * n;                                  // step rewards, gamma
    if ((q->flags & AMC_FALLBACK) && !(q->flags & AMC_SKIP_TAIL))        // fallback kernel
        b += 4 * n * (n + 1) + 2 * 8 * n * n + 5 * 8 * n + 4096;
    *bytes = b;
    return AMC_OK;
}

// ---------------------------------------------------------------------------
// one query on one stream
// ---------------------------------------------------------------------------
