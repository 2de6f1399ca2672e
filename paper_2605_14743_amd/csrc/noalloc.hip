// noalloc.hip -- amc_sweep_static: the sweep of amc_run (counts and global
// centres, no tail) for callers that cannot allocate device memory.
//
// Every device buffer the sweep needs beyond the caller's outputs comes from
// `scratch`, a file-scope device array.  Host code never uses the array's
// name as an address: the name is a host-side stand-in, so each device's
// copy is looked up once with hipGetSymbolAddress (static_scratch_init, at
// context creation with the device current) and that address is what the
// query's arena carves from and what the kernels receive.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "amc.h"
#include "amc_kernels.hpp"
#include "query.hpp"

namespace amc {

namespace {

constexpr size_t kStaticScratchBytes = AMC_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// Per device: the address of its copy of `scratch`, and the lock that keeps
// calls on that device from overlapping (they share the array).
struct DeviceScratch {
    std::mutex mu;
    bool looked_up = false;
    void *ptr = nullptr;
};
DeviceScratch g_scratch[kMaxDevices];

}  // namespace

int static_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return AMC_E_UNSUPPORTED;
    DeviceScratch &d = g_scratch[device];
    std::lock_guard<std::mutex> lk(d.mu);
    if (!d.looked_up) {
        d.looked_up = true;
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p) d.ptr = p;
        else (void)hipGetLastError();
    }
    return d.ptr ? AMC_OK : AMC_E_HIP;
}

}  // namespace amc

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

extern "C" int amc_sweep_static(amc_ctx *ctx, const amc_graph *g, const amc_model *model, const amc_query *q,
                                uint32_t *d_counts, int32_t *d_center, amc_stats *stats) {
    if (!ctx || !g || g->ctx != ctx || !model || !q || !d_counts) return AMC_E_INVALID_ARG;
    const uint32_t allowed = AMC_DIST16 | AMC_DIST32 | AMC_SKIP_TAIL | AMC_SIGMA_GLOBAL;
    if ((q->flags & ~allowed) || q->pool_size != 0 || q->topk != 0 || q->n_debug != 0 || q->hop_radius != 0 ||
        model->p_fail_edge || model->weight_kind == AMC_WEIGHT_TABLE)
        return AMC_E_INVALID_ARG;
    if (ctx->device < 0 || ctx->device >= kMaxDevices) return AMC_E_UNSUPPORTED;
    // the tail's inputs are not used; clearing them keeps the query free of
    // host-side copies
    amc_query qq = *q;
    qq.flags = (q->flags & (AMC_DIST16 | AMC_DIST32 | AMC_SIGMA_GLOBAL)) | AMC_SKIP_TAIL |
               (d_center ? AMC_WANT_CENTER : 0u);
    qq.s = nullptr;
    qq.reward = nullptr;
    qq.gamma = nullptr;
    qq.fb_set = nullptr;
    qq.fb_set_size = 0;
    qq.cert_topk = 0;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceScratch &d = g_scratch[ctx->device];
    std::lock_guard<std::mutex> lk2(d.mu);
    if (!d.ptr) return AMC_E_HIP;
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    // whatever this call enqueued has finished before the array is handed to
    // the next call, on every return path
    struct Drain {
        hipStream_t s;
        ~Drain() { (void)hipStreamSynchronize(s); }
    } drain{st};
    QueryRun R;
    RCHK(qr_init(R, ctx, g, model, &qq));
    R.A.fixed = (char *)d.ptr;
    R.A.fixed_cap = kStaticScratchBytes;
    R.ext_counts = d_counts;
    R.ext_center = d_center;
    RCHK(qr_alloc(R, st));           // carves from the array: AMC_E_SCRATCH before any launch
    RCHK(qr_split_tail(R, st));
    HIPCHK(hipEventRecord(ctx->static_ev[0], st));
    RCHK(qr_enqueue_reset(R, st));   // counts, counters and exchange rows cleared by fill kernels
    RCHK(qr_enqueue_sweep(R, st));
    HIPCHK(hipEventRecord(ctx->static_ev[1], st));
    int herr = 0;
    unsigned long long hs[5] = {0, 0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(&herr, R.d_err, sizeof(herr), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hs, R.P.stats, sizeof(hs), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    R.A.release();
    if (herr & 1) return AMC_E_SIGMA_OVERFLOW;
    if (stats) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ctx->static_ev[0], ctx->static_ev[1]));
        std::memset(stats, 0, sizeof(*stats));
        stats->units = hs[0];
        stats->sum_nK = hs[1];
        stats->sum_AK = hs[2];
        stats->sum_DK = hs[3];
        stats->near_band = hs[4];
        stats->sweep_ms = ms;
        stats->mode = R.pl.mode;
        stats->waves = R.pl.waves;
        stats->tile = R.pl.tile;
        stats->blocks = R.pl.blocks;
        stats->lds_bytes = (int32_t)R.pl.lds;
        stats->launches = R.launches;
        stats->group = R.pl.group;
        stats->adj_bytes = (int32_t)R.pl.adj_bytes;
        stats->dist_bytes = R.pl.dist16 ? 2 : 4;
        stats->b_global = R.pl.b_global ? 1 : 0;
        stats->sig_global = R.pl.sig_global ? 1 : 0;
        stats->state_global = R.pl.state_place;
        stats->tail_split = R.split_tail ? (int32_t)R.tail_R : 0;
        stats->tail_tiles = R.split_tail ? R.P2.tiles_per_r : 0;
    }
    return AMC_OK;
}
