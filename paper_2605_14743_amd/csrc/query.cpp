// query.cpp -- one estimation query on one stream, in stages that contain no
// host synchronisation between them (so a sequence of them can be captured
// into a hipGraph): init (validate, copy inputs, plan) -> alloc (device
// buffers, uploads) -> enqueue reset / sweep / tail -> finish (copy-out).
//
// Paper: Bao, Kontou, Vogiatzis, "Betweenness-Central Nodes Under
// Uncertainty: An Absorbing Markov Chain Approach".
#include "query.hpp"

#include <cmath>
#include <cstring>

#include "amc_kernels.hpp"

namespace amc {

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

static int dev_copy_in(DevArena &A, const void *src, size_t bytes, hipStream_t st, void **out) {
    RCHK(A.alloc(bytes, out));
    if (bytes) HIPCHK(hipMemcpyAsync(*out, src, bytes, hipMemcpyHostToDevice, st));
    return AMC_OK;
}

static int copy_out(void *dst, const void *src, size_t bytes, hipStream_t st) {
    if (dst && bytes) HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
    return AMC_OK;
}

int qr_init(QueryRun &R, amc_ctx *ctx, const amc_graph *g, const amc_model *md, const amc_query *q) {
    RCHK(validate(g, md, q));
    R.ctx = ctx;
    R.g = g;
    R.md = *md;
    R.min.capture(R.md, g->m);
    R.q = *q;
    R.in.capture(R.q, g->n);
    RCHK(plan(ctx, g, &R.md, &R.q, &R.pl));
    R.eta = q->floor_eta < 0.0 ? 0.1 / std::sqrt((double)q->R) : q->floor_eta;
    return AMC_OK;
}

// The descriptor fields every sweep-like launch reads: base graph, network
// law, key, anchor rules and the planned carve-up (uploads the per-edge
// thresholds and the pool mask).
int qr_fill_desc(QueryRun &R, hipStream_t st) {
    DevArena &A = R.A;
    A.stream = st;
    A.async = R.ctx->async_alloc;
    const amc_graph *g = R.g;
    const amc_query *q = &R.q;
    const int n = g->n;
    void *p;
    SweepParams &P = R.P;
    std::memset(&P, 0, sizeof(P));
    P.n = n;
    P.m = g->m;
    P.rp_base = g->d_rp;
    P.col = g->d_col;
    P.slot_edge = g->d_sedge;
    P.eu = g->d_eu;
    P.ev = g->d_ev;
    P.w0 = g->d_w0;
    P.t_fail = prob_threshold(R.md.p_fail);
    if (R.md.p_fail_edge && g->m > 0) {
        R.t_fail_edge.resize((size_t)g->m);
        for (int64_t e = 0; e < g->m; ++e) R.t_fail_edge[e] = prob_threshold(R.md.p_fail_edge[e]);
        RCHK(dev_copy_in(A, R.t_fail_edge.data(), 8 * (size_t)g->m, st, &p));
        P.t_fail_edge = (const uint64_t *)p;
    }
    P.weight_kind = R.md.weight_kind;
    P.w_lo = R.md.w_lo;
    P.w_span = R.md.weight_kind == AMC_WEIGHT_UNIFORM_INT ? R.md.w_hi - R.md.w_lo + 1u
               : R.md.weight_kind == AMC_WEIGHT_TABLE    ? R.md.w_hi
                                                         : 1u;
    if (R.md.weight_kind == AMC_WEIGHT_TABLE && g->m > 0) {
        RCHK(dev_copy_in(A, R.md.w_cdf, 8 * (size_t)g->m * R.md.w_hi, st, &p));
        P.w_cdf = (const uint64_t *)p;
    }
    P.key0 = (uint32_t)q->seed;
    P.key1 = (uint32_t)(q->seed >> 32);
    P.r_begin = q->r_begin;
    P.t_alpha = prob_threshold(q->alpha);
    P.k_min = q->k_min;
    P.tau = q->tie_tau < 0.0 ? 1e-9 : q->tie_tau;
    if (q->pool_size > 0) {
        R.mask.assign((size_t)n, 0);
        for (int k = 0; k < q->pool_size; ++k) R.mask[q->pool[k]] = 1;
        RCHK(dev_copy_in(A, R.mask.data(), (size_t)n, st, &p));
        P.pool = (const uint8_t *)p;
    }
    P.tile = R.pl.tile;
    P.tiles_per_r = R.pl.tiles_per_r;
    P.adj_cap = R.pl.adj_cap;
    P.wave_bytes = R.pl.wave_bytes;
    P.shift = R.pl.shift;
    P.hop_radius = q->hop_radius;
    P.b_global = R.pl.b_global ? 1 : 0;
    return AMC_OK;
}

int qr_alloc(QueryRun &R, hipStream_t st) {
    RCHK(qr_fill_desc(R, st));
    DevArena &A = R.A;
    const amc_graph *g = R.g;
    const amc_query *q = &R.q;
    const int n = g->n;
    const uint32_t Rn = q->R;
    void *p;
    SweepParams &P = R.P;
    const size_t cnt = (size_t)n * (n + 1);
    if (R.ext_counts) P.counts = R.ext_counts;
    else {
        RCHK(A.alloc(4 * cnt, &p));
        P.counts = (uint32_t *)p;
    }
    if (q->pool_size > 0) {
        RCHK(A.alloc(4 * cnt, &p));
        R.cw = (uint32_t *)p;
    }
    if (R.ext_center) P.center_global = R.ext_center;
    else if (q->flags & AMC_WANT_CENTER) {
        RCHK(A.alloc(4 * (size_t)Rn, &p));
        P.center_global = (int32_t *)p;
    }
    if (q->flags & AMC_WANT_NEXT_TABLE) {
        RCHK(A.alloc(4 * (size_t)Rn * n, &p));
        P.next_table = (int32_t *)p;
        if (q->pool_size > 0) {
            RCHK(A.alloc(4 * (size_t)Rn * n, &p));
            R.ntw = (int32_t *)p;
        }
    }
    if (q->flags & AMC_WANT_BSUM) {
        RCHK(A.alloc(8 * (size_t)n, &p));
        P.bsum = (double *)p;
    }
    RCHK(A.alloc(8 * 8, &p)); P.stats = (unsigned long long *)p;
    RCHK(A.alloc(16, &p)); R.d_err = (int *)p;
    P.err = R.d_err;
    RCHK(A.alloc(16, &p)); R.work_ctr = (unsigned int *)p;
    // with k = infinity the sweep applies the pool selector itself; with a
    // finite k the Top-k stage does, from the B(H_r) rows the sweep keeps
    if (q->topk == 0) {
        P.counts_w = R.cw;
        P.next_table_w = R.ntw;
    } else {
        P.keep_rows = 1;
        RCHK(A.alloc(8 * (size_t)n, &p)); R.T.psi = (double *)p;
        RCHK(A.alloc(8 * (size_t)n, &p)); R.T.psi_hat = (double *)p;
        if (q->pool_size > 0) {
            RCHK(A.alloc(8 * (size_t)n, &p)); R.T.psi_w = (double *)p;
            RCHK(A.alloc(8 * (size_t)n, &p)); R.T.psi_w_hat = (double *)p;
        }
        if (q->gamma) {
            RCHK(dev_copy_in(A, q->gamma, 8 * (size_t)n, st, &p));
            R.T.gamma = (double *)p;
        }
        // the Top-k stage's workgroups: their arrays in LDS where they fit,
        // else in global memory (two workgroups per CU)
        const bool gm = topk_lds(n) > (uint32_t)R.ctx->max_lds;
        const uint32_t per_cu =
            gm ? 2u : std::max<uint32_t>(1u, (uint32_t)R.ctx->max_lds / std::max<uint32_t>(topk_lds(n), 1u));
        R.T.topk_blocks = (int)std::min<uint64_t>(Rn, (uint64_t)R.ctx->cu_count * std::min<uint32_t>(per_cu, 8u));
        if (gm) {
            RCHK(A.alloc(topk_global_bytes(n) * (size_t)R.T.topk_blocks, &p));
            R.T.topk_gscr = (unsigned char *)p;
        }
    }
    if (R.pl.tiles_per_r > 1 || P.keep_rows) {
        RCHK(A.alloc(8 * (size_t)Rn * n, &p)); P.Bg = (double *)p;
        RCHK(A.alloc(4 * (size_t)Rn * n, &p)); P.compg = (int32_t *)p;
        RCHK(A.alloc(4 * (size_t)Rn * n, &p)); P.sizeg = (int32_t *)p;
        RCHK(A.alloc(4 * (size_t)Rn, &p)); P.done = (unsigned int *)p;
    }
    if ((q->flags & AMC_WANT_DEBUG) && q->n_debug > 0) {
        RCHK(dev_copy_in(A, q->debug_pairs, 8 * (size_t)q->n_debug, st, &p));
        P.dbg_pairs = (const uint32_t *)p;
        P.n_dbg = q->n_debug;
        RCHK(A.alloc(4 * (size_t)q->n_debug * n, &p)); P.dbg_dist = (uint32_t *)p;
        RCHK(A.alloc(8 * (size_t)q->n_debug * n, &p)); P.dbg_sigma = (unsigned long long *)p;
        RCHK(A.alloc(8 * (size_t)q->n_debug * n, &p)); P.dbg_delta = (double *)p;
    }
    if (R.pl.scratch_words > 0) {
        const int nb = (q->flags & AMC_PLAIN_LAUNCH) ? R.pl.tiles_per_r : R.pl.blocks;
        R.bscratch_words = R.pl.scratch_words;
        RCHK(A.alloc(4 * (size_t)R.bscratch_words * nb, &p));
        R.bscratch = (uint32_t *)p;
    }
    // single-query launch descriptors
    RCHK(dev_copy_in(A, &P, sizeof(SweepParams), st, &p));
    R.d_desc = (SweepParams *)p;
    const uint32_t starts[2] = {0u, (uint32_t)R.pl.items};
    RCHK(dev_copy_in(A, starts, sizeof(starts), st, &p));
    R.d_item_start = (uint32_t *)p;

    // tail buffers
    if (!(q->flags & AMC_SKIP_TAIL)) {
        const size_t nn = (size_t)n * n;
        TailBufs &T = R.T;
        RCHK(A.alloc(8 * nn, &p)); T.Q = (double *)p;
        RCHK(A.alloc(8 * nn, &p)); T.N = (double *)p;
        RCHK(A.alloc(8 * (size_t)n, &p)); T.r = (double *)p;
        RCHK(A.alloc(8 * (size_t)n, &p)); T.mu = (double *)p;
        RCHK(A.alloc(8 * (size_t)n, &p)); T.b = (double *)p;
        RCHK(A.alloc(8 * 8, &p)); T.scal = (double *)p;
        RCHK(A.alloc(4 * 16, &p)); T.top = (int32_t *)p;
        RCHK(A.alloc(4 * (size_t)n, &p)); T.cv = (int32_t *)p;
        RCHK(A.alloc(16, &p)); T.support = (int *)p;
        std::vector<double> s_uni;
        const double *s_host = q->s;
        if (!s_host) {
            s_uni.assign((size_t)n, 1.0 / n);
            s_host = s_uni.data();
        }
        RCHK(dev_copy_in(A, s_host, 8 * (size_t)n, st, &p)); T.s = (double *)p;
        if (q->reward) {
            RCHK(dev_copy_in(A, q->reward, 8 * (size_t)n, st, &p));
            T.f = (double *)p;
        }
        const int k = q->cert_topk;
        if (k > 0) {
            const size_t pairs = (size_t)k * (n - k);
            RCHK(A.alloc(8 * pairs, &p)); T.gap = (double *)p;
            RCHK(A.alloc(8 * pairs, &p)); T.sharp = (double *)p;
            RCHK(A.alloc(8 * pairs, &p)); T.sharp_supp = (double *)p;
            RCHK(A.alloc(pairs, &p)); T.cert_ok = (uint8_t *)p;
        }
        if (q->topk > 0) {
            RCHK(A.alloc(8 * 8, &p));
            T.scal_k = (double *)p;
        }
        if (q->flags & AMC_FALLBACK) {
            std::vector<uint8_t> fm((size_t)n, 0);
            fm[q->fb_node] = 1;
            for (int k = 0; k < q->fb_set_size; ++k) fm[q->fb_set[k]] = 1;
            RCHK(dev_copy_in(A, fm.data(), (size_t)n, st, &p));
            T.fb_mask = (uint8_t *)p;
            HIPCHK(hipStreamSynchronize(st));   // fm is a local vector
            RCHK(A.alloc(4 * (size_t)n * (n + 1), &p)); T.counts_fb = (uint32_t *)p;
            RCHK(A.alloc(8 * nn, &p)); T.Qf = (double *)p;
            RCHK(A.alloc(8 * nn, &p)); T.Nf = (double *)p;
            RCHK(A.alloc(8 * (size_t)n, &p)); T.rf = (double *)p;
            RCHK(A.alloc(8 * (size_t)n, &p)); T.muf = (double *)p;
            RCHK(A.alloc(8 * (size_t)n, &p)); T.bf = (double *)p;
            RCHK(A.alloc(8 * (size_t)n, &p)); T.bcens = (double *)p;
            RCHK(A.alloc(8 * 8, &p)); T.scal_f = (double *)p;
            RCHK(A.alloc(4 * 16, &p)); T.top_f = (int32_t *)p;
            if (!T.scal_k) {
                RCHK(A.alloc(8 * 8, &p));
                T.scal_k = (double *)p;
            }
        }
        if (q->pool_size > 0) {
            RCHK(A.alloc(8 * nn, &p)); T.Qw = (double *)p;
            RCHK(A.alloc(8 * nn, &p)); T.Nw = (double *)p;
            RCHK(A.alloc(8 * (size_t)n, &p)); T.rw = (double *)p;
            RCHK(A.alloc(8 * (size_t)n, &p)); T.muw = (double *)p;
            RCHK(A.alloc(8 * (size_t)n, &p)); T.bw = (double *)p;
            RCHK(A.alloc(8 * (size_t)n, &p)); T.bbar = (double *)p;
            RCHK(A.alloc(8 * (size_t)n, &p)); T.xi = (double *)p;
            RCHK(A.alloc(8 * 8, &p)); T.scal_w = (double *)p;
            RCHK(A.alloc(4 * 16, &p)); T.top_w = (int32_t *)p;
        }
    }
    // the uploads above use pageable host memory: finish them before the
    // host vectors they read from can change
    HIPCHK(hipStreamSynchronize(st));
    return AMC_OK;
}

// Whole realizations leave workgroups idle at the end of the launch (the
// partial last round, and the spread of item times): the last R mod blocks
// realizations, plus one more round of blocks when R >= 2 blocks, run as a
// second descriptor over the same counts and tables, each split into tiles
// of at most n / 16 sources (their partial B rows meet in an exchange buffer
// as in any split realization).  Items are handed out in order, so the short
// tiles come last.  With the rows kept for the finite-k Top-k stage, the
// tail's tiles assemble their rows in place in the kept rows.
int qr_split_tail(QueryRun &R, hipStream_t st) {
    const amc_query &q = R.q;
    Plan &pl = R.pl;
    if ((q.flags & AMC_PLAIN_LAUNCH) || pl.anchored || pl.tiles_per_r != 1 || R.P.n_dbg) return AMC_OK;
    const uint32_t B = (uint32_t)pl.blocks, Rn = q.R;
    if (B < 2 || Rn <= B) return AMC_OK;
    // the partial last round, plus one full round when there are enough
    // realizations, so that the items at the end are short
    const uint32_t tail = Rn % B + (Rn >= 2 * B ? B : 0u);
    if (tail == 0) return AMC_OK;
    const int n = R.g->n;
    const uint32_t want = std::max<uint32_t>(16u, (B + tail - 1) / tail);
    int tile = (int)((n + want - 1) / want);
    tile = std::min(std::max(tile, pl.waves), n);
    const int tiles = (n + tile - 1) / tile;
    if (tiles < 2) return AMC_OK;
    DevArena &A = R.A;
    void *p;
    SweepParams P2 = R.P;
    const uint32_t R0 = Rn - tail;
    P2.r_begin = R.P.r_begin + R0;
    P2.tile = tile;
    P2.tiles_per_r = tiles;
    if (P2.center_global) P2.center_global += R0;
    if (P2.next_table) P2.next_table += (size_t)R0 * n;
    if (P2.next_table_w) P2.next_table_w += (size_t)R0 * n;
    if (R.P.keep_rows) {
        P2.Bg = R.P.Bg + (size_t)R0 * n;
        P2.compg = R.P.compg + (size_t)R0 * n;
        P2.sizeg = R.P.sizeg + (size_t)R0 * n;
        P2.done = R.P.done + R0;
    } else {
        RCHK(A.alloc(8 * (size_t)tail * n, &p)); P2.Bg = (double *)p;
        RCHK(A.alloc(4 * (size_t)tail * n, &p)); P2.compg = (int32_t *)p;
        RCHK(A.alloc(4 * (size_t)tail * n, &p)); P2.sizeg = (int32_t *)p;
        RCHK(A.alloc(4 * (size_t)tail, &p)); P2.done = (unsigned int *)p;
    }
    const SweepParams descs[2] = {R.P, P2};
    RCHK(dev_copy_in(A, descs, sizeof(descs), st, &p));
    R.d_desc = (SweepParams *)p;
    const uint32_t starts[3] = {0u, R0, R0 + tail * (uint32_t)tiles};
    RCHK(dev_copy_in(A, starts, sizeof(starts), st, &p));
    R.d_item_start = (uint32_t *)p;
    R.P2 = P2;
    R.split_tail = true;
    R.tail_R = tail;
    R.nq = 2;
    pl.items = starts[2];
    HIPCHK(hipStreamSynchronize(st));   // descs and starts are locals
    return AMC_OK;
}

int qr_enqueue_reset(QueryRun &R, hipStream_t st) {
    const SweepParams &P = R.P;
    const int n = R.g->n;
    const uint32_t Rn = R.q.R;
    const size_t cnt = (size_t)n * (n + 1);
    HIPCHK(fill_u32(P.counts, cnt, 0u, st));
    if (R.cw) HIPCHK(fill_u32(R.cw, cnt, 0u, st));
    if (R.T.psi) HIPCHK(fill_u32(R.T.psi, 2 * (size_t)n, 0u, st));
    if (R.T.psi_w) HIPCHK(fill_u32(R.T.psi_w, 2 * (size_t)n, 0u, st));
    if (P.bsum) HIPCHK(fill_u32(P.bsum, 2 * (size_t)n, 0u, st));
    HIPCHK(fill_u32(P.stats, 16, 0u, st));
    HIPCHK(fill_u32(R.d_err, 4, 0u, st));
    HIPCHK(fill_u32(R.work_ctr, 4, 0u, st));
    if (P.Bg) {
        HIPCHK(fill_u32(P.Bg, 2 * (size_t)Rn * n, 0u, st));
        HIPCHK(fill_u32(P.done, Rn, 0u, st));
    }
    if (R.split_tail) {
        HIPCHK(fill_u32(R.P2.Bg, 2 * (size_t)R.tail_R * n, 0u, st));
        HIPCHK(fill_u32(R.P2.done, R.tail_R, 0u, st));
    }
    if (P.dbg_dist) {
        HIPCHK(fill_u32(P.dbg_dist, (size_t)P.n_dbg * n, 0xFFFFFFFFu, st));
        HIPCHK(fill_u32(P.dbg_sigma, 2 * (size_t)P.n_dbg * n, 0u, st));
        HIPCHK(fill_u32(P.dbg_delta, 2 * (size_t)P.n_dbg * n, 0u, st));
    }
    if (R.T.support) HIPCHK(fill_u32(R.T.support, 1, 0u, st));
    return AMC_OK;
}

static hipError_t launch_plan(const Plan &pl, const LaunchCtl &LC, int blocks, hipStream_t st) {
    if (pl.anchored) return launch_anchored(LC, pl.weighted, pl.adj_bytes, blocks, pl.waves, pl.lds, st);
    if (pl.mode == AMC_MODE_WAVE || pl.mode == AMC_MODE_WAVE_L2)
        return launch_sweep_wave(LC, pl.weighted, pl.mode == AMC_MODE_WAVE_L2, pl.dist16, pl.sig_global, pl.group,
                                 pl.adj_bytes,
                                 blocks, pl.waves, pl.lds, st);
    return launch_sweep_block(LC, pl.weighted, pl.state_place, blocks, pl.threads, pl.lds, st);
}

int qr_enqueue_sweep(QueryRun &R, hipStream_t st) {
    LaunchCtl LC;
    std::memset(&LC, 0, sizeof(LC));
    LC.descs = R.d_desc;
    LC.item_start = R.d_item_start;
    LC.nq = R.nq;
    LC.work_ctr = R.work_ctr;
    LC.bscratch = R.bscratch;
    LC.bscratch_words = R.bscratch_words;
    R.launches = 0;
    if (R.q.flags & AMC_PLAIN_LAUNCH) {
        LC.static_items = 1;
        LC.n_items = (uint32_t)R.pl.tiles_per_r;
        for (uint32_t rl = 0; rl < R.q.R; ++rl) {
            LC.item_base = rl * (uint32_t)R.pl.tiles_per_r;
            HIPCHK(launch_plan(R.pl, LC, R.pl.tiles_per_r, st));
            ++R.launches;
        }
    } else {
        LC.static_items = 0;
        LC.n_items = (uint32_t)R.pl.items;
        LC.item_base = 0;
        HIPCHK(launch_plan(R.pl, LC, R.pl.blocks, st));
        R.launches = 1;
    }
    return AMC_OK;
}

// Chain algebra of one kernel: Q -> A = I - Q -> N -> mu, b, rewards.
static int tail_chain(int n, const uint32_t *d_counts, uint32_t Rn, double eta, double *Q, double *r, double *N,
                      double *mu, double *b, const double *s, const double *f, const uint8_t *pool, double *bbar,
                      double r_lower, int topk, int32_t *top, double *scal, int *d_err, bool from_Q,
                      hipStream_t st) {
    if (from_Q) HIPCHK(tail_kernel_from_Q(n, Q, r, N, st));
    else HIPCHK(tail_kernel_from_counts(n, d_counts, Rn, eta, Q, r, N, st));
    HIPCHK(tail_invert(n, N, d_err, st));
    HIPCHK(tail_visits(n, N, s, mu, b, f, pool, bbar, pool ? nullptr : r, r_lower, topk, top, scal, st));
    return AMC_OK;
}

// Finite-k Top-k stage (after the sweep): ranks every realization's
// components and accumulates the step rewards and the pool selector.
int qr_enqueue_post(QueryRun &R, hipStream_t st) {
    if (!R.g || R.q.topk == 0) return AMC_OK;
    const SweepParams &P = R.P;
    TopkArgs A;
    A.n = R.g->n;
    A.R = R.q.R;
    A.r_begin = R.q.r_begin;
    A.key0 = P.key0;
    A.key1 = P.key1;
    A.t_alpha = P.t_alpha;
    A.k_min = P.k_min;
    A.tau = P.tau;
    A.topk = R.q.topk;
    A.Bg = P.Bg;
    A.compg = P.compg;
    A.sizeg = P.sizeg;
    A.pool = P.pool;
    A.gamma = R.T.gamma;
    A.psi = R.T.psi;
    A.psi_w = R.T.psi_w;
    A.counts_w = R.cw;
    A.next_table_w = R.ntw;
    A.gscr = R.T.topk_gscr;
    A.gscr_bytes = topk_global_bytes(A.n);
    HIPCHK(launch_topk_reduce(A, R.T.topk_blocks, st));
    // estimated expected step rewards: the sums over the R draws / R
    HIPCHK(tail_div(A.n, R.T.psi, (double)A.R, R.T.psi_hat, st));
    if (R.T.psi_w) HIPCHK(tail_div(A.n, R.T.psi_w, (double)A.R, R.T.psi_w_hat, st));
    return AMC_OK;
}

int qr_enqueue_tail(QueryRun &R, hipStream_t st, bool from_Q) {
    if (R.q.flags & AMC_SKIP_TAIL) return AMC_OK;
    TailBufs &T = R.T;
    const int n = R.g ? R.g->n : R.n_chain;
    const amc_query &q = R.q;
    RCHK(tail_chain(n, R.P.counts, q.R, R.eta, T.Q, T.r, T.N, T.mu, T.b, T.s, T.f, nullptr, nullptr, q.r_lower,
                    q.cert_topk, T.top, T.scal, R.d_err, from_Q, st));
    HIPCHK(tail_certificates(n, q.cert_topk, T.Q, T.N, T.mu, T.top, T.cv, q.eps, q.r_lower, T.gap, T.sharp,
                             T.sharp_supp, T.cert_ok, T.support, st));
    if (R.cw && R.P.pool) {   // constrained kernel P^W (Section 7), same pipeline
        HIPCHK(tail_xi(n, R.cw, q.R, T.xi, st));
        RCHK(tail_chain(n, R.cw, q.R, R.eta, T.Qw, T.rw, T.Nw, T.muw, T.bw, T.s, T.f, R.P.pool, T.bbar, 0.0,
                        0, T.top_w, T.scal_w, R.d_err, false, st));
    }
    // reward-AFCs of the Top-k step rewards (Sections 6.2-6.3)
    if (R.g && q.topk > 0) {
        HIPCHK(tail_reward_afc(n, T.mu, T.scal, T.psi_hat, &T.scal_k[0], st));
        if (T.psi_w_hat) HIPCHK(tail_reward_afc(n, T.mu, T.scal, T.psi_w_hat, &T.scal_k[1], st));
    }
    // fallback kernel P^{W,fb} (Section 7.3) and the censored profile (Section 7.4)
    if (T.counts_fb) {
        HIPCHK(tail_fb_counts(n, R.P.counts, R.cw, q.fb_node, T.counts_fb, st));
        RCHK(tail_chain(n, T.counts_fb, q.R, R.eta, T.Qf, T.rf, T.Nf, T.muf, T.bf, T.s, T.f, R.P.pool, nullptr, 0.0,
                        0, T.top_f, T.scal_f, R.d_err, false, st));
        HIPCHK(tail_censor(n, T.bf, T.fb_mask, T.bcens, &T.scal_k[2], st));
    }
    return AMC_OK;
}

int qr_finish(QueryRun &R, amc_result *out, hipStream_t st) {
    const SweepParams &P = R.P;
    const amc_query &q = R.q;
    const int n = R.g ? R.g->n : R.n_chain;
    const uint32_t Rn = q.R;
    unsigned long long hstats[8] = {0};
    int herr = 0;
    RCHK(copy_out(&herr, R.d_err, 4, st));
    if (P.stats) RCHK(copy_out(hstats, P.stats, 8 * 5, st));
    HIPCHK(hipStreamSynchronize(st));
    if (herr & 1) return AMC_E_SIGMA_OVERFLOW;
    if (herr & 2) return AMC_E_SINGULAR;
    if (R.g) {
        const size_t cnt = (size_t)n * (n + 1);
        RCHK(copy_out(out->counts, P.counts, 4 * cnt, st));
        if (R.cw) RCHK(copy_out(out->counts_w, R.cw, 4 * cnt, st));
        if (P.center_global) RCHK(copy_out(out->center_global, P.center_global, 4 * (size_t)Rn, st));
        if (P.next_table) RCHK(copy_out(out->next_table, P.next_table, 4 * (size_t)Rn * n, st));
        if (R.ntw && out->next_table_w) RCHK(copy_out(out->next_table_w, R.ntw, 4 * (size_t)Rn * n, st));
        if (P.bsum) RCHK(copy_out(out->bsum, P.bsum, 8 * (size_t)n, st));
        if (R.T.psi_hat && out->psi) RCHK(copy_out(out->psi, R.T.psi_hat, 8 * (size_t)n, st));
        if (R.T.psi_w_hat && out->psi_w) RCHK(copy_out(out->psi_w, R.T.psi_w_hat, 8 * (size_t)n, st));
        if (P.dbg_dist) {
            RCHK(copy_out(out->dbg_dist, P.dbg_dist, 4 * (size_t)q.n_debug * n, st));
            RCHK(copy_out(out->dbg_sigma, P.dbg_sigma, 8 * (size_t)q.n_debug * n, st));
            RCHK(copy_out(out->dbg_delta, P.dbg_delta, 8 * (size_t)q.n_debug * n, st));
        }
        out->stats.units = hstats[0];
        out->stats.sum_nK = hstats[1];
        out->stats.sum_AK = hstats[2];
        out->stats.sum_DK = hstats[3];
        out->stats.near_band = hstats[4];
        out->stats.mode = R.pl.mode;
        out->stats.waves = R.pl.waves;
        out->stats.tile = R.pl.tile;
        out->stats.blocks = (q.flags & AMC_PLAIN_LAUNCH) ? R.pl.tiles_per_r : R.pl.blocks;
        out->stats.lds_bytes = (int32_t)R.pl.lds;
        out->stats.launches = R.launches;
        out->stats.group = R.pl.group;
        out->stats.adj_bytes = (int32_t)R.pl.adj_bytes;
        out->stats.dist_bytes = R.pl.dist16 ? 2 : 4;
        out->stats.b_global = R.pl.b_global ? 1 : 0;
        out->stats.sig_global = R.pl.sig_global ? 1 : 0;
        out->stats.state_global = R.pl.state_place;
        out->stats.tail_split = R.split_tail ? (int32_t)R.tail_R : 0;
        out->stats.tail_tiles = R.split_tail ? R.P2.tiles_per_r : 0;
    }
    if (!(q.flags & AMC_SKIP_TAIL)) {
        const TailBufs &T = R.T;
        const size_t nn = (size_t)n * n;
        double hs[8] = {0}, hw[8] = {0};
        int hsupport = 0;
        RCHK(copy_out(out->Q, T.Q, 8 * nn, st));
        RCHK(copy_out(out->r, T.r, 8 * (size_t)n, st));
        if (q.flags & AMC_WANT_N) RCHK(copy_out(out->N, T.N, 8 * nn, st));
        RCHK(copy_out(out->mu, T.mu, 8 * (size_t)n, st));
        RCHK(copy_out(out->b, T.b, 8 * (size_t)n, st));
        RCHK(copy_out(hs, T.scal, 8 * 4, st));
        RCHK(copy_out(&hsupport, T.support, 4, st));
        const int k = q.cert_topk;
        if (k > 0) {
            const size_t pairs = (size_t)k * (n - k);
            RCHK(copy_out(out->top, T.top, 4 * (size_t)k, st));
            RCHK(copy_out(out->cert_v, T.cv, 4 * (size_t)(n - k), st));
            RCHK(copy_out(out->cert_gap, T.gap, 8 * pairs, st));
            RCHK(copy_out(out->cert_sharp, T.sharp, 8 * pairs, st));
            RCHK(copy_out(out->cert_sharp_supp, T.sharp_supp, 8 * pairs, st));
            RCHK(copy_out(out->cert_ok, T.cert_ok, pairs, st));
        }
        if (T.bw) {
            RCHK(copy_out(out->b_w, T.bw, 8 * (size_t)n, st));
            RCHK(copy_out(out->b_w_bar, T.bbar, 8 * (size_t)n, st));
            RCHK(copy_out(out->xi, T.xi, 8 * (size_t)n, st));
            RCHK(copy_out(hw, T.scal_w, 8 * 4, st));
        }
        double hk[8] = {0}, hf[8] = {0};
        if (T.scal_k) RCHK(copy_out(hk, T.scal_k, 8 * 4, st));
        if (T.counts_fb) {
            if (out->b_fb) RCHK(copy_out(out->b_fb, T.bf, 8 * (size_t)n, st));
            if (out->b_cens) RCHK(copy_out(out->b_cens, T.bcens, 8 * (size_t)n, st));
            RCHK(copy_out(hf, T.scal_f, 8 * 4, st));
        }
        HIPCHK(hipStreamSynchronize(st));
        if (R.g && q.topk > 0) {
            out->b_k = hk[0];
            out->b_kw = T.psi_w_hat ? hk[1] : 0.0;
        }
        if (T.counts_fb) {
            out->E_T_fb = hf[0];
            out->m_w_fb = hf[2];
            out->c_fb = hk[2];
        }
        out->E_T = hs[0];
        out->b_f = q.reward ? hs[1] : 0.0;
        out->admissible = hs[3] > 0.5 ? 1 : 0;
        out->epsbar = (double)n * q.eps;
        out->epsbar_supp = (double)hsupport * q.eps;
        out->cert_crude = q.r_lower > 0 ? 2.0 * out->epsbar / (q.r_lower * q.r_lower) : 0.0;
        out->cert_crude_supp = q.r_lower > 0 ? 2.0 * out->epsbar_supp / (q.r_lower * q.r_lower) : 0.0;
        if (T.bw) {
            out->E_T_w = hw[0];
            out->b_w_f = q.reward ? hw[1] : 0.0;
            out->m_w = hw[2];
        }
    }
    HIPCHK(hipStreamSynchronize(st));
    return AMC_OK;
}

void qr_release(QueryRun &R, hipStream_t st) {
    (void)hipStreamSynchronize(st);
    R.A.release();
}

// One complete query on stream `st`, with HIP-event timings of the sweep and
// of the tail (used by amc_run and the serving loop).
int run_query(amc_ctx *ctx, const amc_graph *g, const amc_model *md, const amc_query *q, amc_result *out,
              hipStream_t st) {
    if (!out || !out->counts) return AMC_E_INVALID_ARG;
    if (q && q->pool_size > 0 && !out->counts_w) return AMC_E_INVALID_ARG;
    if (q && q->topk > 0 && (!out->psi || (q->pool_size > 0 && !out->psi_w))) return AMC_E_INVALID_ARG;
    QueryRun R;
    RCHK(qr_init(R, ctx, g, md, q));
    struct Guard {
        QueryRun &r;
        hipStream_t s;
        ~Guard() { qr_release(r, s); }
    } guard{R, st};
    RCHK(qr_alloc(R, st));
    RCHK(qr_split_tail(R, st));
    hipEvent_t ev[4];
    for (auto &e : ev) HIPCHK(hipEventCreate(&e));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() {
            for (int k = 0; k < 4; ++k) (void)hipEventDestroy(e[k]);
        }
    } evg{ev};
    RCHK(qr_enqueue_reset(R, st));
    HIPCHK(hipEventRecord(ev[0], st));
    RCHK(qr_enqueue_sweep(R, st));
    HIPCHK(hipEventRecord(ev[1], st));
    RCHK(qr_enqueue_post(R, st));
    HIPCHK(hipEventRecord(ev[2], st));
    RCHK(qr_enqueue_tail(R, st, false));
    HIPCHK(hipEventRecord(ev[3], st));
    RCHK(qr_finish(R, out, st));
    float ms_sweep = 0.f, ms_post = 0.f, ms_tail = 0.f;
    HIPCHK(hipEventElapsedTime(&ms_sweep, ev[0], ev[1]));
    HIPCHK(hipEventElapsedTime(&ms_post, ev[1], ev[2]));
    HIPCHK(hipEventElapsedTime(&ms_tail, ev[2], ev[3]));
    out->stats.sweep_ms = ms_sweep;
    out->stats.topk_ms = q->topk > 0 ? ms_post : 0.0;
    out->stats.tail_ms = (q->flags & AMC_SKIP_TAIL) ? 0.0 : ms_tail;
    return AMC_OK;
}

}  // namespace amc

using namespace amc;

extern "C" int amc_run(amc_ctx *ctx, const amc_graph *g, const amc_model *model, const amc_query *q,
                       amc_result *out) {
    if (!ctx || !g || g->ctx != ctx || !model || !q) return AMC_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return AMC_E_HIP;
    return run_query(ctx, g, model, q, out, ctx->stream);
}

extern "C" int amc_chain(amc_ctx *ctx, int32_t n, const double *Q, const amc_query *q, amc_result *out) {
    if (!ctx || !Q || !q || !out || n < 1) return AMC_E_INVALID_ARG;
    if (q->cert_topk < 0 || q->cert_topk > 16 || (q->cert_topk > 0 && q->cert_topk >= n)) return AMC_E_INVALID_ARG;
    if (q->cert_topk > 0 && !(q->r_lower > 0.0)) return AMC_E_INVALID_ARG;
    if (!(q->eps >= 0.0)) return AMC_E_INVALID_ARG;
    for (size_t k = 0; k < (size_t)n * n; ++k)
        if (!(Q[k] >= 0.0 && Q[k] <= 1.0)) return AMC_E_INVALID_ARG;
    for (int i = 0; i < n; ++i) {
        double t = 0.0;
        for (int j = 0; j < n; ++j) t += Q[(size_t)i * n + j];
        if (t > 1.0 + 1e-12) return AMC_E_INVALID_ARG;
    }
    if (q->s) {
        double t = 0.0;
        for (int i = 0; i < n; ++i) {
            if (!(q->s[i] >= 0.0)) return AMC_E_INVALID_ARG;
            t += q->s[i];
        }
        if (std::fabs(t - 1.0) > 1e-9) return AMC_E_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return AMC_E_HIP;
    hipStream_t st = ctx->stream;
    QueryRun R;
    R.ctx = ctx;
    R.n_chain = n;
    R.q = *q;
    R.q.flags &= ~(uint32_t)(AMC_SKIP_TAIL | AMC_FALLBACK);
    R.q.pool_size = 0;
    R.q.topk = 0;
    R.q.R = 1;
    struct Guard {
        QueryRun &r;
        hipStream_t s;
        ~Guard() { qr_release(r, s); }
    } guard{R, st};
    DevArena &A = R.A;
    A.stream = st;
    A.async = ctx->async_alloc;
    void *p;
    const size_t nn = (size_t)n * n;
    TailBufs &T = R.T;
    RCHK(dev_copy_in(A, Q, 8 * nn, st, &p)); T.Q = (double *)p;
    RCHK(A.alloc(8 * nn, &p)); T.N = (double *)p;
    RCHK(A.alloc(8 * (size_t)n, &p)); T.r = (double *)p;
    RCHK(A.alloc(8 * (size_t)n, &p)); T.mu = (double *)p;
    RCHK(A.alloc(8 * (size_t)n, &p)); T.b = (double *)p;
    RCHK(A.alloc(8 * 8, &p)); T.scal = (double *)p;
    RCHK(A.alloc(4 * 16, &p)); T.top = (int32_t *)p;
    RCHK(A.alloc(4 * (size_t)n, &p)); T.cv = (int32_t *)p;
    RCHK(A.alloc(16, &p)); T.support = (int *)p;
    RCHK(A.alloc(16, &p)); R.d_err = (int *)p;
    std::vector<double> s_uni((size_t)n, 1.0 / n);
    RCHK(dev_copy_in(A, q->s ? q->s : s_uni.data(), 8 * (size_t)n, st, &p)); T.s = (double *)p;
    if (q->reward) {
        RCHK(dev_copy_in(A, q->reward, 8 * (size_t)n, st, &p));
        T.f = (double *)p;
    }
    if (q->cert_topk > 0) {
        const size_t pairs = (size_t)q->cert_topk * (n - q->cert_topk);
        RCHK(A.alloc(8 * pairs, &p)); T.gap = (double *)p;
        RCHK(A.alloc(8 * pairs, &p)); T.sharp = (double *)p;
        RCHK(A.alloc(8 * pairs, &p)); T.sharp_supp = (double *)p;
        RCHK(A.alloc(pairs, &p)); T.cert_ok = (uint8_t *)p;
    }
    if (hipStreamSynchronize(st) != hipSuccess) return AMC_E_HIP;
    if (fill_u32(R.d_err, 4, 0u, st) != hipSuccess || fill_u32(T.support, 1, 0u, st) != hipSuccess) return AMC_E_HIP;
    RCHK(qr_enqueue_tail(R, st, true));
    return qr_finish(R, out, st);
}
