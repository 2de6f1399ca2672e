// query.hpp -- staged execution of one query (see query.cpp).
#pragma once

#include <vector>

#include "amc_dev.hpp"
#include "amc_runtime.hpp"

namespace amc {

struct TailBufs {
    double *Q = nullptr, *N = nullptr, *r = nullptr, *mu = nullptr, *b = nullptr, *scal = nullptr;
    double *s = nullptr, *f = nullptr;
    int32_t *top = nullptr, *cv = nullptr;
    int *support = nullptr;
    double *gap = nullptr, *sharp = nullptr, *sharp_supp = nullptr;
    uint8_t *cert_ok = nullptr;
    // constrained kernel P^W
    double *Qw = nullptr, *Nw = nullptr, *rw = nullptr, *muw = nullptr, *bw = nullptr, *bbar = nullptr;
    double *xi = nullptr, *scal_w = nullptr;
    int32_t *top_w = nullptr;
    // finite-k Top-k rewards and the fallback kernel P^{W,fb}
    double *psi = nullptr, *psi_w = nullptr;      // sums over draws (sweep stage)
    double *gamma = nullptr;
    double *psi_hat = nullptr, *psi_w_hat = nullptr, *scal_k = nullptr;
    unsigned char *topk_gscr = nullptr;          // Top-k stage arrays in global memory, or nullptr
    int topk_blocks = 0;
    uint32_t *counts_fb = nullptr;
    uint8_t *fb_mask = nullptr;
    double *Qf = nullptr, *Nf = nullptr, *rf = nullptr, *muf = nullptr, *bf = nullptr, *bcens = nullptr;
    double *scal_f = nullptr;
    int32_t *top_f = nullptr;
};

struct QueryRun {
    amc_ctx *ctx = nullptr;
    const amc_graph *g = nullptr;
    int n_chain = 0;                       // amc_chain: size of the given kernel
    amc_model md{};
    amc_query q{};
    ModelInputs min;
    QueryInputs in;
    std::vector<uint64_t> t_fail_edge;
    std::vector<uint8_t> mask;
    Plan pl;
    double eta = 0.0;
    DevArena A;
    SweepParams P{};                       // host copy of the descriptor
    SweepParams *d_desc = nullptr;         // device copy (single-query launches)
    uint32_t *d_item_start = nullptr;
    unsigned int *work_ctr = nullptr;
    uint32_t *bscratch = nullptr;
    uint32_t bscratch_words = 0;
    int *d_err = nullptr;
    int launches = 0;
    uint32_t *cw = nullptr;                // pool-selector counts (sweep or Top-k stage)
    int32_t *ntw = nullptr;                // pool-selector table
    // the last R mod blocks realizations split into tiles (second descriptor)
    bool split_tail = false;
    uint32_t tail_R = 0;
    SweepParams P2{};
    int nq = 1;
    TailBufs T;
    // caller-owned device outputs used instead of allocated ones (no-allocation entry point)
    uint32_t *ext_counts = nullptr;
    int32_t *ext_center = nullptr;
};

int qr_init(QueryRun &R, amc_ctx *ctx, const amc_graph *g, const amc_model *md, const amc_query *q);
int qr_fill_desc(QueryRun &R, hipStream_t st);
int qr_alloc(QueryRun &R, hipStream_t st);
int qr_split_tail(QueryRun &R, hipStream_t st);
int qr_enqueue_reset(QueryRun &R, hipStream_t st);
int qr_enqueue_sweep(QueryRun &R, hipStream_t st);
int qr_enqueue_post(QueryRun &R, hipStream_t st);
int qr_enqueue_tail(QueryRun &R, hipStream_t st, bool from_Q);
int qr_finish(QueryRun &R, amc_result *out, hipStream_t st);
void qr_release(QueryRun &R, hipStream_t st);

}  // namespace amc
