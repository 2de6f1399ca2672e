// amc_runtime.hpp -- host-side state behind the opaque handles of amc.h.
#pragma once

#include <hip/hip_runtime.h>

#include <condition_variable>
#include <deque>
#include <map>
#include <string>
#include <tuple>
#include <mutex>
#include <thread>
#include <vector>

#include "amc.h"

namespace amc {

// Stream-ordered device allocations of one query, released together.  With
// `fixed` set, alloc() carves 256-byte aligned pieces out of that caller-given
// device region instead (no allocator call of any kind; AMC_E_SCRATCH when
// the region is full) and release() forgets them.
struct DevArena {
    hipStream_t stream = nullptr;    // allocation stream
    bool async = false;              // stream-ordered allocator available
    std::vector<void *> ptrs;
    char *fixed = nullptr;
    size_t fixed_cap = 0, fixed_used = 0;
    int alloc(size_t bytes, void **out);
    void release();
};

// Workgroups per CU of the modes that give every workgroup a global scratch.
constexpr uint32_t kMaxScratchBlocksPerCu = 4;
// The per-realization reduction borrows the wavefront regions of a workgroup:
// two u64 and two i32 arrays over the vertices.
constexpr uint64_t kReduceBytesPerVertex = 24;
// Vertex ids in a wavefront region's settled order keep bit 15 for the
// segment tags.
constexpr int kMaxWaveVertices = 0x7FFF;

struct Plan {
    int mode = 0;
    bool weighted = false;
    int group = 8;                  // lanes per vertex in the LDS mode
    uint32_t adj_bytes = 4;         // LDS adjacency entry: 2 (packed) or 4 bytes
    uint32_t shift = 16;            // neighbour bits of an adjacency entry
    int waves = 0, threads = 0;
    uint32_t lds = 0, wave_bytes = 0, adj_cap = 0;
    int tile = 0, tiles_per_r = 1;
    uint64_t items = 0;
    int blocks = 0;
    uint32_t scratch_words = 0;     // per-workgroup global scratch (block and L2 modes)
    bool anchored = false;          // anchored r-hop neighbourhoods (own kernel)
    bool dist16 = false;            // 16-bit distance entries in the wavefront regions
    bool b_global = false;          // L2 mode: B(H_r) in the global scratch instead of LDS
    bool sig_global = false;        // L2 mode: path counts in the global scratch instead of LDS
    int state_place = 0;            // workgroup mode: per-source state in LDS (0), in the global scratch
                                    // but for distances and row offsets (1), all in the scratch (2)
};

// Private copies of the arrays a query points to (inputs are never retained):
// capture() copies them and redirects the query's pointers to the copies.
struct ModelInputs {
    std::vector<double> p_fail_edge;
    std::vector<uint64_t> w_cdf;
    void capture(amc_model &md, int64_t m);
};

struct QueryInputs {
    std::vector<double> s, reward, gamma;
    std::vector<int32_t> pool, fb_set;
    std::vector<uint32_t> dbg;
    void capture(amc_query &q, int n);
};

struct Server;

// Shape key of the autotuner cache: n, m, weight law, largest weight.
using TuneKey = std::tuple<int32_t, int64_t, int32_t, uint32_t>;
struct TuneChoice {
    int32_t mode, group, waves;
    double units_per_s;
};

}  // namespace amc

struct amc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t own = nullptr;
    uint64_t budget = 0;
    int cu_count = 0;
    int max_lds = 65536;
    bool async_alloc = false;
    std::mutex mu;                   // serialises amc_run / amc_chain on the context stream
    std::mutex server_mu;
    amc::Server *server = nullptr;
    std::mutex tune_mu;
    std::map<amc::TuneKey, amc::TuneChoice> tune;
    std::string tune_path;
    hipEvent_t static_ev[2] = {nullptr, nullptr};   // timing events of amc_sweep_static (made at creation)
};

struct amc_graph {
    amc_ctx *ctx = nullptr;
    int32_t n = 0;
    int64_t m = 0;
    std::vector<int32_t> eu, ev, rp;
    std::vector<uint32_t> w0;
    int32_t max_deg = 0;
    int32_t *d_rp = nullptr;
    uint16_t *d_col = nullptr;
    int32_t *d_sedge = nullptr;
    int32_t *d_eu = nullptr, *d_ev = nullptr;
    uint32_t *d_w0 = nullptr;
    amc::DevArena arena;
};

namespace amc {

uint64_t model_wmax(const amc_graph *g, const amc_model *md);
int validate(const amc_graph *g, const amc_model *md, const amc_query *q);
int plan(const amc_ctx *ctx, const amc_graph *g, const amc_model *md, const amc_query *q, Plan *pl);
uint64_t prob_threshold(double p);
TuneKey tune_key(const amc_graph *g, const amc_model *md);
void tune_load(amc_ctx *ctx);
int run_query(amc_ctx *ctx, const amc_graph *g, const amc_model *md, const amc_query *q, amc_result *out,
              hipStream_t st);
void server_stop(amc_ctx *ctx);
// Looks up, once per device (the device current), the address of that
// device's copy of the no-allocation scratch array.
int static_scratch_init(int device);

}  // namespace amc
