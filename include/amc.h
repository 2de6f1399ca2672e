/*
 * amc.h -- C-ABI of the MI355X engine for absorbing-frequency centrality (AFC).
 *
 * Paper: W. Bao, E. Kontou, C. Vogiatzis, "Betweenness-Central Nodes Under
 * Uncertainty: An Absorbing Markov Chain Approach".
 *
 * The library estimates the absorbing Markov chain (AMC) on reported local
 * betweenness centres by the row-wise Monte Carlo construction of Alg. 1 /
 * Alg. 2 and turns the estimated kernel into AFC and its companions:
 *
 *   for every realization r and every anchor i:
 *     next(r,i) = bottom              if the exogenous stop coin fires
 *                                     or |K(i;H_r)| < k_min        (Section 3.2)
 *               = c_loc(i;H_r)        the tie-broken maximiser of the
 *                                     betweenness B(H_r) over K(i;H_r)
 *                                                       (eq. local-center)
 *   counts C[i][j] = #{r : next(r,i) = j}                       (Alg. 2)
 *   N = (I - Q)^{-1}, mu = sN, E_s[T] = mu 1, b = mu / mu 1
 *                                    (eqs. fundamental, visits, afc-def)
 *
 * Conventions shared by every call:
 *   - Vertices are 0 .. n-1.  The base graph is undirected and simple and is
 *     passed as a canonical edge list: eu[e] < ev[e] and the pairs strictly
 *     increasing in lexicographic order.  Anything else is AMC_E_INVALID_ARG.
 *   - Realization r of the network state (Section 3.1) is a pure function of
 *     (seed, r): edge (u,v) survives and draws its integer weight from the
 *     Philox4x32-10 block of counter (r, u, v, 0) and key (seed mod 2^32,
 *     seed >> 32); the stop coin of anchor i uses counter (r, i, 2^32-1, 1).
 *     An event of probability p fires when the first 32-bit word is below
 *     floor(p * 2^32); an integer weight uniform on [lo, hi] is
 *     lo + ((x1 * (hi - lo + 1)) >> 32).
 *   - Ties (Corollary on deterministic tie-breaking): inside a vertex set the
 *     reported vertex is the smallest index v with
 *     max_B - B_v <= tie_tau * max(max_B, 1).
 *   - Pointers in the structs below are host pointers unless stated.  Inputs
 *     are read during the call and never retained.  Result buffers are owned
 *     by the caller and must stay valid until amc_run returns (or until
 *     amc_wait / a successful amc_poll for amc_submit).
 *   - Every call returns AMC_OK (0) or a negative status; no exception
 *     crosses the ABI.  A failed call leaves result buffers unspecified.
 */
#ifndef AMC_H
#define AMC_H

#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define AMC_API __attribute__((visibility("default")))
#else
#define AMC_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define AMC_OK 0
#define AMC_E_INVALID_ARG (-1)    /* bad size, range, edge list or option   */
#define AMC_E_OOM (-2)            /* device or host allocation failed       */
#define AMC_E_HIP (-3)            /* a HIP runtime call failed              */
#define AMC_E_SIGMA_OVERFLOW (-4) /* a shortest-path count exceeded 2^64-1  */
#define AMC_E_SINGULAR (-5)       /* I - Q singular (row never absorbs, no floor) */
#define AMC_E_ADMISSION (-6)      /* query footprint exceeds the context budget */
#define AMC_E_NOT_READY (-7)      /* amc_poll: the request is still running */
#define AMC_E_UNSUPPORTED (-8)    /* the shape exceeds an engine limit      */
#define AMC_E_SCRATCH (-9)        /* amc_sweep_static: the query needs more than the static scratch */

/* ------------------------------------------------------------ weight law */
#define AMC_WEIGHT_UNIT 0         /* every surviving edge has weight 1 (BFS)   */
#define AMC_WEIGHT_UNIFORM_INT 1  /* integer weight uniform on [w_lo, w_hi]    */
#define AMC_WEIGHT_FIXED 2        /* the graph's own integer weights w0        */
#define AMC_WEIGHT_TABLE 3        /* per-call resampled weight from a per-edge law (Section 9.2) */

/* --------------------------------------------------------- sweep mode */
#define AMC_MODE_AUTO 0           /* pick from the shape (autotuner)           */
#define AMC_MODE_WAVE 1           /* graph staged in LDS, one wavefront per (r, s) */
#define AMC_MODE_BLOCK 2          /* one workgroup per (r, s), frontier queues */
#define AMC_MODE_WAVE_L2 3        /* one wavefront per (r, s); realized graph and B in an
                                     L2-resident per-workgroup scratch, LDS for per-source state */

/* ----------------------------------------------------------- query flags */
#define AMC_WANT_N (1u << 0)          /* copy the fundamental matrix N           */
#define AMC_WANT_BSUM (1u << 1)       /* sum over r of B(H_r)                     */
#define AMC_WANT_NEXT_TABLE (1u << 2) /* next(r,i) for every r, i                 */
#define AMC_WANT_CENTER (1u << 3)     /* global centre c(H_r) (eq. central-node)  */
#define AMC_WANT_DEBUG (1u << 4)      /* d, sigma, delta of listed (r, s) pairs   */
#define AMC_SKIP_TAIL (1u << 5)       /* counts only, no chain algebra            */
#define AMC_PLAIN_LAUNCH (1u << 6)    /* one kernel launch per realization        */
#define AMC_FALLBACK (1u << 7)        /* fallback kernel P^{W,fb} with v_fb = fb_node */
#define AMC_DIST32 (1u << 8)          /* per-source distance entries of 32 bits ...          */
#define AMC_DIST16 (1u << 9)          /* ... or of 16 bits (needs n * w_max < 0xFFFF); without
                                         either flag the planner picks the width that keeps
                                         more sources in flight.  Results are identical.
                                         Both flags: AMC_E_INVALID_ARG.  The workgroup-per-
                                         source and anchored kernels keep 32-bit entries. */
#define AMC_STATE_GLOBAL (1u << 11)   /* workgroup-per-source mode with the whole per-source state
                                         (distances, path counts, visit order, B(H_r), labels, realized
                                         row offsets) in the per-workgroup global scratch instead of LDS.
                                         Without the flag the planner moves the state there by itself
                                         when no other mode fits (graphs up to 65535 vertices), keeping
                                         distances and row offsets in LDS while they fit (8 n bytes).
                                         Mode AUTO or BLOCK, not with AMC_SIGMA_GLOBAL or hop_radius.
                                         Results are identical. */
#define AMC_SIGMA_GLOBAL (1u << 10)   /* L2 mode with every wavefront's path counts in the per-workgroup
                                         global scratch instead of LDS (more sources in flight on large
                                         graphs); needs a lane-per-vertex mapping (group 0 .. 3) and
                                         mode AUTO or WAVE_L2.  Without it the path counts stay in LDS.
                                         Results are identical. */

typedef struct amc_ctx amc_ctx;
typedef struct amc_graph amc_graph;
typedef struct amc_request amc_request;
typedef struct amc_batch amc_batch;

/* Network-state law (Section 3.1: availability set and positive weights). */
typedef struct amc_model {
    double p_fail;              /* failure probability of every edge, in [0,1]   */
    const double *p_fail_edge;  /* optional per-edge failure probabilities (m)   */
    int32_t weight_kind;        /* AMC_WEIGHT_*                                   */
    uint32_t w_lo, w_hi;        /* AMC_WEIGHT_UNIFORM_INT: 1 <= w_lo <= w_hi <= 65535;
                                   AMC_WEIGHT_TABLE: w_hi = w_max <= 255             */
    /* AMC_WEIGHT_TABLE: m x w_max cumulative thresholds, row e nondecreasing with
     * T[e][w_max-1] = 2^32; edge e of a realization weighs the smallest v in
     * 1..w_max with x1 < T[e][v-1] (x1 the second word of its Philox block) */
    const uint64_t *w_cdf;
} amc_model;

/* One estimation query (Alg. 2 plus the post-processing of Section 8.3). */
typedef struct amc_query {
    uint64_t seed;              /* realization key                                 */
    uint32_t R;                 /* realizations in this call (samples per row), >= 1 */
    uint32_t r_begin;           /* first realization index (split runs / resume)   */
    double alpha;               /* exogenous stop probability, in (0, 1]            */
    uint32_t k_min;             /* smallest valid component size (Section 3.2)      */
    double tie_tau;             /* tie band; < 0 selects 1e-9                       */
    double floor_eta;           /* floor on an empty absorption column; < 0 selects
                                   0.1/sqrt(R); 0 disables (Section 8.2)            */
    const double *s;            /* initial distribution (n) or NULL for uniform     */
    const int32_t *pool;        /* candidate pool W (Section 7.1) or NULL           */
    int32_t pool_size;
    const double *reward;       /* node values f (n) or NULL (eq. mr-inner-product) */
    double eps;                 /* row-wise radius of every entry eps_ij (Section 5.1) */
    double r_lower;             /* leak lower bound of every row, in (0, 1]         */
    int32_t cert_topk;          /* nominal Top-k whose boundary pairs are certified (0 = none) */
    uint32_t flags;             /* AMC_WANT_* / AMC_SKIP_TAIL / AMC_PLAIN_LAUNCH     */
    int32_t mode;               /* AMC_MODE_*                                        */
    int32_t tile;               /* sources per work item; 0 = chosen by the engine   */
    int32_t waves;              /* wavefronts per workgroup; 0 = chosen by the engine */
    int32_t group;              /* AMC_MODE_WAVE / _WAVE_L2 vertex mapping: 1 / 2 / 3 = one lane per vertex with
                                   4 / 2 / 8 adjacency slots in flight; 4, 8, 16 = lanes per vertex;
                                   0 = engine */
    const uint32_t *debug_pairs; /* AMC_WANT_DEBUG: n_debug pairs (r, s), r absolute */
    int32_t n_debug;            /* at most 64                                        */
    /* Finite-k local Top-k (Section 3.3, eq. local-topk).  topk = 0 keeps k
     * infinite: the pool selector takes the tie-broken maximiser of B over
     * K(i;H_r) ∩ W.  With 1 <= topk <= AMC_MAX_TOPK (and n <= AMC_MAX_TOPK_N)
     * every component is ranked by applying the tie rule repeatedly (the
     * maximiser, then the maximiser of the rest, ...); C_k(i) is the first
     * min(k, |K|) ranked vertices on a valid draw, empty otherwise
     * (eq. realized-topk-set).  The run then reports the Top-k step rewards
     * psi_i = E_i[sum of gamma over C_k(i)] and psi_W,i = E_i[sum of gamma over
     * C_k(i) ∩ W] (Sections 6.2-6.3) with their reward-AFCs, and the pool
     * selector becomes the highest-ranked member of C_k(i) ∩ W (Section 7.1). */
    int32_t topk;
    const double *gamma;        /* node values gamma (n, >= 0) or NULL for 1         */
    /* Fallback kernel P^{W,fb} (Section 7.3) and censoring (Section 7.4),
     * with AMC_FALLBACK: fb_node = v_fb (needs a pool), fb_set = V_fb
     * (fb_set_size vertices, disjoint from W, containing fb_node).  fb_set =
     * NULL takes V_fb = {fb_node}, and then fb_node may lie in W, as in the
     * structure-constrained experiment of Section 9 (v_fb = the smallest
     * vertex of the first chosen 3-clique). */
    int32_t fb_node;
    const int32_t *fb_set;
    int32_t fb_set_size;
    /* Anchored r-hop neighbourhoods (Section 9.2), hop_radius = r > 0: anchor
     * i's step ranks the betweenness of the subgraph of H_r induced by S_r(i),
     * the vertices within r surviving hops of i, and is invalid when |S_r(i)|
     * < k_min (or the coin fires).  Each anchor then needs its own
     * betweenness: the work counters count |S_r(i)| source passes per anchor.
     * Not combined with topk, AMC_WANT_CENTER, AMC_WANT_BSUM, AMC_WANT_DEBUG
     * or AMC_PLAIN_LAUNCH; runs in LDS mode only.  0 = off. */
    int32_t hop_radius;
} amc_query;

#define AMC_MAX_TOPK 64
#define AMC_MAX_TOPK_N 65535   /* the graph limit: past the LDS the stage's arrays go to global memory */

/* Counters of one run.  units = R n (one (r, s) pass each); sum_nK, sum_AK and
 * sum_DK add, over every (r, s), the reached vertices |K(s;H_r)|, the surviving
 * directed adjacency slots inside K(s;H_r) and the base directed slots of its
 * vertices. near_band counts set members whose gap to the set maximum lies in
 * [band/4, 4 band]. */
typedef struct amc_stats {
    uint64_t units, sum_nK, sum_AK, sum_DK, near_band;
    double sweep_ms;            /* HIP-event time of the sweep kernel(s) on the context stream */
    double tail_ms;             /* HIP-event time of the tail kernels                          */
    int32_t mode, waves, tile, blocks, lds_bytes, launches, group, adj_bytes;
    double topk_ms;             /* HIP-event time of the finite-k Top-k stage (topk > 0) */
    int32_t dist_bytes;         /* bytes per distance entry of the per-source state (2 or 4) */
    int32_t b_global;           /* L2 mode: 1 = B(H_r) in the L2-resident scratch, 0 = in LDS */
    int32_t tail_split;         /* last realizations run split into tiles (R mod blocks), 0 = none */
    int32_t tail_tiles;         /* tiles per such realization                                   */
    int32_t sig_global;         /* L2 mode: 1 = path counts in the global scratch, 0 = in LDS    */
    int32_t state_global;       /* workgroup mode: per-source state 0 = in LDS, 1 = in the global
                                   scratch but for distances and row offsets, 2 = all in the scratch */
} amc_stats;

/* Caller-owned host buffers; NULL pointers are skipped. */
typedef struct amc_result {
    uint32_t *counts;           /* n x (n+1), column n = bottom (required)      */
    uint32_t *counts_w;         /* n x (n+1) counts of the pool kernel P^W       */
    int32_t *center_global;     /* R: c(H_r) (AMC_WANT_CENTER)                   */
    int32_t *next_table;        /* R x n, -1 = bottom (AMC_WANT_NEXT_TABLE)      */
    int32_t *next_table_w;      /* R x n, pool kernel                            */
    double *bsum;               /* n: sum_r B(H_r) (AMC_WANT_BSUM)               */
    double *Q, *r;              /* n x n, n: stabilised kernel                   */
    double *N;                  /* n x n (AMC_WANT_N)                            */
    double *mu, *b;             /* n, n                                          */
    double *b_w, *xi, *b_w_bar; /* n each: AFC, feasibility and within-pool profile of P^W */
    int32_t *top;               /* cert_topk: nominal Top-k by b (ties to the smaller index) */
    int32_t *cert_v;            /* n - cert_topk: the complement, increasing     */
    double *cert_gap;           /* cert_topk x (n-cert_topk): G_uv (eq. pm-gap)  */
    double *cert_sharp;         /* same shape: sharp thresholds (eq. sharp-gap)  */
    double *cert_sharp_supp;    /* same shape, support-restricted radii          */
    uint32_t *dbg_dist;         /* n_debug x n (0xFFFFFFFF = unreachable)        */
    uint64_t *dbg_sigma;        /* n_debug x n                                    */
    double *dbg_delta;          /* n_debug x n                                    */
    /* scalars written by the call */
    double E_T, b_f;            /* E_s[T] and b . f                                */
    double E_T_w, m_w, b_w_f;   /* pool kernel: E_s[T], pool mass m_W (eq. settopk-bPsi), b^W . f */
    double cert_crude, epsbar;  /* 2 epsbar / r_lower^2 and epsbar = n eps        */
    double cert_crude_supp, epsbar_supp; /* support-restricted variants           */
    int32_t admissible;         /* 1 when every r_i >= r_lower                    */
    amc_stats stats;
    /* finite-k Top-k rows (topk > 0) */
    double *psi;                /* n: estimated Top-k step reward psi_i (sum over draws / R) */
    double *psi_w;              /* n: pool-restricted step reward (needs a pool)  */
    double b_k, b_kw;           /* reward-AFCs s N psi / s N 1 (eq. mr-afc-def, eq. mr-pool-afc) */
    /* fallback kernel (AMC_FALLBACK) */
    double *b_fb;               /* n: AFC of P^{W,fb}                             */
    double *b_cens;             /* n: censored profile, 0 on V_fb (Section 7.4)   */
    double E_T_fb, m_w_fb, c_fb;/* E_s[T], pool mass and mass off V_fb under P^{W,fb} */
    /* certificates of the boundary pairs (cert_topk x (n-cert_topk), Section 5.5):
     * bit 0: G_uv above the sharp threshold (eq. sharp-gap), so u ahead of v is
     * certified; bit 1: the same with the support-restricted radii; bit 2: G_uv
     * above the crude threshold 2 epsbar / r_lower^2 */
    uint8_t *cert_ok;
} amc_result;

/* Context: one device, one stream, an HBM budget for admission (0 = free HBM). */
AMC_API int amc_ctx_create(int device, uint64_t hbm_budget_bytes, amc_ctx **out);
AMC_API void amc_ctx_destroy(amc_ctx *ctx);
/* Launch on a caller stream (a hipStream_t, e.g. a torch stream); NULL = own stream. */
AMC_API int amc_ctx_set_stream(amc_ctx *ctx, void *hip_stream);
/* The context stream (hipStream_t), for callers that time or order work on it. */
AMC_API void *amc_ctx_stream(amc_ctx *ctx);

/* Stage a base graph G(V,E) (Section 3.1) on the device.  n >= 1, m >= 0,
 * canonical edge list as above; w0 (m) is required for AMC_WEIGHT_FIXED and
 * may be NULL otherwise.  Limits: n <= 65535, w0[e] in [1, 65535]. */
AMC_API int amc_graph_create(amc_ctx *ctx, int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                     const uint32_t *w0, amc_graph **out);
AMC_API void amc_graph_destroy(amc_graph *g);

/* Device bytes a query needs beyond the staged graph. */
AMC_API int amc_footprint(const amc_graph *g, const amc_query *q, uint64_t *bytes);

/* Synchronous estimation: sweep (Alg. 1 for every anchor over R realizations,
 * counted as in Alg. 2) followed, unless AMC_SKIP_TAIL, by the tail. */
AMC_API int amc_run(amc_ctx *ctx, const amc_graph *g, const amc_model *model, const amc_query *q, amc_result *out);

/* Asynchronous estimation through the context's serving loop: the query is
 * admitted when its footprint fits the budget and a slot is free, runs
 * overlapped with other admitted queries, and completes into `out`.
 * Returns AMC_E_ADMISSION at once if the footprint can never fit. */
AMC_API int amc_submit(amc_ctx *ctx, const amc_graph *g, const amc_model *model, const amc_query *q, amc_result *out,
               amc_request **req);
AMC_API int amc_poll(amc_request *req);        /* AMC_E_NOT_READY, or the final status */
AMC_API int amc_wait(amc_request *req);        /* blocks; returns the final status     */
AMC_API void amc_request_destroy(amc_request *req);
/* Serving timestamps of a finished request, seconds on a monotonic clock:
 * t[0] submit, t[1] admitted, t[2] finished. */
AMC_API int amc_request_times(amc_request *req, double t[3]);

/* Counters of the context's serving loop since its start (all zero before the
 * first amc_submit): the admission budget and the largest sum of admitted
 * footprints (never above the budget), queries admitted and completed, the
 * sweep launches the loop issued, how many of them carried work items of two
 * or more queries, the most queries admitted at one time and the most
 * queries that shared one launch. */
typedef struct amc_server_stats {
    uint64_t budget;            /* admission budget, bytes                       */
    uint64_t peak_in_use;       /* largest sum of admitted footprints, bytes      */
    uint64_t admitted, completed;
    uint64_t launches;          /* sweep launches issued by the loop              */
    uint64_t shared_launches;   /* launches carrying items of >= 2 queries         */
    int32_t peak_active;        /* most queries admitted at one time              */
    int32_t max_members;        /* most queries in one launch                     */
} amc_server_stats;
AMC_API int amc_server_info(amc_ctx *ctx, amc_server_stats *out);

/* Persistent fused batch (Alg. 2 for several queries at once).  The queries
 * are grouped by kernel variant; each group is one persistent launch whose
 * work queue holds every member's (realization, source tile) items, largest
 * queries first.  The device sequence (counter resets, sweeps, tails) is
 * captured once into a hipGraph; amc_batch_run replays it and fills
 * results[0 .. count-1] exactly as count separate amc_run calls would (the
 * per-query sweep_ms is the time of the whole replay).  Inputs are copied at
 * creation.  AMC_PLAIN_LAUNCH is not accepted here. */
AMC_API int amc_batch_create(amc_ctx *ctx, int32_t count, const amc_graph *const *graphs, const amc_model *models,
                             const amc_query *queries, amc_batch **out);
AMC_API int amc_batch_run(amc_batch *b, amc_result *results);
/* Number of fused launches and of work items of a batch. */
AMC_API int amc_batch_info(amc_batch *b, int32_t *n_launches, int32_t *items);
AMC_API void amc_batch_destroy(amc_batch *b);

/* Autotuner: times the feasible sweep configurations (LDS mode with each
 * vertex mapping, workgroup-per-source mode) on probe_R realizations of this
 * graph and query, and records the fastest for the graph's shape (n, m,
 * weight law, largest weight) in the context.  Later calls with mode, group
 * and waves left at 0 use it.  With the environment variable AMC_TUNE_CACHE
 * naming a file, choices are loaded from it at context creation and appended
 * to it here. */
typedef struct amc_tune_result {
    int32_t mode, group, waves;     /* chosen configuration                     */
    double units_per_s;             /* its probe rate, realization-sources / s  */
    int32_t candidates;             /* configurations timed                     */
} amc_tune_result;
AMC_API int amc_tune(amc_ctx *ctx, const amc_graph *g, const amc_model *model, const amc_query *q, uint32_t probe_R,
                     amc_tune_result *out);

/* Trajectory simulator (Section 4.3): episodes of the network process itself.
 * Episode e starts at x0[e]; at step t the anchor X_t draws its stop coin and
 * a fresh network state from the Philox counters (e, X_t, 2^32-1, 2 + t) and
 * (e, u, v, 2 + t) (disjoint from the row-wise counters), the step is invalid
 * when the coin fires or |K(X_t;H)| < k_min (X_{t+1} = bottom), otherwise
 * X_{t+1} = c_loc(X_t;H) with the same tie rule as amc_run.  T_e counts the
 * pre-absorption states X_0 .. X_{T-1}; an episode reaching max_steps of them
 * is cut there and counted as truncated.  The outputs give the length-biased
 * estimators of the uniform-step equivalence: b_hat_v = visits_v / sum T
 * estimates b_v(s) for s the law of x0, survival_t = #{T_e > t} / sum T the
 * weights w_t of the survival-weighted decomposition, reward_f / sum T the
 * node-reward AFC b . f, and switches / sum T the switching-rate reward.
 * Layouts: AMC_MODE_WAVE stages each step's realized graph in LDS;
 * AMC_MODE_WAVE_L2 keeps it in a per-workgroup global scratch (L2-resident)
 * with K(X_t;H) in LDS and B in LDS or in that scratch, for lane-per-vertex
 * mappings (group 1 / 2 / 3); AMC_MODE_AUTO takes the layout that fits the
 * most wavefronts per workgroup, weighted by their measured relative rates.
 * In the L2 layout a step's sources after X_t are open to workgroups that
 * have run out of episodes (they read the step's realized graph from the
 * owner's scratch), so the last long episodes do not run alone.
 * Every layout produces identical results.  flags: AMC_WANT_PATHS;
 * AMC_DIST16 / AMC_DIST32 fix the distance width; AMC_TRAJ_B_LDS /
 * AMC_TRAJ_B_GLOBAL fix B's place in the L2 layout.  A graph that fits no
 * layout returns AMC_E_UNSUPPORTED. */
#define AMC_WANT_PATHS (1u << 0)
#define AMC_TRAJ_B_LDS (1u << 1)
#define AMC_TRAJ_B_GLOBAL (1u << 2)
typedef struct amc_traj_query {
    uint64_t seed;
    int32_t episodes;           /* >= 1                                       */
    const int32_t *x0;          /* episodes start states in [0, n)            */
    double alpha;               /* stop probability, in (0, 1]                */
    uint32_t k_min;
    double tie_tau;             /* < 0 selects 1e-9                           */
    int32_t max_steps;          /* >= 1: cap on pre-absorption states          */
    const double *f;            /* node reward (n, >= 0) or NULL               */
    uint32_t flags;             /* AMC_WANT_PATHS, AMC_DIST16 / 32, AMC_TRAJ_B_* */
    int32_t group, waves;       /* vertex mapping / wavefronts, 0 = engine    */
    int32_t mode;               /* AMC_MODE_AUTO, AMC_MODE_WAVE or AMC_MODE_WAVE_L2 */
} amc_traj_query;

typedef struct amc_traj_result {
    int32_t *lengths;           /* episodes: T_e (required)                   */
    int32_t *paths;             /* episodes x max_steps, -1 past T_e (AMC_WANT_PATHS) */
    uint64_t *visits;           /* n (required)                               */
    double *b_hat;              /* n: visits / sum T                           */
    double *survival;           /* max_steps: #{T_e > t} / sum T               */
    double reward_f;            /* sum over episodes and t < T_e of f(X_t)     */
    uint64_t switches;          /* steps with X_{t+1} in V and X_{t+1} != X_t  */
    uint64_t total_steps;       /* sum T_e                                     */
    uint64_t sources;           /* single-source passes run (throughput unit)  */
    int32_t truncated;
    double sweep_ms;            /* HIP-event time of the trajectory kernel     */
    int32_t mode, waves;        /* layout and wavefronts per workgroup used    */
    int32_t dist16, b_global;   /* 16-bit distances; B in the global scratch  */
    uint64_t shared_sources;    /* L2 layout: sources of a step run by workgroups
                                   that had run out of episodes               */
} amc_traj_result;
AMC_API int amc_trajectories(amc_ctx *ctx, const amc_graph *g, const amc_model *model, const amc_traj_query *q,
                             amc_traj_result *out);

/* Robust tail on a given transient block Q0 (n x n, row sums < 1), e.g. the
 * stabilised kernel amc_run returns in `Q`:
 *  - transition reward-AFCs (Section 6.4), with f: switching, eta(i,j) =
 *    1{j in V, j != i}, and improvement, eta(i,j) = (f_j - f_i)_+ for j in V;
 *  - `samples` admissible kernels of the row-wise set (Section 5.1) drawn as in
 *    the robust experiment of Section 9.1: Q_ij = clip(Q0_ij (1 + delta
 *    (2u - 1)), 0, 1), u the 53-bit fraction of the Philox block of counter
 *    (sample, i, j, 3) under key `seed`, each row scaled down to sum 1 - r_min
 *    when it exceeds it; for each, KL(b(P) || b0) and total variation
 *    |b(P) - b0|_1 / 2, and the AFC at both maximisers;
 *  - the first-order sensitivity of Section 5.4 for E = Q* - Q0 (Q* the KL
 *    maximiser): b_lin, and in infinity norms |N0 E|, |N0|, the remainder
 *    bound |N0 E|^2 |N0| / (1 - |N0 E|) (infinite when |N0 E| >= 1) and the
 *    actual |N* - N0 - N0 E N0|;
 *  - with a base topology (m > 0 edges eu, ev, canonical as for
 *    amc_graph_create, connected, n <= AMC_MAX_W1_N): the Wasserstein-1
 *    distance W1(b(P), b0) of every sample on the shortest-path metric of
 *    that topology (robust experiments of Sections 9.1 and 9.2) -- every edge
 *    of length 1 (the hop metric) or, with w, of the integer length w[e] in
 *    [1, 65535] (e.g. the fixed weights of the graph) -- computed exactly as
 *    the cheapest transshipment of b(P) - b0 over its edges, and the AFC at
 *    the W1 maximiser.
 * Errors: AMC_E_INVALID_ARG for a bad size, range or edge list, a
 * disconnected topology, or a Q0 row that does not absorb; AMC_E_UNSUPPORTED
 * for n > AMC_MAX_W1_N with a topology, or when the W1 solver exceeds its
 * iteration bounds; AMC_E_SINGULAR, AMC_E_OOM, AMC_E_HIP as for amc_run.
 * Output arrays are caller-owned host buffers (NULL = skip). */
#define AMC_MAX_W1_N 7500
typedef struct amc_robust_query {
    const double *s;            /* initial distribution (n) or NULL for uniform  */
    const double *f;            /* node values (n, >= 0) or NULL (no transition rewards) */
    int32_t samples;            /* 0 .. 4096                                     */
    double delta;               /* relative radius, >= 0                          */
    double r_min;               /* leak lower bound, in (0, 1]                    */
    uint64_t seed;
    int64_t m;                  /* edges of the base topology for W1 (0 = no W1)  */
    const int32_t *eu, *ev;     /* m each, eu < ev, lexicographically increasing   */
    const uint32_t *w;          /* m edge lengths in [1, 65535], or NULL for the hop metric */
} amc_robust_query;

typedef struct amc_robust_result {
    double *b0;                 /* n                                             */
    double b_sw, b_imp;
    double *kl, *tv;            /* samples                                       */
    int32_t kl_arg, tv_arg;     /* -1 without samples                            */
    double *b_kl, *b_tv, *b_lin;/* n each                                        */
    double norm_N0E, norm_N0, rem_bound, rem_actual;
    double tail_ms;             /* HIP-event time of the whole computation        */
    double *w1;                 /* samples: W1(b(P), b0) (needs a topology)       */
    int32_t w1_arg;             /* -1 without samples or topology                 */
    double *b_w1;               /* n: AFC at the W1 maximiser                     */
} amc_robust_result;
AMC_API int amc_robust(amc_ctx *ctx, int32_t n, const double *Q0, const amc_robust_query *q, amc_robust_result *out);

/* Nonparametric bootstrap of the AFC profile (Section 8.4): each row's R draws
 * are resampled with replacement and b is recomputed, B times.
 *
 * next_table: host, R x n row-major int32, entry (t, i) = the next state of
 * row i on draw t (0 .. n-1, or -1 = bottom), as amc_run writes it with
 * AMC_WANT_NEXT_TABLE.  Draw t of row i in replicate beta (0 .. B-1) is the
 * index j = (x * R) >> 32 with x = word (t mod 4) of Philox4x32-10 at counter
 * (beta, i, t / 4, 0x80000004) under `seed`; the replicate counts row i's
 * outcome at draw j.  Each replicate kernel takes the floor rule of amc_run
 * (Section 8.2) and goes through N = (I - Q*)^-1, mu = s N, b = mu / (mu 1).
 * Per node v, over the B replicate values: mean, sample standard deviation
 * (divisor B - 1; 0 when B = 1) and the nearest-rank order statistics of
 * indices ceil((1 - level) B / 2) - 1 and ceil((1 + level) B / 2) - 1 (clamped
 * to 0 .. B-1) of the ascending values.  b0 is b of the given draws.
 *
 * Errors: AMC_E_INVALID_ARG for NULL pointers, n < 1, R < 1, an entry outside
 * -1 .. n-1, replicates outside 1 .. AMC_MAX_BOOT_REPLICATES, level outside
 * (0, 1), floor_eta >= 1, or an s that is negative or does not sum to 1;
 * AMC_E_UNSUPPORTED for n > AMC_MAX_BOOT_N; AMC_E_SINGULAR when a kernel has a
 * row that never absorbs and the floor is disabled; AMC_E_OOM when the device
 * buffers (6 R n bytes for the table, up to 1 GiB of matrices, 8 B n for the
 * replicates) do not fit.  Output arrays are caller-owned host buffers
 * (NULL = skip). */
#define AMC_MAX_BOOT_REPLICATES 4096
#define AMC_MAX_BOOT_N 16383
typedef struct amc_boot_query {
    const double *s;            /* initial distribution (n) or NULL for uniform  */
    double floor_eta;           /* < 0 selects 0.1/sqrt(R); 0 disables            */
    int32_t replicates;         /* B                                             */
    double level;               /* interval coverage, in (0, 1)                  */
    uint64_t seed;
} amc_boot_query;

typedef struct amc_boot_result {
    double *b0;                 /* n                                             */
    double *mean, *sd, *lo, *hi;/* n each                                        */
    double *b_rep;              /* B x n                                         */
    double ms;                  /* HIP-event time of the whole computation        */
} amc_boot_result;
AMC_API int amc_bootstrap(amc_ctx *ctx, int32_t n, uint32_t R, const int32_t *next_table, const amc_boot_query *q,
                          amc_boot_result *out);

/* Rank-stability check of Section 8.4: the estimate at M = q->R realizations
 * (r_begin .. r_begin + M - 1) and at 2M (r_begin .. r_begin + 2M - 1, the
 * first M shared, as a rerun with the same seed draws them), each through the
 * tail of amc_run with its own default floor (q->floor_eta < 0: 0.1/sqrt(M)
 * and 0.1/sqrt(2M)), and whether the Top-k set by b (ties to the smaller
 * index) is unchanged.  Costs 2M realizations of sweep: the second query
 * starts from the first one's counts.  The query's graph-law and anchor rules
 * (seed, alpha, k_min, tie_tau, floor_eta, s) and execution choices (mode,
 * tile, waves, group, AMC_DIST16 / AMC_DIST32 / AMC_PLAIN_LAUNCH) apply; its
 * other flags, reward, eps, r_lower, cert_topk and debug pairs are ignored.
 * Errors: AMC_E_INVALID_ARG for NULL pointers, k outside 1 .. min(16, n-1),
 * R = 0 or 2R past 2^31, r_begin + 2R past 2^32, a pool, topk > 0 or
 * AMC_FALLBACK; otherwise those of amc_run.  Output arrays are caller-owned
 * host buffers (NULL = skip). */
typedef struct amc_stability_result {
    double *b_M, *b_2M;         /* n each                                        */
    int32_t *top_M, *top_2M;    /* k each, in decreasing b                       */
    uint32_t *counts_2M;        /* n x (n+1) counts over the 2M realizations     */
    int32_t same_set;           /* 1 when the two Top-k sets are equal as sets    */
    int32_t overlap;            /* members the two sets share                     */
    double max_abs_diff;        /* max over v of |b_2M[v] - b_M[v]|               */
    double sweep_ms;            /* HIP-event time of the two sweeps               */
} amc_stability_result;
AMC_API int amc_stability(amc_ctx *ctx, const amc_graph *g, const amc_model *model, const amc_query *q, int32_t k,
                          amc_stability_result *out);

/* Sweep without any allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation.  It computes what amc_run computes with AMC_SKIP_TAIL --
 * the counts C (and, with d_center, the global centres c(H_r)) over the
 * realizations r_begin .. r_begin + R - 1, in the same launch plan -- into
 * caller-owned DEVICE buffers:
 *   d_counts  n x (n+1) uint32, row-major, column n = bottom (required;
 *             overwritten, not accumulated into)
 *   d_center  R int32 or NULL
 *   stats     host, or NULL: the run's counters and plan (sweep_ms from the
 *             context's events)
 * Every device buffer the sweep needs beyond these (descriptors, work and
 * statistics counters, error flags, the per-workgroup scratch of the L2 and
 * workgroup-per-source modes, the partial-B exchange of split realizations)
 * is carved from one file-scope device array of AMC_STATIC_SCRATCH_BYTES that
 * each device holds from the library's first context on it until the process
 * ends; no allocator is called.  Calls on one device share that array and
 * keep the last call's contents there (each call clears what it needs); the
 * library serialises them per device, so calls never overlap on one device
 * within a process -- a caller that drives the same device from several
 * threads waits.  The call returns when the sweep has finished on the
 * context stream.
 * Accepted queries: no pool, topk, fallback, debug pairs, hop_radius,
 * per-edge failure probabilities or AMC_WEIGHT_TABLE; flags only AMC_DIST16,
 * AMC_DIST32, AMC_SIGMA_GLOBAL and AMC_SKIP_TAIL (s, reward, eps, r_lower and cert_topk are
 * ignored: there is no tail).  Errors: AMC_E_INVALID_ARG for the above and
 * for what amc_run rejects; AMC_E_SCRATCH when the plan needs more scratch
 * than the array holds (checked before anything is launched); AMC_E_HIP when
 * the array's address could not be obtained on this device; otherwise those
 * of amc_run. */
#define AMC_STATIC_SCRATCH_BYTES (64u << 20)
AMC_API int amc_sweep_static(amc_ctx *ctx, const amc_graph *g, const amc_model *model, const amc_query *q,
                             uint32_t *d_counts, int32_t *d_center, amc_stats *stats);

/* Chain algebra alone on a given transient block Q (n x n, row sums < 1) with
 * absorption r = 1 - Q 1: N, mu, E_T, b, rewards and certificates exactly as
 * the tail of amc_run (Sections 4 and 5.5).  q supplies s, reward, eps,
 * r_lower, cert_topk; counts-related fields of `out` are ignored. */
AMC_API int amc_chain(amc_ctx *ctx, int32_t n, const double *Q, const amc_query *q, amc_result *out);

AMC_API const char *amc_strerror(int status);
AMC_API int amc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* AMC_H */
