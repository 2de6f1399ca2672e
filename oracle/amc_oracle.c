/*
 * amc_oracle.c -- CPU oracle for absorbing-frequency centrality (AFC).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, single-threaded,
 * obviously-correct FP64 statement of what the GPU library computes.  Only the
 * test-suite, the package smoke check and the benchmark's CPU-baseline leg may
 * load it; the product path never does.  It shares no source, header, helper
 * or generated table with the GPU library: its Philox generator, its
 * shortest-path code, its betweenness, its centre selection and its chain
 * algebra are all written here from their published definitions.
 *
 * Paper: W. Bao, E. Kontou, C. Vogiatzis, "Betweenness-Central Nodes Under
 * Uncertainty: An Absorbing Markov Chain Approach".  Section / equation
 * citations below refer to that paper.
 *
 * Readings of points the paper leaves open:
 *   - realizations are drawn with Philox4x32-10 keyed by the 64-bit seed; the
 *     edge (u<v) of realization r uses counter (r, u, v, 0), the exogenous stop
 *     coin of anchor i uses counter (r, i, 0xFFFFFFFF, 1);
 *   - uniforms are mapped to events with integers only: an event of
 *     probability p fires when the 32-bit draw is below floor(p * 2^32);
 *     integer weights in [lo, hi] are lo + ((x * (hi-lo+1)) >> 32);
 *   - every realization serves every anchor (one realization count R = M);
 *   - the deterministic tie rule is "smallest index inside a relative tie
 *     band": v is a co-maximiser of a set when max - B_v <= tau*max(max, 1);
 *   - the floor on an empty absorption column is eta (default 0.1/sqrt(R));
 *   - the bootstrap redraws each row's R draws from Philox4x32-10 at counter
 *     (replicate, row, t / 4, 0x80000004), index (word * R) >> 32;
 *   - W1 of the robust experiment uses the hop metric of the base topology.
 *
 * Parity pins: every exported function below is pinned by the CPU tests
 * (tests/test_oracle_*.py) against closed forms, brute force, the values the
 * paper prints for its worked examples, or an independent library.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_ARG (-1)
#define OR_E_NOMEM (-2)
#define OR_E_SIGMA (-4)
#define OR_E_SINGULAR (-5)

#define OR_WEIGHT_UNIT 0
#define OR_WEIGHT_UNIFORM 1
#define OR_WEIGHT_FIXED 2
#define OR_WEIGHT_TABLE 3

#define OR_INF UINT64_MAX

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies with the */
/* round keys bumped by the Weyl constants between rounds.                   */
/* ------------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    int round;
    for (round = 0; round < 10; ++round) {
        uint64_t p0, p1;
        uint32_t y0, y1, y2, y3;
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        y1 = (uint32_t)p1;
        y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* An event of probability p fires for a uniform 32-bit draw x iff x < T(p),
 * T(p) = floor(p * 2^32) clamped to [0, 2^32].  Multiplying by 2^32 and the
 * floor are exact in binary64, so T is a pure function of p. */
uint64_t or_prob_threshold(double p)
{
    if (!(p > 0.0)) return 0;
    if (p >= 1.0) return 4294967296ull;
    return (uint64_t)floor(p * 4294967296.0);
}

/* ------------------------------------------------------------------------ */
/* Base graph: undirected, simple, canonical edge list (u < v, sorted).     */
/* Section 3.1: base topology G(V,E).                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n;
    int64_t m;
    const int32_t *eu, *ev;      /* canonical edges, eu[e] < ev[e]         */
    int64_t *off;                /* adjacency offsets, length n+1           */
    int32_t *nbr;                /* neighbour of each adjacency slot        */
    int64_t *eid;                /* edge id of each adjacency slot          */
} or_graph;

static void or_graph_free(or_graph *g)
{
    free(g->off); free(g->nbr); free(g->eid);
    g->off = NULL; g->nbr = NULL; g->eid = NULL;
}

/* Builds adjacency lists of the base graph.  Rejects self-loops, vertices out
 * of range, non-canonical (u >= v) and repeated edges. */
static int or_graph_init(or_graph *g, int32_t n, int64_t m, const int32_t *eu, const int32_t *ev)
{
    int64_t e, *fill;
    int32_t v;
    memset(g, 0, sizeof(*g));
    if (n < 1 || m < 0) return OR_E_ARG;
    for (e = 0; e < m; ++e) {
        if (eu[e] < 0 || ev[e] >= n || eu[e] >= ev[e]) return OR_E_ARG;
        if (e > 0 && (eu[e - 1] > eu[e] || (eu[e - 1] == eu[e] && ev[e - 1] >= ev[e]))) return OR_E_ARG;
    }
    g->n = n; g->m = m; g->eu = eu; g->ev = ev;
    g->off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    g->nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    g->eid = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * m + 1));
    fill = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    if (!g->off || !g->nbr || !g->eid || !fill) { free(fill); or_graph_free(g); return OR_E_NOMEM; }
    for (e = 0; e < m; ++e) { g->off[eu[e] + 1]++; g->off[ev[e] + 1]++; }
    for (v = 0; v < n; ++v) g->off[v + 1] += g->off[v];
    for (e = 0; e < m; ++e) {
        int32_t a = eu[e], b = ev[e];
        g->nbr[g->off[a] + fill[a]] = b; g->eid[g->off[a] + fill[a]] = e; fill[a]++;
        g->nbr[g->off[b] + fill[b]] = a; g->eid[g->off[b] + fill[b]] = e; fill[b]++;
    }
    free(fill);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* One network state (Section 3.1): which edges survive and their positive   */
/* integer weights.  Alg. 1 "sample omega" with the integer-only mapping.    */
/* ------------------------------------------------------------------------ */
typedef struct {
    double p_fail;               /* failure probability of every edge       */
    const double *p_fail_edge;   /* optional per-edge failure probabilities */
    int32_t weight_kind;         /* OR_WEIGHT_*                             */
    uint32_t w_lo, w_hi;         /* range of OR_WEIGHT_UNIFORM; w_hi = w_max */
                                 /* of OR_WEIGHT_TABLE                      */
    const uint32_t *w0;          /* weights of OR_WEIGHT_FIXED              */
    const uint64_t *w_cdf;       /* OR_WEIGHT_TABLE: m x w_max thresholds   */
} or_model;

/* Realization with counter words (r, u, v, stream): stream 0 is the row-wise
 * sweep's realization r; the trajectory simulator uses r = episode and
 * stream = 2 + step (see or_trajectories). */
static int or_realize_stream(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev, const or_model *mod,
                             uint64_t seed, uint32_t r, uint32_t stream, uint8_t *alive, uint32_t *w)
{
    int64_t e;
    uint32_t key[2];
    (void)n;
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
    for (e = 0; e < m; ++e) {
        uint32_t ctr[4], x[4];
        double p = mod->p_fail_edge ? mod->p_fail_edge[e] : mod->p_fail;
        ctr[0] = r; ctr[1] = (uint32_t)eu[e]; ctr[2] = (uint32_t)ev[e]; ctr[3] = stream;
        or_philox4x32_10(ctr, key, x);
        alive[e] = ((uint64_t)x[0] >= or_prob_threshold(p)) ? 1 : 0;
        if (mod->weight_kind == OR_WEIGHT_UNIT) {
            w[e] = 1;
        } else if (mod->weight_kind == OR_WEIGHT_UNIFORM) {
            uint64_t span = (uint64_t)mod->w_hi - (uint64_t)mod->w_lo + 1u;
            w[e] = mod->w_lo + (uint32_t)(((uint64_t)x[1] * span) >> 32);
        } else if (mod->weight_kind == OR_WEIGHT_TABLE) {
            /* per-call resampled weight (Section 9.2): the law of edge e is given
             * by its cumulative thresholds T_e(v) = floor(P(w <= v) 2^32); the
             * weight is the smallest v with x1 < T_e(v) (T_e(w_max) = 2^32) */
            const uint64_t *T = mod->w_cdf + (size_t)e * mod->w_hi;
            uint32_t v = 1;
            while (v < mod->w_hi && (uint64_t)x[1] >= T[v - 1]) ++v;
            w[e] = v;
        } else {
            w[e] = mod->w0[e];
        }
    }
    return OR_OK;
}

int or_realize(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev, const or_model *mod,
               uint64_t seed, uint32_t r, uint8_t *alive, uint32_t *w)
{
    return or_realize_stream(n, m, eu, ev, mod, seed, r, 0u, alive, w);
}

/* Exogenous stop coin of anchor i (Alg. 1: the draw omega includes the
 * stopping event; its probability is alpha), counter (r, i, 2^32-1, stream):
 * stream 1 in the row-wise sweep, 2 + step on a trajectory. */
static int or_stop_coin_stream(uint64_t seed, uint32_t r, int32_t i, uint32_t stream, double alpha)
{
    uint32_t ctr[4], key[2], x[4];
    key[0] = (uint32_t)seed; key[1] = (uint32_t)(seed >> 32);
    ctr[0] = r; ctr[1] = (uint32_t)i; ctr[2] = 0xFFFFFFFFu; ctr[3] = stream;
    or_philox4x32_10(ctr, key, x);
    return (uint64_t)x[0] < or_prob_threshold(alpha);
}

int or_stop_coin(uint64_t seed, uint32_t r, int32_t i, double alpha)
{
    return or_stop_coin_stream(seed, r, i, 1u, alpha);
}

/* ------------------------------------------------------------------------ */
/* Single-source shortest paths with path counts on a realization H         */
/* (Section 3.1: d_H(s,t) and sigma_st(H)).  Unit weights: breadth-first     */
/* search; integer weights: Dijkstra with a binary heap.  sigma is an exact  */
/* uint64; an addition that would wrap returns OR_E_SIGMA.  `order` receives */
/* the reached vertices in non-decreasing distance.                          */
/* ------------------------------------------------------------------------ */
typedef struct { uint64_t key; int32_t v; } or_heap_item;

static void heap_push(or_heap_item *h, int64_t *size, uint64_t key, int32_t v)
{
    int64_t i = (*size)++;
    h[i].key = key; h[i].v = v;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h[p].key <= h[i].key) break;
        { or_heap_item t = h[p]; h[p] = h[i]; h[i] = t; }
        i = p;
    }
}

static or_heap_item heap_pop(or_heap_item *h, int64_t *size)
{
    or_heap_item top = h[0];
    int64_t i = 0;
    h[0] = h[--(*size)];
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, s = i;
        if (l < *size && h[l].key < h[s].key) s = l;
        if (r < *size && h[r].key < h[s].key) s = r;
        if (s == i) break;
        { or_heap_item t = h[s]; h[s] = h[i]; h[i] = t; }
        i = s;
    }
    return top;
}

static int add_sigma(uint64_t *dst, uint64_t add)
{
    if (*dst > UINT64_MAX - add) return OR_E_SIGMA;
    *dst += add;
    return OR_OK;
}

static int or_sssp_graph(const or_graph *g, const uint8_t *alive, const uint32_t *w, int unit, int32_t s,
                         uint64_t *dist, uint64_t *sigma, int32_t *order, int32_t *n_order)
{
    int32_t n = g->n, v, cnt = 0;
    for (v = 0; v < n; ++v) { dist[v] = OR_INF; sigma[v] = 0; }
    dist[s] = 0; sigma[s] = 1;
    if (unit) {
        int32_t head = 0;
        order[cnt++] = s;
        while (head < cnt) {
            int32_t x = order[head++];
            int64_t k;
            for (k = g->off[x]; k < g->off[x + 1]; ++k) {
                int32_t y = g->nbr[k];
                if (!alive[g->eid[k]]) continue;
                if (dist[y] == OR_INF) { dist[y] = dist[x] + 1; order[cnt++] = y; }
                if (dist[y] == dist[x] + 1) {
                    if (add_sigma(&sigma[y], sigma[x]) != OR_OK) return OR_E_SIGMA;
                }
            }
        }
    } else {
        int64_t hsize = 0;
        uint8_t *done = (uint8_t *)calloc((size_t)n, 1);
        or_heap_item *heap = (or_heap_item *)malloc(sizeof(or_heap_item) * (size_t)(2 * g->m + 2));
        if (!done || !heap) { free(done); free(heap); return OR_E_NOMEM; }
        heap_push(heap, &hsize, 0, s);
        while (hsize > 0) {
            or_heap_item it = heap_pop(heap, &hsize);
            int32_t x = it.v;
            int64_t k;
            if (done[x] || it.key != dist[x]) continue;
            done[x] = 1;
            order[cnt++] = x;
            for (k = g->off[x]; k < g->off[x + 1]; ++k) {
                int32_t y = g->nbr[k];
                uint64_t nd;
                if (!alive[g->eid[k]]) continue;
                nd = dist[x] + (uint64_t)w[g->eid[k]];
                if (nd < dist[y]) {
                    dist[y] = nd; sigma[y] = sigma[x];
                    heap_push(heap, &hsize, nd, y);
                } else if (nd == dist[y]) {
                    if (add_sigma(&sigma[y], sigma[x]) != OR_OK) { free(done); free(heap); return OR_E_SIGMA; }
                }
            }
        }
        free(done); free(heap);
    }
    *n_order = cnt;
    return OR_OK;
}

/* Dependencies of source s (Brandes' accumulation of the pair terms of the
 * Section 3.1 definition): vertices are taken in non-increasing distance and
 * each one w passes (sigma_v / sigma_w) * (1 + delta_w) to every predecessor v,
 * i.e. every v joined to w by a surviving edge with d_v + w_vw = d_w. */
static void or_dependency(const or_graph *g, const uint8_t *alive, const uint32_t *w, int unit,
                          const uint64_t *dist, const uint64_t *sigma, const int32_t *order,
                          int32_t n_order, double *delta)
{
    int32_t v, k;
    for (v = 0; v < g->n; ++v) delta[v] = 0.0;
    for (k = n_order - 1; k >= 0; --k) {
        int32_t x = order[k];
        int64_t j;
        for (j = g->off[x]; j < g->off[x + 1]; ++j) {
            int32_t y = g->nbr[j];
            uint64_t wt;
            if (!alive[g->eid[j]]) continue;
            wt = unit ? 1u : (uint64_t)w[g->eid[j]];
            if (dist[y] != OR_INF && dist[y] + wt == dist[x])
                delta[y] += ((double)sigma[y] / (double)sigma[x]) * (1.0 + delta[x]);
        }
    }
}

/* Exported single-source dump (for the distance / path-count / dependency
 * parity checks). */
int or_sssp(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev, const uint8_t *alive,
            const uint32_t *w, int unit, int32_t s, uint64_t *dist, uint64_t *sigma, double *delta)
{
    or_graph g;
    int32_t *order, n_order = 0;
    int rc = or_graph_init(&g, n, m, eu, ev);
    if (rc != OR_OK) return rc;
    if (s < 0 || s >= n) { or_graph_free(&g); return OR_E_ARG; }
    order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!order) { or_graph_free(&g); return OR_E_NOMEM; }
    rc = or_sssp_graph(&g, alive, w, unit, s, dist, sigma, order, &n_order);
    if (rc == OR_OK && delta) or_dependency(&g, alive, w, unit, dist, sigma, order, n_order, delta);
    free(order); or_graph_free(&g);
    return rc;
}

/* Non-normalised weighted betweenness B_v(H) of Section 3.1 (ordered pairs,
 * unreachable pairs contribute 0), by summing the dependencies of every
 * source s (delta_s(v), v != s). */
static int or_brandes_graph(const or_graph *g, const uint8_t *alive, const uint32_t *w, int unit,
                            double *B, uint64_t *dist, uint64_t *sigma, int32_t *order, double *delta)
{
    int32_t s, v, n = g->n;
    for (v = 0; v < n; ++v) B[v] = 0.0;
    for (s = 0; s < n; ++s) {
        int32_t n_order = 0;
        int rc = or_sssp_graph(g, alive, w, unit, s, dist, sigma, order, &n_order);
        if (rc != OR_OK) return rc;
        or_dependency(g, alive, w, unit, dist, sigma, order, n_order, delta);
        for (v = 0; v < n; ++v)
            if (v != s) B[v] += delta[v];
    }
    return OR_OK;
}

int or_betweenness(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev, const uint8_t *alive,
                   const uint32_t *w, int unit, double *B)
{
    or_graph g;
    uint64_t *dist, *sigma;
    int32_t *order;
    double *delta;
    int rc = or_graph_init(&g, n, m, eu, ev);
    if (rc != OR_OK) return rc;
    dist = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    sigma = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    delta = (double *)malloc(sizeof(double) * (size_t)n);
    if (!dist || !sigma || !order || !delta) rc = OR_E_NOMEM;
    else rc = or_brandes_graph(&g, alive, w, unit, B, dist, sigma, order, delta);
    free(dist); free(sigma); free(order); free(delta); or_graph_free(&g);
    return rc;
}

/* The same B_v(H) written as the definition of Section 3.1: for every ordered
 * pair (s,t), s != t, both != v, with d(s,t) finite, add the fraction of the
 * shortest s-t paths that run through v, sigma_sv * sigma_vt / sigma_st when
 * d(s,v) + d(v,t) = d(s,t) and 0 otherwise.  O(n^3); used to pin the Brandes
 * form on small graphs. */
int or_betweenness_pairs(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev, const uint8_t *alive,
                         const uint32_t *w, int unit, double *B)
{
    or_graph g;
    uint64_t *D, *S;
    int32_t *order, s, t, v;
    int rc = or_graph_init(&g, n, m, eu, ev);
    if (rc != OR_OK) return rc;
    D = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n * (size_t)n);
    S = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n * (size_t)n);
    order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!D || !S || !order) { free(D); free(S); free(order); or_graph_free(&g); return OR_E_NOMEM; }
    for (s = 0; s < n && rc == OR_OK; ++s) {
        int32_t n_order;
        rc = or_sssp_graph(&g, alive, w, unit, s, D + (size_t)s * n, S + (size_t)s * n, order, &n_order);
    }
    for (v = 0; v < n && rc == OR_OK; ++v) {
        double acc = 0.0;
        for (s = 0; s < n; ++s) {
            uint64_t dsv;
            if (s == v) continue;
            dsv = D[(size_t)s * n + v];
            if (dsv == OR_INF) continue;
            for (t = 0; t < n; ++t) {
                uint64_t dst, dvt;
                if (t == v || t == s) continue;
                dst = D[(size_t)s * n + t];
                dvt = D[(size_t)v * n + t];
                if (dst == OR_INF || dvt == OR_INF) continue;
                if (dsv + dvt == dst)
                    acc += (double)S[(size_t)s * n + v] * (double)S[(size_t)v * n + t] / (double)S[(size_t)s * n + t];
            }
        }
        B[v] = acc;
    }
    free(D); free(S); free(order); or_graph_free(&g);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Components K(i;H) (Section 3.2): comp[v] = smallest vertex index of the   */
/* component containing v, size[v] = |K(v;H)|.                              */
/* ------------------------------------------------------------------------ */
static int or_components_graph(const or_graph *g, const uint8_t *alive, int32_t *comp, int32_t *size,
                               int32_t *queue)
{
    int32_t n = g->n, v;
    for (v = 0; v < n; ++v) comp[v] = -1;
    for (v = 0; v < n; ++v) {
        int32_t head = 0, cnt = 0, k;
        if (comp[v] >= 0) continue;
        comp[v] = v; queue[cnt++] = v;
        while (head < cnt) {
            int32_t x = queue[head++];
            int64_t j;
            for (j = g->off[x]; j < g->off[x + 1]; ++j) {
                int32_t y = g->nbr[j];
                if (!alive[g->eid[j]] || comp[y] >= 0) continue;
                comp[y] = v; queue[cnt++] = y;
            }
        }
        for (k = 0; k < cnt; ++k) size[queue[k]] = cnt;
    }
    return OR_OK;
}

int or_components(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev, const uint8_t *alive,
                  int32_t *comp, int32_t *size)
{
    or_graph g;
    int32_t *queue;
    int rc = or_graph_init(&g, n, m, eu, ev);
    if (rc != OR_OK) return rc;
    queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!queue) { or_graph_free(&g); return OR_E_NOMEM; }
    rc = or_components_graph(&g, alive, comp, size, queue);
    free(queue); or_graph_free(&g);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Tie-broken argmax (eq. central-node, eq. local-center and the canonical   */
/* smallest-index selector of the corollary on deterministic tie-breaking).  */
/* Among the members of a set, v is a co-maximiser when                      */
/*   max_B - B_v <= tau * max(max_B, 1);                                     */
/* the smallest-index co-maximiser is returned (-1 for an empty set).  With  */
/* exact arithmetic and tau -> 0 this is the paper's rule.  `near` counts    */
/* members whose gap lies in [band/4, 4*band], where rounding could matter.  */
/* ------------------------------------------------------------------------ */
int32_t or_band_argmax(int32_t n, const double *B, const uint8_t *member, double tau, int64_t *near)
{
    int32_t v, best = -1;
    double bmax = 0.0, band;
    int any = 0;
    for (v = 0; v < n; ++v) {
        if (!member[v]) continue;
        if (!any || B[v] > bmax) bmax = B[v];
        any = 1;
    }
    if (!any) return -1;
    band = tau * (bmax > 1.0 ? bmax : 1.0);
    for (v = 0; v < n; ++v) {
        double gap;
        if (!member[v]) continue;
        gap = bmax - B[v];
        if (gap <= band && best < 0) best = v;
        if (near && band > 0.0 && gap >= 0.25 * band && gap <= 4.0 * band) (*near)++;
    }
    return best;
}

/* ------------------------------------------------------------------------ */
/* Row-wise Monte Carlo sweep (Alg. 1 SampleNext for every anchor, Alg. 2    */
/* counting).  Realization r in [r_begin, r_begin + R) is drawn once and     */
/* serves every anchor i: next(r,i) = bottom if the stop coin fires or       */
/* |K(i;H_r)| < k_min, else the tie-broken centre of K(i;H_r).  The pool-    */
/* constrained selector of Section 7.1 takes, with k = infinity (topk = 0),  */
/* the tie-broken argmax over K(i;H_r) intersected with W, bottom when that  */
/* is empty; with a finite k it takes the highest-ranked member of W among   */
/* the local Top-k set (eq. local-topk).                                      */
/*                                                                            */
/* Finite k: the ranking pi_{K,H} of a component is the tie rule applied     */
/* repeatedly, i.e. pi(t) is the band argmax over the members not ranked     */
/* before t.  C_k(i) (eq. realized-topk-set) is the first min(k, |K|) of them */
/* on a valid draw, empty otherwise, and the step rewards of Sections 6.2 and */
/* 6.3 add up gamma over C_k(i) and over C_k(i) intersected with W.           */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t seed;
    uint32_t R;
    uint32_t r_begin;
    double alpha;
    uint32_t k_min;
    double tau;
    const uint8_t *pool_mask;    /* length n, NULL when no pool            */
    int32_t topk;                /* 0: k = infinity; else the Top-k size   */
    const double *gamma;         /* node values (length n) or NULL for 1   */
    int32_t hop_radius;          /* > 0: anchored r-hop neighbourhoods      */
} or_query;

/* Anchored r-hop neighbourhoods (Section 9.2): anchor i's step computes the
 * betweenness of the subgraph of H_r induced by S_r(i), the vertices within
 * `radius` surviving hops of i, reports its tie-broken maximiser (over S_r(i)
 * ∩ W for the pool selector), and is invalid when |S_r(i)| < k_min or the
 * coin fires.  Work counters per anchor: |S| source passes, each reaching |S|
 * vertices, the surviving directed slots inside S and the base directed
 * slots of S's vertices. */
static int or_anchored_step(const or_graph *g, const int32_t *eu, const int32_t *ev, const uint8_t *alive,
                            const uint32_t *w, int unit, int32_t i, int32_t radius, double tau,
                            const uint8_t *pool_mask, uint8_t *inS, uint8_t *aliveS, int32_t *queue, int32_t *hop,
                            double *B, uint64_t *dist, uint64_t *sigma, int32_t *order, double *delta,
                            uint8_t *member, int32_t *size_out, int32_t *c_out, int32_t *cw_out, uint64_t *ak_out,
                            uint64_t *dk_out)
{
    int32_t n = g->n, v, head = 0, cnt = 0, rc;
    int64_t e, k, ak = 0, dk = 0;
    for (v = 0; v < n; ++v) { inS[v] = 0; hop[v] = -1; }
    hop[i] = 0; queue[cnt++] = i;
    while (head < cnt) {                                   /* breadth-first hops over surviving edges */
        int32_t x = queue[head++];
        if (hop[x] == radius) continue;
        for (k = g->off[x]; k < g->off[x + 1]; ++k) {
            int32_t y = g->nbr[k];
            if (!alive[g->eid[k]] || hop[y] >= 0) continue;
            hop[y] = hop[x] + 1;
            queue[cnt++] = y;
        }
    }
    for (v = 0; v < cnt; ++v) inS[queue[v]] = 1;
    for (e = 0; e < g->m; ++e) {
        aliveS[e] = alive[e] && inS[eu[e]] && inS[ev[e]];
        ak += 2 * aliveS[e];
    }
    for (v = 0; v < cnt; ++v) dk += g->off[queue[v] + 1] - g->off[queue[v]];
    rc = or_brandes_graph(g, aliveS, w, unit, B, dist, sigma, order, delta);
    if (rc != OR_OK) return rc;
    for (v = 0; v < n; ++v) member[v] = inS[v];
    *c_out = or_band_argmax(n, B, member, tau, NULL);
    *cw_out = -1;
    if (pool_mask) {
        for (v = 0; v < n; ++v) member[v] = inS[v] && pool_mask[v];
        *cw_out = or_band_argmax(n, B, member, tau, NULL);
    }
    *size_out = cnt;
    *ak_out = (uint64_t)ak;
    *dk_out = (uint64_t)dk;
    return OR_OK;
}

typedef struct {
    uint32_t *counts;            /* n x (n+1), column n is bottom          */
    uint32_t *counts_w;          /* n x (n+1) or NULL                      */
    int32_t *center_global;      /* R or NULL                              */
    int32_t *next_table;         /* R x n or NULL (-1 = bottom)            */
    int32_t *next_table_w;       /* R x n or NULL                          */
    double *bsum;                /* n or NULL: sum over r of B(H_r)        */
    uint64_t stats[8];           /* units, sum n_K, sum A_K, sum D_K,      */
                                 /* near-band count, 0, 0, 0               */
    double *psi, *psi_w;         /* n each or NULL (topk > 0): sum over r  */
                                 /* of the Top-k step rewards               */
} or_sweep_out;

int or_sweep(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev, const or_model *mod,
             const or_query *q, or_sweep_out *out)
{
    or_graph g;
    uint8_t *alive = NULL, *member = NULL;
    uint32_t *w = NULL;
    uint64_t *dist = NULL, *sigma = NULL;
    int32_t *order = NULL, *comp = NULL, *size = NULL, *cc = NULL, *cw = NULL;
    double *B = NULL, *delta = NULL;
    int64_t *k_alive = NULL, *k_deg = NULL;
    int32_t *fw = NULL;
    uint8_t *ranked = NULL;
    double *gs = NULL, *gw = NULL;
    uint32_t rr;
    int32_t v, i;
    int unit = (mod->weight_kind == OR_WEIGHT_UNIT);
    int rc = or_graph_init(&g, n, m, eu, ev);
    if (rc != OR_OK) return rc;
    memset(out->stats, 0, sizeof(out->stats));
    alive = (uint8_t *)malloc((size_t)m + 1);
    member = (uint8_t *)malloc((size_t)n);
    w = (uint32_t *)malloc(sizeof(uint32_t) * ((size_t)m + 1));
    dist = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    sigma = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    comp = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    size = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    cc = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    cw = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    B = (double *)malloc(sizeof(double) * (size_t)n);
    delta = (double *)malloc(sizeof(double) * (size_t)n);
    k_alive = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    k_deg = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    fw = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    ranked = (uint8_t *)malloc((size_t)n);
    gs = (double *)malloc(sizeof(double) * (size_t)n);
    gw = (double *)malloc(sizeof(double) * (size_t)n);
    if (!alive || !member || !w || !dist || !sigma || !order || !comp || !size || !cc || !cw || !B || !delta ||
        !k_alive || !k_deg || !fw || !ranked || !gs || !gw) { rc = OR_E_NOMEM; goto done; }

    if (q->hop_radius > 0) {                               /* anchored r-hop neighbourhoods */
        uint8_t *inS = (uint8_t *)malloc((size_t)n), *aliveS = (uint8_t *)malloc((size_t)m + 1);
        int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int32_t *hop = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        if (!inS || !aliveS || !queue || !hop) rc = OR_E_NOMEM;
        for (rr = 0; rr < q->R && rc == OR_OK; ++rr) {
            uint32_t r = q->r_begin + rr;
            or_realize(n, m, eu, ev, mod, q->seed, r, alive, w);
            for (i = 0; i < n && rc == OR_OK; ++i) {
                int32_t sz, c, cwi;
                uint64_t ak, dk;
                int coin, valid;
                rc = or_anchored_step(&g, eu, ev, alive, w, unit, i, q->hop_radius, q->tau, q->pool_mask, inS,
                                      aliveS, queue, hop, B, dist, sigma, order, delta, member, &sz, &c, &cwi, &ak,
                                      &dk);
                if (rc != OR_OK) break;
                coin = or_stop_coin(q->seed, r, i, q->alpha);
                valid = !coin && (uint32_t)sz >= q->k_min;
                out->counts[(size_t)i * (n + 1) + (valid ? c : n)] += 1u;
                if (out->next_table) out->next_table[(size_t)rr * n + i] = valid ? c : -1;
                if (out->counts_w) {
                    int32_t nw = (valid && cwi >= 0) ? cwi : -1;
                    out->counts_w[(size_t)i * (n + 1) + (nw >= 0 ? nw : n)] += 1u;
                    if (out->next_table_w) out->next_table_w[(size_t)rr * n + i] = nw;
                }
                out->stats[0] += (uint64_t)sz;
                out->stats[1] += (uint64_t)sz * (uint64_t)sz;
                out->stats[2] += (uint64_t)sz * ak;
                out->stats[3] += (uint64_t)sz * dk;
            }
        }
        free(inS); free(aliveS); free(queue); free(hop);
        goto done;
    }

    for (rr = 0; rr < q->R; ++rr) {
        uint32_t r = q->r_begin + rr;
        int32_t cg;
        int64_t e;
        or_realize(n, m, eu, ev, mod, q->seed, r, alive, w);
        rc = or_brandes_graph(&g, alive, w, unit, B, dist, sigma, order, delta);
        if (rc != OR_OK) goto done;
        or_components_graph(&g, alive, comp, size, order);

        /* global centre c(H) (eq. central-node) */
        for (v = 0; v < n; ++v) member[v] = 1;
        cg = or_band_argmax(n, B, member, q->tau, (int64_t *)&out->stats[4]);
        if (out->center_global) out->center_global[rr] = cg;

        /* component centres (eq. local-center) and pool-constrained centres */
        for (v = 0; v < n; ++v) { cc[v] = -1; cw[v] = -1; }
        for (v = 0; v < n; ++v) {
            int32_t c = comp[v], u;
            if (cc[c] >= 0 || v != c) continue;          /* once per component, at its label */
            for (u = 0; u < n; ++u) member[u] = (comp[u] == c);
            cc[c] = or_band_argmax(n, B, member, q->tau, (int64_t *)&out->stats[4]);
            if (q->pool_mask) {
                for (u = 0; u < n; ++u) member[u] = (comp[u] == c) && q->pool_mask[u];
                cw[c] = or_band_argmax(n, B, member, q->tau, (int64_t *)&out->stats[4]);
            }
        }

        /* finite k: rank each component by repeated band argmax and keep, per
         * component label, the gamma mass of its Top-k set, of that set's
         * pool members, and its highest-ranked pool member */
        if (q->topk > 0) {
            for (v = 0; v < n; ++v) { ranked[v] = 0; gs[v] = 0.0; gw[v] = 0.0; fw[v] = -1; }
            for (v = 0; v < n; ++v) {
                int32_t c = comp[v], u, t;
                if (v != c) continue;
                for (t = 0; t < q->topk && t < size[v]; ++t) {
                    int32_t pick;
                    double gv;
                    for (u = 0; u < n; ++u) member[u] = (comp[u] == c) && !ranked[u];
                    pick = or_band_argmax(n, B, member, q->tau, NULL);
                    ranked[pick] = 1;
                    gv = q->gamma ? q->gamma[pick] : 1.0;
                    gs[c] += gv;
                    if (q->pool_mask && q->pool_mask[pick]) {
                        gw[c] += gv;
                        if (fw[c] < 0) fw[c] = pick;
                    }
                }
            }
        }

        /* anchors: Alg. 1 for every i, counted as in Alg. 2 */
        for (i = 0; i < n; ++i) {
            int coin = or_stop_coin(q->seed, r, i, q->alpha);
            int valid = !coin && (uint32_t)size[i] >= q->k_min;
            int32_t nx = valid ? cc[comp[i]] : -1;
            out->counts[(size_t)i * (n + 1) + (nx >= 0 ? nx : n)] += 1u;
            if (out->next_table) out->next_table[(size_t)rr * n + i] = nx;
            if (q->topk > 0 && valid) {
                if (out->psi) out->psi[i] += gs[comp[i]];
                if (out->psi_w) out->psi_w[i] += gw[comp[i]];
            }
            if (out->counts_w) {
                int32_t nw = (valid && q->pool_mask) ? (q->topk > 0 ? fw[comp[i]] : cw[comp[i]]) : -1;
                out->counts_w[(size_t)i * (n + 1) + (nw >= 0 ? nw : n)] += 1u;
                if (out->next_table_w) out->next_table_w[(size_t)rr * n + i] = nw;
            }
        }
        if (out->bsum)
            for (v = 0; v < n; ++v) out->bsum[v] += B[v];

        /* work accounting per (r, s): n_K = |K(s)|, A_K = surviving directed
         * slots inside K(s), D_K = base directed slots of K(s)'s vertices */
        for (v = 0; v < n; ++v) { k_alive[v] = 0; k_deg[v] = 0; }
        for (v = 0; v < n; ++v) k_deg[comp[v]] += g.off[v + 1] - g.off[v];
        for (e = 0; e < m; ++e)
            if (alive[e]) k_alive[comp[eu[e]]] += 2;
        for (v = 0; v < n; ++v) {
            out->stats[0] += 1;
            out->stats[1] += (uint64_t)size[v];
            out->stats[2] += (uint64_t)k_alive[comp[v]];
            out->stats[3] += (uint64_t)k_deg[comp[v]];
        }
    }
done:
    free(alive); free(member); free(w); free(dist); free(sigma); free(order); free(comp); free(size);
    free(cc); free(cw); free(B); free(delta); free(k_alive); free(k_deg);
    free(fw); free(ranked); free(gs); free(gw);
    or_graph_free(&g);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Trajectory simulator (Section 4.3): episodes of the stochastic network    */
/* process itself.  Episode e starts at X_0 = x0[e]; at step t the anchor    */
/* X_t draws a fresh network state and stop coin, counters (e, u, v, 2 + t)  */
/* for edge (u, v) and (e, X_t, 2^32-1, 2 + t) for the coin; the step is     */
/* invalid (X_{t+1} = bottom) when the coin fires or |K(X_t;H)| < k_min,      */
/* otherwise X_{t+1} = c_loc(X_t;H).  T = number of pre-absorption states.    */
/* Outputs feed the length-biased estimators of Definition on length-biased   */
/* sampling: visits(v) / sum T estimates b_v (Proposition on uniform-step     */
/* equivalence), sum f(X_t) / sum T the node-reward AFC, and the switch count */
/* the transition reward 1{X_{t+1} in V, X_{t+1} != X_t} (Section 6.4).       */
/* Episodes that reach max_steps pre-absorption states are truncated.         */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t seed;
    int32_t episodes;
    const int32_t *x0;           /* episodes                                  */
    double alpha;
    uint32_t k_min;
    double tau;
    int32_t max_steps;
    const double *f;             /* node reward (length n) or NULL            */
} or_traj_query;

typedef struct {
    int32_t *lengths;            /* episodes: T_e                             */
    int32_t *paths;              /* episodes x max_steps (-1 past T_e) or NULL */
    uint64_t *visits;            /* n                                         */
    double reward_f;             /* sum over episodes and t < T of f(X_t)     */
    uint64_t switches;
    uint64_t total_steps;
    int32_t truncated;
} or_traj_out;

int or_trajectories(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev, const or_model *mod,
                    const or_traj_query *q, or_traj_out *out)
{
    or_graph g;
    uint8_t *alive = NULL, *member = NULL;
    uint32_t *w = NULL;
    uint64_t *dist = NULL, *sigma = NULL;
    int32_t *order = NULL, *comp = NULL, *size = NULL;
    double *B = NULL, *delta = NULL;
    int32_t e, v;
    int unit = (mod->weight_kind == OR_WEIGHT_UNIT);
    int rc = or_graph_init(&g, n, m, eu, ev);
    if (rc != OR_OK) return rc;
    alive = (uint8_t *)malloc((size_t)m + 1);
    member = (uint8_t *)malloc((size_t)n);
    w = (uint32_t *)malloc(sizeof(uint32_t) * ((size_t)m + 1));
    dist = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    sigma = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    comp = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    size = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    B = (double *)malloc(sizeof(double) * (size_t)n);
    delta = (double *)malloc(sizeof(double) * (size_t)n);
    if (!alive || !member || !w || !dist || !sigma || !order || !comp || !size || !B || !delta) {
        rc = OR_E_NOMEM;
        goto done;
    }
    memset(out->visits, 0, sizeof(uint64_t) * (size_t)n);
    out->reward_f = 0.0;
    out->switches = 0;
    out->total_steps = 0;
    out->truncated = 0;
    for (e = 0; e < q->episodes; ++e) {
        int32_t x = q->x0[e], t = 0;
        for (;;) {
            int32_t nx = -1;
            uint32_t stream = 2u + (uint32_t)t;
            if (out->paths) out->paths[(size_t)e * q->max_steps + t] = x;
            out->visits[x] += 1;
            if (q->f) out->reward_f += q->f[x];
            ++t;
            if (!or_stop_coin_stream(q->seed, (uint32_t)e, x, stream, q->alpha)) {
                or_realize_stream(n, m, eu, ev, mod, q->seed, (uint32_t)e, stream, alive, w);
                rc = or_brandes_graph(&g, alive, w, unit, B, dist, sigma, order, delta);
                if (rc != OR_OK) goto done;
                or_components_graph(&g, alive, comp, size, order);
                if ((uint32_t)size[x] >= q->k_min) {
                    for (v = 0; v < n; ++v) member[v] = (comp[v] == comp[x]);
                    nx = or_band_argmax(n, B, member, q->tau, NULL);
                }
            }
            if (nx >= 0 && nx != x) out->switches += 1;
            if (nx < 0) break;
            if (t == q->max_steps) { out->truncated += 1; break; }
            x = nx;
        }
        out->lengths[e] = t;
        out->total_steps += (uint64_t)t;
        if (out->paths)
            for (v = t; v < q->max_steps; ++v) out->paths[(size_t)e * q->max_steps + v] = -1;
    }
done:
    free(alive); free(member); free(w); free(dist); free(sigma); free(order); free(comp); free(size);
    free(B); free(delta);
    or_graph_free(&g);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Chain algebra (Section 4, eq. amc ... eq. afc-def).                       */
/* ------------------------------------------------------------------------ */

/* Empirical kernel of Alg. 2 with the stabilisation of Section 8.2: P_ij =
 * C_ij / R; when an anchor never absorbed (C_i,bottom = 0) and eta > 0, the
 * absorption entry is floored to eta and the row renormalised, i.e. the
 * transient entries are scaled by (1 - eta). */
int or_counts_to_kernel(int32_t n, const uint32_t *counts, uint32_t R, double eta, double *Q, double *r)
{
    int32_t i, j;
    if (n < 1 || R == 0) return OR_E_ARG;
    for (i = 0; i < n; ++i) {
        const uint32_t *row = counts + (size_t)i * (n + 1);
        if (row[n] == 0 && eta > 0.0) {
            for (j = 0; j < n; ++j) Q[(size_t)i * n + j] = (1.0 - eta) * ((double)row[j] / (double)R);
            r[i] = eta;
        } else {
            for (j = 0; j < n; ++j) Q[(size_t)i * n + j] = (double)row[j] / (double)R;
            r[i] = (double)row[n] / (double)R;
        }
    }
    return OR_OK;
}

/* Fundamental matrix N = (I - Q)^{-1} (eq. fundamental) by LU factorisation
 * with partial pivoting and one forward/back substitution per unit column. */
int or_fundamental(int32_t n, const double *Q, double *N)
{
    double *A = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
    int32_t *piv = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    int32_t i, j, k, c;
    int rc = OR_OK;
    if (!A || !piv || !x) { free(A); free(piv); free(x); return OR_E_NOMEM; }
    for (i = 0; i < n; ++i)
        for (j = 0; j < n; ++j) A[(size_t)i * n + j] = (i == j ? 1.0 : 0.0) - Q[(size_t)i * n + j];
    for (k = 0; k < n; ++k) {
        int32_t p = k;
        double amax = fabs(A[(size_t)k * n + k]);
        for (i = k + 1; i < n; ++i)
            if (fabs(A[(size_t)i * n + k]) > amax) { amax = fabs(A[(size_t)i * n + k]); p = i; }
        if (amax == 0.0) { rc = OR_E_SINGULAR; goto out; }
        piv[k] = p;
        if (p != k)
            for (j = 0; j < n; ++j) {
                double t = A[(size_t)k * n + j]; A[(size_t)k * n + j] = A[(size_t)p * n + j]; A[(size_t)p * n + j] = t;
            }
        for (i = k + 1; i < n; ++i) {
            double l = A[(size_t)i * n + k] / A[(size_t)k * n + k];
            A[(size_t)i * n + k] = l;
            for (j = k + 1; j < n; ++j) A[(size_t)i * n + j] -= l * A[(size_t)k * n + j];
        }
    }
    for (c = 0; c < n; ++c) {
        for (i = 0; i < n; ++i) x[i] = (i == c) ? 1.0 : 0.0;
        for (k = 0; k < n; ++k)                       /* apply the row swaps */
            if (piv[k] != k) { double t = x[k]; x[k] = x[piv[k]]; x[piv[k]] = t; }
        for (i = 1; i < n; ++i)                       /* L y = P e_c */
            for (k = 0; k < i; ++k) x[i] -= A[(size_t)i * n + k] * x[k];
        for (i = n - 1; i >= 0; --i) {                /* U x = y */
            for (k = i + 1; k < n; ++k) x[i] -= A[(size_t)i * n + k] * x[k];
            x[i] /= A[(size_t)i * n + i];
        }
        for (i = 0; i < n; ++i) N[(size_t)i * n + c] = x[i];
    }
out:
    free(A); free(piv); free(x);
    return rc;
}

/* Visits mu(s) = sN (eq. visits), E_s[T] = mu 1 (eq. expected-length) and
 * AFC b(s) = mu / mu 1 (eq. afc-def). */
void or_visits(int32_t n, const double *N, const double *s, double *mu, double *ET, double *b)
{
    int32_t i, j;
    double tot = 0.0;
    for (j = 0; j < n; ++j) {
        double acc = 0.0;
        for (i = 0; i < n; ++i) acc += s[i] * N[(size_t)i * n + j];
        mu[j] = acc;
    }
    for (j = 0; j < n; ++j) tot += mu[j];
    *ET = tot;
    for (j = 0; j < n; ++j) b[j] = mu[j] / tot;
}

/* Top-k of b by decreasing value, ties to the smaller index. */
static void or_topk(int32_t n, const double *b, int32_t k, int32_t *top)
{
    int32_t t, v;
    uint8_t *taken = (uint8_t *)calloc((size_t)n, 1);
    for (t = 0; t < k; ++t) {
        int32_t best = -1;
        for (v = 0; v < n; ++v)
            if (!taken[v] && (best < 0 || b[v] > b[best])) best = v;
        top[t] = best; taken[best] = 1;
    }
    free(taken);
}

/* Visit-gap certificates of Section 5.5.  For the pair (u, v):
 *   G_uv = mu_u - mu_v (eq. pm-gap);
 *   crude threshold 2 * epsbar / r_min^2;
 *   sharp threshold (epsbar / r_min) * max_i |N_iu - N_iv| (eq. sharp-gap).
 * The order u > v is certified when G_uv exceeds the threshold. */
void or_pair_certificate(int32_t n, const double *N, const double *mu, double epsbar, double r_min,
                         int32_t u, int32_t v, double *gap, double *crude, double *sharp)
{
    int32_t i;
    double mx = 0.0;
    for (i = 0; i < n; ++i) {
        double d = fabs(N[(size_t)i * n + u] - N[(size_t)i * n + v]);
        if (d > mx) mx = d;
    }
    *gap = mu[u] - mu[v];
    *crude = 2.0 * epsbar / (r_min * r_min);
    *sharp = epsbar / r_min * mx;
}

/* The whole tail for one query (Sections 4, 5.5, 6.4, 7.1-7.2, 8.2-8.3).     */
typedef struct {
    double eta;                  /* floor on an empty absorption column     */
    const double *s;             /* initial distribution (length n)         */
    const double *f;             /* node reward f (length n) or NULL        */
    const uint8_t *pool_mask;    /* W (length n) or NULL                    */
    double eps;                  /* row-wise radius of every entry          */
    double r_lower;              /* leak lower bound                         */
    int32_t cert_topk;           /* size of the nominal Top-k, 0 = none     */
    const double *psi, *psi_w;   /* Top-k step-reward sums over R draws or NULL */
    int32_t fb_node;             /* fallback representative v_fb, -1 = none */
    const uint8_t *fb_mask;      /* fallback set V_fb (length n) or NULL    */
} or_tail_in;

typedef struct {
    double *Q, *r, *N;           /* n*n, n, n*n                             */
    double *mu, *b;              /* n, n                                     */
    double ET, b_f;
    double *b_w, *xi;            /* n, n   (pool kernel)                     */
    double ET_w, m_w, b_w_f;
    double *b_w_bar;             /* n: b_w / m_w on W, 0 off W              */
    int32_t *top;                /* cert_topk                                */
    double *cert_gap, *cert_sharp;  /* cert_topk x (n - cert_topk)           */
    int32_t *cert_v;             /* the complement, in increasing index     */
    double cert_crude, epsbar, epsbar_supp;
    double cert_crude_supp;
    double *cert_sharp_supp;     /* cert_topk x (n - cert_topk)             */
    int32_t admissible;          /* nominal kernel inside the set: r_i >= r_lower */
    double *psi_hat, *psi_w_hat; /* n each: estimated expected step rewards  */
    double b_k, b_kw;            /* valued Top-k reward-AFCs (eq. mr-afc-def, eq. mr-pool-afc) */
    double *b_fb, *b_cens;       /* n each: fallback-kernel AFC, censored profile */
    double ET_fb, m_w_fb, c_fb;  /* fallback kernel: E[T], pool mass, non-fallback mass */
} or_tail_out;

int or_tail(int32_t n, const uint32_t *counts, const uint32_t *counts_w, uint32_t R, const or_tail_in *in,
            or_tail_out *out)
{
    int32_t i, j, k = in->cert_topk;
    int rc = or_counts_to_kernel(n, counts, R, in->eta, out->Q, out->r);
    if (rc != OR_OK) return rc;
    rc = or_fundamental(n, out->Q, out->N);
    if (rc != OR_OK) return rc;
    or_visits(n, out->N, in->s, out->mu, &out->ET, out->b);
    out->b_f = 0.0;
    if (in->f)
        for (j = 0; j < n; ++j) out->b_f += out->b[j] * in->f[j];   /* eq. mr-inner-product */

    out->admissible = 1;
    for (i = 0; i < n; ++i)
        if (out->r[i] < in->r_lower) out->admissible = 0;
    out->epsbar = (double)n * in->eps;                /* dense radii: epsbar = max_i sum_j eps_ij */
    {
        int32_t supp_max = 0;
        for (i = 0; i < n; ++i) {
            int32_t c = 0;
            for (j = 0; j < n; ++j) c += (out->Q[(size_t)i * n + j] > 0.0);
            if (c > supp_max) supp_max = c;
        }
        out->epsbar_supp = (double)supp_max * in->eps;
    }
    out->cert_crude = 2.0 * out->epsbar / (in->r_lower * in->r_lower);
    out->cert_crude_supp = 2.0 * out->epsbar_supp / (in->r_lower * in->r_lower);
    if (k > 0 && k < n) {
        int32_t a, c = 0, v;
        uint8_t *intop = (uint8_t *)calloc((size_t)n, 1);
        or_topk(n, out->b, k, out->top);
        for (a = 0; a < k; ++a) intop[out->top[a]] = 1;
        for (v = 0; v < n; ++v)
            if (!intop[v]) out->cert_v[c++] = v;
        for (a = 0; a < k; ++a)
            for (c = 0; c < n - k; ++c) {
                double gap, crude, sharp;
                or_pair_certificate(n, out->N, out->mu, out->epsbar, in->r_lower, out->top[a], out->cert_v[c],
                                    &gap, &crude, &sharp);
                out->cert_gap[(size_t)a * (n - k) + c] = gap;
                out->cert_sharp[(size_t)a * (n - k) + c] = sharp;
                if (out->cert_sharp_supp) {      /* eq. sharp-gap with the support-restricted radii */
                    double g2, c2, s2;
                    or_pair_certificate(n, out->N, out->mu, out->epsbar_supp, in->r_lower, out->top[a],
                                        out->cert_v[c], &g2, &c2, &s2);
                    out->cert_sharp_supp[(size_t)a * (n - k) + c] = s2;
                }
            }
        free(intop);
    }

    /* reward-AFC of a step reward (Proposition on reward-AFC): s N psi / s N 1
     * = mu . psi / E[T], with psi estimated by its average over the R draws */
    out->b_k = 0.0;
    out->b_kw = 0.0;
    if (in->psi) {
        for (j = 0; j < n; ++j) {
            double ph = in->psi[j] / (double)R;
            if (out->psi_hat) out->psi_hat[j] = ph;
            out->b_k += out->mu[j] * ph;
        }
        out->b_k /= out->ET;
    }
    if (in->psi_w) {
        for (j = 0; j < n; ++j) {
            double ph = in->psi_w[j] / (double)R;
            if (out->psi_w_hat) out->psi_w_hat[j] = ph;
            out->b_kw += out->mu[j] * ph;
        }
        out->b_kw /= out->ET;
    }

    /* fallback kernel P^{W,fb} (Section 7.3): valid draws whose selection is
     * empty move to v_fb instead of absorbing; with the same counts, the
     * valid-but-empty draws of row i are C^W_i,bottom - C_i,bottom.  Then
     * the censored profile of Section 7.4 renormalises b^{W,fb} off V_fb. */
    if (counts_w && in->pool_mask && in->fb_node >= 0 && out->b_fb) {
        uint32_t *cf = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n * (size_t)(n + 1));
        double *Qf = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
        double *rf = (double *)malloc(sizeof(double) * (size_t)n);
        double *Nf = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
        double *muf = (double *)malloc(sizeof(double) * (size_t)n);
        if (!cf || !Qf || !rf || !Nf || !muf) { free(cf); free(Qf); free(rf); free(Nf); free(muf); return OR_E_NOMEM; }
        for (i = 0; i < n; ++i) {
            const uint32_t *rw = counts_w + (size_t)i * (n + 1);
            uint32_t *rowf = cf + (size_t)i * (n + 1);
            for (j = 0; j < n; ++j) rowf[j] = rw[j];
            rowf[in->fb_node] += rw[n] - counts[(size_t)i * (n + 1) + n];
            rowf[n] = counts[(size_t)i * (n + 1) + n];
        }
        rc = or_counts_to_kernel(n, cf, R, in->eta, Qf, rf);
        if (rc == OR_OK) rc = or_fundamental(n, Qf, Nf);
        if (rc == OR_OK) {
            or_visits(n, Nf, in->s, muf, &out->ET_fb, out->b_fb);
            out->m_w_fb = 0.0;
            out->c_fb = 0.0;
            for (j = 0; j < n; ++j) {
                if (in->pool_mask[j]) out->m_w_fb += out->b_fb[j];
                if (!(in->fb_mask && in->fb_mask[j])) out->c_fb += out->b_fb[j];
            }
            if (out->b_cens)
                for (j = 0; j < n; ++j)
                    out->b_cens[j] = (!(in->fb_mask && in->fb_mask[j]) && out->c_fb > 0.0) ? out->b_fb[j] / out->c_fb
                                                                                         : 0.0;
        }
        free(cf); free(Qf); free(rf); free(Nf); free(muf);
        if (rc != OR_OK) return rc;
    }

    if (counts_w && in->pool_mask) {                   /* constrained kernel P^W (Section 7) */
        double *Qw = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
        double *rw = (double *)malloc(sizeof(double) * (size_t)n);
        double *Nw = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
        double *muw = (double *)malloc(sizeof(double) * (size_t)n);
        if (!Qw || !rw || !Nw || !muw) { free(Qw); free(rw); free(Nw); free(muw); return OR_E_NOMEM; }
        for (i = 0; i < n; ++i)                         /* eq. settopk-xi, raw frequencies */
            out->xi[i] = 1.0 - (double)counts_w[(size_t)i * (n + 1) + n] / (double)R;
        rc = or_counts_to_kernel(n, counts_w, R, in->eta, Qw, rw);
        if (rc == OR_OK) rc = or_fundamental(n, Qw, Nw);
        if (rc == OR_OK) {
            or_visits(n, Nw, in->s, muw, &out->ET_w, out->b_w);
            out->m_w = 0.0; out->b_w_f = 0.0;
            for (j = 0; j < n; ++j) {
                if (in->pool_mask[j]) out->m_w += out->b_w[j];      /* eq. settopk-bPsi */
                if (in->f) out->b_w_f += out->b_w[j] * in->f[j];
            }
            for (j = 0; j < n; ++j)
                out->b_w_bar[j] = (in->pool_mask[j] && out->m_w > 0.0) ? out->b_w[j] / out->m_w : 0.0;
        }
        free(Qw); free(rw); free(Nw); free(muw);
    }
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Robust tail on a given transient block Q0 (Sections 5.1, 5.4, 6.4 and the */
/* robust experiment of Section 9.1).                                        */
/*  - transition rewards (Section 6.4): switching eta(i,j) = 1{j != i} and     */
/*    improvement eta(i,j) = (f_j - f_i)_+ for j in V (0 on absorption), with  */
/*    psi_i = sum_j Q_ij eta(i,j) and the reward-AFC mu . psi / E[T];          */
/*  - sampled admissible kernels: Q_ij = Q0_ij (1 + delta (2u - 1)) clipped to */
/*    [0, 1], u uniform from Philox counter (sample, i, j, 3) as a 53-bit      */
/*    fraction, and each row scaled down to sum 1 - r_min when it exceeds it;  */
/*    for each sample b(P), KL(b(P) || b0) and TV = |b(P) - b0|_1 / 2;         */
/*  - first-order sensitivity (Section 5.4) for E = Q* - Q0, Q* the KL         */
/*    maximiser: b_lin = b0 + mu0 E N0 / (mu0 1) - b0 (mu0 E N0 1) / (mu0 1),  */
/*    the remainder bound |N0 E|^2 |N0| / (1 - |N0 E|) and the actual          */
/*    |N* - N0 - N0 E N0| (infinity norms).                                    */
/* ------------------------------------------------------------------------ */
static double or_u53(uint64_t seed, uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t ctr[4], key[2], x[4];
    key[0] = (uint32_t)seed; key[1] = (uint32_t)(seed >> 32);
    ctr[0] = a; ctr[1] = b; ctr[2] = c; ctr[3] = 3u;
    or_philox4x32_10(ctr, key, x);
    return (double)((((uint64_t)x[0]) << 21) ^ (((uint64_t)x[1]) >> 11)) * (1.0 / 9007199254740992.0);
}

void or_perturbed_kernel(int32_t n, const double *Q0, uint64_t seed, int32_t sample, double delta, double r_min,
                         double *Q)
{
    int32_t i, j;
    for (i = 0; i < n; ++i) {
        double tot = 0.0, cap = 1.0 - r_min;
        for (j = 0; j < n; ++j) {
            double u = or_u53(seed, (uint32_t)sample, (uint32_t)i, (uint32_t)j);
            double f = 1.0 + delta * (2.0 * u - 1.0);
            double q = Q0[(size_t)i * n + j] * f;
            if (q < 0.0) q = 0.0;
            if (q > 1.0) q = 1.0;
            Q[(size_t)i * n + j] = q;
            tot += q;
        }
        if (tot > cap)
            for (j = 0; j < n; ++j) Q[(size_t)i * n + j] *= cap / tot;
    }
}

static double or_inf_norm(int32_t n, const double *A)
{
    int32_t i, j;
    double best = 0.0;
    for (i = 0; i < n; ++i) {
        double t = 0.0;
        for (j = 0; j < n; ++j) t += fabs(A[(size_t)i * n + j]);
        if (t > best) best = t;
    }
    return best;
}

static void or_matmul(int32_t n, const double *A, const double *B, double *C)
{
    int32_t i, j, k;
    for (i = 0; i < n; ++i)
        for (j = 0; j < n; ++j) {
            double acc = 0.0;
            for (k = 0; k < n; ++k) acc += A[(size_t)i * n + k] * B[(size_t)k * n + j];
            C[(size_t)i * n + j] = acc;
        }
}

typedef struct {
    const double *s;             /* n                                          */
    const double *f;             /* n or NULL (no transition rewards)          */
    int32_t samples;             /* sampled admissible kernels                 */
    double delta;                /* relative radius                            */
    double r_min;                /* leak lower bound                           */
    uint64_t seed;
} or_robust_in;

typedef struct {
    double *b0;                  /* n                                          */
    double b_sw, b_imp;          /* transition reward-AFCs                      */
    double *kl, *tv;             /* samples                                    */
    int32_t kl_arg, tv_arg;
    double *b_kl, *b_tv;         /* n: AFC at the maximisers                    */
    double *b_lin;               /* n: first-order AFC for E = Q_kl - Q0        */
    double norm_N0E, norm_N0, rem_bound, rem_actual;
} or_robust_out;

int or_robust(int32_t n, const double *Q0, const or_robust_in *in, or_robust_out *out)
{
    size_t nn = (size_t)n * (size_t)n;
    double *N0 = (double *)malloc(sizeof(double) * nn), *Qs = (double *)malloc(sizeof(double) * nn);
    double *Ns = (double *)malloc(sizeof(double) * nn), *M1 = (double *)malloc(sizeof(double) * nn);
    double *M2 = (double *)malloc(sizeof(double) * nn);
    double *mu0 = (double *)malloc(sizeof(double) * (size_t)n), *mus = (double *)malloc(sizeof(double) * (size_t)n);
    double *bs = (double *)malloc(sizeof(double) * (size_t)n), *v = (double *)malloc(sizeof(double) * (size_t)n);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    double ET0, ETs;
    int32_t i, j, k;
    int rc = OR_OK;
    if (!N0 || !Qs || !Ns || !M1 || !M2 || !mu0 || !mus || !bs || !v || !w) { rc = OR_E_NOMEM; goto done; }
    rc = or_fundamental(n, Q0, N0);
    if (rc != OR_OK) goto done;
    or_visits(n, N0, in->s, mu0, &ET0, out->b0);
    out->b_sw = 0.0;
    out->b_imp = 0.0;
    if (in->f) {
        for (i = 0; i < n; ++i) {
            double sw = 0.0, im = 0.0;
            for (j = 0; j < n; ++j) {
                double q = Q0[(size_t)i * n + j], d = in->f[j] - in->f[i];
                if (j != i) sw += q;
                if (d > 0.0) im += q * d;
            }
            out->b_sw += mu0[i] * sw;
            out->b_imp += mu0[i] * im;
        }
        out->b_sw /= ET0;
        out->b_imp /= ET0;
    }
    out->kl_arg = -1;
    out->tv_arg = -1;
    for (k = 0; k < in->samples; ++k) {
        double kl = 0.0, tv = 0.0;
        or_perturbed_kernel(n, Q0, in->seed, k, in->delta, in->r_min, Qs);
        rc = or_fundamental(n, Qs, Ns);
        if (rc != OR_OK) goto done;
        or_visits(n, Ns, in->s, mus, &ETs, bs);
        for (j = 0; j < n; ++j) {
            if (bs[j] > 0.0) kl += bs[j] * log(bs[j] / out->b0[j]);
            tv += fabs(bs[j] - out->b0[j]);
        }
        tv *= 0.5;
        out->kl[k] = kl;
        out->tv[k] = tv;
        if (out->kl_arg < 0 || kl > out->kl[out->kl_arg]) {
            out->kl_arg = k;
            memcpy(out->b_kl, bs, sizeof(double) * (size_t)n);
        }
        if (out->tv_arg < 0 || tv > out->tv[out->tv_arg]) {
            out->tv_arg = k;
            memcpy(out->b_tv, bs, sizeof(double) * (size_t)n);
        }
    }
    if (out->kl_arg >= 0) {
        double tot = 0.0, vs = 0.0;
        or_perturbed_kernel(n, Q0, in->seed, out->kl_arg, in->delta, in->r_min, Qs);
        for (k = 0; k < (int32_t)nn; ++k) Qs[k] -= Q0[k];                 /* E */
        for (j = 0; j < n; ++j) {                                          /* w = mu0 E */
            double acc = 0.0;
            for (i = 0; i < n; ++i) acc += mu0[i] * Qs[(size_t)i * n + j];
            w[j] = acc;
        }
        for (j = 0; j < n; ++j) {                                          /* v = mu0 E N0 */
            double acc = 0.0;
            for (i = 0; i < n; ++i) acc += w[i] * N0[(size_t)i * n + j];
            v[j] = acc;
            vs += acc;
        }
        for (j = 0; j < n; ++j) tot += mu0[j];
        for (j = 0; j < n; ++j) out->b_lin[j] = out->b0[j] + v[j] / tot - out->b0[j] * vs / tot;
        or_matmul(n, N0, Qs, M1);                                          /* N0 E */
        out->norm_N0E = or_inf_norm(n, M1);
        out->norm_N0 = or_inf_norm(n, N0);
        out->rem_bound = out->norm_N0E < 1.0
                             ? out->norm_N0E * out->norm_N0E * out->norm_N0 / (1.0 - out->norm_N0E) : INFINITY;
        or_matmul(n, M1, N0, M2);                                          /* N0 E N0 */
        or_perturbed_kernel(n, Q0, in->seed, out->kl_arg, in->delta, in->r_min, Qs);   /* Q* again */
        rc = or_fundamental(n, Qs, Ns);
        if (rc != OR_OK) goto done;
        for (k = 0; k < (int32_t)nn; ++k) Ns[k] -= N0[k] + M2[k];
        out->rem_actual = or_inf_norm(n, Ns);
    }
done:
    free(N0); free(Qs); free(Ns); free(M1); free(M2); free(mu0); free(mus); free(bs); free(v); free(w);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Nonparametric bootstrap of the AFC profile (Section 8.4: resample each    */
/* row's M draws with replacement and recompute b).  Replicate beta redraws, */
/* for every row i, R draw indices uniformly from {0 .. R-1}: draw t takes   */
/* word (t mod 4) of the Philox block at counter (beta, i, t / 4,            */
/* 0x80000004), index = (word * R) >> 32; the replicate's counts of row i    */
/* are those of next(index, i).  The replicate kernel is built as for the    */
/* estimate itself (P-hat = C / R, floor eta on an empty absorption column), */
/* and b* = s N* / (s N* 1).  Per node: mean and standard deviation (divisor */
/* B - 1) over the B replicates, and the nearest-rank percentiles of the     */
/* sorted values at (1 - level) / 2 and (1 + level) / 2 (rank ceil(q B)).    */
/* ------------------------------------------------------------------------ */
void or_boot_counts(int32_t n, uint32_t R, const int32_t *next_table, uint64_t seed, uint32_t beta,
                    uint32_t *counts)
{
    uint32_t key[2], ctr[4], x[4], t;
    int32_t i;
    key[0] = (uint32_t)seed; key[1] = (uint32_t)(seed >> 32);
    memset(counts, 0, sizeof(uint32_t) * (size_t)n * (size_t)(n + 1));
    for (i = 0; i < n; ++i) {
        for (t = 0; t < R; ++t) {
            uint32_t j;
            int32_t nx;
            if ((t & 3u) == 0u) {
                ctr[0] = beta; ctr[1] = (uint32_t)i; ctr[2] = t >> 2; ctr[3] = 0x80000004u;
                or_philox4x32_10(ctr, key, x);
            }
            j = (uint32_t)(((uint64_t)x[t & 3u] * (uint64_t)R) >> 32);
            nx = next_table[(size_t)j * n + i];
            counts[(size_t)i * (n + 1) + (nx >= 0 ? nx : n)] += 1u;
        }
    }
}

static int or_cmp_double(const void *a, const void *b)
{
    const double x = *(const double *)a, y = *(const double *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

typedef struct {
    uint64_t seed;
    int32_t replicates;          /* B >= 1                                     */
    double level;                /* interval coverage in (0, 1)                */
    double eta;                  /* floor (R10); 0 disables                    */
    const double *s;             /* n                                          */
} or_boot_in;

typedef struct {
    double *b0;                  /* n: AFC of the given draws                  */
    double *mean, *sd, *lo, *hi; /* n each                                     */
    double *b_rep;               /* B x n                                      */
} or_boot_out;

int or_bootstrap(int32_t n, uint32_t R, const int32_t *next_table, const or_boot_in *in, or_boot_out *out)
{
    const size_t nn = (size_t)n * (size_t)n;
    const int32_t B = in->replicates;
    uint32_t *counts = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n * (size_t)(n + 1));
    double *Q = (double *)malloc(sizeof(double) * nn), *N = (double *)malloc(sizeof(double) * nn);
    double *r = (double *)malloc(sizeof(double) * (size_t)n), *mu = (double *)malloc(sizeof(double) * (size_t)n);
    double *col = (double *)malloc(sizeof(double) * (size_t)(B > 0 ? B : 1));
    double ET;
    int32_t i, v, b;
    uint32_t t;
    int rc = OR_OK;
    if (!counts || !Q || !N || !r || !mu || !col) { rc = OR_E_NOMEM; goto done; }
    if (n < 1 || R == 0 || B < 1 || !(in->level > 0.0 && in->level < 1.0)) { rc = OR_E_ARG; goto done; }
    /* the estimate itself */
    memset(counts, 0, sizeof(uint32_t) * (size_t)n * (size_t)(n + 1));
    for (t = 0; t < R; ++t)
        for (i = 0; i < n; ++i) {
            const int32_t nx = next_table[(size_t)t * n + i];
            counts[(size_t)i * (n + 1) + (nx >= 0 ? nx : n)] += 1u;
        }
    or_counts_to_kernel(n, counts, R, in->eta, Q, r);
    rc = or_fundamental(n, Q, N);
    if (rc != OR_OK) goto done;
    or_visits(n, N, in->s, mu, &ET, out->b0);
    /* replicates */
    for (b = 0; b < B; ++b) {
        or_boot_counts(n, R, next_table, in->seed, (uint32_t)b, counts);
        or_counts_to_kernel(n, counts, R, in->eta, Q, r);
        rc = or_fundamental(n, Q, N);
        if (rc != OR_OK) goto done;
        or_visits(n, N, in->s, mu, &ET, out->b_rep + (size_t)b * n);
    }
    /* per-node summaries */
    for (v = 0; v < n; ++v) {
        double m = 0.0, ss = 0.0;
        int32_t klo, khi;
        for (b = 0; b < B; ++b) { col[b] = out->b_rep[(size_t)b * n + v]; m += col[b]; }
        m /= (double)B;
        for (b = 0; b < B; ++b) ss += (col[b] - m) * (col[b] - m);
        out->mean[v] = m;
        out->sd[v] = B > 1 ? sqrt(ss / (double)(B - 1)) : 0.0;
        qsort(col, (size_t)B, sizeof(double), or_cmp_double);
        klo = (int32_t)ceil(0.5 * (1.0 - in->level) * (double)B) - 1;
        khi = (int32_t)ceil(0.5 * (1.0 + in->level) * (double)B) - 1;
        if (klo < 0) klo = 0;
        if (khi > B - 1) khi = B - 1;
        out->lo[v] = col[klo];
        out->hi[v] = col[khi];
    }
done:
    free(counts); free(Q); free(N); free(r); free(mu); free(col);
    return rc;
}

/* ------------------------------------------------------------------------
 * Wasserstein-1 between two profiles on the shortest-path metric of the base
 * topology (robust experiment of Section 9.1; W1 as an integral probability
 * metric over 1-Lipschitz functions, Section 4), with every edge of length 1
 * (hop metric, cost == NULL) or of the positive integer length cost[e].
 *
 * On a graph metric W1(p, q) is the cost of the cheapest flow that moves the
 * surplus p - q over the edges at cost c_e per unit on edge e (the
 * transshipment form of the transport problem).  It is computed by successive
 * shortest paths: every round runs Bellman-Ford from all nodes with remaining
 * surplus over the residual graph (an edge carrying flow f from u to v offers
 * v -> u at cost -c_e for up to f, and u -> v at cost +c_e without limit; a
 * flow-free edge offers both directions at +c_e), takes the nearest node with remaining
 * deficit (smallest index among the nearest), and pushes along the
 * predecessor path the largest amount that neither overdraws the surplus,
 * the deficit, nor a cancelled flow.  Augmenting along shortest paths keeps
 * the flow optimal for the amount moved, so the final cost is W1.
 * Returns OR_E_ARG for a disconnected graph with unbalanced components or an
 * exhausted round budget.
 * ---------------------------------------------------------------------- */
int or_w1(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev, const uint32_t *cost, const double *p,
          const double *q, double *w1)
{
    double *ex = (double *)malloc(sizeof(double) * (size_t)n);
    double *f = (double *)calloc((size_t)(m > 0 ? m : 1), sizeof(double));
    int64_t *dist = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *pred = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);   /* 2e + dir, -1 = none */
    const int64_t INF = INT64_MAX / 4;
    int64_t round, e, max_rounds = 16 * ((int64_t)n + m) + 16;
    int32_t v;
    int rc = OR_OK;
    if (!ex || !f || !dist || !pred) { rc = OR_E_NOMEM; goto out; }
    for (v = 0; v < n; ++v) ex[v] = p[v] - q[v];
    for (round = 0;; ++round) {
        int has_src = 0, has_snk = 0, changed, pass;
        int32_t t = -1, s, x;
        double th;
        for (v = 0; v < n; ++v) { has_src |= ex[v] > 0.0; has_snk |= ex[v] < 0.0; }
        if (!has_src || !has_snk) break;
        if (round >= max_rounds) { rc = OR_E_ARG; goto out; }
        for (v = 0; v < n; ++v) { dist[v] = ex[v] > 0.0 ? 0 : INF; pred[v] = -1; }
        /* Bellman-Ford with strict improvements (no negative cycle exists in
         * the residual graph of an optimal flow) */
        for (pass = 0, changed = 1; changed; ++pass) {
            if (pass > n + 1) { rc = OR_E_ARG; goto out; }
            changed = 0;
            for (e = 0; e < m; ++e) {
                const int32_t a = eu[e], b = ev[e];
                const int64_t c = cost ? (int64_t)cost[e] : 1;
                const int64_t c_ab = f[e] < 0.0 ? -c : c;   /* a -> b */
                const int64_t c_ba = f[e] > 0.0 ? -c : c;   /* b -> a */
                if (dist[a] < INF && dist[a] + c_ab < dist[b]) { dist[b] = dist[a] + c_ab; pred[b] = 2 * e; changed = 1; }
                if (dist[b] < INF && dist[b] + c_ba < dist[a]) { dist[a] = dist[b] + c_ba; pred[a] = 2 * e + 1; changed = 1; }
            }
        }
        for (v = 0; v < n; ++v)
            if (ex[v] < 0.0 && dist[v] < INF && (t < 0 || dist[v] < dist[t])) t = v;
        if (t < 0) { rc = OR_E_ARG; goto out; }              /* surplus cannot reach any deficit */
        /* bottleneck along the path back to its source */
        th = -ex[t];
        for (x = t, s = t, pass = 0; pred[x] >= 0; ++pass) {
            if (pass > n) { rc = OR_E_ARG; goto out; }
            const int64_t a = pred[x], ee = a >> 1;
            const int fwd = (a & 1) == 0;                     /* eu -> ev */
            if (fwd && f[ee] < 0.0 && -f[ee] < th) th = -f[ee];
            if (!fwd && f[ee] > 0.0 && f[ee] < th) th = f[ee];
            x = fwd ? eu[ee] : ev[ee];
            s = x;
        }
        if (ex[s] < th) th = ex[s];
        for (x = t; pred[x] >= 0; ) {
            const int64_t a = pred[x], ee = a >> 1;
            const int fwd = (a & 1) == 0;
            f[ee] += fwd ? th : -th;
            x = fwd ? eu[ee] : ev[ee];
        }
        ex[s] -= th;
        ex[t] += th;
    }
    *w1 = 0.0;
    for (e = 0; e < m; ++e) *w1 += (cost ? (double)cost[e] : 1.0) * fabs(f[e]);
out:
    free(ex); free(f); free(dist); free(pred);
    return rc;
}
