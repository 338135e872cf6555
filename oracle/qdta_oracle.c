/*
 * qdta_oracle.c -- plain CPU oracle for the quasi-dynamic traffic assignment
 * (QDTA) hot path of Chan et al., "Quasi-Dynamic Traffic Assignment using
 * High Performance Computing" (arXiv 2104.12911).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header, table or helper with
 * the GPU library.
 *
 * What it computes, in the paper's order, with its numeric contract:
 *   - link costs by the BPR curve (Eq. 1), FP64 per link, rounded to FP32;
 *   - destination-rooted shortest-path trees (Get_shortest_path of Alg. 3 and
 *     Alg. 7): D_q(v) = min over out-links (v,w) of fl32(D_q(w) + c), found
 *     with a binary-heap Dijkstra on the reverse graph; the successor of v is
 *     the lowest-id out-link that is tight (fl32(D(w)+c) == D(v)) and strict
 *     (D(w) < D(v)); where FP32 absorption leaves no strict tight link, the
 *     lowest-id tight link one hop closer to q in the tight subgraph;
 *   - route truncation (Eq. 2, Truncate_path) and loading of the truncated
 *     path onto links (Eq. 5, Alg. 3, Alg. 7), flows in int64 units of
 *     2^-20 vehicle;
 *   - the Beckmann / "Rosenthal potential" objective (Eq. 6) and its
 *     derivative along the Frank-Wolfe direction (Eq. 8-9), summed exactly as
 *     int128 multiples of 2^-16;
 *   - the step rules: K-section on the sign of C'(alpha), the quasi-Newton
 *     search of Alg. 8 with the finite differences of Eq. 10 (Alg. 9), and
 *     MSA;
 *   - the link-flow Frank-Wolfe loop of Alg. 6 with the relative-gap or the
 *     objective-change (Eq. 7) stop rule;
 *   - residual demand after an interval (Alg. 4) and the interval chain of
 *     Alg. 1.
 *
 * Readings where the paper is garbled or silent (stop node, path keys,
 * flow units, stop rule, tie rule, ...) are the ones listed in the design
 * notes; each function states the one it applies.
 *
 * Build: gcc -std=c11 -O2 -ffp-contract=off -fno-fast-math -fopenmp -fPIC -shared
 * -ffp-contract=off is required: the contract forbids fused multiply-add.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __int128 i128;

#define ORC_OK 0
#define ORC_EARG (-1)
#define ORC_ECSR (-2)
#define ORC_EVAL (-3)
#define ORC_EUNREACH (-4)
#define ORC_EOVF (-5)
#define ORC_WARN_ABSORB 1

#define OBJ_UE 0   /* user equilibrium: Beckmann objective (Eq. 6), BPR costs route */
#define OBJ_SO 1   /* system optimum: total travel time, marginal costs route */

#define RULE_NONE 0
#define RULE_CEIL 1
#define RULE_FLOOR 2
#define RULE_PROGRESS 3

#define LS_KSECTION 0
#define LS_QN 1
#define LS_MSA 2

#define STOP_GAP 0
#define STOP_OBJ 1

static const double FX_SCALE = 1048576.0;     /* 2^20: vehicles -> fixed point */
static const double FX_INV = 1.0 / 1048576.0; /* exact power of two */
static const double SUM_SCALE = 65536.0;      /* 2^16: exact-sum quantum */

/* ------------------------------------------------------------------------ */
/* Fixed point and exact sums                                               */
/* ------------------------------------------------------------------------ */

/* trips -> int64 units of 2^-20 vehicle, round half to even. */
int64_t orc_trips_to_fx(double trips) { return (int64_t)rint(trips * FX_SCALE); }

/* Q(x) = round-half-even(x * 2^16) as int128; *bad set when not finite or
 * beyond the int128 range. */
static i128 quant(double x, int *bad) {
    double v = rint(x * SUM_SCALE);
    if (!isfinite(v) || fabs(v) >= 1.7e38) { *bad = 1; return 0; }
    return (i128)v;
}

static void put128(i128 v, int64_t *out) {
    out[0] = (int64_t)(uint64_t)((unsigned __int128)v);        /* low limb */
    out[1] = (int64_t)(v >> 64);                               /* high limb */
}

static i128 get128(const int64_t *in) {
    return (i128)(((unsigned __int128)(uint64_t)in[1] << 64) | (uint64_t)in[0]);
}

/* Correctly rounded int128 -> double (the C conversion rounds to nearest). */
double orc_i128_to_double(const int64_t *limbs) { return (double)get128(limbs); }

/* ------------------------------------------------------------------------ */
/* BPR link cost, Eq. 1 (section 3.2)                                        */
/* ------------------------------------------------------------------------ */

/* kappa turns vehicles in the interval into an hourly rate: 3600/dt for a
 * finite interval of dt seconds, 1 for plain static assignment (the demand is
 * then read as veh/h). */
double orc_kappa(double dt_s) { return isfinite(dt_s) ? 3600.0 / dt_s : 1.0; }

/* c_a = c0_a * (1 + alpha * (kappa F_a / C_a)^beta), FP64, no FMA, power by
 * left-to-right repeated multiplication, rounded once to FP32.  With
 * `marginal`, the marginal cost d(F c_a)/dF = c0_a (1 + (alpha (beta+1)) p)
 * that routes the system optimum (total travel time; the second of
 * Wardrop's principles, section 3). */
static double bpr64(double F, float c0, float cap, double alpha, int beta, double kappa, int marginal) {
    double r = (F * kappa) / (double)cap;
    double p = r;
    for (int k = 1; k < beta; ++k) p = p * r;
    double g = marginal ? alpha * (double)(beta + 1) : alpha;
    return (double)c0 * (1.0 + g * p);
}

int orc_bpr_obj(int32_t m, const int64_t *f_fx, const float *c0, const float *cap, double alpha,
                int32_t beta, double kappa, int32_t marginal, float *c_out) {
    if (m < 0 || beta < 1) return ORC_EARG;
    int bad = 0;
    for (int32_t a = 0; a < m; ++a) {
        double c = bpr64((double)f_fx[a] * FX_INV, c0[a], cap[a], alpha, beta, kappa, marginal);
        float c32 = (float)c;
        if (!isfinite(c32)) bad = 1;
        c_out[a] = c32;
    }
    return bad ? ORC_EOVF : ORC_OK;
}

int orc_bpr(int32_t m, const int64_t *f_fx, const float *c0, const float *cap, double alpha,
            int32_t beta, double kappa, float *c_out) {
    return orc_bpr_obj(m, f_fx, c0, cap, alpha, beta, kappa, 0, c_out);
}

/* Exact sum over links of Q(c_a * x_a * 2^-20): S_cf with x = f, S_cy with x = y. */
int orc_sum_cx(int32_t m, const float *c, const int64_t *x_fx, int64_t *out) {
    i128 s = 0;
    int bad = 0;
    for (int32_t a = 0; a < m; ++a) s += quant((double)c[a] * ((double)x_fx[a] * FX_INV), &bad);
    put128(s, out);
    return bad ? ORC_EOVF : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Graph helpers                                                            */
/* ------------------------------------------------------------------------ */

int orc_check_csr(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *col) {
    if (n <= 0 || m < 0 || row_ptr[0] != 0 || row_ptr[n] != m) return ORC_ECSR;
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] < row_ptr[v]) return ORC_ECSR;
    for (int32_t e = 0; e < m; ++e)
        if (col[e] < 0 || col[e] >= n) return ORC_ECSR;
    return ORC_OK;
}

typedef struct {
    int32_t n, m;
    const int32_t *row_ptr, *col;
    int32_t *tail;     /* tail node of each link */
    int32_t *rptr;     /* reverse CSR: in-links of each node */
    int32_t *rlink;    /* link ids, ascending within a node */
} graph_t;

static int graph_build(graph_t *g, int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *col) {
    g->n = n; g->m = m; g->row_ptr = row_ptr; g->col = col;
    g->tail = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    g->rptr = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    g->rlink = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    if (!g->tail || !g->rptr || !g->rlink) return ORC_EARG;
    for (int32_t v = 0; v < n; ++v)
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) g->tail[e] = v;
    for (int32_t e = 0; e < m; ++e) g->rptr[col[e] + 1]++;
    for (int32_t v = 0; v < n; ++v) g->rptr[v + 1] += g->rptr[v];
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    memcpy(fill, g->rptr, sizeof(int32_t) * (size_t)n);
    for (int32_t e = 0; e < m; ++e) g->rlink[fill[col[e]]++] = e;
    free(fill);
    return ORC_OK;
}

static void graph_free(graph_t *g) {
    free(g->tail); free(g->rptr); free(g->rlink);
}

/* ------------------------------------------------------------------------ */
/* Shortest-path tree rooted at a destination (Alg. 3 Get_shortest_path)   */
/* ------------------------------------------------------------------------ */

typedef struct { float key; int32_t node; } hitem;

typedef struct { hitem *a; int32_t size, cap; } heap_t;

static void heap_push(heap_t *h, float key, int32_t node) {
    if (h->size == h->cap) {
        h->cap = h->cap ? 2 * h->cap : 1024;
        h->a = (hitem *)realloc(h->a, sizeof(hitem) * (size_t)h->cap);
    }
    int32_t i = h->size++;
    while (i > 0) {
        int32_t p = (i - 1) / 2;
        if (h->a[p].key <= key) break;
        h->a[i] = h->a[p];
        i = p;
    }
    h->a[i].key = key; h->a[i].node = node;
}

static hitem heap_pop(heap_t *h) {
    hitem top = h->a[0];
    hitem last = h->a[--h->size];
    int32_t i = 0;
    for (;;) {
        int32_t l = 2 * i + 1, r = l + 1, s = i;
        float ks = last.key;
        if (l < h->size && h->a[l].key < ks) { s = l; ks = h->a[l].key; }
        if (r < h->size && h->a[r].key < ks) { s = r; }
        if (s == i) break;
        h->a[i] = h->a[s];
        i = s;
    }
    if (h->size > 0) h->a[i] = last;
    return top;
}

/* FP32 Dijkstra on the reverse graph: D[v] = fl32 min-plus time from v to q.
 * fl32(x + c) >= x and is monotone in x for c >= 0, so the label-setting
 * order is valid and D is the least fixed point of
 * D(v) = min_e fl32(D(head e) + c_e), which every label-correcting method
 * reaches too. */
static void dijkstra_to(const graph_t *g, const float *cost, int32_t q, float *D, heap_t *h) {
    for (int32_t v = 0; v < g->n; ++v) D[v] = INFINITY;
    D[q] = 0.0f;
    h->size = 0;
    heap_push(h, 0.0f, q);
    while (h->size > 0) {
        hitem it = heap_pop(h);
        int32_t u = it.node;
        if (it.key > D[u]) continue;            /* stale entry */
        for (int32_t i = g->rptr[u]; i < g->rptr[u + 1]; ++i) {
            int32_t e = g->rlink[i];
            int32_t v = g->tail[e];
            float cand = D[u] + cost[e];
            if (cand < D[v]) {
                D[v] = cand;
                heap_push(h, cand, v);
            }
        }
    }
}

/* Successor links under the tie rule.  Returns 1 when the absorption
 * fallback was needed for some node, 0 otherwise.  succ[q] = -1, and -1 for
 * nodes that cannot reach q. */
static int successors(const graph_t *g, const float *cost, int32_t q, const float *D,
                      int32_t *succ, int32_t *hop, int32_t *queue) {
    int need = 0;
    for (int32_t v = 0; v < g->n; ++v) {
        succ[v] = -1;
        if (v == q || !isfinite(D[v])) continue;
        for (int32_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e) {
            float w = D[g->col[e]];
            if (w < D[v] && (float)(w + cost[e]) == D[v]) { succ[v] = e; break; }
        }
        if (succ[v] < 0) need = 1;
    }
    if (!need) return 0;
    /* hop depth to q inside the tight subgraph, breadth-first from q */
    for (int32_t v = 0; v < g->n; ++v) hop[v] = -1;
    int32_t head = 0, tail = 0;
    hop[q] = 0;
    queue[tail++] = q;
    while (head < tail) {
        int32_t u = queue[head++];
        for (int32_t i = g->rptr[u]; i < g->rptr[u + 1]; ++i) {
            int32_t e = g->rlink[i];
            int32_t v = g->tail[e];
            if (hop[v] < 0 && isfinite(D[v]) && (float)(D[u] + cost[e]) == D[v]) {
                hop[v] = hop[u] + 1;
                queue[tail++] = v;
            }
        }
    }
    for (int32_t v = 0; v < g->n; ++v) {
        if (v == q || !isfinite(D[v]) || succ[v] >= 0) continue;
        for (int32_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e) {
            int32_t w = g->col[e];
            if ((float)(D[w] + cost[e]) == D[v] && hop[w] == hop[v] - 1) { succ[v] = e; break; }
        }
    }
    return 1;
}

/* One tree: D (float[n]) and succ (int32[n]).  Returns 0 or ORC_WARN_ABSORB. */
int orc_tree(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *col, const float *cost,
             int32_t q, float *D, int32_t *succ) {
    if (orc_check_csr(n, m, row_ptr, col) || q < 0 || q >= n) return ORC_EARG;
    graph_t g;
    if (graph_build(&g, n, m, row_ptr, col)) return ORC_EARG;
    heap_t h = {0};
    int32_t *hop = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *qu = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    dijkstra_to(&g, cost, q, D, &h);
    int w = successors(&g, cost, q, D, succ, hop, qu);
    free(hop); free(qu); free(h.a);
    graph_free(&g);
    return w ? ORC_WARN_ABSORB : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Truncated walk of one leg (Eq. 2 read as CEIL/FLOOR, Eq. 5)               */
/* ------------------------------------------------------------------------ */

/* Walks the successor path of leg (s0 -> q) and calls back for every loaded
 * link.  tau accumulates fl32 times with `tcost` (the interval's costs in the
 * Frank-Wolfe loop, the final costs in Alg. 4), starting from tau0.
 *   CEIL : a link entered before dt is loaded; stop at the first node reached
 *          at or after dt (the worked example of section 6).
 *   FLOOR: a link is loaded only if it is left by dt.
 *   NONE : walk to q.
 *   PROGRESS (the remedy section 3 suggests for intervals shorter than a
 *          link: track how far a trip got along its link): links are loaded
 *          as under CEIL, when entered before dt, but a trip that is still on
 *          a link at dt stops there, at the link's head with the time it still
 *          needs to reach it, *delay_out = fl32(tau - dt) > 0.  A leg that
 *          starts with tau0 >= dt is still on its way to s0: it stops there
 *          with delay fl32(tau0 - dt).  A trip on the last link of its path
 *          has loaded every link and completes (stop node q).
 * Returns the stop node (q when the leg completes); *delay_out (may be NULL)
 * receives the remaining delay, 0 unless PROGRESS stops a trip on a link.
 * pq > 0 (PROGRESS only): every delay a leg leaves with is rounded up to a
 * whole multiple of pq seconds, fl32(pq * ceil(x / pq)) in FP64, so that
 * legs stopped on the same link for the same destination merge into one
 * (reading R24: with exact delays every (iterate, leg) leaves a leg of its
 * own and the pending legs multiply from interval to interval). */
typedef void (*load_fn)(void *ctx, int32_t link);

static float progress_delay(float x, double pq) {
    if (!(pq > 0.0)) return x;
    return (float)(pq * ceil((double)x / pq));
}

static int32_t walk_leg(const int32_t *col, const int32_t *succ, const float *tcost, int32_t s0,
                        int32_t q, float dt32, int rule, float tau0, load_fn fn, void *ctx, float *delay_out,
                        double pq) {
    int32_t u = s0;
    float tau = tau0;
    if (delay_out) *delay_out = 0.0f;
    if (rule == RULE_PROGRESS && tau >= dt32) {
        if (delay_out) *delay_out = progress_delay(tau - dt32, pq);
        return s0;
    }
    while (u != q) {
        if ((rule == RULE_CEIL || rule == RULE_PROGRESS) && tau >= dt32) return u;
        int32_t e = succ[u];
        if (e < 0) return -1;
        float nt = tau + tcost[e];
        if (rule == RULE_FLOOR && nt > dt32) return u;
        if (fn) fn(ctx, e);
        tau = nt;
        u = col[e];
        if (rule == RULE_PROGRESS && tau > dt32) {
            if (u == q) return q;
            if (delay_out) *delay_out = progress_delay(tau - dt32, pq);
            return u;
        }
    }
    return q;
}

typedef struct { int64_t *y; int64_t d; } addctx;

static void add_link(void *ctx, int32_t e) {
    addctx *a = (addctx *)ctx;
#pragma omp atomic
    a->y[e] += a->d;
}

/* Group leg indices by destination (stable, ascending leg index). */
static int32_t *legs_by_dest(int32_t n, int32_t P, const int32_t *dest, int32_t **qptr_out) {
    int32_t *qptr = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(P > 0 ? P : 1));
    for (int32_t p = 0; p < P; ++p) qptr[dest[p] + 1]++;
    for (int32_t v = 0; v < n; ++v) qptr[v + 1] += qptr[v];
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    memcpy(fill, qptr, sizeof(int32_t) * (size_t)n);
    for (int32_t p = 0; p < P; ++p) idx[fill[dest[p]]++] = p;
    free(fill);
    *qptr_out = qptr;
    return idx;
}

static int effective_rule(double dt_s, int rule) { return isfinite(dt_s) ? rule : RULE_NONE; }

/* All-or-nothing assignment (Alg. 3 / Alg. 7 on one process): for every leg
 * with d > 0 and origin != destination, shortest path to its destination,
 * truncated, demand added to each loaded link.  y (int64[m]) is overwritten,
 * stop (int32[P], may be NULL) receives the stop node of each leg (q when it
 * completes, -1 when skipped).  Returns 0, ORC_WARN_ABSORB or an error. */
int orc_aon_d(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *col, const float *cost,
              const float *tcost, int32_t P, const int32_t *orig, const int32_t *dest, const int64_t *d_fx,
              const float *tau0, double dt_s, int32_t rule, int64_t *y, int32_t *stop, float *stop_delay,
              double pq, int32_t nthreads) {
    if (!tcost) tcost = cost;
    if (orc_check_csr(n, m, row_ptr, col)) return ORC_ECSR;
    for (int32_t p = 0; p < P; ++p)
        if (orig[p] < 0 || orig[p] >= n || dest[p] < 0 || dest[p] >= n || d_fx[p] < 0) return ORC_EARG;
    graph_t g;
    if (graph_build(&g, n, m, row_ptr, col)) return ORC_EARG;
    memset(y, 0, sizeof(int64_t) * (size_t)m);
    int32_t *qptr;
    int32_t *idx = legs_by_dest(n, P, dest, &qptr);
    int eff = effective_rule(dt_s, rule);
    float dt32 = (float)dt_s;
    int absorb = 0, unreach = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel reduction(| : absorb, unreach)
    {
        float *D = (float *)malloc(sizeof(float) * (size_t)n);
        int32_t *succ = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int32_t *hop = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int32_t *qu = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        heap_t h = {0};
#pragma omp for schedule(dynamic, 1)
        for (int32_t q = 0; q < n; ++q) {
            int32_t b = qptr[q], e = qptr[q + 1];
            int any = 0;
            for (int32_t i = b; i < e; ++i)
                if (d_fx[idx[i]] > 0 && orig[idx[i]] != q) { any = 1; break; }
            if (!any) {
                if (stop) for (int32_t i = b; i < e; ++i) stop[idx[i]] = -1;
                continue;
            }
            dijkstra_to(&g, cost, q, D, &h);
            absorb |= successors(&g, cost, q, D, succ, hop, qu);
            for (int32_t i = b; i < e; ++i) {
                int32_t p = idx[i];
                if (stop_delay) stop_delay[p] = 0.0f;
                if (d_fx[p] <= 0 || orig[p] == q) { if (stop) stop[p] = -1; continue; }
                if (!isfinite(D[orig[p]])) { unreach = 1; if (stop) stop[p] = -1; continue; }
                addctx ac = {y, d_fx[p]};
                float dl = 0.0f;
                int32_t s = walk_leg(col, succ, tcost, orig[p], q, dt32, eff, tau0 ? tau0[p] : 0.0f, add_link, &ac,
                                     &dl, pq);
                if (stop) stop[p] = s;
                if (stop_delay) stop_delay[p] = dl;
            }
        }
        free(D); free(succ); free(hop); free(qu); free(h.a);
    }
    free(idx); free(qptr);
    graph_free(&g);
    if (unreach) return ORC_EUNREACH;
    return absorb ? ORC_WARN_ABSORB : ORC_OK;
}

/* Legs that all start at their origin node at the start of the interval. */
int orc_aon_t(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *col, const float *cost,
              const float *tcost, int32_t P, const int32_t *orig, const int32_t *dest, const int64_t *d_fx,
              double dt_s, int32_t rule, int64_t *y, int32_t *stop, int32_t nthreads) {
    return orc_aon_d(n, m, row_ptr, col, cost, tcost, P, orig, dest, d_fx, NULL, dt_s, rule, y, stop, NULL, 0.0,
                     nthreads);
}

/* The trees' own costs clock the truncation (user equilibrium). */
int orc_aon(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *col, const float *cost,
            int32_t P, const int32_t *orig, const int32_t *dest, const int64_t *d_fx,
            double dt_s, int32_t rule, int64_t *y, int32_t *stop, int32_t nthreads) {
    return orc_aon_t(n, m, row_ptr, col, cost, NULL, P, orig, dest, d_fx, dt_s, rule, y, stop, nthreads);
}

/* Truncated paths (the link incidence of Eq. 5 under one set of trees): for
 * every leg, the links the walk of orc_aon loads, in walk order.  ptr
 * (int64[P+1]) always receives the offsets; links (int32[ptr[P]]) is filled
 * when not NULL.  Legs that orc_aon skips (d <= 0 or origin == destination)
 * have empty paths.  Single-threaded. */
typedef struct { int32_t *links; int64_t at; } pathctx;

static void put_link(void *ctx, int32_t e) {
    pathctx *pc = (pathctx *)ctx;
    if (pc->links) pc->links[pc->at] = e;
    pc->at++;
}

int orc_paths(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *col, const float *cost,
              int32_t P, const int32_t *orig, const int32_t *dest, const int64_t *d_fx, double dt_s,
              int32_t rule, int64_t *ptr, int32_t *links) {
    if (orc_check_csr(n, m, row_ptr, col)) return ORC_ECSR;
    for (int32_t p = 0; p < P; ++p)
        if (orig[p] < 0 || orig[p] >= n || dest[p] < 0 || dest[p] >= n) return ORC_EARG;
    graph_t g;
    if (graph_build(&g, n, m, row_ptr, col)) return ORC_EARG;
    int eff = effective_rule(dt_s, rule);
    float dt32 = (float)dt_s;
    float *D = (float *)malloc(sizeof(float) * (size_t)n);
    int32_t *succ = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *hop = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *qu = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *len = (int64_t *)calloc((size_t)(P > 0 ? P : 1), sizeof(int64_t));
    heap_t h = {0};
    int32_t *qptr;
    int32_t *idx = legs_by_dest(n, P, dest, &qptr);
    int rc = ORC_OK;
    /* pass 1: lengths */
    for (int32_t q = 0; q < n && rc >= 0; ++q) {
        if (qptr[q] == qptr[q + 1]) continue;
        dijkstra_to(&g, cost, q, D, &h);
        if (successors(&g, cost, q, D, succ, hop, qu)) rc = ORC_WARN_ABSORB;
        for (int32_t i = qptr[q]; i < qptr[q + 1]; ++i) {
            int32_t p = idx[i];
            if (d_fx[p] <= 0 || orig[p] == q) continue;
            if (!isfinite(D[orig[p]])) { rc = ORC_EUNREACH; break; }
            pathctx pc = {NULL, 0};
            walk_leg(col, succ, cost, orig[p], q, dt32, eff, 0.0f, put_link, &pc, NULL, 0.0);
            len[p] = pc.at;
        }
    }
    ptr[0] = 0;
    for (int32_t p = 0; p < P; ++p) ptr[p + 1] = ptr[p] + len[p];
    /* pass 2: the links, written at each leg's offset */
    if (links && rc >= 0) {
        for (int32_t q = 0; q < n; ++q) {
            if (qptr[q] == qptr[q + 1]) continue;
            dijkstra_to(&g, cost, q, D, &h);
            successors(&g, cost, q, D, succ, hop, qu);
            for (int32_t i = qptr[q]; i < qptr[q + 1]; ++i) {
                int32_t p = idx[i];
                if (d_fx[p] <= 0 || orig[p] == q) continue;
                pathctx pc = {links + ptr[p], 0};
                walk_leg(col, succ, cost, orig[p], q, dt32, eff, 0.0f, put_link, &pc, NULL, 0.0);
            }
        }
    }
    free(idx); free(qptr); free(len);
    free(D); free(succ); free(hop); free(qu); free(h.a);
    graph_free(&g);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Line search (Eq. 6, Eq. 8-10, Alg. 8-9)                                   */
/* ------------------------------------------------------------------------ */

/* Per-link terms at step alpha on f + alpha (y - f):
 *   obj = int_0^v c0 (1 + a (kappa s / C)^b) ds = c0 (v + a v p / (b+1)), p = (kappa v / C)^b
 *   der = (y - f) * c(v)          (d obj / d alpha)                         */
static void ls_terms(double F, double Y, float c0, float cap, double ab, int beta, double kappa,
                     double alpha, int so, double *obj, double *der) {
    double t = Y - F;
    double v = F + alpha * t;
    double r = (v * kappa) / (double)cap;
    double p = r;
    for (int k = 1; k < beta; ++k) p = p * r;
    double cost = (double)c0 * (1.0 + ab * p);
    if (so) {
        /* system optimum: total travel time v c(v) and its derivative
         * t (c + v c') = t c0 (1 + (ab (beta+1)) p) */
        double mc = (double)c0 * (1.0 + (ab * (double)(beta + 1)) * p);
        *obj = v * cost;
        *der = t * mc;
        return;
    }
    double g = ab * v;
    g = g * p;
    g = g / (double)(beta + 1);
    *obj = (double)c0 * (v + g);
    *der = t * cost;
}

/* Exact sums C(alpha_k) = sum Q(obj), C'(alpha_k) = sum Q(der) for K step
 * sizes (the batched form of Alg. 9's per-link partial sums).
 * Cs, Ds: int64[2K] (low, high limb per k). */
int orc_ls_eval(int32_t m, const int64_t *f, const int64_t *y, const float *c0, const float *cap,
                double ab, int32_t beta, double kappa, int32_t K, const double *alphas,
                int64_t *Cs, int64_t *Ds, int32_t objective) {
    int bad = 0;
    for (int32_t k = 0; k < K; ++k) {
        i128 sc = 0, sd = 0;
        for (int32_t a = 0; a < m; ++a) {
            double obj, der;
            ls_terms((double)f[a] * FX_INV, (double)y[a] * FX_INV, c0[a], cap[a], ab, beta, kappa,
                     alphas[k], objective, &obj, &der);
            sc += quant(obj, &bad);
            sd += quant(der, &bad);
        }
        put128(sc, Cs + 2 * k);
        put128(sd, Ds + 2 * k);
    }
    return bad ? ORC_EOVF : ORC_OK;
}

typedef struct {
    int32_t ls_mode;     /* LS_KSECTION, LS_QN, LS_MSA */
    int32_t K;           /* step sizes per K-section pass */
    int32_t passes;      /* K-section passes */
    int32_t max_ls;      /* quasi-Newton iteration cap L */
    double T1, T2, dx;   /* Alg. 8 thresholds and Eq. 10 stencil */
    int32_t objective;   /* OBJ_UE (Beckmann, Eq. 6) or OBJ_SO (total travel time) */
} ls_opts;

typedef struct {
    double alpha;
    int32_t evals;       /* passes over the links */
    int32_t qn_iters;
} ls_info;

static double q2d(i128 v) { return (double)v; }

/* K-section: bracket the root of C' (C is convex in alpha) on [0,1]. */
static int ksection(int32_t m, const int64_t *f, const int64_t *y, const float *c0, const float *cap,
                    double ab, int32_t beta, double kappa, int32_t K, int32_t passes, int32_t so,
                    ls_info *info) {
    double lo = 0.0, hi = 1.0;
    double *al = (double *)malloc(sizeof(double) * (size_t)K);
    int64_t *Cs = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)K);
    int64_t *Ds = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)K);
    i128 dlo = 0, dhi = 0;
    int rc = ORC_OK;
    double result = NAN;
    for (int32_t pass = 0; pass < passes; ++pass) {
        for (int32_t k = 0; k < K; ++k) al[k] = lo + ((hi - lo) * (double)k) / (double)(K - 1);
        rc = orc_ls_eval(m, f, y, c0, cap, ab, beta, kappa, K, al, Cs, Ds, so);
        info->evals++;
        if (rc) break;
        int32_t kk = -1;
        for (int32_t k = 0; k < K; ++k)
            if (get128(Ds + 2 * k) >= 0) { kk = k; break; }
        if (kk == 0) { result = al[0]; break; }
        if (kk < 0) { result = al[K - 1]; break; }
        lo = al[kk - 1]; hi = al[kk];
        dlo = get128(Ds + 2 * (kk - 1));
        dhi = get128(Ds + 2 * kk);
    }
    if (rc == ORC_OK && isnan(result)) {
        /* one secant step on the last bracket, from the exact sums */
        double a = lo, b = hi, da = q2d(dlo), db = q2d(dhi);
        result = a - (da * (b - a)) / (db - da);
    }
    info->alpha = result;
    free(al); free(Cs); free(Ds);
    return rc;
}

/* Quasi-Newton search of Alg. 8: start at 2/(2+j), three-point stencil of
 * Eq. 10 for C' and C'', |C'| < T1 or |step| < T2 stops, alpha kept in [0,1];
 * a non-positive C'' falls back to the K-section search. */
static int qn_search(int32_t m, const int64_t *f, const int64_t *y, const float *c0, const float *cap,
                     double ab, int32_t beta, double kappa, int32_t j, const ls_opts *o, ls_info *info) {
    double alpha = 2.0 / (2.0 + (double)j);
    double al[3];
    int64_t Cs[6], Ds[6];
    for (int32_t l = 0; l < o->max_ls; ++l) {
        al[0] = alpha - o->dx; al[1] = alpha; al[2] = alpha + o->dx;
        int rc = orc_ls_eval(m, f, y, c0, cap, ab, beta, kappa, 3, al, Cs, Ds, o->objective);
        info->evals++;
        info->qn_iters++;
        if (rc) return rc;
        double cm = q2d(get128(Cs)) / SUM_SCALE, c0v = q2d(get128(Cs + 2)) / SUM_SCALE,
               cp = q2d(get128(Cs + 4)) / SUM_SCALE;
        double d1 = (cp - cm) / (2.0 * o->dx);
        double d2 = ((cm - 2.0 * c0v) + cp) / (o->dx * o->dx);
        if (fabs(d1) < o->T1) { info->alpha = alpha; return ORC_OK; }
        if (!(d2 > 0.0)) return ksection(m, f, y, c0, cap, ab, beta, kappa, o->K, o->passes, o->objective, info);
        double an = alpha - d1 / d2;
        if (an < 0.0) an = 0.0;
        if (an > 1.0) an = 1.0;
        if (fabs(an - alpha) < o->T2) { info->alpha = an; return ORC_OK; }
        alpha = an;
    }
    info->alpha = alpha;
    return ORC_OK;
}

int orc_line_search(int32_t m, const int64_t *f, const int64_t *y, const float *c0, const float *cap,
                    double ab, int32_t beta, double kappa, int32_t j, const ls_opts *o, ls_info *info) {
    info->alpha = NAN; info->evals = 0; info->qn_iters = 0;
    if (o->ls_mode == LS_MSA) { info->alpha = 1.0 / ((double)j + 1.0); return ORC_OK; }
    if (o->ls_mode == LS_QN) return qn_search(m, f, y, c0, cap, ab, beta, kappa, j, o, info);
    if (o->K < 2 || o->passes < 1) return ORC_EARG;
    return ksection(m, f, y, c0, cap, ab, beta, kappa, o->K, o->passes, o->objective, info);
}

/* f <- f + rint(alpha * (y - f)) (Alg. 6 link-flow update). */
void orc_fw_update(int32_t m, int64_t *f, const int64_t *y, double alpha) {
    for (int32_t a = 0; a < m; ++a) f[a] += (int64_t)rint(alpha * (double)(y[a] - f[a]));
}

/* Beckmann objective of f alone (C at alpha = 0 with y = f), exact. */
static i128 objective(int32_t m, const int64_t *f, const float *c0, const float *cap, double ab,
                      int32_t beta, double kappa, int32_t so, int *bad) {
    i128 s = 0;
    for (int32_t a = 0; a < m; ++a) {
        double obj, der, F = (double)f[a] * FX_INV;
        ls_terms(F, F, c0[a], cap[a], ab, beta, kappa, 0.0, so, &obj, &der);
        s += quant(obj, bad);
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* FP64 reference of an iterate's relative gap and objective                 */
/* ------------------------------------------------------------------------ */

/* The relative gap (sum c F - sum c Y) / sum c F and the objective of flows f
 * with all-or-nothing direction y, free of the numeric contract: no FP32
 * rounding of the costs, no fixed-point quantisation of the terms, every
 * cost, term and sum in long double (64-bit mantissa), the power by powl.
 *   cost    c = c0 (1 + ab (kappa F / C)^beta)               (Eq. 1)
 *           (system optimum: the marginal cost c0 (1 + ab (beta+1) (kappa F / C)^beta))
 *   Beckmann integral  int_0^F c0 (1 + ab (kappa s / C)^beta) ds
 *           = c0 F (1 + ab (kappa F / C)^beta / (beta + 1))  (Eq. 6)
 *           (system optimum: the total travel time F c(F))
 * out[0] = sum c F, out[1] = sum c Y (veh s), out[2] = gap, out[3] = objective.
 * A reference for the contract's exact sums, which quantise every term to
 * 2^-16 and route by FP32 costs. */
void orc_ref_fp64(int32_t m, const int64_t *f, const int64_t *y, const float *c0, const float *cap,
                  double ab, int32_t beta, double kappa, int32_t so, double *out) {
    long double scf = 0.0L, scy = 0.0L, obj = 0.0L;
    for (int32_t a = 0; a < m; ++a) {
        long double F = (long double)f[a] / 1048576.0L;
        long double Y = (long double)y[a] / 1048576.0L;
        long double p = powl((long double)kappa * F / (long double)cap[a], (long double)beta);
        long double tt = (long double)c0[a] * (1.0L + (long double)ab * p);
        long double route = so ? (long double)c0[a] * (1.0L + (long double)ab * (long double)(beta + 1) * p) : tt;
        scf += route * F;
        scy += route * Y;
        obj += so ? F * tt : (long double)c0[a] * F * (1.0L + (long double)ab * p / (long double)(beta + 1));
    }
    out[0] = (double)scf;
    out[1] = (double)scy;
    out[2] = (double)((scf - scy) / scf);
    out[3] = (double)obj;
}

/* ------------------------------------------------------------------------ */
/* Frank-Wolfe for one interval (Alg. 2 in its link-flow form, Alg. 6)       */
/* ------------------------------------------------------------------------ */

typedef struct {
    double alpha_b;      /* BPR alpha */
    int32_t beta;        /* BPR beta (integer >= 1) */
    int32_t rule;        /* truncation rule */
    double dt_s;         /* interval length, inf for plain static assignment */
    int32_t stop_rule;   /* STOP_GAP or STOP_OBJ */
    double tol;          /* relative-gap tolerance, or T0 of Eq. 7 */
    int32_t max_iter;    /* iteration cap */
    int32_t fixed_iters; /* > 0: exactly this many updates, no stop test */
    ls_opts ls;
    int32_t nthreads;
} fw_opts;

typedef struct {
    int32_t iters;       /* updates applied */
    int32_t ls_evals;    /* line-search passes over the links */
    int32_t qn_iters;
    int32_t absorb;      /* absorption fallback used */
    int32_t stopped_by;  /* 0 cap/fixed, 1 gap, 2 objective, 3 stalled (alpha* = 0) */
    double gap;          /* relative gap at the returned iterate */
    double objective;    /* Beckmann objective at the returned iterate (veh s) */
    double last_alpha;
    double gap_fp64;     /* the same gap and objective by orc_ref_fp64 (no FP32 costs, no */
    double objective_fp64; /* quantised terms): the FP64 reference of each reported result */
} fw_stats;

/* tau0: float[P] or NULL, each leg's time still needed to reach its origin
 * (the PROGRESS rule's carried delay; 0 for new demand).
 * hist_alpha: double[max_iter+1], hist_cost: float[(max_iter+1) * m] (may be
 * NULL): alpha_j and the costs that defined AON j, j = 0 is the initial
 * free-flow AON (alpha_0 = 1).  gap_hist: double[max_iter+1] or NULL. */
int orc_fw_solve(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *col, const float *c0,
                 const float *cap, int32_t P, const int32_t *orig, const int32_t *dest,
                 const int64_t *d_fx, const float *tau0, const fw_opts *o, int64_t *f, fw_stats *st,
                 double *hist_alpha, float *hist_cost, double *gap_hist) {
    memset(st, 0, sizeof(*st));
    double kappa = orc_kappa(o->dt_s);
    /* the system optimum routes by marginal costs; its trips still take the
     * actual travel times, which clock the truncation */
    const int so = o->ls.objective == OBJ_SO;
    float *c = (float *)malloc(sizeof(float) * (size_t)(m > 0 ? m : 1));
    float *tc = so ? (float *)malloc(sizeof(float) * (size_t)(m > 0 ? m : 1)) : NULL;
    int64_t *y = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    int64_t *zero = (int64_t *)calloc((size_t)(m > 0 ? m : 1), sizeof(int64_t));
    int rc, bad = 0;
    int cap_iter = o->fixed_iters > 0 ? o->fixed_iters : o->max_iter;
    /* initial AON at free flow: BPR(0) = c0 exactly (the marginal cost too) */
    rc = orc_bpr_obj(m, zero, c0, cap, o->alpha_b, o->beta, kappa, so, c);
    if (rc < 0) goto done;
    if (so) orc_bpr(m, zero, c0, cap, o->alpha_b, o->beta, kappa, tc);
    rc = orc_aon_d(n, m, row_ptr, col, c, tc, P, orig, dest, d_fx, tau0, o->dt_s, o->rule, f, NULL, NULL, 0.0,
                   o->nthreads);
    if (rc < 0) goto done;
    st->absorb |= (rc == ORC_WARN_ABSORB);
    if (hist_alpha) hist_alpha[0] = 1.0;
    if (hist_cost) memcpy(hist_cost, c, sizeof(float) * (size_t)m);
    for (int32_t j = 1;; ++j) {
        rc = orc_bpr_obj(m, f, c0, cap, o->alpha_b, o->beta, kappa, so, c);
        if (rc < 0) goto done;
        if (so) orc_bpr(m, f, c0, cap, o->alpha_b, o->beta, kappa, tc);
        rc = orc_aon_d(n, m, row_ptr, col, c, tc, P, orig, dest, d_fx, tau0, o->dt_s, o->rule, y, NULL, NULL, 0.0,
                       o->nthreads);
        if (rc < 0) goto done;
        st->absorb |= (rc == ORC_WARN_ABSORB);
        int64_t scf[2], scy[2];
        orc_sum_cx(m, c, f, scf);
        orc_sum_cx(m, c, y, scy);
        i128 a = get128(scf), b = get128(scy);
        st->gap = q2d(a - b) / q2d(a);
        if (gap_hist) gap_hist[j - 1] = st->gap;
        if (o->fixed_iters <= 0 && o->stop_rule == STOP_GAP && fabs(st->gap) < o->tol) {
            st->stopped_by = 1;
            break;
        }
        if (j > cap_iter) break;
        ls_info li;
        rc = orc_line_search(m, f, y, c0, cap, o->alpha_b, o->beta, kappa, j, &o->ls, &li);
        if (rc < 0) goto done;
        st->ls_evals += li.evals;
        st->qn_iters += li.qn_iters;
        if (o->fixed_iters <= 0 && o->stop_rule == STOP_OBJ) {
            /* Converged(f, f_new) of Eq. 7 on the objective (Beckmann, or the total
             * travel time of the system optimum) */
            int64_t *fn = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
            memcpy(fn, f, sizeof(int64_t) * (size_t)m);
            orc_fw_update(m, fn, y, li.alpha);
            double b0 = q2d(objective(m, f, c0, cap, o->alpha_b, o->beta, kappa, so, &bad));
            double b1 = q2d(objective(m, fn, c0, cap, o->alpha_b, o->beta, kappa, so, &bad));
            free(fn);
            if (fabs((b0 - b1) / b0) < o->tol) { st->stopped_by = 2; break; }
        }
        if (o->fixed_iters <= 0 && li.alpha == 0.0) {
            /* alpha* = 0 leaves f unchanged and the next iteration would repeat
             * this one: under truncation the AON direction need not descend */
            st->stopped_by = 3;
            break;
        }
        orc_fw_update(m, f, y, li.alpha);
        st->iters = j;
        st->last_alpha = li.alpha;
        if (hist_alpha) hist_alpha[j] = li.alpha;
        if (hist_cost) memcpy(hist_cost + (size_t)j * (size_t)m, c, sizeof(float) * (size_t)m);
    }
    st->objective = q2d(objective(m, f, c0, cap, o->alpha_b, o->beta, kappa, so, &bad)) / SUM_SCALE;
    {
        /* y holds the direction of the last test, the one the gap was taken on */
        double ref[4];
        orc_ref_fp64(m, f, y, c0, cap, o->alpha_b, o->beta, kappa, so, ref);
        st->gap_fp64 = ref[2];
        st->objective_fp64 = ref[3];
    }
    rc = bad ? ORC_EOVF : ORC_OK;
done:
    free(c); free(tc); free(y); free(zero);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Residual demand after an interval (Alg. 4)                                */
/* ------------------------------------------------------------------------ */

/* tau0 (may be NULL) and r_delay (may be NULL): the legs' carried delays in
 * and the residual legs' delays out (the PROGRESS rule; 0 otherwise).
 * Path flows are keyed by full shortest paths: iterate j routed every leg on
 * the trees of cost vector c_j, and the converged mixture weights them by
 * lambda_j = alpha_j * prod_{k>j} (1 - alpha_k) (alpha_0 = 1).  Every path is
 * re-truncated with the final costs c_fin = BPR(f); a leg that stops at
 * s != q leaves rint(lambda_j d) at s, to be carried into the next interval
 * as demand (s, q).  Output legs are unmerged (one per j and leg);
 * out arrays must hold (J+1) * P entries.  *n_out receives the count, and
 * *done_fx the fixed-point demand that completed. */
int orc_residual(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *col, const float *c0,
                 const float *cap, double alpha_b, int32_t beta, double dt_s, int32_t rule,
                 const int64_t *f, int32_t J, const double *hist_alpha, const float *hist_cost,
                 int32_t P, const int32_t *orig, const int32_t *dest, const int64_t *d_fx, const float *tau0,
                 double pq, int32_t *r_orig, int32_t *r_dest, int64_t *r_fx, float *r_delay, int64_t *n_out,
                 int64_t *done_fx, double *lambda_out) {
    double kappa = orc_kappa(dt_s);
    int eff = effective_rule(dt_s, rule);
    float dt32 = (float)dt_s;
    float *cfin = (float *)malloc(sizeof(float) * (size_t)(m > 0 ? m : 1));
    int rc = orc_bpr(m, f, c0, cap, alpha_b, beta, kappa, cfin);
    if (rc < 0) { free(cfin); return rc; }
    double *lam = (double *)malloc(sizeof(double) * (size_t)(J + 1));
    for (int32_t j = 0; j <= J; ++j) {
        double l = (j == 0) ? 1.0 : hist_alpha[j];
        for (int32_t k = j + 1; k <= J; ++k) l = l * (1.0 - hist_alpha[k]);
        lam[j] = l;
        if (lambda_out) lambda_out[j] = l;
    }
    graph_t g;
    graph_build(&g, n, m, row_ptr, col);
    int32_t *qptr;
    int32_t *idx = legs_by_dest(n, P, dest, &qptr);
    /* trees of different (iterate, destination) pairs are independent: they
     * run in parallel, each leg's outcome goes to its own slot j * P + i (i =
     * its rank among the legs sorted by destination), and the slots are
     * gathered afterwards in the order (j, destination, leg) */
    size_t nslot = (size_t)(J + 1) * (size_t)(P > 0 ? P : 1);
    int32_t *t_orig = (int32_t *)malloc(sizeof(int32_t) * nslot);
    int64_t *t_w = (int64_t *)calloc(nslot, sizeof(int64_t));
    float *t_dl = (float *)malloc(sizeof(float) * nslot);
    int64_t done = 0;
    for (int32_t j = 0; j <= J; ++j) {
        if (!(lam[j] > 0.0)) continue;
        const float *cj = hist_cost + (size_t)j * (size_t)m;
#pragma omp parallel reduction(+ : done)
        {
            float *D = (float *)malloc(sizeof(float) * (size_t)n);
            int32_t *succ = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
            int32_t *hop = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
            int32_t *qu = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
            heap_t h = {0};
#pragma omp for schedule(dynamic, 1)
            for (int32_t q = 0; q < n; ++q) {
                int32_t b = qptr[q], e = qptr[q + 1];
                if (b == e) continue;
                int any = 0;
                for (int32_t i = b; i < e; ++i)
                    if (d_fx[idx[i]] > 0 && orig[idx[i]] != q) { any = 1; break; }
                if (!any) continue;
                dijkstra_to(&g, cj, q, D, &h);
                successors(&g, cj, q, D, succ, hop, qu);
                for (int32_t i = b; i < e; ++i) {
                    int32_t p = idx[i];
                    if (d_fx[p] <= 0 || orig[p] == q) continue;
                    int64_t w = (int64_t)rint(lam[j] * (double)d_fx[p]);
                    float dl = 0.0f;
                    int32_t s = walk_leg(col, succ, cfin, orig[p], q, dt32, eff, tau0 ? tau0[p] : 0.0f, NULL, NULL,
                                         &dl, pq);
                    if (s == q) { done += w; continue; }
                    size_t k = (size_t)j * (size_t)P + (size_t)i;
                    t_orig[k] = s;
                    t_w[k] = w;
                    t_dl[k] = dl;
                }
            }
            free(D); free(succ); free(hop); free(qu); free(h.a);
        }
    }
    int64_t cnt = 0;
    for (int32_t j = 0; j <= J; ++j)
        for (int32_t i = 0; i < P; ++i) {
            size_t k = (size_t)j * (size_t)P + (size_t)i;
            if (t_w[k] == 0) continue;
            r_orig[cnt] = t_orig[k]; r_dest[cnt] = dest[idx[i]]; r_fx[cnt] = t_w[k];
            if (r_delay) r_delay[cnt] = t_dl[k];
            cnt++;
        }
    free(t_orig); free(t_w); free(t_dl);
    *n_out = cnt;
    *done_fx = done;
    free(idx); free(qptr); free(lam); free(cfin);
    graph_free(&g);
    return ORC_OK;
}
