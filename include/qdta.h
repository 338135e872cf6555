/*
 * qdta.h -- C ABI of the MI355X (gfx950) hot path of quasi-dynamic traffic
 * assignment (QDTA), after Chan et al., "Quasi-Dynamic Traffic Assignment
 * using High Performance Computing" (arXiv 2104.12911).
 *
 * One Frank-Wolfe (FW) iteration of the paper's link-flow form (Alg. 6) is:
 *   BPR link costs (Eq. 1) -> all-or-nothing assignment (Alg. 3 / Alg. 7:
 *   shortest paths to every destination, route truncation by Eq. 2, loading
 *   by the truncated incidence of Eq. 5) -> convergence test (Eq. 7, or the
 *   relative gap) -> line search on the Beckmann objective (Eq. 6, Eq. 8-10,
 *   Alg. 8-9) -> link-flow update.  After an interval, residual demand is
 *   carried to the next one (Alg. 4, Alg. 1).
 *
 * Also: the system optimum in place of the user equilibrium
 * (opts->objective, Wardrop's second principle, section 3); checkpoint and
 * resume between intervals (qdta_get_residual / qdta_set_residual); and the
 * derivative of a solved interval's flows in the demand and the capacities
 * at frozen paths, for OD calibration (qdta_adjoint_record,
 * qdta_model_forward, qdta_model_backward; not in the paper).
 *
 * Conventions (all entry points):
 *   - Return value: QDTA_OK (0) on success, a negative QDTA_E* code on error
 *     (the context's last-error text says why), a positive QDTA_W* code for a
 *     warning.  No exception crosses the ABI.  A call that fails leaves the
 *     context usable unless it returns QDTA_EHIP.
 *   - Pointers named host_* or documented as host are ordinary host memory.
 *     All other arrays are device pointers on the context's device (e.g.
 *     torch tensors' data_ptr()), owned by the caller, which must keep them
 *     alive until the context's stream has executed the call.
 *   - Calls that take device pointers enqueue work on the context's stream
 *     and return without synchronising, unless documented otherwise.
 *   - Flows are int64 fixed point in units of 2^-20 vehicle ("fx");
 *     trips are converted with round-half-even(trips * 2^20).
 *   - Times are seconds.  Capacities are vehicles per hour.  Within an
 *     interval of dt seconds, a link's flow F (vehicles) enters the BPR curve
 *     as the hourly rate kappa*F, kappa = 3600/dt; dt = +inf means plain
 *     static assignment (kappa = 1, demand read as veh/h, no truncation).
 *   - A context holds one or more network instances ("batched" solve: every
 *     instance advances one FW iteration per launch sequence).  Node ids and
 *     link ids passed in and out are local to an instance; device arrays over
 *     "all links" are the instances' links concatenated in instance order
 *     (qdta_layout() gives the offsets).
 *   - A link's id ("uid") is its position in the caller's CSR.  Shortest-path
 *     ties are broken towards the lowest uid.
 *   - Sizes: nodes, links and legs, each summed over a context's instances,
 *     stay below 2^31 (QDTA_EARG otherwise).
 *   - Contexts are not thread-safe; use one per host thread.
 */
#ifndef QDTA_H
#define QDTA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QDTA_OK 0
#define QDTA_EARG (-1)      /* bad argument (null pointer, size, option range) */
#define QDTA_ECSR (-2)      /* malformed CSR (row_ptr not monotone, col out of range) */
#define QDTA_EVAL (-3)      /* free-flow time or capacity <= 0 or not finite */
#define QDTA_EUNREACH (-4)  /* a leg's destination is unreachable from its origin */
#define QDTA_EOVF (-5)      /* fixed-point, cost or exact-sum overflow */
#define QDTA_ENOMEM (-6)    /* device allocation failed, or the bound workspace is too small */
#define QDTA_EHIP (-7)      /* HIP runtime error (text in last error) */
#define QDTA_ESTATE (-8)    /* call out of order (e.g. solve before demand) */
#define QDTA_WABSORB 1      /* FP32 absorption: the tie-rule fallback was used */

#define QDTA_RULE_NONE 0    /* no truncation: walk to the destination */
#define QDTA_RULE_CEIL 1    /* load a link entered before dt; stop at the first node reached at or after dt */
#define QDTA_RULE_FLOOR 2   /* load a link only if it is left by dt */
/* Link progress (section 3's remedy for intervals shorter than a link): load
 * as CEIL, but a trip still on a link at dt stops at the link's head with the
 * time it still needs to get there (its delay); the next interval starts it
 * with that delay on its clock, and a leg whose delay is at or above dt stays
 * on its way (delay - dt).  A trip on the last link of its path completes.
 * Residual legs carry their delays (qdta_get_residual, qdta_set_residual)
 * and merge by (destination, origin, delay).  Not taken by the frozen-path
 * model (qdta_adjoint_record). */
#define QDTA_RULE_PROGRESS 3

#define QDTA_LS_KSECTION 0  /* K step sizes per pass, bracket the root of C'(alpha) */
#define QDTA_LS_QN 1        /* quasi-Newton search of Alg. 8 with the stencil of Eq. 10 */
#define QDTA_LS_MSA 2       /* alpha_j = 1/(j+1) */

#define QDTA_STOP_GAP 0     /* relative gap (sum c f - sum c y) / sum c f below tol */
#define QDTA_STOP_OBJ 1     /* relative change of the objective below tol (Eq. 7) */

/* Which of Wardrop's two principles (section 3) the interval solves: the user
 * equilibrium the paper adopts (trees by the BPR costs, Beckmann objective of
 * Eq. 6), or the system optimum (trees by the marginal costs
 * c + F dc/dF = c0 (1 + alpha (beta+1) (kappa F / C)^beta), objective the total
 * travel time sum F c(F)).  In both the truncation (Eq. 2) is clocked by the
 * travel times BPR(f), and the gap and stop rules use the routing costs. */
#define QDTA_OBJ_UE 0
#define QDTA_OBJ_SO 1

typedef struct qdta_ctx qdta_ctx;

/* Solver options.  qdta_default_opts() fills the paper's values:
 * BPR alpha 0.15, beta 4; CEIL truncation; K-section with K = 32, 3 passes;
 * T1 = T2 = dx = 1e-4 (Alg. 8, Eq. 10); relative-gap stop at 1e-4. */
typedef struct {
    double alpha;          /* BPR alpha (Eq. 1), >= 0 */
    int32_t beta;          /* BPR beta (Eq. 1), integer 1..16 */
    int32_t trunc_rule;    /* QDTA_RULE_* (ignored for dt = +inf) */
    int32_t ls_mode;       /* QDTA_LS_* */
    int32_t K;             /* K-section points per pass, 3..64 */
    int32_t passes;        /* K-section passes, 1..8 */
    int32_t max_ls;        /* quasi-Newton iteration cap L, 1..100 */
    double T1, T2, dx;     /* Alg. 8 thresholds (slope, step) and Eq. 10 stencil */
    int32_t stop_rule;     /* QDTA_STOP_* */
    double tol;            /* tolerance of the stop rule */
    int32_t max_iter;      /* FW iteration cap */
    int32_t fixed_iters;   /* > 0: exactly this many updates, stop rule ignored */
    int32_t keep_history;  /* record (alpha_j, c_j) per iteration; needed by qdta_advance_interval */
    int32_t waves_per_cu;  /* shortest-path wavefronts in flight per compute unit (a tree takes
                              tree_waves of them): 0 auto (28 for the chain-contracted search, 24
                              for the other kernels with four wavefronts per tree, 32 with one),
                              else 1..32 */
    double delta_scale;    /* delta-stepping bucket width as a multiple of the instance's geometric-mean
                              link cost: 0 auto (10.0); any value > 0 gives the same trees, only the speed
                              changes */
    int32_t sssp_shape;    /* shortest-path kernel shape, nodes per lane per step x links per lane per
                              chunk, 0 auto (3); four wavefronts per tree: 1 (1,2), 2 (1,4), 3 (2,4),
                              4 (4,4), 5 (2,2), 6 (4,2); one: 1 (1,4), 2 (2,4), 3 (4,4), 4 (4,8),
                              5 (8,8), 6 (1,1) */
    int32_t launch_form;   /* 0 batched: every tree of every instance in one launch, all K step sizes in
                              one pass, one FW iteration replayed as a captured HIP graph when possible
                              (K-section or MSA); 1 batched with direct launches; 2 plain: one launch per
                              destination tree and per step size (same results, for comparison) */
    int32_t tree_waves;    /* wavefronts that grow one shortest-path tree: 0 auto (4), 4 (a whole
                              workgroup per tree, a quarter as many trees in flight), or 1 */
    int32_t history_mib;   /* with keep_history: device memory for the iterates' labels, in MiB:
                              0 auto (without a workspace: the free device memory less 16 GiB; with
                              one: what the workspace has left), < 0 none (the residual step grows
                              every tree again); never changes results */
    int32_t objective;     /* QDTA_OBJ_UE (default) or QDTA_OBJ_SO */
    int32_t sssp_kernel;   /* shortest-path kernel: 0 auto (4, or 1 when tree_waves = 1), 1 node queue
                              (tree_waves and sssp_shape as above), 2 block-local (a block of node ids is
                              relaxed to closure in LDS per load; sssp_shape 1..4 = blocks of 128, 128
                              (two per wavefront per step), 64, 256 nodes; instances of at most 8,192
                              blocks, else the node queue), 3 node queue with each thread relaxing its own
                              nodes' in-links (sssp_shape 1..4 = nodes x links per thread 1x4, 2x4, 2x2,
                              1x2), 4 node queue (one workgroup per tree, sssp_shape as above) over the
                              chain-contracted network: nodes with exactly two neighbours that are no
                              tree's destination are left out of the search, each run of at most 8 of them
                              between two kept nodes is relaxed as one link applying its link costs one
                              by one, and their labels are filled from the run's ends after the search
                              (built on the host when first needed and again when a destination is a
                              left-out node; networks of fewer than 2^30 nodes in all, QDTA_EARG
                              otherwise).  The trees are the same whichever runs */
    int32_t load_form;     /* loading of plain intervals (dt = +inf, every instance plain): 0 auto (walk),
                              1 walk every leg to its destination, 2 merge the legs' paths children before
                              parents (two passes over the legs, each link loaded once per tree with the sum
                              of the demand through it; same int64 flows); truncated intervals always walk */
    int32_t pad1;
    double progress_quantum_s; /* link-progress rule only: every delay a leg leaves an interval with is rounded
                              up to a whole multiple of this many seconds, fl32(q * ceil(x / q)) in FP64, so
                              that legs stopped on the same link for the same destination merge (default
                              60; 0 keeps exact delays, with which every (iterate, leg) leaves a pending leg
                              of its own and a long day's pending legs multiply) */
} qdta_opts;

/* Per-instance results of qdta_solve. */
typedef struct {
    int32_t iters;         /* FW updates applied */
    int32_t ls_evals;      /* line-search passes over the links */
    int32_t qn_iters;      /* quasi-Newton iterations (QDTA_LS_QN) */
    int32_t absorb;        /* 1 when the FP32-absorption tie fallback was used */
    int32_t stopped_by;    /* 0 iteration cap / fixed count, 1 gap, 2 objective change,
                              3 stalled: the line search returned alpha* = 0, so f cannot change */
    int32_t status;        /* QDTA_OK or an error code for this instance */
    double gap;            /* relative gap at the returned iterate */
    double objective;      /* objective at the returned iterate (veh s): Beckmann, or the total travel
                              time under QDTA_OBJ_SO */
    double last_alpha;     /* last step size applied */
} qdta_stats;

/* Layout of the concatenated arrays (host output of qdta_layout). */
typedef struct {
    int32_t n_instances;
    int64_t total_nodes, total_links, total_legs, total_dests;
} qdta_layout_info;

void qdta_default_opts(qdta_opts *opts);
const char *qdta_strerror(int code);
/* Text of the last error on this context (never NULL; "" when none). */
const char *qdta_last_error(const qdta_ctx *ctx);

/* Create a context on HIP device `device`, enqueuing on `stream` (a
 * hipStream_t; NULL = the default stream).  *out receives the context. */
int qdta_create(qdta_ctx **out, int device, void *stream);
/* Free the context and the device memory it allocated (a bound workspace
 * stays the caller's).  Synchronises its stream. */
int qdta_destroy(qdta_ctx *ctx);
/* Change the stream later calls enqueue on. */
int qdta_set_stream(qdta_ctx *ctx, void *stream);

/* ---- Device memory owned by the caller ------------------------------------
 * By default the library allocates its own device memory (hipMalloc) as the
 * networks, the demand and the options need it, and frees it in
 * qdta_destroy.  A caller that owns the device memory (a torch tensor,
 * memory shared with other work) sizes a workspace with
 * qdta_workspace_query and hands it over with qdta_bind_workspace; from then
 * on every device buffer of the context -- network copies, demand tables,
 * shortest-path labels and queues, Frank-Wolfe state, per-iterate costs and
 * labels, the residual accumulator of Alg. 4 -- is carved from it and the
 * library calls hipMalloc no more.  The inputs are those of the problem
 * statement (section 3.1: the network, the interval's demand, the BPR and
 * step-rule options).
 *
 * qdta_workspace_query: *bytes (host) receives the device memory a solve
 * (and, with opts->keep_history, qdta_advance_interval) needs for the
 * networks added so far and the current demand, or for max_legs legs and
 * max_dests destinations (over all instances) if these are larger (0: the
 * current demand's).  max_legs also bounds the residual legs an interval
 * leaves (before merging, at most one per leg and iterate with weight > 0).
 * With keep_history, it covers opts->history_mib MiB of
 * iterate labels when that is > 0 (when it is 0, the labels get whatever the
 * workspace has left).  The maxima are remembered: once bound, buffers sized
 * by the demand are carved at them, so later intervals up to those sizes
 * reuse them.  Host-only: it allocates nothing.
 * qdta_bind_workspace: dev_ptr (device, aligned to 256 bytes, owned by the
 * caller, alive until qdta_destroy) of `bytes` bytes.  Call once, after the
 * networks and demand are set and before any call that uses device memory
 * (QDTA_ESTATE otherwise).  A call that needs more than is left returns
 * QDTA_ENOMEM (the text names the size): query again with larger maxima and
 * bind a larger workspace in a new context (qdta_get_residual /
 * qdta_set_residual carry the state between intervals).  The label-history
 * and path-record extras (qdta_adjoint_record, qdta_trees' temporaries) are
 * carved from what is left.  The library still allocates a small pinned host
 * mirror of the per-instance state.
 * qdta_alloc_count: *hip_mallocs (host, may be NULL) receives the number of
 * hipMalloc calls the context has made, *ws_in_use (may be NULL) the
 * workspace bytes currently carved -- for callers and tests that check that
 * no allocation happens. */
int qdta_workspace_query(qdta_ctx *ctx, const qdta_opts *opts, int64_t max_legs, int64_t max_dests,
                         size_t *bytes);
int qdta_bind_workspace(qdta_ctx *ctx, void *dev_ptr, size_t bytes);
int qdta_alloc_count(const qdta_ctx *ctx, int64_t *hip_mallocs, size_t *ws_in_use);

/* Add a network instance (section 3.1 notation: graph G(V,A), capacity C_a,
 * free-flow time c_0,a).  Host arrays: row_ptr int32[n+1] (row_ptr[0] = 0,
 * non-decreasing, row_ptr[n] = m), col int32[m] (head node of each link,
 * 0 <= col < n), fftt float[m] (> 0, finite, s), cap float[m] (> 0, finite,
 * veh/h).  Copied; the caller may free them on return.  *inst_out receives
 * the instance index (0, 1, ...).  Errors: QDTA_EARG, QDTA_ECSR, QDTA_EVAL. */
int qdta_add_network(qdta_ctx *ctx, int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *col,
                     const float *fftt, const float *cap, int32_t *inst_out);

/* Set the original demand d^o(i) of instance `inst` for the next interval
 * (Alg. 1): host arrays orig, dest int32[P] (local node ids), trips
 * double[P] (>= 0, vehicles departing in the interval).  Legs with
 * orig == dest or zero trips are dropped (Alg. 3 visits non-zero entries).
 * Residual demand d^r(i) left by qdta_advance_interval is merged in
 * (d(i) = d^o(i) + d^r(i)); legs with equal (orig, dest) are summed.
 * dt_s: interval length in s, or +inf for plain static assignment.
 * Errors: QDTA_EARG (ids out of range, negative or non-finite trips),
 * QDTA_EOVF (trips beyond the fixed-point range). */
int qdta_set_demand(qdta_ctx *ctx, int32_t inst, int32_t P, const int32_t *orig, const int32_t *dest,
                    const double *trips, double dt_s);

/* Sizes of the concatenated device arrays (host output). */
int qdta_layout(qdta_ctx *ctx, qdta_layout_info *info);
/* Host outputs: per-instance first node / first link / first leg / first
 * destination in the concatenated order (each int64[n_instances+1]). */
int qdta_offsets(qdta_ctx *ctx, int64_t *node_off, int64_t *link_off, int64_t *leg_off, int64_t *dest_off);

/* A1 -- link costs by Eq. 1 over all links: cost[a] = fl32(c0 (1 + alpha
 * (kappa F / C)^beta)), F = f_fx[a] * 2^-20, evaluated in FP64 without fused
 * multiply-add, the power by repeated multiplication.  f_fx int64[total_links],
 * cost float[total_links] (device).  Uses opts->alpha, opts->beta and each
 * instance's dt; under opts->objective = QDTA_OBJ_SO the routing costs
 * fl32(c0 (1 + (alpha (beta+1)) p)) instead.  Returns QDTA_EOVF (after the
 * stream completes: this call synchronises) if a cost is not finite. */
int qdta_bpr(qdta_ctx *ctx, const qdta_opts *opts, const int64_t *f_fx, float *cost);

/* A2 -- shortest-path trees (Get_shortest_path of Alg. 3) on one instance:
 * for each of the nq destinations (device int32[nq], local ids), the FP32
 * min-plus time to it from every node, dist float[nq][n] (+inf when
 * unreachable), and the successor link on the tree, succ int32[nq][n]
 * (local uid; -1 at the destination and where unreachable).  The successor is
 * the lowest-uid out-link (v,w) with fl32(dist[w] + cost) == dist[v] and
 * dist[w] < dist[v]; where FP32 absorption leaves none, the lowest-uid tight
 * link to a node one hop closer to the destination in the tight subgraph
 * (then QDTA_WABSORB is returned; this call synchronises).  cost is the
 * instance's float[m] (device). */
int qdta_trees(qdta_ctx *ctx, const qdta_opts *opts, int32_t inst, const float *cost, int32_t nq,
               const int32_t *dest, float *dist, int32_t *succ);

/* A2 + A3 -- all-or-nothing assignment of the current demand (Alg. 3 /
 * Alg. 7) under cost float[total_links]: y_fx int64[total_links] (device,
 * overwritten) receives the truncated loading; stop int32[total_legs] (device,
 * may be NULL) the stop node of each leg in qdta_get_legs() order (its
 * destination when the leg completes); stop_delay float[total_legs] (device,
 * may be NULL) the time the leg still needs to reach its stop node (link-
 * progress rule; 0 otherwise).  Synchronises; returns QDTA_EUNREACH,
 * QDTA_WABSORB or QDTA_OK. */
int qdta_aon(qdta_ctx *ctx, const qdta_opts *opts, const float *cost, int64_t *y_fx, int32_t *stop,
             float *stop_delay);

/* The current legs of all instances, in the order qdta_aon reports them:
 * grouped by instance, then by destination (then origin, then delay).  Host
 * outputs of int32/int32/int64/float[total_legs], local node ids, fixed-point
 * demand, and each leg's carried delay (link-progress rule; 0 for new
 * demand); any may be NULL. */
int qdta_get_legs(qdta_ctx *ctx, int32_t *host_orig, int32_t *host_dest, int64_t *host_d_fx, float *host_delay);

/* A5 -- exact line-search sums (Alg. 9 batched over K step sizes): for every
 * instance i and k < K, C_i(alpha) = sum_a Q(obj_a) and C'_i(alpha) =
 * sum_a Q(der_a) at alpha = alphas[i*K + k] (device double), where on
 * v = F + alpha (Y - F): obj = c0 (v + alpha_b v p / (beta+1)),
 * p = (kappa v / C)^beta, der = (Y - F) c0 (1 + alpha_b p), and
 * Q(x) = round-half-even(x * 2^16) summed exactly as int128.
 * sums: device int64[n_instances][K][2][2] = (C, C') x (low, high limb). */
int qdta_ls_eval(qdta_ctx *ctx, const qdta_opts *opts, const int64_t *f_fx, const int64_t *y_fx,
                 int32_t K, const double *alphas, int64_t *sums);

/* qdta_ls_eval for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same sums, bit for bit, with no hipMalloc, hipFree or allocating library
 * call.  Its scratch (error flags and the exact accumulators) is a static
 * array each device holds for the life of the process, looked up once per
 * device by qdta_create: at most n_instances x K = 4,096 (e.g. 64 instances
 * at K = 64); larger is QDTA_EARG.  The context must already be laid out on
 * the device (any earlier call that uses it, e.g. qdta_layout; QDTA_ESTATE
 * otherwise).  Every call on a device shares that device's scratch and keeps
 * the last call's contents (each call clears what it uses first): calls that
 * overlap on one device, on any streams or contexts, race.  Synchronises. */
int qdta_ls_eval_noalloc(qdta_ctx *ctx, const qdta_opts *opts, const int64_t *f_fx, const int64_t *y_fx,
                         int32_t K, const double *alphas, int64_t *sums);

/* A5 -- the step size of FW iteration j for every instance by opts->ls_mode
 * (K-section, quasi-Newton of Alg. 8, or MSA), alpha_out double[n_instances]
 * (device).  Synchronises. */
int qdta_line_search(qdta_ctx *ctx, const qdta_opts *opts, const int64_t *f_fx, const int64_t *y_fx,
                     int32_t j, double *alpha_out);

/* A6 -- link-flow update f <- f + rint(alpha_i (y - f)) with alpha of each
 * link's instance (device double[n_instances]). */
int qdta_fw_update(qdta_ctx *ctx, int64_t *f_fx, const int64_t *y_fx, const double *alpha);

/* A1-A7 -- Frank-Wolfe on the current demand of every instance (Alg. 6):
 * initial AON at free flow, then BPR, AON, stop test, line search, update,
 * until each instance's stop rule fires (its pre-update iterate is returned)
 * or the cap is reached.  host_stats: qdta_stats[n_instances] (host).
 * Synchronises once per FW iteration.  Returns the worst per-instance code. */
int qdta_solve(qdta_ctx *ctx, const qdta_opts *opts, qdta_stats *host_stats);

/* The same Frank-Wolfe loop one iteration at a time.  qdta_fw_begin resets
 * the state and runs the initial free-flow AON; each qdta_fw_step runs one
 * iteration (BPR, AON, stop test, line search, update) for every instance
 * whose stop rule has not fired, fills host_stats[n_instances] (host; may be
 * NULL) and sets *live_out (host) to 0 once every instance has stopped.
 * Synchronises once per call. */
int qdta_fw_begin(qdta_ctx *ctx, const qdta_opts *opts);
int qdta_fw_step(qdta_ctx *ctx, const qdta_opts *opts, qdta_stats *host_stats, int32_t *live_out);

/* Copies of the link flows (int64 fx) and costs BPR(f) (float) over all
 * links, device outputs, of the solved interval or, during qdta_fw_begin /
 * qdta_fw_step, of the current iterate. */
int qdta_get_flows(qdta_ctx *ctx, int64_t *f_fx);
int qdta_get_costs(qdta_ctx *ctx, const qdta_opts *opts, float *cost);

/* A8 -- residual demand after the solved interval (Alg. 4): every iterate's
 * paths (weights lambda_j = alpha_j prod_{k>j}(1 - alpha_k), alpha_0 = 1) are
 * re-truncated under the final costs BPR(f); a leg stopping at s != q leaves
 * rint(lambda_j d) as demand (s, q), merged into the next qdta_set_demand.
 * Needs opts->keep_history during qdta_solve.  With keep_history, the solve
 * keeps each iterate's shortest-path labels in device memory while it lasts
 * (sized at qdta_fw_begin from the free memory, leaving 16 GiB free, held
 * until the context is destroyed); this pass walks those and grows trees
 * again only for the iterates that did not fit.  Residual legs are kept in
 * (destination, origin) order.  Synchronises. */
int qdta_advance_interval(qdta_ctx *ctx, const qdta_opts *opts);

/* The pending residual demand of instance inst (host outputs).  Call with
 * NULL arrays to get *count; arrays then hold at least *count entries.
 * host_delay (may be NULL): each residual leg's delay (link-progress rule). */
int qdta_get_residual(qdta_ctx *ctx, int32_t inst, int64_t *count, int32_t *host_orig,
                      int32_t *host_dest, int64_t *host_w_fx, int64_t *host_done_fx, float *host_delay);

/* Resume (Alg. 1): the whole state carried from interval i to i+1 is the
 * residual demand d^r(i+1), so a day stopped after qdta_advance_interval and
 * qdta_get_residual continues, bit for bit, in another context on the same
 * network: qdta_set_residual replaces instance inst's pending residual with
 * count legs (host inputs, copied) in the order qdta_get_residual returns
 * them, strictly increasing by (destination, origin, delay), origin !=
 * destination, w_fx > 0, delays finite and >= 0 (host_delay NULL: all 0);
 * the next qdta_set_demand merges them as it merges its own.
 * count = 0 clears it.  Errors: QDTA_EARG (ids out of range, order, weights). */
int qdta_set_residual(qdta_ctx *ctx, int32_t inst, int64_t count, const int32_t *host_orig,
                      const int32_t *host_dest, const int64_t *host_w_fx, const float *host_delay);

/* ---- Derivatives for OD calibration (not in the paper) -------------------
 * The frozen-path model of a solved interval: its J applied Frank-Wolfe
 * updates are replayed with every iterate's trees and truncation frozen,
 * as a function of the demand d (veh per leg) and the capacities C:
 *     f = L_0 d;  for j = 1..J:  y_j = L_j d,  alpha_j = line search of
 *     (f, y_j) under C (Eq. 6, opts->ls_mode),  f += rint(alpha_j (y_j - f)),
 * where L_j loads each leg along its truncated path under iterate j's trees
 * (Eq. 2, Eq. 5).  At the solve's own demand and capacities it reproduces the
 * solve's flows bit for bit.  The reverse pass treats alpha_j as the root of
 * C'(alpha) = 0 (implicit-function theorem; a step at 0 or 1, or an MSA step,
 * has zero derivative) and the rounding as the identity.  One instance only.
 *
 * qdta_adjoint_record: after qdta_solve with opts->keep_history, walks every
 * leg under every iterate's trees (stored labels, else grown again from the
 * recorded costs) and keeps the paths in device memory (about 4 bytes per
 * loaded link per iterate).  Errors: QDTA_ESTATE (no solved interval, no
 * history, more than one instance, FP32 absorption on a path).
 * Synchronises. */
int qdta_adjoint_record(qdta_ctx *ctx, const qdta_opts *opts);

/* Forward pass of the model.  d: double[total_legs] (device), veh per leg in
 * the context's leg order (qdta_get_legs); cap: float[total_links] (device)
 * or NULL for the network's capacities; f_out: double[total_links] (device),
 * veh.  Keeps the iterates for qdta_model_backward and writes the id of this
 * forward pass to *fwd_id_out (host, may be NULL).  Errors: QDTA_ESTATE (no
 * record for the current solve), QDTA_EOVF (non-finite demand or costs).
 * Synchronises. */
int qdta_model_forward(qdta_ctx *ctx, const qdta_opts *opts, const double *d, const float *cap,
                       double *f_out, uint64_t *fwd_id_out);

/* Reverse pass of the forward pass fwd_id (the id qdta_model_forward
 * returned in *fwd_id_out; the context keeps the iterates of its last
 * forward pass only): given fbar = dL/df (double[total_links], device),
 * writes dbar = dL/dd (double[total_legs]) and capbar = dL/dC
 * (double[total_links]), device outputs.  Errors: QDTA_ESTATE when another
 * forward pass ran after fwd_id (its iterates are gone; run that forward
 * again).  Enqueued on the stream, no synchronisation. */
int qdta_model_backward(qdta_ctx *ctx, uint64_t fwd_id, const double *fbar, double *dbar, double *capbar);

/* Autotuner: times the shortest-path launch of the current demand (every
 * instance, under the costs BPR(f) of the running solve's iterate or of the
 * last solved one, free-flow costs otherwise; the running solve's next
 * qdta_fw_step recomputes whatever the trials overwrote) for a grid of
 * kernel shapes, bucket widths and
 * wavefronts per tree, stopping once about budget_ms of GPU time is spent,
 * and writes the fastest into opts->sssp_shape, opts->delta_scale and
 * opts->tree_waves.  The configuration passed in (zero fields read as the
 * defaults) is timed first, after one untimed launch, and is kept unless
 * another is at least 5% faster.  When opts->load_form is 0 and every
 * instance is plain (no truncation), the loading by per-leg walks and by
 * merged paths are timed on the same trees and opts->load_form becomes 2
 * if the merged paths are at least 5% faster, else 1.  Other fields are
 * unchanged.  Results never depend on these fields, only the speed does.
 * *best_ms_out (host, may be NULL) receives the shortest-path time of the
 * configuration chosen.  Synchronises. */
int qdta_autotune(qdta_ctx *ctx, qdta_opts *opts, double budget_ms, double *best_ms_out);

/* Per-phase timers: HIP events recorded on the context's stream around each
 * phase of the Frank-Wolfe iteration; durations are added at the iteration's
 * synchronisation.  Phases: 0 BPR costs, 1 shortest-path trees, 2 loading
 * walk (with the tie fallback), 3 gap sums and stop test, 4 line search,
 * 5 flow update, 6 a whole iteration replayed as a HIP graph (the phases
 * inside a graph are not timed separately), 7 the labels of the nodes the
 * chain-contracted search leaves out (filled after phase 1's search).  qdta_profile_enable(ctx, 1) resets and starts the timers,
 * 0 stops them; qdta_profile_read copies the totals (host output; synchronises).  The work
 * counters (sssp_nodes, sssp_links) add up over every shortest-path launch, graph replays
 * included, from the last qdta_profile_enable on. */
typedef struct {
    double ms[8];        /* summed duration per phase, milliseconds */
    int64_t count[8];    /* timed occurrences per phase */
    int64_t sssp_nodes;  /* nodes taken off the shortest-path queues since qdta_profile_enable (a node
                            taken twice counts twice; the one-wavefront-per-tree kernel does not count) */
    int64_t sssp_links;  /* in-links relaxed by them */
} qdta_profile;

int qdta_profile_enable(qdta_ctx *ctx, int32_t on);
int qdta_profile_read(qdta_ctx *ctx, qdta_profile *out);

#ifdef __cplusplus
}
#endif
#endif /* QDTA_H */
