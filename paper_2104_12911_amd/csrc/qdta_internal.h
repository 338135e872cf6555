// Private declarations shared by the library's kernels (qdta_kernels.hip)
// and its host runtime (qdta_runtime.cpp).  Not installed, not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qdta {

constexpr int kWG = 256;                 // threads per workgroup (4 wavefronts of 64)
constexpr int kChunk = 2048;             // links per workgroup in link-parallel kernels
constexpr uint32_t kInfBits = 0x7f800000u;
constexpr int kMaxK = 64;                // step sizes per line-search pass
// block-local shortest-path kernel: blocks per tree its LDS bitmap covers
// (instances up to kBlkMaxBits * block-size nodes)
constexpr int kBlkMaxBits = 8192;
// chain-contracted search: most nodes one chain holds (longer runs of
// two-neighbour nodes are cut by keeping a node)
constexpr int kChainMax = 8;
constexpr int kFillChunk = 1024;         // chains per work item of the fill after the contracted search
// A kept node's row of contracted records packed in one word, (first record
// << 6) | count, carried by the records that name the node as their source
// and by its queue entries so that a pop need not read the row pointers;
// kNoRow when the row does not fit (64 records or more, or a first record at
// 2^26 or beyond) or the record has no room for it.
constexpr uint32_t kNoRow = 0xffffffffu;
constexpr int kRowCountBits = 6;
__host__ __device__ inline uint32_t pack_row(int64_t e0, int64_t count) {
    return (count < (1 << kRowCountBits) && e0 < ((int64_t)1 << (32 - kRowCountBits)))
               ? (uint32_t)(e0 << kRowCountBits) | (uint32_t)count
               : kNoRow;
}
// allocation-free line search: 16 words of flags, then the exact accumulators
// (three 64-bit chunks per sum, two sums per step size) of up to 64 instances
// at K = 64
constexpr int kNoAllocFlagWords = 16;
constexpr int kNoAllocWords = kNoAllocFlagWords + 64 * kMaxK * 6;

// One shortest-path label word: (not-queued flag << 31) | FP32 bits of the
// distance.
typedef uint32_t label_t;

// Static description of one instance inside the concatenated layout.
struct InstDev {
    int32_t node0, n;        // first global node, node count
    int32_t link0, m;        // first global link, link count
    int32_t q0, nq;          // first global destination index, count
    int32_t leg0, nleg;      // first global leg, count
    int32_t rule;            // effective truncation rule (NONE when dt = inf)
    float dt32;              // interval length rounded to FP32
    double kappa;            // 3600/dt, or 1 for dt = inf
    double pq;               // link-progress rule: delays rounded up to multiples of this (0: exact)
};

// Per-instance Frank-Wolfe / line-search state, resident on the device.
struct InstState {
    int32_t active;          // instance has legs in this solve
    int32_t converged;       // stop rule fired or cap reached: f is final
    int32_t ls_done;         // line search finished for this iteration
    int32_t iter;            // FW iteration j being computed (1-based)
    int32_t stopped_by;      // 0 cap/fixed, 1 gap, 2 objective change, 3 stalled (alpha* = 0)
    int32_t ls_evals;        // passes over the links (accumulated)
    int32_t qn_iters;        // quasi-Newton iterations (accumulated)
    int32_t iters;           // updates applied
    int32_t ls_pass;         // passes in the current line search
    int32_t pad0;
    double gap;              // relative gap of the last test
    double alpha;            // step size chosen for this iteration
    double last_alpha;       // last applied step size
    double lo, hi;           // K-section bracket
    long long dlo[2], dhi[2];// C' at lo and hi (int128 limbs: low, high)
    double qn_alpha;         // quasi-Newton iterate
    double obj;              // objective (veh s) of the returned iterate
};

// Kernel arguments ---------------------------------------------------------

struct NetDev {
    const int32_t* row_ptr;  // [N+1] global forward CSR
    const int32_t* col;      // [M]   head (global node)
    const float* c0;         // [M]
    const float* cap;        // [M]
    const int32_t* rptr;     // [N+1] reverse CSR
    const int32_t* rsrc;     // [M]   tail (global node) of each in-link
    const int32_t* rlink;    // [M]   global link id of each in-link
    const int32_t* revpos;   // [M]   position of link a in the reverse arrays
    uint2* fadj;             // [M]   forward records (head, cost bits): the costs the trees are grown with
    const uint32_t* frow;    // [M]   the head's forward row packed as pack_row does (first link, count)
    const InstDev* inst;     // [ninst]
    // chain contraction (NULL until built): the search's reverse CSR over the
    // kept nodes, whose records are 4 words: source | form << 30, then the
    // cost bits in the order they are added, one for a plain link (form 0),
    // two or three for a chain of one or two nodes (forms 1, 2); form 3, a
    // longer chain, holds the word offset of its cost block (count, then the
    // costs) instead; cslot[a] is the word that holds link a's cost (-1 none)
    const int32_t* crptr;    // [N+1]
    uint32_t* cbuf;          // records, cost blocks, then the chains' fill blocks
    const int2* cslot;       // [M] (record word, fill word) holding link a's cost, -1 none
    const uint2* anc;        // [N] nodes whose labels must be final before the node's own is (itself if kept)
    const int32_t* inst_chain;// [ninst+1] chains of each instance
    // [C] chain headers (u, v, k, word offset in cbuf of the fill block), u
    // next to the chain's first node and v next to its last; the block holds
    // per chain node its id, the cost of its link toward v and of its link
    // toward u (+inf bits where the link is missing)
    const int4* ch_hdr;
    int32_t fill_chunks;     // most chunks of kFillChunk chains in one instance
    const int32_t* blk_inst; // [nblk] instance of each link chunk
    const int32_t* blk_start;// [nblk] first global link of each chunk
    int32_t ninst, nblk;
    int64_t N, M;
    int32_t objective;       // 0 user equilibrium (BPR costs route, Beckmann objective, Eq. 6);
                             // 1 system optimum (marginal costs route, total travel time)
};

struct DemDev {
    const int32_t* dest_node;// [Q] global node of each destination
    const int32_t* dest_inst;// [Q]
    const int64_t* dest_lab; // [Q] offset in labels of the tree's label of node 0 (a multiple of 32)
    const int32_t* qptr;     // [Q+1] legs of each destination (global leg index)
    const int32_t* leg_orig; // [P] global origin node
    const int64_t* leg_dfx;  // [P]
    const int32_t* leg_q;    // [P] global destination index
    const float* leg_delay;  // [P] time a leg still needs to reach its origin node (link-progress rule), or NULL
    int32_t Q, P;
};

// Per-wavefront scratch of the shortest-path kernel (also the workgroup
// scratch of the tie fallback, slot = workgroup there).
struct Scratch {
    // near queue (ring of n + 1) and far queue of each slot: nmax entries of
    // the node (1 word; contracted search: the node and its packed row, 2
    // words) and of (node, label) (2 words; contracted search: node, label,
    // packed row and a pad word, 4 words)
    int32_t* nearq;
    int32_t* farq;
    int64_t nmax;            // >= largest n + 65
    int32_t* work;           // tree work counter
    int32_t nslots;          // slots allocated (a launch is clamped to them)
    unsigned long long* stats; // [2] nodes taken and in-links relaxed, added up by the kernels
};

struct FlagsDev {
    int* err_overflow;       // set on non-finite cost / exact-sum overflow
    int* err_unreach;        // set when a leg's origin cannot reach its destination
    int* absorb_count;       // legs interrupted by FP32 absorption
    int32_t* absorb_q;       // [Q] destination flagged for the tie fallback
    int32_t* int_node;       // [P] node where an interrupted leg stopped (-1 none)
    float* int_tau;          // [P] its elapsed time there
};

// Launchers (qdta_kernels.hip) ---------------------------------------------

hipError_t launch_fill_u32(hipStream_t s, uint32_t* p, uint32_t v, int64_t count);
hipError_t launch_fill_i64(hipStream_t s, int64_t* p, int64_t v, int64_t count);

// cost: the routing costs (marginal ones under net.objective = 1); tcost (may
// be NULL): the travel times BPR(f) as well
hipError_t launch_bpr(hipStream_t s, const NetDev& net, const int64_t* f, double alpha, int beta,
                      float* cost, uint2* radj, const InstState* st, int only_active, int* err,
                      float* tcost = nullptr);

hipError_t launch_gap_sums(hipStream_t s, const NetDev& net, const float* cost, const int64_t* f,
                           const int64_t* y, long long* acc /*[ninst][2][3]*/, const InstState* st, int* err);

hipError_t launch_gap_decide(hipStream_t s, int ninst, const long long* acc, InstState* st, int stop_rule,
                             double tol, int fixed_iters, int cap_iter);

hipError_t launch_ls_begin(hipStream_t s, int ninst, InstState* st, double* alphas, int K, int ls_mode,
                           double dx, long long* ls_acc, int only_fallback);

hipError_t launch_ls_eval(hipStream_t s, const NetDev& net, const int64_t* f, const int64_t* y,
                          double alpha_b, int beta, int K, const double* alphas, long long* ls_acc,
                          const InstState* st, int only_pending, int* err, int k0 = 0, int kstride = 0);

hipError_t launch_ls_decide(hipStream_t s, int ninst, InstState* st, double* alphas, int K, int ls_mode,
                            int passes, int max_ls, double T1, double T2, double dx, long long* ls_acc);

hipError_t launch_stall_check(hipStream_t s, int ninst, InstState* st, int fixed_iters);
hipError_t launch_ls_export(hipStream_t s, int ninst, const long long* ls_acc, int K, int64_t* sums);
// device address of the static scratch of the allocation-free line search on
// `device` (which must be current); looked up once per device
hipError_t noalloc_scratch(int device, long long** out);

hipError_t launch_obj_pair(hipStream_t s, const NetDev& net, const int64_t* f, const int64_t* y,
                           double alpha_b, int beta, long long* acc /*[ninst][2][3]*/, const InstState* st,
                           int use_alpha, int* err);

hipError_t launch_obj_decide(hipStream_t s, int ninst, const long long* acc, InstState* st, double tol,
                             int apply_rule);

hipError_t launch_fw_update(hipStream_t s, const NetDev& net, int64_t* f, const int64_t* y,
                            const double* alpha_per_inst, const InstState* st);

hipError_t launch_copy_alpha(hipStream_t s, int ninst, const InstState* st, double* out);
hipError_t launch_after_update(hipStream_t s, int ninst, InstState* st);
hipError_t launch_scatter_rcost(hipStream_t s, const NetDev& net, const float* cost, uint2* radj);
// contracted records' costs from the forward link records (after a rebuild)
hipError_t launch_cslot_init(hipStream_t s, const NetDev& net);

hipError_t launch_delta(hipStream_t s, const NetDev& net, const float* cost, double delta_scale, float* delta_inst,
                        double* logsum);
// The contracted search's trees (variant >= 32) are complete only after
// launch_chain_fill of the same trees; fill = true launches it right after.
hipError_t launch_trees(hipStream_t s, const NetDev& net, const DemDev& dem, const uint2* radj, label_t* labels,
                        const Scratch& scr, int slots, const InstState* st, const float* delta_inst, int variant,
                        int early, int t_begin, int t_end, bool fill = true);
hipError_t launch_sssp(hipStream_t s, const NetDev& net, const DemDev& dem, const float* cost, const uint2* radj,
                       label_t* labels, const Scratch& scr, int slots, const InstState* st, double delta_scale,
                       float* delta_inst, double* logsum, int variant, int early, bool fill = true);
hipError_t launch_chain_fill(hipStream_t s, const NetDev& net, const DemDev& dem, label_t* labels,
                             const InstState* st, int t_begin, int t_end);

// time_cost NULL: the trees' own costs (held in the forward records)
// Legs the link-progress rule leaves on a link (residual mode): appended as
// (destination index, node, delay, weight) while fewer than cap are held.
struct TransitOut {
    int32_t* q;
    int32_t* node;
    float* delay;
    int64_t* w;
    unsigned int* n;         // entries appended (may pass cap: then QDTA_EOVF)
    unsigned int cap;
};

hipError_t launch_walk(hipStream_t s, const NetDev& net, const DemDev& dem, const label_t* labels,
                       const float* time_cost, int64_t* y, int32_t* stop,
                       const InstState* st, const FlagsDev& fl, int residual_mode, const double* lambda,
                       int64_t* r_dense,
                       unsigned long long* done_fx, int l_begin = 0, int l_end = -1, float* stop_delay = nullptr,
                       const TransitOut* tr = nullptr);

// plain-interval loading by children-before-parent accumulation (see the
// kernels); cnt and acc: scratch indexed like the labels, all zero before and
// after; every instance must be plain (no truncation)
hipError_t launch_sweep(hipStream_t s, const NetDev& net, const DemDev& dem, const label_t* labels,
                        int64_t* y, int32_t* stop, float* stop_delay, const InstState* st, const FlagsDev& fl,
                        uint32_t* cnt, int64_t* acc);

hipError_t launch_fallback(hipStream_t s, const NetDev& net, const DemDev& dem, const label_t* labels,
                           const float* tree_cost, const float* time_cost, int64_t* y, int32_t* stop,
                           const InstState* st, const FlagsDev& fl, const Scratch& scr, int slots,
                           int residual_mode, const double* lambda, int64_t* r_dense,
                           unsigned long long* done_fx,
                           int trees_mode, int32_t* succ_out, int32_t n_out, float* stop_delay = nullptr,
                           const TransitOut* tr = nullptr);

// residual accumulator (indexed like the labels) -> legs in (destination, origin) order
hipError_t launch_resid_count(hipStream_t s, const NetDev& net, const DemDev& dem, const int64_t* r_dense,
                              int64_t* cnt);
hipError_t launch_resid_write(hipStream_t s, const NetDev& net, const DemDev& dem, int64_t* r_dense,
                              const int64_t* off, int32_t* r_orig, int32_t* r_q, int64_t* r_w);

hipError_t launch_trees_out(hipStream_t s, const NetDev& net, const DemDev& dem, const label_t* labels,
                            const float* cost_local, int32_t inst, float* dist, int32_t* succ,
                            int32_t* absorb_q);

// frozen-path model and its reverse pass (OD calibration)
hipError_t launch_path_walk(hipStream_t s, const NetDev& net, const DemDev& dem, const label_t* labels,
                            const int64_t* ptr, int32_t* links, int32_t* leg_of, int64_t* len, int* bad);
hipError_t launch_path_load(hipStream_t s, int64_t total, const int32_t* links, const int32_t* leg_of,
                            const double* d, int64_t* y, int* err);
hipError_t launch_path_gather(hipStream_t s, int P, const int64_t* ptr, const int32_t* links, const double* g,
                              double* dbar, int accumulate);
hipError_t launch_adj_step(hipStream_t s, const NetDev& net, const int64_t* f, const int64_t* y,
                           const double* alpha, int is_root, double ab, int beta, double* fbar, double* ybar,
                           double* capbar, double* part /*[2 x 1024]*/, double* sbuf);
hipError_t launch_fx_to_veh(hipStream_t s, int64_t M, const int64_t* f, double* out);

}  // namespace qdta
