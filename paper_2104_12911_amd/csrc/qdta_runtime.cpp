// qdta_runtime.cpp -- host side of the QDTA library: argument validation,
// the concatenated device layout of all instances, the Frank-Wolfe driver
// (Alg. 6), the residual-demand step (Alg. 4) and the C ABI of qdta.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "qdta.h"
#include "qdta_internal.h"

using namespace qdta;

namespace {

struct Instance {
    int32_t n = 0, m = 0;
    std::vector<int32_t> row_ptr, col;
    std::vector<float> fftt, cap;
    // merged demand of the current interval, sorted by (dest, orig)
    bool has_demand = false;
    double dt_s = INFINITY;
    std::vector<int32_t> orig, dest;
    std::vector<int64_t> dfx;
    std::vector<float> delay;            // time each leg still needs to reach its origin (link-progress rule)
    // residual carried into the next interval (Alg. 4 output)
    std::vector<int32_t> r_orig, r_dest;
    std::vector<int64_t> r_w;
    std::vector<float> r_delay;
    int64_t r_done = 0;
    // per-iteration step sizes of the last solve (alpha_0 = 1)
    std::vector<double> hist_alpha;
    int32_t solved_iters = -1;
};

template <class T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
};

}  // namespace

struct qdta_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int cus = 256;
    std::vector<Instance> inst;
    bool net_dirty = true, dem_dirty = true;
    std::vector<void*> allocs;    // buffers this context got from hipMalloc
    int64_t n_hip_malloc = 0;     // hipMalloc calls made (qdta_alloc_count)
    // caller-owned workspace (qdta_bind_workspace): while one is bound, every
    // device buffer is carved from it and hipMalloc is never called
    char* ws_base = nullptr;
    size_t ws_size = 0;
    std::map<size_t, size_t> ws_free;   // offset -> length of each free run (coalesced)
    std::map<size_t, size_t> ws_used;   // offset -> length of each carved buffer
    int64_t ws_max_legs = 0, ws_max_dests = 0;  // maxima the workspace was sized for
    long long* noalloc = nullptr; // device address of the allocation-free line search's static scratch

    // network layout
    int64_t N = 0, M = 0;
    int nblk = 0;
    std::vector<InstDev> h_inst;
    std::vector<int64_t> node_off, link_off, leg_off, dest_off;
    DBuf<int32_t> row_ptr, col, rptr, rsrc, rlink, revpos, blk_inst, blk_start;
    DBuf<float> c0, cap;
    DBuf<InstDev> d_inst;

    // demand layout
    int64_t Q = 0, P = 0, nmax = 0;
    int slots = 0, scr_slots = 0;
    int64_t scr_nmax = 0;
    bool scr_wide = false;             // queues sized for the contracted search's entries
    size_t label_count = 0;
    DBuf<int32_t> dest_node, dest_inst, qptr, leg_orig, leg_q;
    DBuf<int64_t> dest_lab, leg_dfx;
    DBuf<float> leg_delay;
    // legs the link-progress rule leaves on a link during the residual pass
    DBuf<int32_t> tr_q, tr_node;
    DBuf<float> tr_delay;
    DBuf<int64_t> tr_w;
    DBuf<unsigned int> tr_n;
    std::vector<int32_t> h_dest_inst, h_dest_node, h_qptr;
    DBuf<label_t> labels;         // 32-bit label words, tree-major, each tree 128-byte aligned
    DBuf<int32_t> nearq, farq;

    DBuf<int32_t> work;
    DBuf<uint32_t> sw_cnt;            // plain-interval loading: arrival counts and accumulators,
    DBuf<int64_t> sw_acc;             // indexed like the labels, zero between launches
    DBuf<unsigned long long> sssp_stats;  // nodes taken, in-links relaxed (reset by qdta_profile_enable)
    DBuf<float> delta_inst;
    DBuf<double> logsum;

    // chain contraction of the search (opts.sssp_kernel = 4), built for the
    // roots (destinations) seen so far
    std::vector<uint8_t> croot, cleft;   // nodes kept as roots; nodes the search leaves out
    bool c_built = false;
    int64_t c_chains = 0, c_left = 0;
    DBuf<int32_t> crptr, inst_chain;
    DBuf<int4> ch_hdr;
    DBuf<uint32_t> cbuf;
    DBuf<uint2> anc;
    DBuf<int2> cslot;
    int32_t c_fill_chunks = 0;         // most chain chunks of one instance (k_chain_fill items)

    // Frank-Wolfe state
    DBuf<int64_t> f, y;
    DBuf<float> cost, cfin, tcost;    // routing costs, final times, travel times (system optimum)
    DBuf<uint2> radj;             // reverse adjacency records (source node, cost)
    DBuf<uint2> fadj;             // forward link records (head node, cost)
    DBuf<uint32_t> frow;          // per link its head's forward row, packed (pack_row)
    DBuf<InstState> st;
    DBuf<long long> acc, ls_acc;
    DBuf<double> alphas, alpha_arr;
    DBuf<int> flags;              // [0] overflow, [1] unreach, [2] absorb count, [3] path-record faults
    DBuf<int32_t> absorb_q, int_node;
    DBuf<float> int_tau;
    DBuf<float> hist_cost;
    size_t hist_iters_cap = 0;
    // residual output
    DBuf<int32_t> r_orig, r_dest;
    DBuf<int64_t> r_w, r_dense, r_cnt;
    size_t r_dense_zero = 0;      // leading accumulator words known to be zero
    DBuf<InstState> st_hist;      // per-iterate instance state of a residual pass
    // labels of the solve's iterates, kept while device memory allows, so the
    // residual pass walks them instead of growing the trees again
    DBuf<label_t> lab_hist;
    std::vector<char> lab_hist_ok;  // iterate j's labels are at lab_hist + j * label_count
    DBuf<double> lam_hist;
    DBuf<unsigned long long> done_fx;
    uint64_t gen = 0;             // bumped on every (re)allocation and every rebuild of the
                                  // network or demand tables: a captured iteration is valid
                                  // only for the generation it was captured in
    // captured FW iteration
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    uint64_t graph_gen = 0;
    qdta_opts graph_opts;
    InstState* h_st = nullptr;    // pinned mirror
    int h_st_n = 0;
    bool solved = false;
    int fw_j = -1;                // FW iteration of the running solve (-1: none)
    bool fw_live = false;
    uint64_t solve_id = 0;        // bumped by every qdta_fw_begin
    // frozen-path model (OD calibration): each leg's truncated path under
    // every iterate's trees, and the states of the last model forward pass
    int adj_J = -1;
    uint64_t adj_gen = 0, adj_solve = 0;
    bool adj_fwd = false;
    uint64_t adj_fwd_id = 0;      // bumped by every model forward; a backward names the one it reverses
    int adj_is_root = 1, adj_beta = 4;
    double adj_ab = 0.15;
    std::vector<DBuf<int64_t>> adj_ptr;   // [J+1] offsets of each leg's path
    std::vector<DBuf<int32_t>> adj_links; // [J+1] link ids in walk order
    std::vector<DBuf<int32_t>> adj_leg;   // [J+1] the leg of each entry
    std::vector<int64_t> adj_total;       // [J+1] entries per iterate
    DBuf<int64_t> adj_len, adj_f, adj_y, adj_cur;
    DBuf<double> adj_alpha, adj_fbar, adj_ybar, adj_part, adj_s;
    DBuf<float> adj_cap;
    // per-phase HIP-event timers (qdta_profile_enable)
    int prof_on = 0;
    hipEvent_t prof_ev[8][2] = {};
    int prof_open[8] = {};
    double prof_ms[8] = {};
    int64_t prof_n[8] = {};
};

namespace {

void drop_graph(qdta_ctx* c);

int set_err(qdta_ctx* c, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    c->err = buf;
    return code;
}

#define RC0(x)                  \
    do {                        \
        int rc0_ = (x);         \
        if (rc0_ < 0) return rc0_; \
    } while (0)

#define HIPCHECK(ctx, expr)                                                                          \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) return set_err(ctx, QDTA_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

void evict_label_history(qdta_ctx* c);

// Device memory: from the bound workspace (first fit over its free runs),
// else from hipMalloc.
int dev_alloc(qdta_ctx* c, size_t bytes, void** out) {
    *out = nullptr;
    bytes = align_up(std::max<size_t>(bytes, 1));
    if (c->ws_base) {
        for (auto it = c->ws_free.begin(); it != c->ws_free.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, len = it->second;
            c->ws_free.erase(it);
            if (len > bytes) c->ws_free[off + bytes] = len - bytes;
            c->ws_used[off] = bytes;
            *out = c->ws_base + off;
            return QDTA_OK;
        }
        size_t largest = 0;
        for (const auto& r : c->ws_free) largest = std::max(largest, r.second);
        return set_err(c, QDTA_ENOMEM, "workspace too small: a buffer of %zu bytes does not fit (largest free run %zu "
                       "of %zu bytes); query again and bind a larger workspace", bytes, largest, c->ws_size);
    }
    hipError_t e = hipMalloc(out, bytes);
    c->n_hip_malloc++;
    if (e != hipSuccess && c->lab_hist.p) {
        // the label history only saves the residual pass from growing the
        // trees again, and it was sized from the free memory: give it back
        // (the pass then grows them) and try once more
        (void)hipGetLastError();
        evict_label_history(c);
        e = hipMalloc(out, bytes);
        c->n_hip_malloc++;
    }
    if (e != hipSuccess) {
        *out = nullptr;
        (void)hipGetLastError();
        return set_err(c, QDTA_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    c->allocs.push_back(*out);
    return QDTA_OK;
}

void dev_free(qdta_ctx* c, void* p) {
    if (!p) return;
    if (c->ws_base) {
        auto u = c->ws_used.find((size_t)((char*)p - c->ws_base));
        if (u == c->ws_used.end()) return;
        size_t off = u->first, len = u->second;
        c->ws_used.erase(u);
        auto nx = c->ws_free.lower_bound(off);
        if (nx != c->ws_free.end() && nx->first == off + len) {   // merge with the next run
            len += nx->second;
            nx = c->ws_free.erase(nx);
        }
        if (nx != c->ws_free.begin()) {                            // and the previous one
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += len;
                return;
            }
        }
        c->ws_free[off] = len;
        return;
    }
    (void)hipFree(p);
    auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
    if (it != c->allocs.end()) c->allocs.erase(it);
}

template <class T>
void dfree(qdta_ctx* c, DBuf<T>& b) {
    dev_free(c, (void*)b.p);
    b.p = nullptr;
    b.n = 0;
}

void evict_label_history(qdta_ctx* c) {
    (void)hipStreamSynchronize(c->stream);   // work queued on it may still read the history
    dfree(c, c->lab_hist);
    c->lab_hist_ok.clear();
    c->gen++;                        // a captured iteration may copy labels into it
}

template <class T>
int dalloc(qdta_ctx* c, DBuf<T>& b, size_t n) {
    if (b.p && b.n >= n && n > 0) return QDTA_OK;
    if (b.p) dfree(c, b);
    void* p = nullptr;
    RC0(dev_alloc(c, std::max<size_t>(n, 1) * sizeof(T), &p));
    b.p = (T*)p;
    b.n = std::max<size_t>(n, 1);
    c->gen++;
    return QDTA_OK;
}

// With a workspace bound, buffers sized by the demand are carved at the
// maxima the workspace was sized for (qdta_workspace_query), so later
// intervals reuse them instead of carving again.
size_t plan_legs(const qdta_ctx* c, size_t n) { return c->ws_base ? std::max<size_t>(n, (size_t)c->ws_max_legs) : n; }
size_t plan_dests(const qdta_ctx* c, size_t n) { return c->ws_base ? std::max<size_t>(n, (size_t)c->ws_max_dests) : n; }

template <class T>
int upload(qdta_ctx* c, DBuf<T>& b, const std::vector<T>& h, size_t min_n = 0) {
    int rc = dalloc(c, b, std::max(h.size(), min_n));
    if (rc) return rc;
    if (!h.empty()) HIPCHECK(c, hipMemcpyAsync(b.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
    return QDTA_OK;
}

#define RC(x)                  \
    do {                       \
        int rc_ = (x);         \
        if (rc_ < 0) return rc_; \
    } while (0)

bool opts_ok(qdta_ctx* c, const qdta_opts* o) {
    if (!o) { set_err(c, QDTA_EARG, "opts is NULL"); return false; }
    if (!(o->alpha >= 0.0 && std::isfinite(o->alpha))) { set_err(c, QDTA_EARG, "alpha must be finite and >= 0"); return false; }
    if (o->beta < 1 || o->beta > 16) { set_err(c, QDTA_EARG, "beta must be in 1..16"); return false; }
    if (o->trunc_rule < 0 || o->trunc_rule > 3) { set_err(c, QDTA_EARG, "bad trunc_rule"); return false; }
    if (o->ls_mode < 0 || o->ls_mode > 2) { set_err(c, QDTA_EARG, "bad ls_mode"); return false; }
    if (o->K < 3 || o->K > kMaxK) { set_err(c, QDTA_EARG, "K must be in 3..64"); return false; }
    if (o->passes < 1 || o->passes > 8) { set_err(c, QDTA_EARG, "passes must be in 1..8"); return false; }
    if (o->max_ls < 1 || o->max_ls > 100) { set_err(c, QDTA_EARG, "max_ls must be in 1..100"); return false; }
    if (o->stop_rule < 0 || o->stop_rule > 1) { set_err(c, QDTA_EARG, "bad stop_rule"); return false; }
    if (!(o->tol >= 0.0) || !(o->dx > 0.0) || !(o->T1 >= 0.0) || !(o->T2 >= 0.0)) {
        set_err(c, QDTA_EARG, "tol, T1, T2 must be >= 0 and dx > 0");
        return false;
    }
    if (o->max_iter < 0 || o->fixed_iters < 0) { set_err(c, QDTA_EARG, "negative iteration count"); return false; }
    if (o->waves_per_cu < 0 || o->waves_per_cu > 32) { set_err(c, QDTA_EARG, "waves_per_cu must be in 0..32"); return false; }
    if (o->sssp_shape < 0 || o->sssp_shape > 6) { set_err(c, QDTA_EARG, "sssp_shape must be in 0..6"); return false; }
    if (o->sssp_kernel < 0 || o->sssp_kernel > 4) { set_err(c, QDTA_EARG, "sssp_kernel must be 0..4"); return false; }
    if (o->load_form < 0 || o->load_form > 2) { set_err(c, QDTA_EARG, "load_form must be 0, 1 or 2"); return false; }
    if (o->launch_form < 0 || o->launch_form > 2) { set_err(c, QDTA_EARG, "launch_form must be 0, 1 or 2"); return false; }
    if (o->tree_waves != 0 && o->tree_waves != 1 && o->tree_waves != 4) {
        set_err(c, QDTA_EARG, "tree_waves must be 0, 1 or 4");
        return false;
    }
    if (!(o->progress_quantum_s >= 0.0) || !std::isfinite(o->progress_quantum_s)) {
        set_err(c, QDTA_EARG, "progress_quantum_s must be finite and >= 0");
        return false;
    }
    if (!(o->delta_scale >= 0.0) || !std::isfinite(o->delta_scale)) {
        set_err(c, QDTA_EARG, "delta_scale must be finite and >= 0");
        return false;
    }
    if (o->objective != QDTA_OBJ_UE && o->objective != QDTA_OBJ_SO) {
        set_err(c, QDTA_EARG, "objective must be QDTA_OBJ_UE or QDTA_OBJ_SO");
        return false;
    }
    return true;
}

// wavefronts per tree: one only for the node-queue kernel asked to run one
// tree per wavefront; the block-local kernel always takes a workgroup
int tree_waves(const qdta_opts* o) { return (o->sssp_kernel < 2 && o->tree_waves == 1) ? 1 : 4; }
// FW updates a solve may apply (iterates 1..this, plus the initial AON)
int hist_iters(const qdta_opts* o) { return o->fixed_iters > 0 ? o->fixed_iters : std::max(o->max_iter, 0); }
bool uses_contraction(const qdta_opts* o);
// wavefronts in flight per CU by default: what the kernels' registers allow
// (one tree per wavefront: 32; the contracted <2, 4> form: 28; else 24)
int waves_per_cu(const qdta_opts* o) {
    if (o->waves_per_cu) return o->waves_per_cu;
    return tree_waves(o) == 1 ? 32 : uses_contraction(o) ? 28 : 24;
}
double delta_scale(const qdta_opts* o) { return o->delta_scale > 0.0 ? o->delta_scale : 10.0; }
// Block size of each block-local shape (qdta_opts.sssp_shape 1..4)
int blk_nodes(int shape) { return shape == 3 ? 64 : shape == 4 ? 256 : 128; }
// the chain-contracted search runs for kernel 4, and by default (kernel 0)
// unless one wavefront per tree was asked for
bool uses_contraction(const qdta_opts* o) {
    return o->sssp_kernel == 4 || (o->sssp_kernel == 0 && o->tree_waves != 1);
}

// Shortest-path kernel variant (see qdta_opts.sssp_kernel / sssp_shape).
// Variants 0-5: node queue, one wavefront per tree; 8-13: node queue, one
// workgroup per tree; 16-19: block-local, one workgroup per tree; 24-27:
// node-per-thread queue; 32-37: the node queue over the chain-contracted
// search (shapes as 8-13).  The
// block-local kernel needs every instance within its block bitmap.
int sssp_variant(const qdta_ctx* c, const qdta_opts* o) {
    int64_t nmax = 0;
    for (const Instance& I : c->inst) nmax = std::max<int64_t>(nmax, I.n);
    const bool fits = nmax <= (int64_t)kBlkMaxBits * blk_nodes(o->sssp_shape);
    if (o->sssp_kernel == 2 && fits) {
        const int v = (o->sssp_shape >= 1 && o->sssp_shape <= 4) ? o->sssp_shape - 1 : 1;
        return 16 + v;
    }
    if (o->sssp_kernel == 3) {
        const int v = (o->sssp_shape >= 1 && o->sssp_shape <= 4) ? o->sssp_shape - 1 : 1;
        return 24 + v;
    }
    const int v = (o->sssp_shape >= 1 && o->sssp_shape <= 6) ? o->sssp_shape - 1 : 2;
    if (uses_contraction(o)) return 32 + v;
    return tree_waves(o) == 1 ? v : v + 8;
}

// ---------------------------------------------------------------------------
// network layout: instances concatenated, reverse CSR, link chunks
// ---------------------------------------------------------------------------
int ensure_network(qdta_ctx* c) {
    if (!c->net_dirty) return QDTA_OK;
    if (c->inst.empty()) return set_err(c, QDTA_ESTATE, "no network added");
    int ni = (int)c->inst.size();
    c->node_off.assign(ni + 1, 0);
    c->link_off.assign(ni + 1, 0);
    for (int i = 0; i < ni; ++i) {
        c->node_off[i + 1] = c->node_off[i] + c->inst[i].n;
        c->link_off[i + 1] = c->link_off[i] + c->inst[i].m;
    }
    c->N = c->node_off[ni];
    c->M = c->link_off[ni];
    if (c->N >= INT32_MAX || c->M >= INT32_MAX) return set_err(c, QDTA_EARG, "total size beyond int32 ids");
    std::vector<int32_t> rp(c->N + 1), col(c->M), rptr(c->N + 1, 0), rsrc(c->M), rlink(c->M), revpos(c->M);
    std::vector<float> c0(c->M), cap(c->M);
    std::vector<int32_t> bi, bs;
    for (int i = 0; i < ni; ++i) {
        const Instance& I = c->inst[i];
        int32_t n0 = (int32_t)c->node_off[i], l0 = (int32_t)c->link_off[i];
        for (int v = 0; v < I.n; ++v) rp[n0 + v] = l0 + I.row_ptr[v];
        for (int a = 0; a < I.m; ++a) {
            col[l0 + a] = n0 + I.col[a];
            c0[l0 + a] = I.fftt[a];
            cap[l0 + a] = I.cap[a];
        }
        for (int a0 = 0; a0 < I.m; a0 += kChunk) {
            bi.push_back(i);
            bs.push_back(l0 + a0);
        }
    }
    rp[c->N] = (int32_t)c->M;
    // reverse CSR (in-links of each node), link ids ascending within a node
    std::vector<int32_t> tail(c->M);
    for (int64_t v = 0; v < c->N; ++v)
        for (int32_t a = rp[v]; a < rp[v + 1]; ++a) tail[a] = (int32_t)v;
    for (int64_t a = 0; a < c->M; ++a) rptr[col[a] + 1]++;
    for (int64_t v = 0; v < c->N; ++v) rptr[v + 1] += rptr[v];
    std::vector<int32_t> fill(rptr.begin(), rptr.end() - 1);
    for (int64_t a = 0; a < c->M; ++a) {
        int32_t pos = fill[col[a]]++;
        rsrc[pos] = tail[a];
        rlink[pos] = (int32_t)a;
        revpos[a] = pos;
    }
    c->h_inst.assign(ni, InstDev{});
    for (int i = 0; i < ni; ++i) {
        InstDev& d = c->h_inst[i];
        d.node0 = (int32_t)c->node_off[i];
        d.n = c->inst[i].n;
        d.link0 = (int32_t)c->link_off[i];
        d.m = c->inst[i].m;
        d.rule = QDTA_RULE_NONE;
        d.dt32 = INFINITY;
        d.kappa = 1.0;
    }
    c->nblk = (int)bi.size();
    RC(upload(c, c->row_ptr, rp));
    RC(upload(c, c->col, col));
    RC(upload(c, c->c0, c0));
    RC(upload(c, c->cap, cap));
    RC(upload(c, c->rptr, rptr));
    RC(upload(c, c->rsrc, rsrc));
    RC(upload(c, c->rlink, rlink));
    RC(upload(c, c->revpos, revpos));
    RC(upload(c, c->blk_inst, bi));
    RC(upload(c, c->blk_start, bs));
    RC(upload(c, c->d_inst, c->h_inst));
    RC(dalloc(c, c->f, c->M));
    RC(dalloc(c, c->y, c->M));
    RC(dalloc(c, c->cost, c->M));
    {
        std::vector<uint2> ra(c->M), fa(c->M);
        std::vector<uint32_t> fr(c->M);
        for (int64_t k = 0; k < c->M; ++k) {
            ra[k] = make_uint2((uint32_t)rsrc[k], 0u);
            fa[k] = make_uint2((uint32_t)col[k], 0u);
            fr[k] = pack_row(rp[col[k]], rp[col[k] + 1] - rp[col[k]]);
        }
        RC(upload(c, c->radj, ra));
        RC(upload(c, c->fadj, fa));
        RC(upload(c, c->frow, fr));
    }
    RC(dalloc(c, c->cfin, c->M));
    RC(dalloc(c, c->tcost, c->M));
    RC(dalloc(c, c->st, ni));
    RC(dalloc(c, c->acc, (size_t)ni * 6));
    RC(dalloc(c, c->ls_acc, (size_t)ni * kMaxK * 6));
    RC(dalloc(c, c->alphas, (size_t)ni * kMaxK));
    RC(dalloc(c, c->alpha_arr, ni));
    RC(dalloc(c, c->flags, 4));
    RC(dalloc(c, c->done_fx, ni));
    if (c->h_st_n < ni) {
        if (c->h_st) (void)hipHostFree(c->h_st);
        HIPCHECK(c, hipHostMalloc((void**)&c->h_st, sizeof(InstState) * ni, hipHostMallocDefault));
        c->h_st_n = ni;
    }
    c->net_dirty = false;
    c->dem_dirty = true;
    c->c_built = false;                // the contraction is rebuilt for the new layout
    c->croot.clear();
    c->gen++;                          // sizes baked into a captured iteration are stale
    return QDTA_OK;
}

// o (may be NULL): the solve options, whose objective selects the routing
// costs and the objective terms; NULL = user equilibrium (travel times).
NetDev net_view(qdta_ctx* c, const qdta_opts* o = nullptr) {
    NetDev v;
    v.objective = o ? o->objective : 0;
    v.row_ptr = c->row_ptr.p;
    v.col = c->col.p;
    v.c0 = c->c0.p;
    v.cap = c->cap.p;
    v.rptr = c->rptr.p;
    v.rsrc = c->rsrc.p;
    v.rlink = c->rlink.p;
    v.revpos = c->revpos.p;
    v.fadj = c->fadj.p;
    v.frow = c->frow.p;
    v.inst = c->d_inst.p;
    const bool ct = c->c_built;
    v.crptr = ct ? c->crptr.p : nullptr;
    v.cbuf = ct ? c->cbuf.p : nullptr;
    v.cslot = ct ? c->cslot.p : nullptr;
    v.anc = ct ? c->anc.p : nullptr;
    v.inst_chain = ct ? c->inst_chain.p : nullptr;
    v.ch_hdr = ct ? c->ch_hdr.p : nullptr;
    v.fill_chunks = ct ? c->c_fill_chunks : 0;
    v.blk_inst = c->blk_inst.p;
    v.blk_start = c->blk_start.p;
    v.ninst = (int32_t)c->inst.size();
    v.nblk = c->nblk;
    v.N = c->N;
    v.M = c->M;
    return v;
}

// ---------------------------------------------------------------------------
// chain contraction of the shortest-path search (opts.sssp_kernel = 4)
// ---------------------------------------------------------------------------
// A node is left out of the search when it is no root (destination) of any
// tree, has exactly two distinct neighbours (links taken both ways), one or
// two links in and out, no parallel links and no self-loop.  A run x1..xk of
// such nodes (k <= kChainMax; longer runs keep every (kChainMax+1)-th node)
// between kept nodes u (next to x1) and v (next to xk) is a chain.  When every
// link u->x1->...->xk->v exists, the search holds one record at v with source
// u whose cost list is c(xk->v), ..., c(x1->x2), c(u->x1): the candidate label
// of u is v's label plus each cost in turn, rounded to FP32 after each
// addition, which is what the same relaxations link by link would give; the
// same for v->xk->...->x1->u at u.  After a tree's search, each chain node's
// label is the lesser of the two folds from the ends' labels (see the kernel).
// Records are 4 words: (source | form << 30, then up to three costs in the
// order they are added).  Form 0 is a plain link (one cost), forms 1 and 2 a
// chain of one or two nodes (two or three costs inline), form 3 a longer
// chain, whose second word is the offset of its cost block (count, then the
// costs).  Inline costs spare the search a dependent read per relaxation.
// The last word of forms 0, 1 and 3 holds the source's packed row
// (pack_row), which the search queues with the node.
// After the records and cost blocks, one fill block per chain: per chain
// node x1..xk its id, the cost of its link toward v and of its link toward u
// (+inf bits where the link is missing); the chain's header (u, v, k, word
// offset of the block) is in ch_hdr.  k_chain_fill labels the chain nodes.
// Words at most: one record per link at most (a chain's record stands for
// two links or more), per chain of k > 2 nodes two cost blocks of
// ceil((k + 2) / 4) * 4 words (under 6 words per left-out node), and per
// chain a fill block of 3k words.
constexpr int kInlineCosts = 3;
size_t contraction_words(int64_t N, int64_t M) { return 4 * (size_t)M + 4 + 9 * (size_t)N; }

int build_contraction(qdta_ctx* c) {
    const int64_t N = c->N;
    if (N >= (int64_t)1 << 30) return set_err(c, QDTA_EARG, "the contracted search takes fewer than 2^30 nodes");
    const int ni = (int)c->inst.size();
    std::vector<int32_t> crp(N + 1, 0), ch_ptr{0}, ch_node, inst_chain(ni + 1, 0);
    std::vector<int2> cslot(c->M, make_int2(-1, -1));   // (record word, fill word) holding each link's cost
    std::vector<int2> ch_end, ch_link;
    std::vector<uint2> anc(N);
    for (int64_t v = 0; v < N; ++v) anc[v] = make_uint2((uint32_t)v, (uint32_t)v);
    // records per head node: plain (source, link) and shortcuts (source, chain, direction)
    struct Rec {
        int32_t head, src, link, chain, dir;   // link >= 0: plain; else shortcut of chain in direction dir
    };
    std::vector<Rec> recs;
    std::vector<std::vector<int32_t>> sc_links;   // cost links of each shortcut, in fold order
    for (int i = 0; i < ni; ++i) {
        const Instance& I = c->inst[i];
        const int n = I.n;
        const int32_t n0 = (int32_t)c->node_off[i], l0 = (int32_t)c->link_off[i];
        const std::vector<int32_t>& rp = I.row_ptr;
        const std::vector<int32_t>& col = I.col;
        inst_chain[i] = (int32_t)ch_end.size();
        // in-links (local)
        std::vector<int32_t> rrp(n + 1, 0), rin(I.m);
        for (int a = 0; a < I.m; ++a) rrp[col[a] + 1]++;
        for (int v = 0; v < n; ++v) rrp[v + 1] += rrp[v];
        {
            std::vector<int32_t> fill(rrp.begin(), rrp.end() - 1);
            for (int v = 0; v < n; ++v)
                for (int a = rp[v]; a < rp[v + 1]; ++a) rin[fill[col[a]]++] = v;
        }
        auto link_to = [&](int x, int y) -> int32_t {
            for (int a = rp[x]; a < rp[x + 1]; ++a)
                if (col[a] == y) return a;
            return -1;
        };
        // candidates and their two neighbours
        std::vector<int32_t> nb0(n, -1), nb1(n, -1);
        std::vector<char> cand(n, 0);
        for (int v = 0; v < n; ++v) {
            if (c->croot[n0 + v]) continue;
            const int od = rp[v + 1] - rp[v], id = rrp[v + 1] - rrp[v];
            if (od < 1 || od > 2 || id < 1 || id > 2) continue;
            int nb[4], k = 0;
            bool ok = true;
            for (int a = rp[v]; a < rp[v + 1]; ++a) nb[k++] = col[a];
            if (od == 2 && nb[0] == nb[1]) ok = false;
            for (int e = rrp[v]; e < rrp[v + 1]; ++e) nb[k++] = rin[e];
            if (id == 2 && rin[rrp[v]] == rin[rrp[v] + 1]) ok = false;
            int a0 = -1, a1 = -1;
            for (int j = 0; j < k && ok; ++j) {
                if (nb[j] == v) ok = false;
                else if (a0 < 0 || nb[j] == a0) a0 = nb[j];
                else if (a1 < 0 || nb[j] == a1) a1 = nb[j];
                else ok = false;
            }
            if (!ok || a1 < 0) continue;
            cand[v] = 1;
            nb0[v] = a0;
            nb1[v] = a1;
        }
        auto other = [&](int x, int from) { return nb0[x] == from ? nb1[x] : nb0[x]; };
        std::vector<char> seen(n, 0);
        std::vector<int32_t> run;
        for (int s = 0; s < n; ++s) {
            if (!cand[s] || seen[s]) continue;
            // extend from s both ways through candidates to the kept ends
            std::vector<int32_t> left;
            int prev = s, cur = nb0[s];
            bool ring = false;
            while (cand[cur]) {
                if (cur == s) { ring = true; break; }
                left.push_back(cur);
                const int nx = other(cur, prev);
                prev = cur;
                cur = nx;
            }
            if (ring) {                  // a ring of candidates with no kept node: keep them all
                seen[s] = 1;
                for (int x : left) seen[x] = 1;
                cand[s] = 0;
                for (int x : left) cand[x] = 0;
                continue;
            }
            const int u = cur;
            std::vector<int32_t> right;
            prev = s;
            cur = nb1[s];
            while (cand[cur]) {
                right.push_back(cur);
                const int nx = other(cur, prev);
                prev = cur;
                cur = nx;
            }
            const int v = cur;
            run.assign(left.rbegin(), left.rend());
            run.push_back(s);
            run.insert(run.end(), right.begin(), right.end());
            for (int x : run) seen[x] = 1;
            // cut into pieces of at most kChainMax nodes; the cut nodes are kept
            int a_end = u;
            size_t p = 0;
            while (p < run.size()) {
                const size_t q = std::min(run.size(), p + kChainMax);
                const int b_end = q < run.size() ? run[q] : v;
                if (q < run.size()) cand[run[q]] = 0;
                // chain run[p..q) between a_end and b_end
                const int k = (int)(q - p);
                const int cid = (int32_t)ch_end.size();
                std::vector<int32_t> rl(k), ll(k);
                for (int j = 0; j < k; ++j) {
                    const int x = run[p + j];
                    const int nxt = j + 1 < k ? run[p + j + 1] : b_end;
                    const int prv = j > 0 ? run[p + j - 1] : a_end;
                    rl[j] = link_to(x, nxt);
                    ll[j] = link_to(x, prv);
                }
                std::vector<char> ok_r(k), ok_l(k);
                for (int j = k - 1; j >= 0; --j) ok_r[j] = rl[j] >= 0 && (j == k - 1 || ok_r[j + 1]);
                for (int j = 0; j < k; ++j) ok_l[j] = ll[j] >= 0 && (j == 0 || ok_l[j - 1]);
                ch_end.push_back(make_int2(n0 + a_end, n0 + b_end));
                for (int j = 0; j < k; ++j) {
                    const int x = run[p + j];
                    ch_node.push_back(n0 + x);
                    ch_link.push_back(make_int2(rl[j] >= 0 ? l0 + rl[j] : -1, ll[j] >= 0 ? l0 + ll[j] : -1));
                    const int ar = ok_r[j] ? b_end : (ok_l[j] ? a_end : x);
                    const int al = ok_l[j] ? a_end : (ok_r[j] ? b_end : x);
                    anc[n0 + x] = make_uint2((uint32_t)(n0 + ar), (uint32_t)(n0 + al));
                }
                ch_ptr.push_back((int32_t)ch_node.size());
                if (a_end != b_end) {
                    const int32_t in_a = link_to(a_end, run[p]), in_b = link_to(b_end, run[q - 1]);
                    if (in_a >= 0 && ok_r[0]) {              // a_end -> x1 -> ... -> b_end, held at b_end
                        std::vector<int32_t> ls;
                        for (int j = k - 1; j >= 0; --j) ls.push_back(l0 + rl[j]);
                        ls.push_back(l0 + in_a);
                        recs.push_back({n0 + b_end, n0 + a_end, -1, (int32_t)sc_links.size(), 0});
                        sc_links.push_back(std::move(ls));
                    }
                    if (in_b >= 0 && ok_l[k - 1]) {          // b_end -> xk -> ... -> a_end, held at a_end
                        std::vector<int32_t> ls;
                        for (int j = 0; j < k; ++j) ls.push_back(l0 + ll[j]);
                        ls.push_back(l0 + in_b);
                        recs.push_back({n0 + a_end, n0 + b_end, -1, (int32_t)sc_links.size(), 1});
                        sc_links.push_back(std::move(ls));
                    }
                }
                (void)cid;
                a_end = b_end;
                p = q + (q < run.size() ? 1 : 0);
            }
        }
        // plain records: links between kept nodes
        for (int x = 0; x < n; ++x) {
            if (cand[x]) continue;
            for (int a = rp[x]; a < rp[x + 1]; ++a)
                if (!cand[col[a]]) recs.push_back({n0 + col[a], n0 + x, l0 + a, -1, 0});
        }
    }
    inst_chain[ni] = (int32_t)ch_end.size();
    // contracted reverse CSR: records grouped by head, plain ones in link order first
    std::stable_sort(recs.begin(), recs.end(), [](const Rec& a, const Rec& b) {
        if (a.head != b.head) return a.head < b.head;
        if ((a.link >= 0) != (b.link >= 0)) return a.link >= 0;
        return a.link >= 0 ? a.link < b.link : a.chain < b.chain;
    });
    for (const Rec& r : recs) crp[r.head + 1]++;
    for (int64_t v = 0; v < N; ++v) crp[v + 1] += crp[v];
    size_t words = 4 * recs.size();
    std::vector<size_t> blk(sc_links.size(), 0);
    for (size_t s = 0; s < sc_links.size(); ++s) {
        if (sc_links[s].size() <= (size_t)kInlineCosts) continue;
        blk[s] = words;
        words += (1 + sc_links[s].size() + 3) / 4 * 4;
    }
    std::vector<uint32_t> cbuf(words, 0u);
    for (size_t k = 0; k < recs.size(); ++k) {
        const Rec& r = recs[k];
        // the last word carries the source's packed row where no cost takes it
        const uint32_t row = pack_row(crp[r.src], crp[r.src + 1] - crp[r.src]);
        cbuf[4 * k + 3] = row;
        if (r.link >= 0) {
            cbuf[4 * k] = (uint32_t)r.src;
            cslot[r.link].x = (int32_t)(4 * k + 1);
            continue;
        }
        const std::vector<int32_t>& ls = sc_links[r.chain];
        if (ls.size() <= (size_t)kInlineCosts) {
            cbuf[4 * k] = (uint32_t)r.src | (uint32_t)(ls.size() - 1) << 30;
            for (size_t j = 0; j < ls.size(); ++j) cslot[ls[j]].x = (int32_t)(4 * k + 1 + j);
        } else {
            const size_t b = blk[r.chain];
            cbuf[4 * k] = (uint32_t)r.src | 3u << 30;
            cbuf[4 * k + 1] = (uint32_t)b;
            cbuf[b] = (uint32_t)ls.size();
            for (size_t j = 0; j < ls.size(); ++j) cslot[ls[j]].x = (int32_t)(b + 1 + j);
        }
    }
    // fill blocks and chain headers
    const size_t nch = ch_end.size();
    std::vector<int4> ch_hdr(nch);
    for (size_t ch = 0; ch < nch; ++ch) {
        const int k = ch_ptr[ch + 1] - ch_ptr[ch];
        ch_hdr[ch] = make_int4(ch_end[ch].x, ch_end[ch].y, k, (int32_t)std::min(words, (size_t)INT32_MAX));
        words += 3 * (size_t)k;
    }
    if (words >= (size_t)INT32_MAX) return set_err(c, QDTA_EARG, "contracted records beyond int32 offsets");
    cbuf.resize(words, 0u);
    for (size_t ch = 0; ch < nch; ++ch) {
        const size_t b = (size_t)ch_hdr[ch].w;
        const int j0 = ch_ptr[ch], k = ch_ptr[ch + 1] - j0;
        for (int j = 0; j < k; ++j) {
            const size_t q = b + 3 * (size_t)j;
            cbuf[q] = (uint32_t)ch_node[j0 + j];
            const int2 lk = ch_link[j0 + j];
            cbuf[q + 1] = kInfBits;               // a missing link stops the fold
            cbuf[q + 2] = kInfBits;
            if (lk.x >= 0) cslot[lk.x].y = (int32_t)(q + 1);
            if (lk.y >= 0) cslot[lk.y].y = (int32_t)(q + 2);
        }
    }
    c->c_fill_chunks = 0;
    for (int i = 0; i < ni; ++i) {
        const int32_t chunks = (inst_chain[i + 1] - inst_chain[i] + kFillChunk - 1) / kFillChunk;
        c->c_fill_chunks = std::max(c->c_fill_chunks, chunks);
    }
    c->c_chains = (int64_t)ch_end.size();
    c->c_left = (int64_t)ch_node.size();
    c->cleft.assign(N, 0);
    for (int32_t x : ch_node) c->cleft[x] = 1;
    // inside a workspace every buffer is carved at its bound once (see
    // contraction_words), so later rebuilds fit in place
    const bool ws = c->ws_base != nullptr;
    RC(upload(c, c->crptr, crp));
    RC(upload(c, c->cbuf, cbuf, ws ? contraction_words(N, c->M) : 0));
    RC(upload(c, c->cslot, cslot));
    RC(upload(c, c->anc, anc));
    RC(upload(c, c->ch_hdr, ch_hdr, ws ? (size_t)N : 0));
    RC(upload(c, c->inst_chain, inst_chain));
    c->c_built = true;
    c->gen++;
    // the records' costs from the forward records, which hold the current routing costs
    NetDev net = net_view(c);
    HIPCHECK(c, launch_cslot_init(c->stream, net));
    return QDTA_OK;
}

// Roots (global node ids) must stay in the search: the contraction is built
// on first use and again when a root is a node it leaves out.
int ensure_contraction(qdta_ctx* c, const int32_t* roots, size_t nroots) {
    if ((int64_t)c->croot.size() != c->N) {
        c->croot.assign(c->N, 0);
        c->c_built = false;
    }
    bool again = !c->c_built;
    for (size_t k = 0; k < nroots; ++k) {
        c->croot[roots[k]] = 1;
        if (c->c_built && c->cleft[roots[k]]) again = true;
    }
    return again ? build_contraction(c) : QDTA_OK;
}


// before a search of the current demand's trees
int ensure_contract(qdta_ctx* c, const qdta_opts* o) {
    if (!uses_contraction(o)) return QDTA_OK;
    // queues sized for the other search's narrower entries: widen them in place
    if (!c->scr_wide && c->scr_slots > 0) {
        RC(dalloc(c, c->nearq, (size_t)c->scr_slots * (size_t)c->scr_nmax * 2));
        RC(dalloc(c, c->farq, (size_t)c->scr_slots * (size_t)c->scr_nmax * 4));
        c->scr_wide = true;
    }
    return ensure_contraction(c, c->h_dest_node.data(), c->h_dest_node.size());
}

// Destinations of an instance are in ascending node order; tree t's labels
// are n 32-bit words at dest_lab[t], each tree padded to 32 words (128 bytes).
int64_t tree_words(int64_t n) { return (n + 31) / 32 * 32; }

// c->slots: wavefronts of a shortest-path launch (whole workgroups of four).
// Scratch: one slot per tree in flight, i.e. per wavefront (tree_waves 1) or
// per workgroup (tree_waves 4); launches never use more slots than exist.
int ensure_scratch(qdta_ctx* c, int64_t trees, int64_t nmax, int wpc, int tw, bool wide) {
    // every tree takes tw wavefronts; never more than wpc per CU
    int slots = (int)std::min<int64_t>(std::max<int64_t>(trees, 1) * (tw == 1 ? 1 : 4), (int64_t)c->cus * wpc);
    slots = (slots + 3) / 4 * 4;
    c->slots = slots;
    const int need = tw == 1 ? slots : slots / 4;
    nmax = std::max<int64_t>(nmax, 1) + 65;      // near rings: n queued nodes in n + (up to 64) slots
    // the contracted search's queue entries are twice as wide (see Scratch)
    if (need > c->scr_slots || nmax > c->scr_nmax || (wide && !c->scr_wide)) {
        int64_t ns = std::max<int64_t>(need, c->scr_slots), nm = std::max<int64_t>(nmax, c->scr_nmax);
        const bool w = wide || c->scr_wide;
        RC(dalloc(c, c->nearq, (size_t)ns * nm * (w ? 2 : 1)));
        RC(dalloc(c, c->farq, (size_t)ns * nm * (w ? 4 : 2)));
        c->scr_slots = (int)ns;
        c->scr_nmax = nm;
        c->scr_wide = w;
    }
    RC(dalloc(c, c->work, 1));
    if (!c->sssp_stats.p) {
        RC(dalloc(c, c->sssp_stats, 2));
        HIPCHECK(c, launch_fill_i64(c->stream, reinterpret_cast<int64_t*>(c->sssp_stats.p), 0, 2));
    }
    RC(dalloc(c, c->delta_inst, c->inst.size()));
    RC(dalloc(c, c->logsum, c->inst.size()));
    return QDTA_OK;
}

// wpc = 0: the demand tables only (no shortest-path scratch).
int ensure_demand(qdta_ctx* c, int wpc, int tw = 1, bool wide = false) {
    RC(ensure_network(c));
    if (!c->dem_dirty)
        return wpc > 0 ? ensure_scratch(c, (int64_t)plan_dests(c, (size_t)c->Q), c->nmax, wpc, tw, wide) : QDTA_OK;
    int64_t total_legs = 0;
    for (const Instance& I : c->inst) total_legs += (int64_t)I.orig.size();
    if (total_legs >= INT32_MAX) return set_err(c, QDTA_EARG, "total legs beyond int32 ids");
    int ni = (int)c->inst.size();
    std::vector<int32_t> qptr{0}, leg_orig, leg_q, dest_node, dest_inst;
    std::vector<int64_t> leg_dfx, dest_lab;
    std::vector<float> leg_delay;
    c->leg_off.assign(ni + 1, 0);
    c->dest_off.assign(ni + 1, 0);
    int64_t nmax = 0, lab = 0;
    for (int i = 0; i < ni; ++i) {
        Instance& I = c->inst[i];
        InstDev& d = c->h_inst[i];
        bool fin = std::isfinite(I.dt_s);
        d.kappa = fin ? 3600.0 / I.dt_s : 1.0;
        d.dt32 = (float)I.dt_s;
        d.rule = QDTA_RULE_NONE;
        d.q0 = (int32_t)dest_node.size();
        d.leg0 = (int32_t)leg_orig.size();
        size_t p = 0;
        while (p < I.orig.size()) {
            int32_t q = I.dest[p];
            int32_t qi = (int32_t)dest_node.size();
            dest_node.push_back(d.node0 + q);
            dest_inst.push_back(i);
            dest_lab.push_back(lab);
            lab += tree_words(I.n);
            while (p < I.orig.size() && I.dest[p] == q) {
                leg_orig.push_back(d.node0 + I.orig[p]);
                leg_dfx.push_back(I.dfx[p]);
                leg_delay.push_back(p < I.delay.size() ? I.delay[p] : 0.0f);
                leg_q.push_back(qi);
                ++p;
            }
            qptr.push_back((int32_t)leg_orig.size());
        }
        d.nq = (int32_t)dest_node.size() - d.q0;
        d.nleg = (int32_t)I.orig.size();
        c->leg_off[i + 1] = c->leg_off[i] + d.nleg;
        c->dest_off[i + 1] = c->dest_off[i] + d.nq;
        nmax = std::max<int64_t>(nmax, I.n);
    }
    c->Q = (int64_t)dest_node.size();
    c->P = (int64_t)leg_orig.size();
    c->nmax = nmax;
    c->label_count = (size_t)lab;
    c->h_dest_inst = dest_inst;
    c->h_dest_node = dest_node;
    c->h_qptr = qptr;
    const size_t pq = plan_dests(c, (size_t)c->Q), pp = plan_legs(c, (size_t)c->P);
    RC(upload(c, c->dest_node, dest_node, pq));
    RC(upload(c, c->dest_inst, dest_inst, pq));
    RC(upload(c, c->dest_lab, dest_lab, pq));
    RC(upload(c, c->qptr, qptr, pq + 1));
    RC(upload(c, c->leg_orig, leg_orig, pp));
    RC(upload(c, c->leg_dfx, leg_dfx, pp));
    RC(upload(c, c->leg_q, leg_q, pp));
    RC(upload(c, c->leg_delay, leg_delay, pp));
    RC(upload(c, c->d_inst, c->h_inst));
    RC(dalloc(c, c->labels, std::max(c->label_count, c->ws_base ? pq * (size_t)tree_words(nmax) : 0)));
    RC(dalloc(c, c->absorb_q, pq));
    RC(dalloc(c, c->int_node, pp));
    RC(dalloc(c, c->int_tau, pp));
    if (wpc > 0) RC(ensure_scratch(c, (int64_t)pq, nmax, wpc, tw, wide));
    c->dem_dirty = false;
    c->solved = false;
    c->lab_hist_ok.clear();
    c->gen++;                          // Q and P are baked into a captured iteration
    return QDTA_OK;
}

// The truncation rule comes with the options; it is stored per instance
// (NONE for plain intervals, dt = inf) in the device descriptors.
int apply_rule(qdta_ctx* c, const qdta_opts* o) {
    bool changed = false;
    for (size_t i = 0; i < c->inst.size(); ++i) {
        int32_t r = std::isfinite(c->inst[i].dt_s) ? o->trunc_rule : QDTA_RULE_NONE;
        if (c->h_inst[i].rule != r || c->h_inst[i].pq != o->progress_quantum_s) {
            c->h_inst[i].rule = r;
            c->h_inst[i].pq = o->progress_quantum_s;
            changed = true;
        }
    }
    if (changed) RC(upload(c, c->d_inst, c->h_inst));
    return QDTA_OK;
}

DemDev dem_view(qdta_ctx* c) {
    DemDev v;
    v.dest_node = c->dest_node.p;
    v.dest_inst = c->dest_inst.p;
    v.dest_lab = c->dest_lab.p;
    v.qptr = c->qptr.p;
    v.leg_orig = c->leg_orig.p;
    v.leg_dfx = c->leg_dfx.p;
    v.leg_q = c->leg_q.p;
    v.leg_delay = c->leg_delay.p;
    v.Q = (int32_t)c->Q;
    v.P = (int32_t)c->P;
    return v;
}

Scratch scr_view(qdta_ctx* c) {
    Scratch s;
    s.nearq = c->nearq.p;
    s.farq = c->farq.p;
    s.nmax = c->scr_nmax;
    s.work = c->work.p;
    s.nslots = c->scr_slots;
    s.stats = c->sssp_stats.p;
    return s;
}

FlagsDev flags_view(qdta_ctx* c) {
    FlagsDev f;
    f.err_overflow = c->flags.p;
    f.err_unreach = c->flags.p + 1;
    f.absorb_count = c->flags.p + 2;
    f.absorb_q = c->absorb_q.p;
    f.int_node = c->int_node.p;
    f.int_tau = c->int_tau.p;
    return f;
}

int clear_flags(qdta_ctx* c) {
    HIPCHECK(c, launch_fill_u32(c->stream, reinterpret_cast<uint32_t*>(c->flags.p), 0u, 4));
    return QDTA_OK;
}

int read_flags(qdta_ctx* c, int* h) {
    HIPCHECK(c, hipMemcpyAsync(h, c->flags.p, 4 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return QDTA_OK;
}

constexpr int kPhases = 8;
enum { PH_BPR = 0, PH_SSSP = 1, PH_WALK = 2, PH_GAP = 3, PH_LS = 4, PH_UPDATE = 5, PH_GRAPH = 6, PH_FILL = 7 };

// Record the start (edge 0) or end (edge 1) of a phase on the stream.
int prof_mark(qdta_ctx* c, int ph, int edge) {
    if (!c->prof_on) return QDTA_OK;
    HIPCHECK(c, hipEventRecord(c->prof_ev[ph][edge], c->stream));
    if (edge == 1) c->prof_open[ph] = 1;
    return QDTA_OK;
}

// After a stream synchronisation: add the closed phases' durations.
void prof_collect(qdta_ctx* c) {
    if (!c->prof_on) return;
    for (int p = 0; p < kPhases; ++p) {
        if (!c->prof_open[p]) continue;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, c->prof_ev[p][0], c->prof_ev[p][1]) == hipSuccess) {
            c->prof_ms[p] += ms;
            c->prof_n[p] += 1;
        } else {
            (void)hipGetLastError();           // a timer is optional: leave no sticky error
        }
        c->prof_open[p] = 0;
    }
}

// One all-or-nothing assignment (A2 + A3) under `cost` (reverse records already set).
// time_cost: the travel times that clock the truncation; NULL = `cost`.
// Plain-interval loading by merged paths: asked for, every instance plain,
// batched launches.
bool use_sweep(const qdta_ctx* c, const qdta_opts* o) {
    if (o->load_form != 2 || o->launch_form == 2) return false;
    for (const InstDev& d : c->h_inst)
        if (d.rule != QDTA_RULE_NONE) return false;
    return true;
}

// Its scratch, allocated (and cleared) before any launch that may be captured.
int ensure_sweep(qdta_ctx* c, const qdta_opts* o) {
    if (!use_sweep(c, o)) return QDTA_OK;
    if (c->sw_cnt.n < c->label_count || !c->sw_cnt.p) {
        RC(dalloc(c, c->sw_cnt, c->label_count));
        HIPCHECK(c, launch_fill_u32(c->stream, c->sw_cnt.p, 0u, (int64_t)c->sw_cnt.n));
    }
    if (c->sw_acc.n < c->label_count || !c->sw_acc.p) {
        RC(dalloc(c, c->sw_acc, c->label_count));
        HIPCHECK(c, launch_fill_i64(c->stream, c->sw_acc.p, 0, (int64_t)c->sw_acc.n));
    }
    return QDTA_OK;
}

int aon_core(qdta_ctx* c, const qdta_opts* o, const float* cost, const float* time_cost, int64_t* y, int32_t* stop,
             const InstState* st, bool marks = true, float* stop_delay = nullptr) {
    NetDev net = net_view(c);
    DemDev dem = dem_view(c);
    FlagsDev fl = flags_view(c);
    if (marks) RC(prof_mark(c, PH_SSSP, 0));
    if (o->launch_form == 2) {
        // plain form: one launch per destination tree (one workgroup each)
        HIPCHECK(c, launch_delta(c->stream, net, cost, delta_scale(o), c->delta_inst.p, c->logsum.p));
        for (int64_t t = 0; t < c->Q; ++t)
            HIPCHECK(c, launch_trees(c->stream, net, dem, c->radj.p, c->labels.p, scr_view(c), 4, st, c->delta_inst.p,
                                     sssp_variant(c, o), 1, (int)t, (int)t + 1, false));
    } else {
        HIPCHECK(c, launch_sssp(c->stream, net, dem, cost, c->radj.p, c->labels.p, scr_view(c), c->slots, st,
                                delta_scale(o), c->delta_inst.p, c->logsum.p, sssp_variant(c, o), 1, false));
    }
    if (marks) RC(prof_mark(c, PH_SSSP, 1));
    if (sssp_variant(c, o) >= 32) {   // the contracted search's left-out chain nodes, timed apart
        if (marks) RC(prof_mark(c, PH_FILL, 0));
        HIPCHECK(c, launch_chain_fill(c->stream, net, dem, c->labels.p, st, 0, (int)c->Q));
        if (marks) RC(prof_mark(c, PH_FILL, 1));
    }
    if (marks) RC(prof_mark(c, PH_WALK, 0));
    HIPCHECK(c, launch_fill_i64(c->stream, y, 0, c->M));
    HIPCHECK(c, launch_fill_u32(c->stream, reinterpret_cast<uint32_t*>(c->absorb_q.p), 0u, c->Q));
    if (use_sweep(c, o)) {
        HIPCHECK(c, launch_sweep(c->stream, net, dem, c->labels.p, y, stop, stop_delay, st, fl, c->sw_cnt.p,
                                 c->sw_acc.p));
    } else if (o->launch_form == 2) {
        for (int64_t qi = 0; qi < c->Q; ++qi)
            HIPCHECK(c, launch_walk(c->stream, net, dem, c->labels.p, time_cost, y, stop, st, fl, 0, nullptr, nullptr,
                                    nullptr, c->h_qptr[qi], c->h_qptr[qi + 1], stop_delay));
    } else {
        HIPCHECK(c, launch_walk(c->stream, net, dem, c->labels.p, time_cost, y, stop, st, fl, 0, nullptr, nullptr,
                                nullptr, 0, -1, stop_delay));
    }
    HIPCHECK(c, launch_fallback(c->stream, net, dem, c->labels.p, cost, time_cost ? time_cost : cost, y, stop, st, fl,
                                scr_view(c),
                                (int)std::min<int64_t>(c->scr_slots, std::max<int64_t>(c->Q, 1)), 0, nullptr, nullptr,
                                nullptr, 0, nullptr, 0, stop_delay));
    if (marks) RC(prof_mark(c, PH_WALK, 1));
    return QDTA_OK;
}

int init_state(qdta_ctx* c, bool all_instances, int iter) {
    int ni = (int)c->inst.size();
    for (int i = 0; i < ni; ++i) {
        InstState s;
        memset(&s, 0, sizeof(s));
        s.active = all_instances ? (c->inst[i].m > 0) : (c->h_inst[i].nleg > 0);
        s.iter = iter;
        c->h_st[i] = s;
    }
    HIPCHECK(c, hipMemcpyAsync(c->st.p, c->h_st, sizeof(InstState) * ni, hipMemcpyHostToDevice, c->stream));
    return QDTA_OK;
}

int pull_state(qdta_ctx* c) {
    int ni = (int)c->inst.size();
    HIPCHECK(c, hipMemcpyAsync(c->h_st, c->st.p, sizeof(InstState) * ni, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return QDTA_OK;
}

// Line search of the current iteration for every live instance (A5).
int line_search_core(qdta_ctx* c, const qdta_opts* o, const int64_t* f, const int64_t* y,
                     const NetDev* net_in = nullptr) {
    NetDev net = net_in ? *net_in : net_view(c, o);
    int ni = (int)c->inst.size();
    int* err = c->flags.p;
    int K = o->ls_mode == QDTA_LS_QN ? 3 : o->K;
    HIPCHECK(c, launch_ls_begin(c->stream, ni, c->st.p, c->alphas.p, K, o->ls_mode, o->dx, c->ls_acc.p, 0));
    if (o->ls_mode == QDTA_LS_MSA) return QDTA_OK;
    const bool plain = o->launch_form == 2;
    if (o->ls_mode == QDTA_LS_KSECTION) {
        for (int p = 0; p < o->passes; ++p) {
            if (plain) {
                for (int k = 0; k < K; ++k)
                    HIPCHECK(c, launch_ls_eval(c->stream, net, f, y, o->alpha, o->beta, 1, c->alphas.p, c->ls_acc.p,
                                               c->st.p, 1, err, k, K));
            } else {
                HIPCHECK(c, launch_ls_eval(c->stream, net, f, y, o->alpha, o->beta, K, c->alphas.p, c->ls_acc.p,
                                           c->st.p, 1, err));
            }
            HIPCHECK(c, launch_ls_decide(c->stream, ni, c->st.p, c->alphas.p, K, 0, o->passes, o->max_ls, o->T1, o->T2,
                                         o->dx, c->ls_acc.p));
        }
        return QDTA_OK;
    }
    // quasi-Newton (Alg. 8): iterate until every live instance is done
    for (int l = 0; l < o->max_ls; ++l) {
        if (plain) {
            for (int k = 0; k < 3; ++k)
                HIPCHECK(c, launch_ls_eval(c->stream, net, f, y, o->alpha, o->beta, 1, c->alphas.p, c->ls_acc.p, c->st.p,
                                           1, err, k, 3));
        } else {
            HIPCHECK(c, launch_ls_eval(c->stream, net, f, y, o->alpha, o->beta, 3, c->alphas.p, c->ls_acc.p, c->st.p, 1,
                                       err));
        }
        HIPCHECK(c, launch_ls_decide(c->stream, ni, c->st.p, c->alphas.p, 3, 1, o->passes, o->max_ls, o->T1, o->T2,
                                     o->dx, c->ls_acc.p));
        RC(pull_state(c));
        bool pending = false, fallback = false;
        for (int i = 0; i < ni; ++i) {
            const InstState& s = c->h_st[i];
            if (!s.active || s.converged) continue;
            if (s.ls_done == 0) pending = true;
            if (s.ls_done == 2) fallback = true;
        }
        if (!pending) {
            if (fallback) {
                // C'' <= 0: K-section for those instances (non-convex stencil)
                HIPCHECK(c, launch_ls_begin(c->stream, ni, c->st.p, c->alphas.p, o->K, 0, o->dx, c->ls_acc.p, 1));
                for (int p = 0; p < o->passes; ++p) {
                    HIPCHECK(c, launch_ls_eval(c->stream, net, f, y, o->alpha, o->beta, o->K, c->alphas.p, c->ls_acc.p,
                                               c->st.p, 1, err));
                    HIPCHECK(c, launch_ls_decide(c->stream, ni, c->st.p, c->alphas.p, o->K, 0, o->passes, o->max_ls,
                                                 o->T1, o->T2, o->dx, c->ls_acc.p));
                }
            }
            break;
        }
    }
    return QDTA_OK;
}

int flag_code(qdta_ctx* c, const int* h) {
    if (h[0]) return set_err(c, QDTA_EOVF, "non-finite link cost or exact-sum overflow");
    if (h[1]) return set_err(c, QDTA_EUNREACH, "a leg's destination is unreachable from its origin");
    return QDTA_OK;
}

// Slots of label history for this solve: as many iterates as fit in the free
// device memory less a reserve for the residual pass (its accumulator and
// outputs) and 16 GiB of headroom, or in opts->history_mib; at most
// max_iter + 1 and 64.
int plan_label_history(qdta_ctx* c, const qdta_opts* o) {
    c->lab_hist_ok.clear();
    const size_t per = c->label_count;
    if (per == 0 || o->history_mib < 0) return QDTA_OK;
    size_t avail = 0, reserve = 0;
    if (c->ws_base) {
        // the workspace's largest free run once the current history is given
        // back, less what the residual pass has still to carve
        dfree(c, c->lab_hist);
        for (const auto& r : c->ws_free) avail = std::max(avail, r.second);
        const int ni = (int)c->inst.size();
        const size_t hcap = (size_t)(hist_iters(o) + 1) * ni;
        const size_t rn = plan_legs(c, (size_t)std::max<int64_t>(c->P, 1));
        if (c->r_dense.n < c->label_count) reserve += align_up(c->label_count * sizeof(int64_t));
        if (c->st_hist.n < hcap) reserve += align_up(hcap * sizeof(InstState));
        if (c->lam_hist.n < hcap) reserve += align_up(hcap * sizeof(double));
        if (c->r_cnt.n < plan_dests(c, (size_t)std::max<int64_t>(c->Q, 1)))
            reserve += align_up(plan_dests(c, (size_t)std::max<int64_t>(c->Q, 1)) * sizeof(int64_t));
        if (c->r_orig.n < rn) reserve += 2 * align_up(rn * sizeof(int32_t)) + align_up(rn * sizeof(int64_t));
    } else {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            (void)hipGetLastError();
            return QDTA_OK;
        }
        avail = free_b + c->lab_hist.n * sizeof(label_t);
        reserve = (size_t)16 << 30;
        if (c->r_dense.n < c->label_count) reserve += (c->label_count - c->r_dense.n) * sizeof(int64_t);
        reserve += (size_t)c->P * 16;
    }
    if (avail <= reserve) return QDTA_OK;
    size_t budget = avail - reserve;
    if (o->history_mib > 0) budget = std::min(budget, (size_t)o->history_mib << 20);
    size_t slots = budget / (per * sizeof(label_t));
    const size_t want = o->fixed_iters > 0 ? (size_t)o->fixed_iters + 1 : (size_t)std::max(o->max_iter, 0) + 1;
    slots = std::min<size_t>(std::min<size_t>(slots, want), 64);
    if (slots == 0) return QDTA_OK;
    if (c->lab_hist.n < slots * per) {
        dfree(c, c->lab_hist);
        if (dalloc(c, c->lab_hist, slots * per) != QDTA_OK) {   // not fatal: recompute instead
            c->err.clear();
            return QDTA_OK;
        }
    }
    c->lab_hist_ok.assign(slots, 0);
    return QDTA_OK;
}

// After iterate j's shortest paths: keep its labels if a slot is free.
int stash_labels(qdta_ctx* c, int j) {
    if (j < 0 || (size_t)j >= c->lab_hist_ok.size()) return QDTA_OK;
    HIPCHECK(c, hipMemcpyAsync(c->lab_hist.p + (size_t)j * c->label_count, c->labels.p,
                               sizeof(label_t) * c->label_count, hipMemcpyDeviceToDevice, c->stream));
    c->lab_hist_ok[j] = 1;
    return QDTA_OK;
}

int ensure_history(qdta_ctx* c, size_t iters) {
    if (c->hist_iters_cap >= iters) return QDTA_OK;
    size_t want = std::max(iters, c->hist_iters_cap * 2);
    DBuf<float> nb;
    RC(dalloc(c, nb, want * (size_t)c->M));
    if (c->hist_cost.p && c->hist_iters_cap)
        HIPCHECK(c, hipMemcpyAsync(nb.p, c->hist_cost.p, c->hist_iters_cap * (size_t)c->M * sizeof(float),
                                   hipMemcpyDeviceToDevice, c->stream));
    if (c->hist_cost.p) {
        HIPCHECK(c, hipStreamSynchronize(c->stream));
        dfree(c, c->hist_cost);
    }
    c->hist_cost = nb;
    c->hist_iters_cap = want;
    return QDTA_OK;
}

int64_t trips_fx(double t) { return (int64_t)std::nearbyint(t * 1048576.0); }

// Sort legs by (dest, orig, delay) and sum equal ones; drop zero and
// orig == dest.  Delays are non-negative floats, which order like their bits.
// Legs of different destinations never merge: they are bucketed by
// destination (counting sort), and the buckets are sorted by (orig, delay)
// packed in 64 bits on several host threads (the link-progress rule leaves
// tens of millions of pending legs at a peak interval).
void merge_legs(std::vector<int32_t>& o, std::vector<int32_t>& d, std::vector<int64_t>& w, std::vector<float>& t) {
    const size_t n = o.size();
    t.resize(n, 0.0f);
    int32_t dmax = -1;
    for (size_t i = 0; i < n; ++i) dmax = std::max(dmax, d[i]);
    std::vector<size_t> start((size_t)dmax + 2, 0), idx(n);
    for (size_t i = 0; i < n; ++i) start[(size_t)d[i] + 1]++;
    for (size_t v = 0; v + 1 < start.size(); ++v) start[v + 1] += start[v];
    {
        std::vector<size_t> fill(start.begin(), start.end() - 1);
        for (size_t i = 0; i < n; ++i) idx[fill[(size_t)d[i]]++] = i;
    }
    // per destination: (orig << 32 | delay bits, weight), sorted and summed
    std::vector<std::vector<std::pair<uint64_t, int64_t>>> out((size_t)dmax + 1);
    std::atomic<int64_t> next{0};
    auto work = [&]() {
        std::vector<std::pair<uint64_t, int64_t>> v;
        for (int64_t b; (b = next.fetch_add(1)) <= dmax;) {
            const size_t b0 = start[(size_t)b], b1 = start[(size_t)b + 1];
            if (b0 == b1) continue;
            v.clear();
            for (size_t k = b0; k < b1; ++k) {
                const size_t i = idx[k];
                v.emplace_back(((uint64_t)(uint32_t)o[i] << 32) | __builtin_bit_cast(uint32_t, t[i]), w[i]);
            }
            std::sort(v.begin(), v.end(), [](const auto& a, const auto& c) { return a.first < c.first; });
            auto& r = out[(size_t)b];
            for (size_t k = 0; k < v.size(); ++k) {
                if (!r.empty() && r.back().first == v[k].first) r.back().second += v[k].second;
                else r.push_back(v[k]);
            }
        }
    };
    const unsigned nt = n < (1u << 16) ? 1u : std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned k = 1; k < nt; ++k) pool.emplace_back(work);
    work();
    for (auto& th : pool) th.join();
    std::vector<int32_t> no, nd;
    std::vector<int64_t> nw;
    std::vector<float> ntl;
    for (int32_t b = 0; b <= dmax; ++b) {
        for (const auto& e : out[(size_t)b]) {
            const int32_t oo = (int32_t)(e.first >> 32);
            if (e.second <= 0 || oo == b) continue;
            no.push_back(oo);
            nd.push_back(b);
            nw.push_back(e.second);
            ntl.push_back(__builtin_bit_cast(float, (uint32_t)(e.first & 0xffffffffu)));
        }
    }
    o.swap(no); d.swap(nd); w.swap(nw); t.swap(ntl);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void qdta_default_opts(qdta_opts* o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->alpha = 0.15;
    o->beta = 4;
    o->trunc_rule = QDTA_RULE_CEIL;
    o->ls_mode = QDTA_LS_KSECTION;
    o->K = 32;
    o->passes = 3;
    o->max_ls = 20;
    o->T1 = 1e-4;
    o->T2 = 1e-4;
    o->dx = 1e-4;
    o->stop_rule = QDTA_STOP_GAP;
    o->tol = 1e-4;
    o->max_iter = 1000;
    o->fixed_iters = 0;
    o->keep_history = 0;
    o->waves_per_cu = 0;
    o->delta_scale = 0.0;
    o->progress_quantum_s = 60.0;
}

const char* qdta_strerror(int code) {
    switch (code) {
        case QDTA_OK: return "ok";
        case QDTA_EARG: return "bad argument";
        case QDTA_ECSR: return "malformed CSR";
        case QDTA_EVAL: return "free-flow time or capacity not positive and finite";
        case QDTA_EUNREACH: return "destination unreachable from origin";
        case QDTA_EOVF: return "overflow";
        case QDTA_ENOMEM: return "device allocation failed";
        case QDTA_EHIP: return "HIP runtime error";
        case QDTA_ESTATE: return "call out of order";
        case QDTA_WABSORB: return "FP32 absorption: tie-rule fallback used";
        default: return "unknown code";
    }
}

const char* qdta_last_error(const qdta_ctx* c) { return c ? c->err.c_str() : "null context"; }

int qdta_create(qdta_ctx** out, int device, void* stream) {
    if (!out) return QDTA_EARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return QDTA_EARG;
    if (hipSetDevice(device) != hipSuccess) return QDTA_EHIP;
    // the allocation-free line search's static scratch on this device
    long long* na = nullptr;
    if (noalloc_scratch(device, &na) != hipSuccess || !na) {
        (void)hipGetLastError();
        return QDTA_EHIP;
    }
    qdta_ctx* c = new qdta_ctx();
    c->device = device;
    c->noalloc = na;
    c->stream = (hipStream_t)stream;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->cus = prop.multiProcessorCount;
    *out = c;
    return QDTA_OK;
}

int qdta_destroy(qdta_ctx* c) {
    if (!c) return QDTA_EARG;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (void* p : c->allocs) (void)hipFree(p);
    if (c->h_st) (void)hipHostFree(c->h_st);
    for (int p = 0; p < 8; ++p)
        for (int e = 0; e < 2; ++e)
            if (c->prof_ev[p][e]) (void)hipEventDestroy(c->prof_ev[p][e]);
    drop_graph(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return QDTA_OK;
}

int qdta_set_stream(qdta_ctx* c, void* stream) {
    if (!c) return QDTA_EARG;
    c->stream = (hipStream_t)stream;
    return QDTA_OK;
}

int qdta_workspace_query(qdta_ctx* c, const qdta_opts* o, int64_t max_legs, int64_t max_dests, size_t* bytes) {
    if (!c) return QDTA_EARG;
    c->err.clear();
    if (!opts_ok(c, o)) return QDTA_EARG;
    if (!bytes || max_legs < 0 || max_dests < 0) return set_err(c, QDTA_EARG, "bad arguments");
    if (c->inst.empty()) return set_err(c, QDTA_ESTATE, "no network added");
    // sizes from the host copies of the networks and the current demand, as
    // ensure_network / ensure_demand / ensure_scratch / the FW and residual
    // passes will carve them (every buffer rounded up to 256 bytes)
    const int ni = (int)c->inst.size();
    int64_t N = 0, M = 0, nblk = 0, Q = 0, P = 0, nmax = 0, words = 0;
    for (const Instance& I : c->inst) {
        N += I.n;
        M += I.m;
        nblk += (I.m + kChunk - 1) / kChunk;
        nmax = std::max<int64_t>(nmax, I.n);
        int64_t q = 0;
        for (size_t p = 0; p < I.orig.size(); ++p)
            if (p == 0 || I.dest[p] != I.dest[p - 1]) ++q;
        Q += q;
        P += (int64_t)I.orig.size();
        words += q * tree_words(I.n);
    }
    if (N >= INT32_MAX || M >= INT32_MAX) return set_err(c, QDTA_EARG, "total size beyond int32 ids");
    const size_t pq = (size_t)std::max(Q, max_dests), pp = (size_t)std::max(P, max_legs);
    const size_t labels = std::max<size_t>((size_t)words, pq * (size_t)tree_words(nmax));
    size_t b = 0;
    auto add = [&](size_t n, size_t sz) { b += align_up(std::max<size_t>(n, 1) * sz); };
    // network and Frank-Wolfe state
    add(N + 1, 4); add(M, 4); add(M, 4); add(M, 4); add(N + 1, 4); add(M, 4); add(M, 4); add(M, 4);
    add(nblk, 4); add(nblk, 4); add(ni, sizeof(InstDev));
    add(M, 8); add(M, 8); add(M, 4); add(M, 8); add(M, 8); add(M, 4); add(M, 4); add(M, 4);
    add(ni, sizeof(InstState)); add((size_t)ni * 6, 8); add((size_t)ni * kMaxK * 6, 8); add((size_t)ni * kMaxK, 8);
    add(ni, 8); add(4, 4); add(ni, 8);
    // demand tables and shortest-path labels
    add(pq, 4); add(pq, 4); add(pq, 8); add(pq + 1, 4); add(pp, 4); add(pp, 8); add(pp, 4); add(pp, 4);
    add(labels, 4); add(pq, 4); add(pp, 4); add(pp, 4);
    if (o->load_form == 2) { add(labels, 4); add(labels, 8); }   // plain-interval loading by merged paths
    if (uses_contraction(o)) {                                    // chain contraction (at its bounds)
        add(N + 1, 4); add(contraction_words(N, M), 4); add(M, 8); add(N, 8);
        add(N, 16); add(ni + 1, 4);
    }
    // shortest-path scratch (as ensure_scratch sizes it)
    {
        const int tw = tree_waves(o), wpc = waves_per_cu(o);
        int slots = (int)std::min<int64_t>(std::max<int64_t>((int64_t)pq, 1) * (tw == 1 ? 1 : 4),
                                           (int64_t)c->cus * wpc);
        slots = (slots + 3) / 4 * 4;
        const int64_t need = tw == 1 ? slots : slots / 4;
        const int64_t nm = std::max<int64_t>(nmax, 1) + 65;
        const size_t qw = uses_contraction(o) || o->sssp_kernel == 0 ? 2 : 1;   // wider entries (Scratch)
        add((size_t)(need * nm) * qw, 4); add((size_t)(need * nm * 2) * qw, 4);
        add(1, 4); add(2, 8); add(ni, 4); add(ni, 8);
    }
    if (o->keep_history) {
        const size_t hcap = (size_t)(hist_iters(o) + 1);
        add((hcap + 1) * (size_t)M, 4);                             // per-iterate costs
        add(hcap * ni, sizeof(InstState)); add(hcap * ni, 8);       // residual pass: states, weights
        add(labels, 8); add(pq, 8); add(pp, 4); add(pp, 4); add(pp, 8);  // accumulator, counts, legs out
        if (o->trunc_rule == QDTA_RULE_PROGRESS) {                       // legs left on links
            const size_t tc = std::max(pp, hcap * (size_t)std::max<int64_t>(P, 1));
            add(tc, 4); add(tc, 4); add(tc, 4); add(tc, 8); add(1, 4);
        }
        if (o->history_mib > 0) b += align_up((size_t)o->history_mib << 20);
    }
    c->ws_max_legs = (int64_t)pp;
    c->ws_max_dests = (int64_t)pq;
    *bytes = b;
    return QDTA_OK;
}

int qdta_bind_workspace(qdta_ctx* c, void* dev_ptr, size_t bytes) {
    if (!c) return QDTA_EARG;
    c->err.clear();
    if (c->ws_base || !c->allocs.empty())
        return set_err(c, QDTA_ESTATE, "bind the workspace once, before any call that uses device memory");
    if (!dev_ptr || bytes == 0 || ((uintptr_t)dev_ptr % kAlign) != 0)
        return set_err(c, QDTA_EARG, "workspace must be a non-empty device range aligned to %zu bytes", kAlign);
    c->ws_base = (char*)dev_ptr;
    c->ws_size = bytes / kAlign * kAlign;
    c->ws_free.clear();
    c->ws_used.clear();
    c->ws_free[0] = c->ws_size;
    return QDTA_OK;
}

int qdta_alloc_count(const qdta_ctx* c, int64_t* hip_mallocs, size_t* ws_in_use) {
    if (!c) return QDTA_EARG;
    if (hip_mallocs) *hip_mallocs = c->n_hip_malloc;
    if (ws_in_use) {
        size_t u = 0;
        for (const auto& r : c->ws_used) u += r.second;
        *ws_in_use = u;
    }
    return QDTA_OK;
}

int qdta_add_network(qdta_ctx* c, int32_t n, int32_t m, const int32_t* row_ptr, const int32_t* col,
                     const float* fftt, const float* cap, int32_t* inst_out) {
    if (!c) return QDTA_EARG;
    c->err.clear();
    if (n <= 0 || m < 0 || !row_ptr || (m > 0 && (!col || !fftt || !cap)))
        return set_err(c, QDTA_EARG, "bad sizes or null arrays");
    if (row_ptr[0] != 0 || row_ptr[n] != m) return set_err(c, QDTA_ECSR, "row_ptr must start at 0 and end at m");
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] < row_ptr[v]) return set_err(c, QDTA_ECSR, "row_ptr decreases at node %d", v);
    for (int32_t a = 0; a < m; ++a) {
        if (col[a] < 0 || col[a] >= n) return set_err(c, QDTA_ECSR, "col[%d] = %d out of range", a, col[a]);
        if (!(fftt[a] > 0.0f) || !std::isfinite(fftt[a])) return set_err(c, QDTA_EVAL, "fftt[%d] not > 0 and finite", a);
        if (!(cap[a] > 0.0f) || !std::isfinite(cap[a])) return set_err(c, QDTA_EVAL, "cap[%d] not > 0 and finite", a);
    }
    Instance I;
    I.n = n;
    I.m = m;
    I.row_ptr.assign(row_ptr, row_ptr + n + 1);
    I.col.assign(col, col + m);
    I.fftt.assign(fftt, fftt + m);
    I.cap.assign(cap, cap + m);
    c->inst.push_back(std::move(I));
    c->net_dirty = true;
    c->dem_dirty = true;
    if (inst_out) *inst_out = (int32_t)c->inst.size() - 1;
    return QDTA_OK;
}

int qdta_set_demand(qdta_ctx* c, int32_t inst, int32_t P, const int32_t* orig, const int32_t* dest,
                    const double* trips, double dt_s) {
    if (!c) return QDTA_EARG;
    c->err.clear();
    if (inst < 0 || inst >= (int32_t)c->inst.size()) return set_err(c, QDTA_EARG, "no instance %d", inst);
    if (P < 0 || (P > 0 && (!orig || !dest || !trips))) return set_err(c, QDTA_EARG, "bad legs");
    if (!(dt_s > 0.0)) return set_err(c, QDTA_EARG, "dt must be > 0 (or +inf)");
    Instance& I = c->inst[inst];
    std::vector<int32_t> o, d;
    std::vector<int64_t> w;
    o.reserve(P + I.r_orig.size());
    for (int32_t p = 0; p < P; ++p) {
        if (orig[p] < 0 || orig[p] >= I.n || dest[p] < 0 || dest[p] >= I.n)
            return set_err(c, QDTA_EARG, "leg %d: node out of range", p);
        if (!(trips[p] >= 0.0) || !std::isfinite(trips[p])) return set_err(c, QDTA_EARG, "leg %d: bad trips", p);
        if (trips[p] * 1048576.0 >= 9.0e18) return set_err(c, QDTA_EOVF, "leg %d: trips beyond fixed point", p);
        o.push_back(orig[p]);
        d.push_back(dest[p]);
        w.push_back(trips_fx(trips[p]));
    }
    // the pending residual is already in (destination, origin, delay) order
    // with positive weights and origin != destination: sort the new legs
    // alone (no delay), then merge the two runs (equal legs add up)
    std::vector<float> t;
    merge_legs(o, d, w, t);
    if (!I.r_orig.empty()) {
        const size_t na = o.size(), nb = I.r_orig.size();
        std::vector<int32_t> mo, md;
        std::vector<int64_t> mw;
        std::vector<float> mt;
        mo.reserve(na + nb);
        md.reserve(na + nb);
        mw.reserve(na + nb);
        mt.reserve(na + nb);
        auto key_a = [&](size_t i) { return std::make_tuple(d[i], o[i], __builtin_bit_cast(uint32_t, t[i])); };
        auto key_b = [&](size_t i) {
            return std::make_tuple(I.r_dest[i], I.r_orig[i], __builtin_bit_cast(uint32_t, I.r_delay[i]));
        };
        size_t a = 0, b = 0;
        while (a < na || b < nb) {
            int cmp;
            if (a == na) cmp = 1;
            else if (b == nb) cmp = -1;
            else cmp = key_a(a) < key_b(b) ? -1 : (key_b(b) < key_a(a) ? 1 : 0);
            if (cmp <= 0) {
                mo.push_back(o[a]);
                md.push_back(d[a]);
                mw.push_back(w[a] + (cmp == 0 ? I.r_w[b] : 0));
                mt.push_back(t[a]);
                ++a;
                if (cmp == 0) ++b;
            } else {
                mo.push_back(I.r_orig[b]);
                md.push_back(I.r_dest[b]);
                mw.push_back(I.r_w[b]);
                mt.push_back(I.r_delay[b]);
                ++b;
            }
        }
        o.swap(mo);
        d.swap(md);
        w.swap(mw);
        t.swap(mt);
    }
    I.orig.swap(o);
    I.dest.swap(d);
    I.dfx.swap(w);
    I.delay.swap(t);
    I.r_orig.clear();
    I.r_dest.clear();
    I.r_w.clear();
    I.r_delay.clear();
    I.dt_s = dt_s;
    I.has_demand = true;
    I.solved_iters = -1;
    c->dem_dirty = true;
    c->solved = false;
    return QDTA_OK;
}

int qdta_layout(qdta_ctx* c, qdta_layout_info* info) {
    if (!c || !info) return QDTA_EARG;
    RC(ensure_network(c));
    if (c->dem_dirty) RC(ensure_demand(c, 0));
    info->n_instances = (int32_t)c->inst.size();
    info->total_nodes = c->N;
    info->total_links = c->M;
    info->total_legs = c->P;
    info->total_dests = c->Q;
    return QDTA_OK;
}

int qdta_offsets(qdta_ctx* c, int64_t* node_off, int64_t* link_off, int64_t* leg_off, int64_t* dest_off) {
    if (!c) return QDTA_EARG;
    RC(ensure_network(c));
    if (c->dem_dirty) RC(ensure_demand(c, 0));
    size_t k = c->inst.size() + 1;
    if (node_off) std::copy(c->node_off.begin(), c->node_off.begin() + k, node_off);
    if (link_off) std::copy(c->link_off.begin(), c->link_off.begin() + k, link_off);
    if (leg_off) std::copy(c->leg_off.begin(), c->leg_off.begin() + k, leg_off);
    if (dest_off) std::copy(c->dest_off.begin(), c->dest_off.begin() + k, dest_off);
    return QDTA_OK;
}

int qdta_get_legs(qdta_ctx* c, int32_t* ho, int32_t* hd, int64_t* hw, float* ht) {
    if (!c) return QDTA_EARG;
    size_t k = 0;
    for (const Instance& I : c->inst) {
        for (size_t p = 0; p < I.orig.size(); ++p, ++k) {
            if (ho) ho[k] = I.orig[p];
            if (hd) hd[k] = I.dest[p];
            if (hw) hw[k] = I.dfx[p];
            if (ht) ht[k] = p < I.delay.size() ? I.delay[p] : 0.0f;
        }
    }
    return QDTA_OK;
}

int qdta_bpr(qdta_ctx* c, const qdta_opts* o, const int64_t* f, float* cost) {
    if (!c) return QDTA_EARG;
    c->err.clear();
    if (!opts_ok(c, o)) return QDTA_EARG;
    if (!f || !cost) return set_err(c, QDTA_EARG, "null array");
    RC(ensure_network(c));
    if (c->dem_dirty) RC(ensure_demand(c, 0));   // kappa of each instance
    RC(clear_flags(c));
    HIPCHECK(c, launch_bpr(c->stream, net_view(c, o), f, o->alpha, o->beta, cost, nullptr, nullptr, 0, c->flags.p));
    int h[4];
    RC(read_flags(c, h));
    return flag_code(c, h);
}

int qdta_trees(qdta_ctx* c, const qdta_opts* o, int32_t inst, const float* cost, int32_t nq, const int32_t* dest,
               float* dist, int32_t* succ) {
    if (!c) return QDTA_EARG;
    c->err.clear();
    if (!opts_ok(c, o)) return QDTA_EARG;
    RC(ensure_network(c));
    if (inst < 0 || inst >= (int32_t)c->inst.size()) return set_err(c, QDTA_EARG, "no instance %d", inst);
    if (nq < 0 || (nq > 0 && (!cost || !dest || !dist || !succ))) return set_err(c, QDTA_EARG, "bad arguments");
    if (nq == 0) return QDTA_OK;
    const InstDev I = c->h_inst[inst];
    std::vector<int32_t> hd(nq);
    HIPCHECK(c, hipMemcpyAsync(hd.data(), dest, sizeof(int32_t) * nq, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    for (int t = 0; t < nq; ++t)
        if (hd[t] < 0 || hd[t] >= I.n) return set_err(c, QDTA_EARG, "dest[%d] out of range", t);
    // one tree per requested destination, in order, labels tree-major
    std::vector<int32_t> dn(nq), di(nq, inst);
    std::vector<int64_t> dl(nq);
    for (int t = 0; t < nq; ++t) {
        dn[t] = I.node0 + hd[t];
        dl[t] = (int64_t)t * tree_words(I.n);
    }
    DBuf<int32_t> ddn, ddi, aq;
    DBuf<int64_t> ddl;
    DBuf<label_t> lab;
    auto cleanup = [&]() {
        for (void* p : {(void*)ddn.p, (void*)ddi.p, (void*)aq.p, (void*)ddl.p, (void*)lab.p}) dev_free(c, p);
    };
    int rc = QDTA_OK;
    do {
        if ((rc = upload(c, ddn, dn))) break;
        if ((rc = upload(c, ddi, di))) break;
        if ((rc = upload(c, ddl, dl))) break;
        if ((rc = dalloc(c, lab, (size_t)nq * tree_words(I.n)))) break;
        if ((rc = dalloc(c, aq, nq))) break;
        int saved_slots = c->slots;
        if ((rc = ensure_scratch(c, nq, std::max<int64_t>(c->nmax, I.n), waves_per_cu(o), tree_waves(o),
                                 uses_contraction(o))))
            break;
        int slots = c->slots;
        c->slots = saved_slots;
        DemDev dem;
        memset(&dem, 0, sizeof(dem));
        dem.dest_node = ddn.p;
        dem.dest_inst = ddi.p;
        dem.dest_lab = ddl.p;
        dem.Q = nq;
        if (uses_contraction(o) && (rc = ensure_contraction(c, dn.data(), dn.size()))) break;
        NetDev net = net_view(c);
        hipError_t e;
        // place the instance's costs in the global link order
        if ((e = hipMemcpyAsync(c->cost.p + I.link0, cost, sizeof(float) * I.m, hipMemcpyDeviceToDevice, c->stream)))
            { rc = set_err(c, QDTA_EHIP, "copy cost: %s", hipGetErrorString(e)); break; }
        if ((e = launch_scatter_rcost(c->stream, net, c->cost.p, c->radj.p)))
            { rc = set_err(c, QDTA_EHIP, "scatter: %s", hipGetErrorString(e)); break; }
        if ((e = launch_sssp(c->stream, net, dem, c->cost.p, c->radj.p, lab.p, scr_view(c), slots, nullptr,
                             delta_scale(o), c->delta_inst.p, c->logsum.p, sssp_variant(c, o), 0)))
            { rc = set_err(c, QDTA_EHIP, "sssp: %s", hipGetErrorString(e)); break; }
        if ((e = launch_fill_u32(c->stream, reinterpret_cast<uint32_t*>(aq.p), 0u, nq)))
            { rc = set_err(c, QDTA_EHIP, "fill: %s", hipGetErrorString(e)); break; }
        if ((e = launch_trees_out(c->stream, net, dem, lab.p, c->cost.p, inst, dist, succ, aq.p)))
            { rc = set_err(c, QDTA_EHIP, "trees_out: %s", hipGetErrorString(e)); break; }
        FlagsDev fl = flags_view(c);
        fl.absorb_q = aq.p;
        if ((e = launch_fallback(c->stream, net, dem, lab.p, c->cost.p, c->cost.p, nullptr, nullptr, nullptr, fl,
                                 scr_view(c), (int)std::min<int64_t>(c->scr_slots, nq), 0, nullptr, nullptr, nullptr,
                                 1, succ, I.n)))
            { rc = set_err(c, QDTA_EHIP, "fallback: %s", hipGetErrorString(e)); break; }
        std::vector<int32_t> ha(nq);
        if ((e = hipMemcpyAsync(ha.data(), aq.p, sizeof(int32_t) * nq, hipMemcpyDeviceToHost, c->stream)))
            { rc = set_err(c, QDTA_EHIP, "copy: %s", hipGetErrorString(e)); break; }
        if ((e = hipStreamSynchronize(c->stream))) { rc = set_err(c, QDTA_EHIP, "sync: %s", hipGetErrorString(e)); break; }
        for (int t = 0; t < nq; ++t)
            if (ha[t]) rc = QDTA_WABSORB;
    } while (0);
    (void)hipStreamSynchronize(c->stream);
    cleanup();
    return rc;
}

int qdta_aon(qdta_ctx* c, const qdta_opts* o, const float* cost, int64_t* y, int32_t* stop, float* stop_delay) {
    if (!c) return QDTA_EARG;
    c->err.clear();
    if (!opts_ok(c, o)) return QDTA_EARG;
    if (!cost || !y) return set_err(c, QDTA_EARG, "null array");
    RC(ensure_demand(c, waves_per_cu(o), tree_waves(o), uses_contraction(o)));
    RC(apply_rule(c, o));
    RC(ensure_sweep(c, o));
    RC(ensure_contract(c, o));
    RC(init_state(c, false, 0));
    RC(clear_flags(c));
    NetDev net = net_view(c);
    HIPCHECK(c, hipMemcpyAsync(c->cost.p, cost, sizeof(float) * c->M, hipMemcpyDeviceToDevice, c->stream));
    HIPCHECK(c, launch_scatter_rcost(c->stream, net, c->cost.p, c->radj.p));
    if (stop) HIPCHECK(c, launch_fill_u32(c->stream, reinterpret_cast<uint32_t*>(stop), 0xffffffffu, c->P));
    if (stop_delay) HIPCHECK(c, launch_fill_u32(c->stream, reinterpret_cast<uint32_t*>(stop_delay), 0u, c->P));
    RC(aon_core(c, o, c->cost.p, nullptr, y, stop, nullptr, true, stop_delay));
    int h[4];
    RC(read_flags(c, h));
    prof_collect(c);
    RC(flag_code(c, h));
    return h[2] ? QDTA_WABSORB : QDTA_OK;
}

int qdta_ls_eval(qdta_ctx* c, const qdta_opts* o, const int64_t* f, const int64_t* y, int32_t K, const double* alphas,
                 int64_t* sums) {
    if (!c) return QDTA_EARG;
    c->err.clear();
    if (!opts_ok(c, o)) return QDTA_EARG;
    if (K < 1 || K > kMaxK || !f || !y || !alphas || !sums) return set_err(c, QDTA_EARG, "bad arguments");
    RC(ensure_network(c));
    if (c->dem_dirty) RC(ensure_demand(c, waves_per_cu(o), tree_waves(o), uses_contraction(o)));
    int ni = (int)c->inst.size();
    RC(clear_flags(c));
    HIPCHECK(c, launch_fill_i64(c->stream, reinterpret_cast<int64_t*>(c->ls_acc.p), 0, (int64_t)ni * K * 6));
    HIPCHECK(c, launch_ls_eval(c->stream, net_view(c, o), f, y, o->alpha, o->beta, K, alphas, c->ls_acc.p, nullptr, 0,
                               c->flags.p));
    HIPCHECK(c, launch_ls_export(c->stream, ni, c->ls_acc.p, K, sums));
    int h[4];
    RC(read_flags(c, h));
    return flag_code(c, h);
}

int qdta_ls_eval_noalloc(qdta_ctx* c, const qdta_opts* o, const int64_t* f, const int64_t* y, int32_t K,
                         const double* alphas, int64_t* sums) {
    if (!c) return QDTA_EARG;
    c->err.clear();
    if (!opts_ok(c, o)) return QDTA_EARG;
    if (K < 1 || K > kMaxK || !f || !y || !alphas || !sums) return set_err(c, QDTA_EARG, "bad arguments");
    if (c->net_dirty || c->dem_dirty)
        return set_err(c, QDTA_ESTATE, "lay the context out first (e.g. qdta_layout): this call allocates nothing");
    const int ni = (int)c->inst.size();
    const int64_t words = (int64_t)ni * K * 6;
    if (words > kNoAllocWords - kNoAllocFlagWords)
        return set_err(c, QDTA_EARG, "n_instances x K = %d x %d exceeds the static scratch (at most %d sums)", ni, K,
                       (kNoAllocWords - kNoAllocFlagWords) / 6);
    int* flags = reinterpret_cast<int*>(c->noalloc);
    long long* acc = c->noalloc + kNoAllocFlagWords;
    // the scratch keeps the last call's contents: clear the flags and the
    // accumulators this call uses (a fill kernel, safe under graph capture)
    HIPCHECK(c, launch_fill_i64(c->stream, reinterpret_cast<int64_t*>(c->noalloc), 0, kNoAllocFlagWords + words));
    HIPCHECK(c, launch_ls_eval(c->stream, net_view(c, o), f, y, o->alpha, o->beta, K, alphas, acc, nullptr, 0, flags));
    HIPCHECK(c, launch_ls_export(c->stream, ni, acc, K, sums));
    int h[4];
    HIPCHECK(c, hipMemcpyAsync(h, flags, 4 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return flag_code(c, h);
}

int qdta_line_search(qdta_ctx* c, const qdta_opts* o, const int64_t* f, const int64_t* y, int32_t j,
                     double* alpha_out) {
    if (!c) return QDTA_EARG;
    c->err.clear();
    if (!opts_ok(c, o)) return QDTA_EARG;
    if (!f || !y || !alpha_out || j < 1) return set_err(c, QDTA_EARG, "bad arguments");
    RC(ensure_network(c));
    if (c->dem_dirty) RC(ensure_demand(c, waves_per_cu(o), tree_waves(o), uses_contraction(o)));
    int ni = (int)c->inst.size();
    RC(init_state(c, true, j));
    RC(clear_flags(c));
    RC(line_search_core(c, o, f, y));
    HIPCHECK(c, launch_copy_alpha(c->stream, ni, c->st.p, alpha_out));
    int h[4];
    RC(read_flags(c, h));
    RC(flag_code(c, h));
    RC(pull_state(c));
    return QDTA_OK;
}

int qdta_fw_update(qdta_ctx* c, int64_t* f, const int64_t* y, const double* alpha) {
    if (!c) return QDTA_EARG;
    c->err.clear();
    if (!f || !y || !alpha) return set_err(c, QDTA_EARG, "null array");
    RC(ensure_network(c));
    HIPCHECK(c, launch_fw_update(c->stream, net_view(c), f, y, alpha, nullptr));
    return QDTA_OK;
}

int qdta_fw_begin(qdta_ctx* c, const qdta_opts* o) {
    if (!c) return QDTA_EARG;
    c->err.clear();
    if (!opts_ok(c, o)) return QDTA_EARG;
    for (const Instance& I : c->inst)
        if (!I.has_demand) return set_err(c, QDTA_ESTATE, "every instance needs qdta_set_demand before solving");
    RC(ensure_demand(c, waves_per_cu(o), tree_waves(o), uses_contraction(o)));
    RC(apply_rule(c, o));
    RC(ensure_sweep(c, o));
    RC(ensure_contract(c, o));
    NetDev net = net_view(c, o);
    RC(init_state(c, false, 0));
    RC(clear_flags(c));
    c->solve_id++;
    // costs of iterates 0..cap+1 (the last one is tested, not applied)
    if (o->keep_history) RC(ensure_history(c, c->ws_base ? (size_t)hist_iters(o) + 2 : 8));
    for (Instance& I : c->inst) {
        I.hist_alpha.assign(1, 1.0);
        I.solved_iters = -1;
    }
    // initial AON at free flow: BPR(0) = c0 exactly (first step of Alg. 6)
    HIPCHECK(c, launch_fill_i64(c->stream, c->f.p, 0, c->M));
    RC(prof_mark(c, PH_BPR, 0));
    float* tc = o->objective == QDTA_OBJ_SO ? c->tcost.p : nullptr;
    HIPCHECK(c, launch_bpr(c->stream, net, c->f.p, o->alpha, o->beta, c->cost.p, c->radj.p, c->st.p, 1, c->flags.p,
                           tc));
    RC(prof_mark(c, PH_BPR, 1));
    c->lab_hist_ok.clear();
    if (o->keep_history) RC(plan_label_history(c, o));
    RC(aon_core(c, o, c->cost.p, tc, c->f.p, nullptr, c->st.p));
    if (o->keep_history) {
        HIPCHECK(c, hipMemcpyAsync(c->hist_cost.p, c->cost.p, sizeof(float) * c->M, hipMemcpyDeviceToDevice, c->stream));
        RC(stash_labels(c, 0));
    }
    c->fw_j = 0;
    c->fw_live = true;
    c->solved = false;
    RC(pull_state(c));
    prof_collect(c);
    return QDTA_OK;
}

namespace {

void fill_stats(qdta_ctx* c, qdta_stats* hs, int worst, const int* h) {
    int ni = (int)c->inst.size();
    for (int i = 0; i < ni && hs; ++i) {
        const InstState& s = c->h_st[i];
        qdta_stats& q = hs[i];
        q.iters = s.iters;
        q.ls_evals = s.ls_evals;
        q.qn_iters = s.qn_iters;
        q.absorb = h[2] ? 1 : 0;
        q.stopped_by = s.stopped_by;
        q.status = worst;
        q.gap = s.active ? s.gap : 0.0;
        q.objective = s.obj;
        q.last_alpha = s.last_alpha;
    }
}

// The kernels of one Frank-Wolfe iteration (Alg. 6): BPR, AON, stop test,
// line search, update, for every live instance.  No host synchronisation
// unless the quasi-Newton search is selected.
int enqueue_iteration(qdta_ctx* c, const qdta_opts* o, bool marks) {
    int ni = (int)c->inst.size();
    NetDev net = net_view(c, o);
    int* err = c->flags.p;
    const int cap_iter = o->fixed_iters > 0 ? o->fixed_iters : o->max_iter;
    if (marks) RC(prof_mark(c, PH_BPR, 0));
    float* tc = o->objective == QDTA_OBJ_SO ? c->tcost.p : nullptr;
    HIPCHECK(c, launch_bpr(c->stream, net, c->f.p, o->alpha, o->beta, c->cost.p, c->radj.p, c->st.p, 1, err, tc));
    if (marks) RC(prof_mark(c, PH_BPR, 1));
    RC(aon_core(c, o, c->cost.p, tc, c->y.p, nullptr, c->st.p, marks));
    if (marks) RC(prof_mark(c, PH_GAP, 0));
    HIPCHECK(c, launch_fill_i64(c->stream, reinterpret_cast<int64_t*>(c->acc.p), 0, (int64_t)ni * 6));
    HIPCHECK(c, launch_gap_sums(c->stream, net, c->cost.p, c->f.p, c->y.p, c->acc.p, c->st.p, err));
    HIPCHECK(c, launch_gap_decide(c->stream, ni, c->acc.p, c->st.p, o->stop_rule, o->tol, o->fixed_iters, cap_iter));
    if (marks) RC(prof_mark(c, PH_GAP, 1));
    if (marks) RC(prof_mark(c, PH_LS, 0));
    RC(line_search_core(c, o, c->f.p, c->y.p));
    if (o->stop_rule == QDTA_STOP_OBJ && o->fixed_iters <= 0) {
        HIPCHECK(c, launch_fill_i64(c->stream, reinterpret_cast<int64_t*>(c->acc.p), 0, (int64_t)ni * 6));
        HIPCHECK(c, launch_obj_pair(c->stream, net, c->f.p, c->y.p, o->alpha, o->beta, c->acc.p, c->st.p, 1, err));
        HIPCHECK(c, launch_obj_decide(c->stream, ni, c->acc.p, c->st.p, o->tol, 1));
    }
    HIPCHECK(c, launch_stall_check(c->stream, ni, c->st.p, o->fixed_iters));
    if (marks) RC(prof_mark(c, PH_LS, 1));
    if (marks) RC(prof_mark(c, PH_UPDATE, 0));
    HIPCHECK(c, launch_copy_alpha(c->stream, ni, c->st.p, c->alpha_arr.p));
    HIPCHECK(c, launch_fw_update(c->stream, net, c->f.p, c->y.p, c->alpha_arr.p, c->st.p));
    HIPCHECK(c, launch_after_update(c->stream, ni, c->st.p));
    if (marks) RC(prof_mark(c, PH_UPDATE, 1));
    return QDTA_OK;
}

bool graph_form(const qdta_opts* o) { return o->launch_form == 0 && o->ls_mode != QDTA_LS_QN; }

void drop_graph(qdta_ctx* c) {
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
}

// Capture one iteration on a side stream; the graph is then launched on the
// context's stream (which may be the null stream, which cannot capture).
int capture_once(qdta_ctx* c, const qdta_opts* o) {
    drop_graph(c);
    if (!c->cap_stream) HIPCHECK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t saved = c->stream;
    c->stream = c->cap_stream;
    for (int p = 0; p < kPhases; ++p) c->prof_open[p] = 0;
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    int rc = e == hipSuccess ? enqueue_iteration(c, o, false) : QDTA_EHIP;
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
    c->stream = saved;
    for (int p = 0; p < kPhases; ++p) c->prof_open[p] = 0;
    if (e != hipSuccess) return set_err(c, QDTA_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    if (rc < 0) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e2 != hipSuccess) return set_err(c, QDTA_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e2));
    c->graph = g;
    HIPCHECK(c, hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0));
    c->graph_gen = c->gen;
    c->graph_opts = *o;
    return QDTA_OK;
}

// Phase events stay out of the graph (event nodes cannot be timed), so a
// profiled replay reports only the whole iteration.
int capture_iteration(qdta_ctx* c, const qdta_opts* o) { return capture_once(c, o); }

// One Frank-Wolfe iteration j, then one host synchronisation.
int fw_iteration(qdta_ctx* c, const qdta_opts* o, int* h) {
    int ni = (int)c->inst.size();
    const int j = ++c->fw_j;
    if (graph_form(o)) {
        if (!c->graph_exec || c->graph_gen != c->gen || memcmp(&c->graph_opts, o, sizeof(qdta_opts)) != 0)
            RC(capture_iteration(c, o));
        RC(prof_mark(c, PH_GRAPH, 0));
        HIPCHECK(c, hipGraphLaunch(c->graph_exec, c->stream));
        RC(prof_mark(c, PH_GRAPH, 1));
    } else {
        RC(enqueue_iteration(c, o, true));
    }
    if (o->keep_history) {
        RC(ensure_history(c, (size_t)j + 1));
        HIPCHECK(c, hipMemcpyAsync(c->hist_cost.p + (size_t)j * c->M, c->cost.p, sizeof(float) * c->M,
                                   hipMemcpyDeviceToDevice, c->stream));
        RC(stash_labels(c, j));
    }
    HIPCHECK(c, hipMemcpyAsync(h, c->flags.p, 4 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    RC(pull_state(c));
    prof_collect(c);
    RC(flag_code(c, h));
    bool live = false;
    for (int i = 0; i < ni; ++i) {
        const InstState& s = c->h_st[i];
        if (!s.active) continue;
        if (!s.converged) {
            live = true;
            c->inst[i].hist_alpha.push_back(s.alpha);
        }
    }
    c->fw_live = live;
    return QDTA_OK;
}

int fw_finish(qdta_ctx* c, const qdta_opts* o, qdta_stats* hs) {
    int ni = (int)c->inst.size();
    NetDev net = net_view(c, o);
    int h[4];
    // objective of the returned iterates
    HIPCHECK(c, launch_fill_i64(c->stream, reinterpret_cast<int64_t*>(c->acc.p), 0, (int64_t)ni * 6));
    HIPCHECK(c, launch_obj_pair(c->stream, net, c->f.p, c->y.p, o->alpha, o->beta, c->acc.p, c->st.p, 0, c->flags.p));
    HIPCHECK(c, launch_obj_decide(c->stream, ni, c->acc.p, c->st.p, o->tol, 0));
    HIPCHECK(c, hipMemcpyAsync(h, c->flags.p, 4 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    RC(pull_state(c));
    int worst = flag_code(c, h);
    for (int i = 0; i < ni; ++i) {
        const InstState& s = c->h_st[i];
        c->inst[i].solved_iters = s.iters;
        c->inst[i].hist_alpha.resize((size_t)s.iters + 1);
    }
    fill_stats(c, hs, worst, h);
    c->solved = true;
    if (worst < 0) return worst;
    return h[2] ? QDTA_WABSORB : QDTA_OK;
}

}  // namespace

int qdta_fw_step(qdta_ctx* c, const qdta_opts* o, qdta_stats* hs, int32_t* live_out) {
    if (!c) return QDTA_EARG;
    c->err.clear();
    if (!opts_ok(c, o)) return QDTA_EARG;
    if (c->fw_j < 0 || c->dem_dirty) return set_err(c, QDTA_ESTATE, "qdta_fw_step needs qdta_fw_begin");
    RC(ensure_sweep(c, o));
    RC(ensure_contract(c, o));
    int h[4] = {0, 0, 0, 0};
    if (c->fw_live) RC(fw_iteration(c, o, h));
    else {
        HIPCHECK(c, hipMemcpyAsync(h, c->flags.p, 4 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
        RC(pull_state(c));
    }
    for (int i = 0; i < (int)c->inst.size(); ++i) c->inst[i].solved_iters = c->h_st[i].iters;
    fill_stats(c, hs, QDTA_OK, h);
    c->solved = true;
    if (live_out) *live_out = c->fw_live ? 1 : 0;
    return h[2] ? QDTA_WABSORB : QDTA_OK;
}

int qdta_solve(qdta_ctx* c, const qdta_opts* o, qdta_stats* hs) {
    RC(qdta_fw_begin(c, o));
    int h[4];
    while (c->fw_live) RC(fw_iteration(c, o, h));
    return fw_finish(c, o, hs);
}

int qdta_autotune(qdta_ctx* c, qdta_opts* o, double budget_ms, double* best_ms_out) {
    if (!c) return QDTA_EARG;
    c->err.clear();
    if (!opts_ok(c, o)) return QDTA_EARG;
    if (!(budget_ms > 0.0)) return set_err(c, QDTA_EARG, "budget_ms must be > 0");
    for (const Instance& I : c->inst)
        if (!I.has_demand) return set_err(c, QDTA_ESTATE, "autotune needs the demand of every instance");
    RC(ensure_demand(c, waves_per_cu(o), 1,               // slots for either kernel form
                     o->sssp_kernel == 0 || o->sssp_kernel == 4));
    RC(apply_rule(c, o));
    if (o->sssp_kernel == 0 || o->sssp_kernel == 4)       // trials of either tree form
        RC(ensure_contraction(c, c->h_dest_node.data(), c->h_dest_node.size()));
    NetDev net = net_view(c, o);
    DemDev dem = dem_view(c);
    // trial costs: BPR of the current flows while a solve runs or after one,
    // else free flow
    if (!c->solved && c->fw_j < 0) HIPCHECK(c, launch_fill_i64(c->stream, c->f.p, 0, c->M));
    RC(clear_flags(c));
    HIPCHECK(c, launch_bpr(c->stream, net, c->f.p, o->alpha, o->beta, c->cost.p, c->radj.p, nullptr, 0, c->flags.p));
    hipEvent_t e0, e1;
    HIPCHECK(c, hipEventCreate(&e0));
    HIPCHECK(c, hipEventCreate(&e1));
    static const int shapes[] = {3, 4, 2, 5};
    static const double scales[] = {10.0, 5.0, 20.0, 2.5, 1.25};
    static const int tws[] = {4, 1};
    // trial order: the bucket widths at the starting shape first (on heavily
    // congested networks the width matters most and trials are slow), then
    // every shape at every width, then one wavefront per tree
    struct Trial { int shape; double scale; int tw; };
    std::vector<Trial> trials;
    // the starting configuration (the caller's, else the defaults) is trial
    // -1, after an untimed launch that takes the first-touch costs; another
    // replaces it only when at least 5% faster (single trials vary by about
    // 2%), so near-ties do not flip the choice from run to run
    const int start_shape = o->sssp_shape ? o->sssp_shape : 3, start_tw = o->tree_waves ? o->tree_waves : 4;
    const double start_scale = delta_scale(o);
    for (double sc : scales)
        if (sc != start_scale) trials.push_back({start_shape, sc, start_tw});
    for (int tw : tws)
        for (double sc : scales)
            for (int sh : shapes)
                if (!(tw == start_tw && sh == start_shape)) trials.push_back({sh, sc, tw});
    int best_shape = start_shape, best_tw = start_tw;
    double best_scale = start_scale, best = 1e300, start_ms = 1e300, spent = 0.0;
    int rc = QDTA_OK;
    for (int k = -2; k < (int)trials.size() && rc == QDTA_OK && (k < 0 || spent < budget_ms); ++k) {
        qdta_opts t = *o;
        t.sssp_shape = k < 0 ? start_shape : trials[k].shape;
        t.delta_scale = k < 0 ? start_scale : trials[k].scale;
        t.tree_waves = k < 0 ? start_tw : trials[k].tw;
        const int sh = t.sssp_shape, tw = t.tree_waves;
        const double sc = t.delta_scale;
        // the trial's own occupancy (the scratch, sized for one wavefront per
        // tree, covers both forms; launches never exceed it)
        int ts = (int)std::min<int64_t>((int64_t)std::max<int64_t>(c->Q, 1) * (tw == 1 ? 1 : 4),
                                        (int64_t)c->cus * waves_per_cu(&t));
        ts = (ts + 3) / 4 * 4;
        hipError_t e = hipEventRecord(e0, c->stream);
        if (e == hipSuccess)
            e = launch_sssp(c->stream, net, dem, c->cost.p, c->radj.p, c->labels.p, scr_view(c), ts, nullptr,
                            delta_scale(&t), c->delta_inst.p, c->logsum.p, sssp_variant(c, &t), 1);
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) { rc = set_err(c, QDTA_EHIP, "autotune trial: %s", hipGetErrorString(e)); break; }
        if (k == -2) continue;                     // warm-up
        spent += ms;
        if (k == -1) start_ms = ms;
        if (ms < best) { best = ms; best_shape = sh; best_scale = sc; best_tw = tw; }
    }
    if (rc == QDTA_OK && best > 0.95 * start_ms) {
        best = start_ms;
        best_shape = start_shape;
        best_scale = start_scale;
        best_tw = start_tw;
    }
    // plain intervals: loading by per-leg walks or by merged paths, on the
    // labels of the last trial (the trees do not depend on the trial)
    int best_load = o->load_form;
    if (rc == QDTA_OK && o->load_form == 0) {
        qdta_opts ts = *o;
        ts.load_form = 2;
        if (use_sweep(c, &ts)) {
            rc = ensure_sweep(c, &ts);
            float ms_w = 0.0f, ms_s = 0.0f;
            FlagsDev fl = flags_view(c);
            for (int k = 0; k < 4 && rc == QDTA_OK; ++k) {
                const bool sweep = k & 1;                   // walk, sweep, walk, sweep (first pair untimed)
                hipError_t e = launch_fill_i64(c->stream, c->y.p, 0, c->M);
                if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
                if (e == hipSuccess)
                    e = sweep ? launch_sweep(c->stream, net, dem, c->labels.p, c->y.p, nullptr, nullptr, nullptr, fl,
                                             c->sw_cnt.p, c->sw_acc.p)
                              : launch_walk(c->stream, net, dem, c->labels.p, nullptr, c->y.p, nullptr, nullptr, fl, 0,
                                            nullptr, nullptr, nullptr, 0, -1);
                if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.0f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) { rc = set_err(c, QDTA_EHIP, "autotune loading: %s", hipGetErrorString(e)); break; }
                if (k >= 2) (sweep ? ms_s : ms_w) = ms;
            }
            if (rc == QDTA_OK) best_load = ms_s < 0.95f * ms_w ? 2 : 1;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc < 0) return rc;
    o->sssp_shape = best_shape;
    o->delta_scale = best_scale;
    o->tree_waves = best_tw;
    o->load_form = best_load;
    if (best_ms_out) *best_ms_out = best;
    return QDTA_OK;
}

int qdta_profile_enable(qdta_ctx* c, int32_t on) {
    if (!c) return QDTA_EARG;
    for (int p = 0; p < kPhases; ++p) {
        c->prof_ms[p] = 0.0;
        c->prof_n[p] = 0;
        c->prof_open[p] = 0;
        if (on && !c->prof_ev[p][0]) {
            HIPCHECK(c, hipEventCreate(&c->prof_ev[p][0]));
            HIPCHECK(c, hipEventCreate(&c->prof_ev[p][1]));
        }
    }
    c->prof_on = on ? 1 : 0;
    if (c->sssp_stats.p)
        HIPCHECK(c, launch_fill_i64(c->stream, reinterpret_cast<int64_t*>(c->sssp_stats.p), 0, 2));
    return QDTA_OK;
}

int qdta_profile_read(qdta_ctx* c, qdta_profile* out) {
    if (!c || !out) return QDTA_EARG;
    memset(out, 0, sizeof(*out));
    for (int p = 0; p < kPhases; ++p) {
        out->ms[p] = c->prof_ms[p];
        out->count[p] = c->prof_n[p];
    }
    if (c->sssp_stats.p) {
        unsigned long long h[2] = {0, 0};
        HIPCHECK(c, hipMemcpyAsync(h, c->sssp_stats.p, sizeof(h), hipMemcpyDeviceToHost, c->stream));
        HIPCHECK(c, hipStreamSynchronize(c->stream));
        out->sssp_nodes = (int64_t)h[0];
        out->sssp_links = (int64_t)h[1];
    }
    return QDTA_OK;
}

int qdta_get_flows(qdta_ctx* c, int64_t* f) {
    if (!c || !f) return QDTA_EARG;
    if (!c->solved && c->fw_j < 0) return set_err(c, QDTA_ESTATE, "no solved or running interval");
    HIPCHECK(c, hipMemcpyAsync(f, c->f.p, sizeof(int64_t) * c->M, hipMemcpyDeviceToDevice, c->stream));
    return QDTA_OK;
}

int qdta_get_costs(qdta_ctx* c, const qdta_opts* o, float* cost) {
    if (!c || !cost) return QDTA_EARG;
    if (!opts_ok(c, o)) return QDTA_EARG;
    if (!c->solved && c->fw_j < 0) return set_err(c, QDTA_ESTATE, "no solved or running interval");
    HIPCHECK(c, launch_bpr(c->stream, net_view(c), c->f.p, o->alpha, o->beta, cost, nullptr, nullptr, 0, c->flags.p));
    return QDTA_OK;
}

int qdta_advance_interval(qdta_ctx* c, const qdta_opts* o) {
    if (!c) return QDTA_EARG;
    c->err.clear();
    if (!opts_ok(c, o)) return QDTA_EARG;
    if (!c->solved) return set_err(c, QDTA_ESTATE, "advance needs a solved interval");
    if (!o->keep_history) return set_err(c, QDTA_ESTATE, "advance needs keep_history during solve");
    RC(apply_rule(c, o));
    RC(ensure_contract(c, o));
    int ni = (int)c->inst.size();
    NetDev net = net_view(c);
    DemDev dem = dem_view(c);
    FlagsDev fl = flags_view(c);
    RC(clear_flags(c));
    // final costs c_fin = BPR(f)
    HIPCHECK(c, launch_bpr(c->stream, net, c->f.p, o->alpha, o->beta, c->cfin.p, nullptr, nullptr, 0, c->flags.p));
    int J = 0;
    for (const Instance& I : c->inst) J = std::max(J, I.solved_iters);
    // lambda_j = alpha_j prod_{k>j} (1 - alpha_k), alpha_0 = 1, per instance;
    // instances with fewer iterations sit out.  All iterates' states go up
    // at once, so the passes below queue without host round trips.
    std::vector<InstState> hst((size_t)(J + 1) * ni);
    std::vector<double> hlam((size_t)(J + 1) * ni, 0.0);
    std::vector<char> any(J + 1, 0);
    for (int j = 0; j <= J; ++j) {
        for (int i = 0; i < ni; ++i) {
            const Instance& I = c->inst[i];
            InstState& s = hst[(size_t)j * ni + i];
            memset(&s, 0, sizeof(s));
            if (I.solved_iters >= j && c->h_inst[i].nleg > 0) {
                double l = (j == 0) ? 1.0 : I.hist_alpha[j];
                for (int k = j + 1; k <= I.solved_iters; ++k) l = l * (1.0 - I.hist_alpha[k]);
                hlam[(size_t)j * ni + i] = l;
                s.active = l > 0.0;
            }
            any[j] |= s.active != 0;
        }
    }
    // with a workspace: room for every iterate the options allow, carved once
    const size_t hcap = c->ws_base ? (size_t)(hist_iters(o) + 1) * ni : hst.size();
    RC(dalloc(c, c->st_hist, std::max(hst.size(), hcap)));
    RC(dalloc(c, c->lam_hist, std::max(hlam.size(), hcap)));
    HIPCHECK(c, hipMemcpy(c->st_hist.p, hst.data(), sizeof(InstState) * hst.size(), hipMemcpyHostToDevice));
    HIPCHECK(c, hipMemcpy(c->lam_hist.p, hlam.data(), sizeof(double) * hlam.size(), hipMemcpyHostToDevice));
    {
        // a reallocated buffer (possibly at the same address) holds anything
        const size_t before = c->r_dense.n;
        RC(dalloc(c, c->r_dense, c->label_count));
        if (c->r_dense.n != before) c->r_dense_zero = 0;
    }
    if (c->r_dense_zero < c->label_count) {
        HIPCHECK(c, launch_fill_i64(c->stream, c->r_dense.p, 0, (int64_t)c->label_count));
        c->r_dense_zero = c->label_count;
    }
    // the walks write only inside the current trees' rows, and the compaction
    // clears every word it finds non-zero there; until it has, nothing is known
    const size_t zero_after = c->r_dense_zero;
    c->r_dense_zero = 0;
    HIPCHECK(c, launch_fill_i64(c->stream, reinterpret_cast<int64_t*>(c->done_fx.p), 0, ni));
    // the link-progress rule leaves legs on links: they go to a transit list
    // (at most one entry per iterate and leg)
    bool progress = false;
    for (int i = 0; i < ni; ++i) progress |= c->h_inst[i].rule == QDTA_RULE_PROGRESS;
    TransitOut tr{nullptr, nullptr, nullptr, nullptr, nullptr, 0u};
    if (progress) {
        const size_t cap = plan_legs(c, (size_t)(J + 1) * (size_t)std::max<int64_t>(c->P, 1));
        if (cap >= UINT32_MAX) return set_err(c, QDTA_EARG, "too many legs in transit for one pass");
        RC(dalloc(c, c->tr_q, cap));
        RC(dalloc(c, c->tr_node, cap));
        RC(dalloc(c, c->tr_delay, cap));
        RC(dalloc(c, c->tr_w, cap));
        RC(dalloc(c, c->tr_n, 1));
        HIPCHECK(c, launch_fill_u32(c->stream, c->tr_n.p, 0u, 1));
        tr = TransitOut{c->tr_q.p, c->tr_node.p, c->tr_delay.p, c->tr_w.p, c->tr_n.p, (unsigned int)cap};
    }
    for (int j = 0; j <= J; ++j) {
        if (!any[j]) continue;
        const InstState* stj = c->st_hist.p + (size_t)j * ni;
        const double* lamj = c->lam_hist.p + (size_t)j * ni;
        const float* cj = c->hist_cost.p + (size_t)j * c->M;
        label_t* lab = c->labels.p;
        // the trees' costs c_j into the link records (the walk's tight test reads them)
        HIPCHECK(c, launch_scatter_rcost(c->stream, net, cj, c->radj.p));
        if ((size_t)j < c->lab_hist_ok.size() && c->lab_hist_ok[j]) {
            lab = c->lab_hist.p + (size_t)j * c->label_count;    // the solve's own trees of iterate j
        } else {
            HIPCHECK(c, launch_sssp(c->stream, net, dem, cj, c->radj.p, c->labels.p, scr_view(c), c->slots, stj,
                                    delta_scale(o), c->delta_inst.p, c->logsum.p, sssp_variant(c, o), 1));
        }
        HIPCHECK(c, launch_fill_u32(c->stream, reinterpret_cast<uint32_t*>(c->absorb_q.p), 0u, c->Q));
        HIPCHECK(c, launch_walk(c->stream, net, dem, lab, c->cfin.p, nullptr, nullptr, stj, fl, 1, lamj,
                                c->r_dense.p, c->done_fx.p, 0, -1, nullptr, progress ? &tr : nullptr));
        HIPCHECK(c, launch_fallback(c->stream, net, dem, lab, cj, c->cfin.p, nullptr, nullptr, stj, fl,
                                    scr_view(c), (int)std::min<int64_t>(c->scr_slots, std::max<int64_t>(c->Q, 1)), 1,
                                    lamj, c->r_dense.p, c->done_fx.p, 0, nullptr, 0, nullptr,
                                    progress ? &tr : nullptr));
    }
    // compact: legs per tree, offsets, then the legs in (destination, origin) order
    RC(dalloc(c, c->r_cnt, plan_dests(c, (size_t)std::max<int64_t>(c->Q, 1))));
    HIPCHECK(c, launch_resid_count(c->stream, net, dem, c->r_dense.p, c->r_cnt.p));
    std::vector<int64_t> cnt((size_t)c->Q), off((size_t)c->Q);
    if (c->Q) HIPCHECK(c, hipMemcpyAsync(cnt.data(), c->r_cnt.p, sizeof(int64_t) * c->Q, hipMemcpyDeviceToHost,
                                         c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    int64_t total = 0;
    for (int64_t t = 0; t < c->Q; ++t) {
        off[t] = total;
        total += cnt[t];
    }
    const size_t rn = plan_legs(c, (size_t)std::max<int64_t>(total, 1));
    RC(dalloc(c, c->r_orig, rn));
    RC(dalloc(c, c->r_dest, rn));
    RC(dalloc(c, c->r_w, rn));
    if (c->Q) HIPCHECK(c, hipMemcpy(c->r_cnt.p, off.data(), sizeof(int64_t) * c->Q, hipMemcpyHostToDevice));
    HIPCHECK(c, launch_resid_write(c->stream, net, dem, c->r_dense.p, c->r_cnt.p, c->r_orig.p, c->r_dest.p,
                                   c->r_w.p));
    std::vector<int32_t> ho((size_t)total), hq((size_t)total);
    std::vector<int64_t> hw((size_t)total);
    if (total) {
        HIPCHECK(c, hipMemcpyAsync(ho.data(), c->r_orig.p, sizeof(int32_t) * total, hipMemcpyDeviceToHost, c->stream));
        HIPCHECK(c, hipMemcpyAsync(hq.data(), c->r_dest.p, sizeof(int32_t) * total, hipMemcpyDeviceToHost, c->stream));
        HIPCHECK(c, hipMemcpyAsync(hw.data(), c->r_w.p, sizeof(int64_t) * total, hipMemcpyDeviceToHost, c->stream));
    }
    std::vector<unsigned long long> done(ni);
    HIPCHECK(c, hipMemcpyAsync(done.data(), c->done_fx.p, sizeof(unsigned long long) * ni, hipMemcpyDeviceToHost,
                               c->stream));
    unsigned int ntr = 0;
    std::vector<int32_t> tq, tnode;
    std::vector<float> tdl;
    std::vector<int64_t> tw;
    if (progress) {
        HIPCHECK(c, hipMemcpyAsync(&ntr, c->tr_n.p, sizeof(ntr), hipMemcpyDeviceToHost, c->stream));
        HIPCHECK(c, hipStreamSynchronize(c->stream));
        ntr = std::min(ntr, tr.cap);
        tq.resize(ntr); tnode.resize(ntr); tdl.resize(ntr); tw.resize(ntr);
        if (ntr) {
            HIPCHECK(c, hipMemcpyAsync(tq.data(), c->tr_q.p, sizeof(int32_t) * ntr, hipMemcpyDeviceToHost, c->stream));
            HIPCHECK(c, hipMemcpyAsync(tnode.data(), c->tr_node.p, sizeof(int32_t) * ntr, hipMemcpyDeviceToHost,
                                       c->stream));
            HIPCHECK(c, hipMemcpyAsync(tdl.data(), c->tr_delay.p, sizeof(float) * ntr, hipMemcpyDeviceToHost,
                                       c->stream));
            HIPCHECK(c, hipMemcpyAsync(tw.data(), c->tr_w.p, sizeof(int64_t) * ntr, hipMemcpyDeviceToHost, c->stream));
        }
    }
    int h[4];
    RC(read_flags(c, h));                  // synchronises the stream
    c->r_dense_zero = zero_after;
    // trees are instance-major, so each instance's legs are one run
    int64_t k = 0;
    for (int i = 0; i < ni; ++i) {
        Instance& I = c->inst[i];
        const int64_t end = c->dest_off[i + 1];
        int64_t k1 = k;
        while (k1 < total && hq[k1] < end) ++k1;
        I.r_orig.assign(ho.begin() + k, ho.begin() + k1);
        I.r_dest.resize(k1 - k);
        for (int64_t x = k; x < k1; ++x) I.r_dest[x - k] = c->h_dest_node[hq[x]] - c->h_inst[i].node0;
        I.r_w.assign(hw.begin() + k, hw.begin() + k1);
        I.r_delay.assign((size_t)(k1 - k), 0.0f);
        I.r_done = (int64_t)done[i];
        k = k1;
    }
    if (ntr) {
        // legs on links join their instance's residual; the merge sorts by
        // (destination, origin, delay) and adds up equal legs
        for (unsigned int x = 0; x < ntr; ++x) {
            const int qi = tq[x];
            Instance& I = c->inst[c->h_dest_inst[qi]];
            I.r_orig.push_back(tnode[x]);
            I.r_dest.push_back(c->h_dest_node[qi] - c->h_inst[c->h_dest_inst[qi]].node0);
            I.r_w.push_back(tw[x]);
            I.r_delay.push_back(tdl[x]);
        }
        for (Instance& I : c->inst) merge_legs(I.r_orig, I.r_dest, I.r_w, I.r_delay);
    }
    c->solved = false;
    RC(flag_code(c, h));
    return h[2] ? QDTA_WABSORB : QDTA_OK;
}

int qdta_get_residual(qdta_ctx* c, int32_t inst, int64_t* count, int32_t* ho, int32_t* hd, int64_t* hw,
                      int64_t* done, float* ht) {
    if (!c || !count) return QDTA_EARG;
    if (inst < 0 || inst >= (int32_t)c->inst.size()) return set_err(c, QDTA_EARG, "no instance %d", inst);
    const Instance& I = c->inst[inst];
    *count = (int64_t)I.r_orig.size();
    if (done) *done = I.r_done;
    if (ho) std::copy(I.r_orig.begin(), I.r_orig.end(), ho);
    if (hd) std::copy(I.r_dest.begin(), I.r_dest.end(), hd);
    if (hw) std::copy(I.r_w.begin(), I.r_w.end(), hw);
    if (ht) std::copy(I.r_delay.begin(), I.r_delay.end(), ht);
    return QDTA_OK;
}

// ---------------------------------------------------------------------------
// Frozen-path model and its reverse pass (OD calibration)
// ---------------------------------------------------------------------------
static bool adj_valid(const qdta_ctx* c) {
    return c->adj_J >= 0 && c->adj_gen == c->gen && c->adj_solve == c->solve_id && !c->dem_dirty && !c->net_dirty;
}

int qdta_adjoint_record(qdta_ctx* c, const qdta_opts* o) {
    if (!c) return QDTA_EARG;
    c->err.clear();
    if (!opts_ok(c, o)) return QDTA_EARG;
    if (o->trunc_rule == QDTA_RULE_PROGRESS)
        return set_err(c, QDTA_EARG, "the frozen-path model does not take the link-progress rule");
    if (c->inst.size() != 1) return set_err(c, QDTA_ESTATE, "the frozen-path model takes exactly one instance");
    if (o->objective != QDTA_OBJ_UE) return set_err(c, QDTA_ESTATE, "the frozen-path model is the user equilibrium's");
    if (!c->solved || c->dem_dirty) return set_err(c, QDTA_ESTATE, "record needs a solved interval");
    if (!o->keep_history) return set_err(c, QDTA_ESTATE, "record needs keep_history during solve");
    const Instance& I = c->inst[0];
    const int J = I.solved_iters;
    if (J < 0 || (int)I.hist_alpha.size() < J + 1 || c->hist_iters_cap < (size_t)J + 1)
        return set_err(c, QDTA_ESTATE, "no iteration history");
    RC(ensure_demand(c, waves_per_cu(o), tree_waves(o), uses_contraction(o)));
    RC(apply_rule(c, o));
    RC(ensure_contract(c, o));
    const int64_t P = c->P, M = c->M;
    c->adj_J = -1;
    c->adj_fwd = false;
    c->adj_ptr.resize((size_t)J + 1);
    c->adj_links.resize((size_t)J + 1);
    c->adj_leg.resize((size_t)J + 1);
    c->adj_total.assign((size_t)J + 1, 0);
    RC(dalloc(c, c->adj_len, (size_t)std::max<int64_t>(P, 1)));
    RC(dalloc(c, c->adj_f, (size_t)(J + 1) * M));
    RC(dalloc(c, c->adj_y, (size_t)(J + 1) * M));
    RC(dalloc(c, c->adj_cur, (size_t)M));
    RC(dalloc(c, c->adj_alpha, (size_t)J + 1));
    RC(dalloc(c, c->adj_fbar, (size_t)M));
    RC(dalloc(c, c->adj_ybar, (size_t)M));
    RC(dalloc(c, c->adj_part, 2 * 1024));
    RC(dalloc(c, c->adj_s, 1));
    RC(dalloc(c, c->adj_cap, (size_t)M));
    std::vector<int64_t> len((size_t)P), ptr((size_t)P + 1);
    for (int j = 0; j <= J; ++j) {
        NetDev net = net_view(c);
        DemDev dem = dem_view(c);
        const float* cj = c->hist_cost.p + (size_t)j * M;
        HIPCHECK(c, launch_scatter_rcost(c->stream, net, cj, c->radj.p));
        const label_t* lab = c->labels.p;
        if ((size_t)j < c->lab_hist_ok.size() && c->lab_hist_ok[j]) {
            lab = c->lab_hist.p + (size_t)j * c->label_count;   // the solve's own trees of iterate j
        } else {
            HIPCHECK(c, launch_sssp(c->stream, net, dem, cj, c->radj.p, c->labels.p, scr_view(c), c->slots, nullptr,
                                    delta_scale(o), c->delta_inst.p, c->logsum.p, sssp_variant(c, o), 1));
        }
        RC(clear_flags(c));
        HIPCHECK(c, launch_path_walk(c->stream, net, dem, lab, nullptr, nullptr, nullptr, c->adj_len.p,
                                     c->flags.p + 3));
        if (P) HIPCHECK(c, hipMemcpyAsync(len.data(), c->adj_len.p, sizeof(int64_t) * P, hipMemcpyDeviceToHost,
                                          c->stream));
        int h[4];
        RC(read_flags(c, h));
        if (h[3] & 1) return set_err(c, QDTA_EUNREACH, "iterate %d: a leg's origin cannot reach its destination", j);
        if (h[3] & 2) return set_err(c, QDTA_ESTATE, "iterate %d: FP32 absorption (tie fallback) on a path", j);
        ptr[0] = 0;
        for (int64_t l = 0; l < P; ++l) ptr[l + 1] = ptr[l] + len[l];
        RC(dalloc(c, c->adj_ptr[j], (size_t)P + 1));
        RC(dalloc(c, c->adj_links[j], (size_t)std::max<int64_t>(ptr[P], 1)));
        RC(dalloc(c, c->adj_leg[j], (size_t)std::max<int64_t>(ptr[P], 1)));
        c->adj_total[j] = ptr[P];
        HIPCHECK(c, hipMemcpyAsync(c->adj_ptr[j].p, ptr.data(), sizeof(int64_t) * (P + 1), hipMemcpyHostToDevice,
                                   c->stream));
        HIPCHECK(c, launch_path_walk(c->stream, net_view(c), dem_view(c), lab, c->adj_ptr[j].p, c->adj_links[j].p,
                                     c->adj_leg[j].p, nullptr, c->flags.p + 3));
        RC(read_flags(c, h));
        if (h[3]) return set_err(c, QDTA_ESTATE, "iterate %d: paths changed between the two walks", j);
    }
    c->adj_J = J;
    c->adj_gen = c->gen;
    c->adj_solve = c->solve_id;
    return QDTA_OK;
}

int qdta_model_forward(qdta_ctx* c, const qdta_opts* o, const double* d, const float* cap, double* f_out,
                       uint64_t* fwd_id_out) {
    if (!c) return QDTA_EARG;
    c->err.clear();
    if (!opts_ok(c, o)) return QDTA_EARG;
    if (!adj_valid(c)) return set_err(c, QDTA_ESTATE, "no recorded paths for the current solve (qdta_adjoint_record)");
    if (!d || !f_out) return set_err(c, QDTA_EARG, "null array");
    const int64_t M = c->M;
    const int J = c->adj_J;
    c->adj_fwd = false;
    HIPCHECK(c, hipMemcpyAsync(c->adj_cap.p, cap ? cap : c->cap.p, sizeof(float) * M, hipMemcpyDeviceToDevice,
                               c->stream));
    NetDev net = net_view(c);
    net.cap = c->adj_cap.p;
    RC(clear_flags(c));
    for (int j = 0; j <= J; ++j) {
        int64_t* yj = c->adj_y.p + (size_t)j * M;
        HIPCHECK(c, launch_fill_i64(c->stream, yj, 0, M));
        HIPCHECK(c, launch_path_load(c->stream, c->adj_total[j], c->adj_links[j].p, c->adj_leg[j].p, d, yj,
                                     c->flags.p));
        if (j == 0) {
            HIPCHECK(c, hipMemcpyAsync(c->adj_cur.p, yj, sizeof(int64_t) * M, hipMemcpyDeviceToDevice, c->stream));
            continue;
        }
        HIPCHECK(c, hipMemcpyAsync(c->adj_f.p + (size_t)j * M, c->adj_cur.p, sizeof(int64_t) * M,
                                   hipMemcpyDeviceToDevice, c->stream));
        RC(init_state(c, true, j));
        RC(line_search_core(c, o, c->adj_cur.p, yj, &net));
        HIPCHECK(c, launch_copy_alpha(c->stream, 1, c->st.p, c->adj_alpha.p + j));
        HIPCHECK(c, launch_fw_update(c->stream, net, c->adj_cur.p, yj, c->adj_alpha.p + j, nullptr));
    }
    HIPCHECK(c, launch_fx_to_veh(c->stream, M, c->adj_cur.p, f_out));
    int h[4];
    RC(read_flags(c, h));
    RC(flag_code(c, h));
    c->adj_fwd = true;
    c->adj_fwd_id++;
    if (fwd_id_out) *fwd_id_out = c->adj_fwd_id;
    c->adj_is_root = o->ls_mode != QDTA_LS_MSA;
    c->adj_ab = o->alpha;
    c->adj_beta = o->beta;
    return QDTA_OK;
}

int qdta_model_backward(qdta_ctx* c, uint64_t fwd_id, const double* fbar, double* dbar, double* capbar) {
    if (!c) return QDTA_EARG;
    c->err.clear();
    if (!adj_valid(c) || !c->adj_fwd) return set_err(c, QDTA_ESTATE, "backward needs a model forward pass first");
    if (fwd_id != c->adj_fwd_id)
        return set_err(c, QDTA_ESTATE, "backward of forward %llu, but the context holds forward %llu's iterates",
                       (unsigned long long)fwd_id, (unsigned long long)c->adj_fwd_id);
    if (!fbar || !dbar || !capbar) return set_err(c, QDTA_EARG, "null array");
    const int64_t M = c->M;
    const int P = (int)c->P, J = c->adj_J;
    NetDev net = net_view(c);
    net.cap = c->adj_cap.p;
    HIPCHECK(c, hipMemcpyAsync(c->adj_fbar.p, fbar, sizeof(double) * M, hipMemcpyDeviceToDevice, c->stream));
    HIPCHECK(c, launch_fill_i64(c->stream, reinterpret_cast<int64_t*>(capbar), 0, M));
    for (int j = J; j >= 1; --j) {
        HIPCHECK(c, launch_adj_step(c->stream, net, c->adj_f.p + (size_t)j * M, c->adj_y.p + (size_t)j * M,
                                    c->adj_alpha.p + j, c->adj_is_root, c->adj_ab, c->adj_beta, c->adj_fbar.p,
                                    c->adj_ybar.p, capbar, c->adj_part.p, c->adj_s.p));
        HIPCHECK(c, launch_path_gather(c->stream, P, c->adj_ptr[j].p, c->adj_links[j].p, c->adj_ybar.p, dbar,
                                       j != J));
    }
    HIPCHECK(c, launch_path_gather(c->stream, P, c->adj_ptr[0].p, c->adj_links[0].p, c->adj_fbar.p, dbar, J > 0));
    return QDTA_OK;
}

int qdta_set_residual(qdta_ctx* c, int32_t inst, int64_t count, const int32_t* ho, const int32_t* hd,
                      const int64_t* hw, const float* ht) {
    if (!c) return QDTA_EARG;
    c->err.clear();
    if (inst < 0 || inst >= (int32_t)c->inst.size()) return set_err(c, QDTA_EARG, "no instance %d", inst);
    if (count < 0 || (count > 0 && (!ho || !hd || !hw))) return set_err(c, QDTA_EARG, "bad residual legs");
    Instance& I = c->inst[inst];
    for (int64_t p = 0; p < count; ++p) {
        if (ho[p] < 0 || ho[p] >= I.n || hd[p] < 0 || hd[p] >= I.n || ho[p] == hd[p])
            return set_err(c, QDTA_EARG, "residual leg %lld: bad nodes", (long long)p);
        if (hw[p] <= 0) return set_err(c, QDTA_EARG, "residual leg %lld: weight <= 0", (long long)p);
        const float tp = ht ? ht[p] : 0.0f;
        if (!(tp >= 0.0f) || !std::isfinite(tp)) return set_err(c, QDTA_EARG, "residual leg %lld: bad delay", (long long)p);
        if (p > 0) {
            const float tq = ht ? ht[p - 1] : 0.0f;
            const auto a = std::make_tuple(hd[p - 1], ho[p - 1], __builtin_bit_cast(uint32_t, tq));
            const auto b = std::make_tuple(hd[p], ho[p], __builtin_bit_cast(uint32_t, tp));
            if (!(a < b))
                return set_err(c, QDTA_EARG, "residual leg %lld: not in (destination, origin, delay) order",
                               (long long)p);
        }
    }
    I.r_orig.assign(ho, ho + count);
    I.r_dest.assign(hd, hd + count);
    I.r_w.assign(hw, hw + count);
    if (ht) I.r_delay.assign(ht, ht + count);
    else I.r_delay.assign((size_t)count, 0.0f);
    I.r_done = 0;
    return QDTA_OK;
}

}  // extern "C"
