// qdta_kernels.hip -- gfx950 kernels of the QDTA hot path.
//
// One Frank-Wolfe iteration of the link-flow form (Alg. 6, section 5.1):
//   k_bpr        link costs by the BPR curve (Eq. 1)
//   k_sssp<SB>   destination-rooted FP32 shortest-path trees, SB trees per
//                workgroup (Get_shortest_path of Alg. 3 / Alg. 7)
//   k_walk       route truncation (Eq. 2) and loading along the successor
//                links (Eq. 5, Alg. 3), int64 fixed-point atomics
//   k_gap_sums   exact sums for the relative gap / stop test
//   k_ls_*       line search on the Beckmann objective (Eq. 6, Eq. 8-10,
//                Alg. 8-9), K step sizes per pass over the links
//   k_fw_update  f <- f + rint(alpha (y - f))
// plus the tie-rule fallback under FP32 absorption and the residual-demand
// walk of Alg. 4.
//
// Numeric contract: FP64 per-link arithmetic with no fused multiply-add (the
// library is compiled with -ffp-contract=off), power by repeated
// multiplication, FP32 min-plus with IEEE round-to-nearest adds, int64 flows
// in units of 2^-20 vehicle, decision sums exact as int128 multiples of 2^-16.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qdta_internal.h"

namespace qdta {

typedef __int128 i128;

#define RULE_NONE 0
#define RULE_CEIL 1
#define RULE_FLOOR 2

static constexpr double kFxInv = 1.0 / 1048576.0;   // 2^-20, exact
static constexpr double kSumQ = 65536.0;            // 2^16

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// Coherent (L2) load of a word that other waves update with atomics.
__device__ __forceinline__ uint32_t ld_coherent(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_coherent(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// round-half-even(x * 2^16) as int128; flags values that are not finite or
// beyond the int128 range.
__device__ __forceinline__ i128 quant(double x, int& bad) {
    double v = __builtin_rint(x * kSumQ);
    if (!(__builtin_fabs(v) < 1.7e38)) { bad = 1; return 0; }
    return (i128)v;
}

// Exact int128 accumulation with 64-bit atomics: the value is kept as three
// chunk sums, v = c2 * 2^84 + c1 * 2^42 + c0, each term split into a signed
// top part and two non-negative 42-bit parts.
__device__ __forceinline__ void acc3_add(long long* acc, i128 v) {
    const unsigned long long m42 = (1ull << 42) - 1;
    unsigned long long lo = (unsigned long long)v & m42;
    unsigned long long mid = (unsigned long long)(v >> 42) & m42;
    long long hi = (long long)(v >> 84);
    if (lo) atomicAdd((unsigned long long*)&acc[0], lo);
    if (mid) atomicAdd((unsigned long long*)&acc[1], mid);
    if (hi) atomicAdd((unsigned long long*)&acc[2], (unsigned long long)hi);
}

__device__ __forceinline__ i128 acc3_value(const long long* acc) {
    return (i128)acc[2] * ((i128)1 << 84) + (i128)acc[1] * ((i128)1 << 42) + (i128)acc[0];
}

__device__ __forceinline__ void put128(long long* out, i128 v) {
    out[0] = (long long)(unsigned long long)v;
    out[1] = (long long)(v >> 64);
}

__device__ __forceinline__ i128 get128(const long long* in) {
    return (i128)(((unsigned __int128)(unsigned long long)in[1] << 64) | (unsigned long long)in[0]);
}

// Workgroup sum of one int128 per thread, added to an exact accumulator.
__device__ void wg_acc_add(i128 v, long long* acc, i128* lds) {
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int s = kWG / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && lds[0] != 0) acc3_add(acc, lds[0]);
    __syncthreads();
}

// BPR curve (Eq. 1): c0 (1 + alpha (kappa F / C)^beta) in FP64.
__device__ __forceinline__ double bpr64(double F, float c0, float cap, double alpha, int beta, double kappa) {
    double r = (F * kappa) / (double)cap;
    double p = r;
    for (int k = 1; k < beta; ++k) p = p * r;
    return (double)c0 * (1.0 + alpha * p);
}

// Beckmann term and its derivative along the FW direction at step alpha.
__device__ __forceinline__ void ls_terms(double F, double Y, float c0, float cap, double ab, int beta, double kappa,
                                         double alpha, double& obj, double& der) {
    double t = Y - F;
    double v = F + alpha * t;
    double r = (v * kappa) / (double)cap;
    double p = r;
    for (int k = 1; k < beta; ++k) p = p * r;
    double cost = (double)c0 * (1.0 + ab * p);
    double g = ab * v;
    g = g * p;
    g = g / (double)(beta + 1);
    obj = (double)c0 * (v + g);
    der = t * cost;
}

// ---------------------------------------------------------------------------
// fills
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_i64(int64_t* p, int64_t v, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static int grid_for(int64_t count) {
    int64_t g = (count + kWG - 1) / kWG;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_fill_u32(hipStream_t s, uint32_t* p, uint32_t v, int64_t count) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(count)), dim3(kWG), 0, s, p, v, count);
    return hipGetLastError();
}
hipError_t launch_fill_i64(hipStream_t s, int64_t* p, int64_t v, int64_t count) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(count)), dim3(kWG), 0, s, p, v, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// A1: link costs (Eq. 1)
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool inst_live(const InstState* st, int i) {
    return st == nullptr || (st[i].active && !st[i].converged);
}

__global__ __launch_bounds__(kWG) void k_bpr(NetDev net, const int64_t* __restrict__ f, double alpha, int beta,
                                             float* __restrict__ cost, float* __restrict__ rcost,
                                             const InstState* st, int only_active, int* err) {
    const int b = blockIdx.x;
    const int inst = net.blk_inst[b];
    if (only_active && !inst_live(st, inst)) return;
    const InstDev I = net.inst[inst];
    const int a0 = net.blk_start[b];
    const int a1 = min(a0 + kChunk, I.link0 + I.m);
    int bad = 0;
    for (int a = a0 + threadIdx.x; a < a1; a += kWG) {
        double c = bpr64((double)f[a] * kFxInv, net.c0[a], net.cap[a], alpha, beta, I.kappa);
        float c32 = (float)c;
        if (!(c32 <= 3.4028234663852886e38f)) bad = 1;
        cost[a] = c32;
        if (rcost) rcost[net.revpos[a]] = c32;
    }
    if (bad) atomicOr(err, 1);
}

hipError_t launch_bpr(hipStream_t s, const NetDev& net, const int64_t* f, double alpha, int beta, float* cost,
                      float* rcost, const InstState* st, int only_active, int* err) {
    if (net.nblk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bpr, dim3(net.nblk), dim3(kWG), 0, s, net, f, alpha, beta, cost, rcost, st, only_active,
                       err);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// A4: exact sums for the relative gap, sum c F and sum c Y
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_gap_sums(NetDev net, const float* __restrict__ cost,
                                                  const int64_t* __restrict__ f, const int64_t* __restrict__ y,
                                                  long long* acc, const InstState* st, int* err) {
    __shared__ i128 lds[kWG];
    const int b = blockIdx.x;
    const int inst = net.blk_inst[b];
    if (!inst_live(st, inst)) return;
    const InstDev I = net.inst[inst];
    const int a0 = net.blk_start[b];
    const int a1 = min(a0 + kChunk, I.link0 + I.m);
    i128 sf = 0, sy = 0;
    int bad = 0;
    for (int a = a0 + threadIdx.x; a < a1; a += kWG) {
        double c = (double)cost[a];
        sf += quant(c * ((double)f[a] * kFxInv), bad);
        sy += quant(c * ((double)y[a] * kFxInv), bad);
    }
    if (bad) atomicOr(err, 1);
    wg_acc_add(sf, acc + inst * 6 + 0, lds);
    wg_acc_add(sy, acc + inst * 6 + 3, lds);
}

hipError_t launch_gap_sums(hipStream_t s, const NetDev& net, const float* cost, const int64_t* f, const int64_t* y,
                           long long* acc, const InstState* st, int* err) {
    if (net.nblk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gap_sums, dim3(net.nblk), dim3(kWG), 0, s, net, cost, f, y, acc, st, err);
    return hipGetLastError();
}

// Stop test of iteration j (Alg. 6): relative gap, or the iteration cap.
__global__ void k_gap_decide(int ninst, const long long* acc, InstState* st, int stop_rule, double tol,
                             int fixed_iters, int cap_iter, int j) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst) return;
    InstState& S = st[i];
    if (!S.active || S.converged) return;
    S.iter = j;
    i128 scf = acc3_value(acc + i * 6), scy = acc3_value(acc + i * 6 + 3);
    S.gap = (double)(scf - scy) / (double)scf;
    if (fixed_iters <= 0 && stop_rule == 0 && __builtin_fabs(S.gap) < tol) {
        S.converged = 1;
        S.stopped_by = 1;
    } else if (S.iter > cap_iter) {
        S.converged = 1;
        S.stopped_by = 0;
    }
}

hipError_t launch_gap_decide(hipStream_t s, int ninst, const long long* acc, InstState* st, int stop_rule,
                             double tol, int fixed_iters, int cap_iter, int j) {
    hipLaunchKernelGGL(k_gap_decide, dim3((ninst + 63) / 64), dim3(64), 0, s, ninst, acc, st, stop_rule, tol,
                       fixed_iters, cap_iter, j);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// A5: line search
// ---------------------------------------------------------------------------
__device__ __forceinline__ void ks_alphas(double lo, double hi, int K, double* out) {
    for (int k = 0; k < K; ++k) out[k] = lo + ((hi - lo) * (double)k) / (double)(K - 1);
}

// Start the line search of iteration j for every live instance.
// only_fallback: restart as K-section only the instances whose quasi-Newton
// search met a non-positive C'' (ls_done == 2).
__global__ void k_ls_begin(int ninst, InstState* st, double* alphas, int K, int ls_mode, double dx,
                           long long* ls_acc, int only_fallback) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst) return;
    InstState& S = st[i];
    if (!S.active || S.converged) return;
    if (only_fallback && S.ls_done != 2) return;
    S.ls_done = 0;
    S.ls_pass = 0;
    for (int k = 0; k < K * 6; ++k) ls_acc[(long long)i * K * 6 + k] = 0;
    double* al = alphas + (long long)i * K;
    if (ls_mode == 2) {                  // MSA
        S.alpha = 1.0 / ((double)S.iter + 1.0);
        S.ls_done = 1;
    } else if (ls_mode == 1) {           // quasi-Newton, Alg. 8 initial guess
        double a = 2.0 / (2.0 + (double)S.iter);
        S.qn_alpha = a;
        al[0] = a - dx; al[1] = a; al[2] = a + dx;
    } else {                              // K-section on [0, 1]
        S.lo = 0.0; S.hi = 1.0;
        ks_alphas(0.0, 1.0, K, al);
    }
}

hipError_t launch_ls_begin(hipStream_t s, int ninst, InstState* st, double* alphas, int K, int ls_mode, double dx,
                           long long* ls_acc, int only_fallback) {
    hipLaunchKernelGGL(k_ls_begin, dim3((ninst + 63) / 64), dim3(64), 0, s, ninst, st, alphas, K, ls_mode, dx,
                       ls_acc, only_fallback);
    return hipGetLastError();
}

// One pass over the links: C(alpha_k) and C'(alpha_k) for all k at once.
// Lanes of a group take the K step sizes of one link; a workgroup covers
// kWG / GK links per step over a 2048-link chunk of one instance.
template <int GK>
__global__ __launch_bounds__(kWG) void k_ls_eval(NetDev net, const int64_t* __restrict__ f,
                                                 const int64_t* __restrict__ y, double alpha_b, int beta, int K,
                                                 const double* __restrict__ alphas, long long* ls_acc,
                                                 const InstState* st, int only_pending, int* err) {
    __shared__ i128 ldsC[kWG];
    __shared__ i128 ldsD[kWG];
    constexpr int LPB = kWG / GK;
    const int b = blockIdx.x;
    const int inst = net.blk_inst[b];
    if (st && (!st[inst].active || st[inst].converged || (only_pending && st[inst].ls_done))) return;
    const InstDev I = net.inst[inst];
    const int a0 = net.blk_start[b];
    const int a1 = min(a0 + kChunk, I.link0 + I.m);
    const int k = threadIdx.x % GK;
    const int g = threadIdx.x / GK;
    const bool live = k < K;
    const double alpha = live ? alphas[(long long)inst * K + k] : 0.0;
    i128 sc = 0, sd = 0;
    int bad = 0;
    if (live) {
        for (int a = a0 + g; a < a1; a += LPB) {
            double obj, der;
            ls_terms((double)f[a] * kFxInv, (double)y[a] * kFxInv, net.c0[a], net.cap[a], alpha_b, beta, I.kappa,
                     alpha, obj, der);
            sc += quant(obj, bad);
            sd += quant(der, bad);
        }
    }
    if (bad) atomicOr(err, 1);
    ldsC[threadIdx.x] = sc;
    ldsD[threadIdx.x] = sd;
    __syncthreads();
    for (int s = LPB / 2; s > 0; s >>= 1) {
        if (g < s) {
            ldsC[threadIdx.x] += ldsC[threadIdx.x + s * GK];
            ldsD[threadIdx.x] += ldsD[threadIdx.x + s * GK];
        }
        __syncthreads();
    }
    if (g == 0 && live) {
        long long* acc = ls_acc + ((long long)inst * K + k) * 6;
        if (ldsC[threadIdx.x] != 0) acc3_add(acc, ldsC[threadIdx.x]);
        if (ldsD[threadIdx.x] != 0) acc3_add(acc + 3, ldsD[threadIdx.x]);
    }
}

hipError_t launch_ls_eval(hipStream_t s, const NetDev& net, const int64_t* f, const int64_t* y, double alpha_b,
                          int beta, int K, const double* alphas, long long* ls_acc, const InstState* st,
                          int only_pending, int* err) {
    if (net.nblk == 0) return hipSuccess;
    dim3 g(net.nblk), blk(kWG);
    if (K <= 4)
        hipLaunchKernelGGL(k_ls_eval<4>, g, blk, 0, s, net, f, y, alpha_b, beta, K, alphas, ls_acc, st, only_pending,
                           err);
    else if (K <= 8)
        hipLaunchKernelGGL(k_ls_eval<8>, g, blk, 0, s, net, f, y, alpha_b, beta, K, alphas, ls_acc, st, only_pending,
                           err);
    else if (K <= 16)
        hipLaunchKernelGGL(k_ls_eval<16>, g, blk, 0, s, net, f, y, alpha_b, beta, K, alphas, ls_acc, st,
                           only_pending, err);
    else if (K <= 32)
        hipLaunchKernelGGL(k_ls_eval<32>, g, blk, 0, s, net, f, y, alpha_b, beta, K, alphas, ls_acc, st,
                           only_pending, err);
    else
        hipLaunchKernelGGL(k_ls_eval<64>, g, blk, 0, s, net, f, y, alpha_b, beta, K, alphas, ls_acc, st,
                           only_pending, err);
    return hipGetLastError();
}

// Decide after a pass: K-section bracket update (root of C', C convex in
// alpha), or one quasi-Newton step (Alg. 8 with Eq. 10).
__global__ void k_ls_decide(int ninst, InstState* st, double* alphas, int K, int ls_mode, int passes, int max_ls,
                            double T1, double T2, double dx, long long* ls_acc) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst) return;
    InstState& S = st[i];
    if (!S.active || S.converged || S.ls_done) return;
    long long* acc = ls_acc + (long long)i * K * 6;
    double* al = alphas + (long long)i * K;
    S.ls_evals++;
    S.ls_pass++;
    if (ls_mode == 0) {
        int kk = -1;
        for (int k = 0; k < K; ++k)
            if (acc3_value(acc + k * 6 + 3) >= 0) { kk = k; break; }
        if (kk == 0) { S.alpha = al[0]; S.ls_done = 1; }
        else if (kk < 0) { S.alpha = al[K - 1]; S.ls_done = 1; }
        else {
            S.lo = al[kk - 1];
            S.hi = al[kk];
            put128(S.dlo, acc3_value(acc + (kk - 1) * 6 + 3));
            put128(S.dhi, acc3_value(acc + kk * 6 + 3));
            if (S.ls_pass >= passes) {
                double a = S.lo, bb = S.hi;
                double da = (double)get128(S.dlo), db = (double)get128(S.dhi);
                S.alpha = a - (da * (bb - a)) / (db - da);
                S.ls_done = 1;
            } else {
                ks_alphas(S.lo, S.hi, K, al);
            }
        }
    } else {
        S.qn_iters++;
        double cm = (double)acc3_value(acc + 0) / kSumQ;
        double c0v = (double)acc3_value(acc + 6) / kSumQ;
        double cp = (double)acc3_value(acc + 12) / kSumQ;
        double d1 = (cp - cm) / (2.0 * dx);
        double d2 = ((cm - 2.0 * c0v) + cp) / (dx * dx);
        double a = S.qn_alpha;
        if (__builtin_fabs(d1) < T1) { S.alpha = a; S.ls_done = 1; }
        else if (!(d2 > 0.0)) { S.ls_done = 2; }          // fall back to K-section
        else {
            double an = a - d1 / d2;
            if (an < 0.0) an = 0.0;
            if (an > 1.0) an = 1.0;
            if (__builtin_fabs(an - a) < T2) { S.alpha = an; S.ls_done = 1; }
            else if (S.ls_pass >= max_ls) { S.alpha = an; S.ls_done = 1; }
            else {
                S.qn_alpha = an;
                al[0] = an - dx; al[1] = an; al[2] = an + dx;
            }
        }
    }
    if (!S.ls_done)
        for (int k = 0; k < K * 6; ++k) acc[k] = 0;
}

hipError_t launch_ls_decide(hipStream_t s, int ninst, InstState* st, double* alphas, int K, int ls_mode, int passes,
                            int max_ls, double T1, double T2, double dx, long long* ls_acc) {
    hipLaunchKernelGGL(k_ls_decide, dim3((ninst + 63) / 64), dim3(64), 0, s, ninst, st, alphas, K, ls_mode, passes,
                       max_ls, T1, T2, dx, ls_acc);
    return hipGetLastError();
}

__global__ void k_ls_export(int ninst, const long long* ls_acc, int K, int64_t* sums) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ninst * K * 2) return;
    i128 v = acc3_value(ls_acc + (long long)t * 3);
    put128((long long*)sums + 2 * (long long)t, v);
}

hipError_t launch_ls_export(hipStream_t s, int ninst, const long long* ls_acc, int K, int64_t* sums) {
    int n = ninst * K * 2;
    hipLaunchKernelGGL(k_ls_export, dim3((n + 63) / 64), dim3(64), 0, s, ninst, ls_acc, K, sums);
    return hipGetLastError();
}

// Beckmann objective of f (slot 0) and of the would-be update f + rint(alpha
// (y - f)) (slot 1), exact -- the Converged test of Eq. 7.
__global__ __launch_bounds__(kWG) void k_obj_pair(NetDev net, const int64_t* __restrict__ f,
                                                  const int64_t* __restrict__ y, double alpha_b, int beta,
                                                  long long* acc, const InstState* st, int use_alpha, int* err) {
    __shared__ i128 lds[kWG];
    const int b = blockIdx.x;
    const int inst = net.blk_inst[b];
    if (st && !st[inst].active) return;
    if (use_alpha && (st[inst].converged)) return;
    const InstDev I = net.inst[inst];
    const int a0 = net.blk_start[b];
    const int a1 = min(a0 + kChunk, I.link0 + I.m);
    const double alpha = use_alpha ? st[inst].alpha : 0.0;
    i128 s0 = 0, s1 = 0;
    int bad = 0;
    for (int a = a0 + threadIdx.x; a < a1; a += kWG) {
        double obj, der;
        double F = (double)f[a] * kFxInv;
        ls_terms(F, F, net.c0[a], net.cap[a], alpha_b, beta, I.kappa, 0.0, obj, der);
        s0 += quant(obj, bad);
        if (use_alpha) {
            int64_t fn = f[a] + (int64_t)__builtin_rint(alpha * (double)(y[a] - f[a]));
            double Fn = (double)fn * kFxInv;
            ls_terms(Fn, Fn, net.c0[a], net.cap[a], alpha_b, beta, I.kappa, 0.0, obj, der);
            s1 += quant(obj, bad);
        }
    }
    if (bad) atomicOr(err, 1);
    wg_acc_add(s0, acc + inst * 6, lds);
    if (use_alpha) wg_acc_add(s1, acc + inst * 6 + 3, lds);
}

hipError_t launch_obj_pair(hipStream_t s, const NetDev& net, const int64_t* f, const int64_t* y, double alpha_b,
                           int beta, long long* acc, const InstState* st, int use_alpha, int* err) {
    if (net.nblk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_obj_pair, dim3(net.nblk), dim3(kWG), 0, s, net, f, y, alpha_b, beta, acc, st, use_alpha,
                       err);
    return hipGetLastError();
}

// apply_rule = 1: Eq. 7 test on (slot 0, slot 1); 0: record slot 0 as the
// objective of the returned iterate.
__global__ void k_obj_decide(int ninst, const long long* acc, InstState* st, double tol, int apply_rule) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst) return;
    InstState& S = st[i];
    if (!S.active) return;
    if (apply_rule) {
        if (S.converged) return;
        double b0 = (double)acc3_value(acc + i * 6), b1 = (double)acc3_value(acc + i * 6 + 3);
        if (__builtin_fabs((b0 - b1) / b0) < tol) { S.converged = 1; S.stopped_by = 2; }
    } else {
        S.obj = (double)acc3_value(acc + i * 6) / kSumQ;
    }
}

hipError_t launch_obj_decide(hipStream_t s, int ninst, const long long* acc, InstState* st, double tol,
                             int apply_rule) {
    hipLaunchKernelGGL(k_obj_decide, dim3((ninst + 63) / 64), dim3(64), 0, s, ninst, acc, st, tol, apply_rule);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// A6: link-flow update
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_fw_update(NetDev net, int64_t* __restrict__ f, const int64_t* __restrict__ y,
                                                   const double* alpha_per_inst, const InstState* st) {
    const int b = blockIdx.x;
    const int inst = net.blk_inst[b];
    if (!inst_live(st, inst)) return;
    const InstDev I = net.inst[inst];
    const int a0 = net.blk_start[b];
    const int a1 = min(a0 + kChunk, I.link0 + I.m);
    const double alpha = alpha_per_inst[inst];
    for (int a = a0 + threadIdx.x; a < a1; a += kWG) {
        int64_t fa = f[a];
        f[a] = fa + (int64_t)__builtin_rint(alpha * (double)(y[a] - fa));
    }
}

hipError_t launch_fw_update(hipStream_t s, const NetDev& net, int64_t* f, const int64_t* y,
                            const double* alpha_per_inst, const InstState* st) {
    if (net.nblk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fw_update, dim3(net.nblk), dim3(kWG), 0, s, net, f, y, alpha_per_inst, st);
    return hipGetLastError();
}

__global__ __launch_bounds__(kWG) void k_scatter_rcost(NetDev net, const float* __restrict__ cost,
                                                       float* __restrict__ rcost) {
    for (int64_t a = blockIdx.x * (int64_t)kWG + threadIdx.x; a < net.M; a += (int64_t)gridDim.x * kWG)
        rcost[net.revpos[a]] = cost[a];
}

hipError_t launch_scatter_rcost(hipStream_t s, const NetDev& net, const float* cost, float* rcost) {
    if (net.M == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_rcost, dim3(grid_for(net.M)), dim3(kWG), 0, s, net, cost, rcost);
    return hipGetLastError();
}

// Bookkeeping after an applied update of iteration j.
__global__ void k_after_update(int ninst, InstState* st) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst) return;
    InstState& S = st[i];
    if (!S.active || S.converged) return;
    S.iters = S.iter;
    S.last_alpha = S.alpha;
}

hipError_t launch_after_update(hipStream_t s, int ninst, InstState* st) {
    hipLaunchKernelGGL(k_after_update, dim3((ninst + 63) / 64), dim3(64), 0, s, ninst, st);
    return hipGetLastError();
}

__global__ void k_copy_alpha(int ninst, const InstState* st, double* out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ninst) out[i] = st[i].alpha;
}

hipError_t launch_copy_alpha(hipStream_t s, int ninst, const InstState* st, double* out) {
    hipLaunchKernelGGL(k_copy_alpha, dim3((ninst + 63) / 64), dim3(64), 0, s, ninst, st, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// A2: shortest-path trees, SB destinations per workgroup
// ---------------------------------------------------------------------------
// Persistent workgroups pull batches of up to SB destinations from a work
// counter.  Labels of a batch are node-major, D[v * SB + t] for tree t, so
// the SB lanes of a group read and write one contiguous row.  Each round
// processes the current queue of nodes whose label improved in some tree
// (dirty[v] holds those trees as a bit mask), relaxing the in-links of each
// such node on the reverse graph: D[u] = min(D[u], fl32(D[w] + c)) by an
// integer atomicMin on the FP32 bit pattern (labels are non-negative, so bit
// order is value order).  An improved node enters the queue of round r+1
// once: stamp[v] records the last round it was queued for (atomicMax), so a
// queue never holds more than n entries.  Pushes are aggregated per
// wavefront with a ballot and a prefix count.  The fixed point reached is the
// least one, the FP32 min-plus distance, whatever the processing order.
template <int SB>
__global__ __launch_bounds__(kWG) void k_sssp(NetDev net, DemDev dem, const float* __restrict__ rcost,
                                              float* labels, Scratch scr, const InstState* st) {
    constexpr int GW = 64 / SB;           // groups per wavefront
    constexpr int NG = kWG / SB;          // groups per workgroup
    constexpr unsigned long long GMASK = (SB == 64) ? ~0ull : ((1ull << SB) - 1);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int slot = lane % SB;
    const int gw = lane / SB;
    const int gid = (tid >> 6) * GW + gw;
    __shared__ int s_batch;
    __shared__ int s_cnt[2];
    int32_t* qbase = scr.queues + (int64_t)blockIdx.x * 2 * scr.nmax;
    uint32_t* dirty = scr.dirty + (int64_t)blockIdx.x * scr.nmax;
    int32_t* stamp = scr.stamp + (int64_t)blockIdx.x * scr.nmax;

    for (;;) {
        if (tid == 0) s_batch = atomicAdd(scr.work, 1);
        __syncthreads();
        const int b = s_batch;
        if (b >= dem.B) break;
        const int inst = dem.b_inst[b];
        if (!inst_live(st, inst)) { __syncthreads(); continue; }
        const InstDev I = net.inst[inst];
        const int n = I.n, node0 = I.node0;
        uint32_t* D = reinterpret_cast<uint32_t*>(labels + dem.b_lab[b]);
        const int nq = dem.b_nq[b];
        const int q_first = dem.b_q[b];

        for (int64_t i = tid; i < (int64_t)n * SB; i += kWG) D[i] = kInfBits;
        for (int i = tid; i < n; i += kWG) { dirty[i] = 0u; stamp[i] = 0; }
        if (tid == 0) { s_cnt[0] = 0; s_cnt[1] = 0; }
        __syncthreads();
        if (tid < nq) {
            int r = dem.dest_node[q_first + tid] - node0;
            D[(int64_t)r * SB + tid] = 0u;
            atomicOr(&dirty[r], 1u << tid);
            if (atomicMax(&stamp[r], 1) < 1) { int pos = atomicAdd(&s_cnt[0], 1); qbase[pos] = r; }
        }
        __syncthreads();

        int cur = 0;
        for (int round = 1;; ++round) {
            const int cnt = s_cnt[cur];
            if (cnt == 0) break;
            const int32_t* qc = qbase + (int64_t)cur * scr.nmax;
            int32_t* qn = qbase + (int64_t)(cur ^ 1) * scr.nmax;
            for (int base = 0; base < cnt; base += NG) {
                const int i = base + gid;
                const bool valid = i < cnt;
                const int w = valid ? qc[i] : 0;
                unsigned mask = 0u;
                if (valid && slot == 0) mask = atomicExch(&dirty[w], 0u);
                mask = __shfl(mask, lane - slot);
                const bool act = (mask >> slot) & 1u;
                float dw = 0.0f;
                if (act) dw = __uint_as_float(ld_coherent(&D[(int64_t)w * SB + slot]));
                int e0 = 0, e1 = 0;
                if (mask) { e0 = net.rptr[node0 + w]; e1 = net.rptr[node0 + w + 1]; }
                for (int e = e0; e < e1; ++e) {
                    const int v = net.rsrc[e] - node0;
                    const float c = rcost[e];
                    bool imp = false;
                    if (act) {
                        const uint32_t cb = __float_as_uint(dw + c);
                        uint32_t* dv = &D[(int64_t)v * SB + slot];
                        if (cb < *dv) {
                            uint32_t old = atomicMin(dv, cb);
                            imp = cb < old;
                        }
                    }
                    const unsigned long long bal = __ballot(imp);
                    const unsigned bits = (unsigned)((bal >> (gw * SB)) & GMASK);
                    bool push = false;
                    if (slot == 0 && bits) {
                        atomicOr(&dirty[v], bits);
                        push = atomicMax(&stamp[v], round + 1) < round + 1;
                    }
                    const unsigned long long pb = __ballot(push);
                    if (pb) {
                        const int leader = __ffsll((long long)pb) - 1;
                        int pos = 0;
                        if (lane == leader) pos = atomicAdd(&s_cnt[cur ^ 1], __popcll(pb));
                        pos = __shfl(pos, leader);
                        if (push) qn[pos + __popcll(pb & ((1ull << lane) - 1ull))] = v;
                    }
                }
            }
            __syncthreads();
            if (tid == 0) s_cnt[cur] = 0;
            cur ^= 1;
            __syncthreads();
        }
        __syncthreads();
    }
}

hipError_t launch_sssp(hipStream_t s, const NetDev& net, const DemDev& dem, const float* rcost, float* labels,
                       const Scratch& scr, int slots, const InstState* st) {
    if (dem.B == 0) return hipSuccess;
    hipError_t e = launch_fill_u32(s, reinterpret_cast<uint32_t*>(scr.work), 0u, 1);
    if (e != hipSuccess) return e;
    dim3 g(slots), blk(kWG);
    switch (dem.sb) {
        case 4: hipLaunchKernelGGL(k_sssp<4>, g, blk, 0, s, net, dem, rcost, labels, scr, st); break;
        case 8: hipLaunchKernelGGL(k_sssp<8>, g, blk, 0, s, net, dem, rcost, labels, scr, st); break;
        case 16: hipLaunchKernelGGL(k_sssp<16>, g, blk, 0, s, net, dem, rcost, labels, scr, st); break;
        case 32: hipLaunchKernelGGL(k_sssp<32>, g, blk, 0, s, net, dem, rcost, labels, scr, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// A3: truncation + loading, and the residual walk of Alg. 4
// ---------------------------------------------------------------------------
// Successor of u on the tree whose labels are lab[(node - node0) * sb]: the
// lowest-uid out-link (u, w) that is tight, fl32(D(w) + c) == D(u), and
// strict, D(w) < D(u).  -1 when FP32 absorption leaves none.
__device__ __forceinline__ int succ_strict(const NetDev& net, const float* lab, int sb, int node0, int u, float du,
                                          const float* tree_cost) {
    const int e1 = net.row_ptr[u + 1];
    for (int e = net.row_ptr[u]; e < e1; ++e) {
        const float dw = lab[(int64_t)(net.col[e] - node0) * sb];
        if (dw < du && dw + tree_cost[e] == du) return e;
    }
    return -1;
}

struct WalkOut {
    int64_t* y;
    int32_t* stop;
    int residual_mode;
    const double* lambda;        // per instance (residual mode)
    int32_t *r_orig, *r_dest;
    int64_t* r_w;
    unsigned long long *r_count, *done_fx;
};

// Residual mode emits (stop node, destination index, rint(lambda d)) for a
// leg that stops short of q, and counts the completed weight otherwise.
__device__ __forceinline__ void finish_leg(const WalkOut& o, int l, int s, int q, int qi, int inst, int node0,
                                           int64_t d) {
    if (!o.residual_mode) {
        if (o.stop) o.stop[l] = s - node0;
        return;
    }
    const int64_t w = (int64_t)__builtin_rint(o.lambda[inst] * (double)d);
    if (s == q) {
        if (w) atomicAdd(&o.done_fx[inst], (unsigned long long)w);
        return;
    }
    if (w == 0) return;
    const unsigned long long k = atomicAdd(o.r_count, 1ull);
    o.r_orig[k] = s - node0;
    o.r_dest[k] = qi;
    o.r_w[k] = w;
}

__global__ __launch_bounds__(kWG) void k_walk(NetDev net, DemDev dem, const float* __restrict__ labels,
                                              const float* __restrict__ tree_cost,
                                              const float* __restrict__ time_cost, const InstState* st,
                                              FlagsDev fl, WalkOut o) {
    const int l = blockIdx.x * kWG + threadIdx.x;
    if (l >= dem.P) return;
    const int qi = dem.leg_q[l];
    const int inst = dem.dest_inst[qi];
    if (!inst_live(st, inst)) return;
    const InstDev I = net.inst[inst];
    const int node0 = I.node0;
    const int q = dem.dest_node[qi];
    const float* lab = labels + dem.dest_lab[qi];
    const int sb = dem.sb;
    const int64_t d = dem.leg_dfx[l];
    int u = dem.leg_orig[l];
    float du = lab[(int64_t)(u - node0) * sb];
    fl.int_node[l] = -1;
    if (!(du <= 3.4028234663852886e38f)) {       // origin cannot reach q
        atomicOr(fl.err_unreach, 1);
        if (o.stop) o.stop[l] = -1;
        return;
    }
    float tau = 0.0f;
    for (int hops = 0; u != q; ++hops) {
        if (I.rule == RULE_CEIL && tau >= I.dt32) break;
        const int e = succ_strict(net, lab, sb, node0, u, du, tree_cost);
        if (e < 0 || hops > I.n) {                // absorption: finish in the fallback
            fl.int_node[l] = u;
            fl.int_tau[l] = tau;
            fl.absorb_q[qi] = 1;
            atomicAdd(fl.absorb_count, 1);
            return;
        }
        const float nt = tau + time_cost[e];
        if (I.rule == RULE_FLOOR && nt > I.dt32) break;
        if (!o.residual_mode) atomicAdd((unsigned long long*)&o.y[e], (unsigned long long)d);
        tau = nt;
        u = net.col[e];
        du = lab[(int64_t)(u - node0) * sb];
    }
    finish_leg(o, l, u, q, qi, inst, node0, d);
}

hipError_t launch_walk(hipStream_t s, const NetDev& net, const DemDev& dem, const float* labels,
                       const float* tree_cost, const float* time_cost, int64_t* y, int32_t* stop,
                       const InstState* st, const FlagsDev& fl, int residual_mode, const double* lambda, int32_t* r_orig,
                       int32_t* r_dest, int64_t* r_w, unsigned long long* r_count, unsigned long long* done_fx) {
    if (dem.P == 0) return hipSuccess;
    WalkOut o{y, stop, residual_mode, lambda, r_orig, r_dest, r_w, r_count, done_fx};
    hipLaunchKernelGGL(k_walk, dim3((dem.P + kWG - 1) / kWG), dim3(kWG), 0, s, net, dem, labels, tree_cost, time_cost,
                       st, fl, o);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tie-rule fallback under FP32 absorption
// ---------------------------------------------------------------------------
// For a flagged tree: hop depth h to q inside the tight subgraph (links with
// fl32(D(w) + c) == D(v)), breadth-first from q; a node without a strict
// tight link then takes the lowest-uid tight link to a node with h - 1.
// Trees mode fills the missing successors; walk mode finishes the legs that
// the walk interrupted.  One workgroup per flagged tree.
__global__ __launch_bounds__(kWG) void k_fallback(NetDev net, DemDev dem, const float* __restrict__ labels,
                                                  const float* __restrict__ tree_cost,
                                                  const float* __restrict__ time_cost, const InstState* st,
                                                  FlagsDev fl, Scratch scr, WalkOut o, int trees_mode,
                                                  int32_t* succ_out, int32_t n_out) {
    __shared__ int s_cnt[2];
    int32_t* hop = reinterpret_cast<int32_t*>(scr.dirty) + (int64_t)blockIdx.x * scr.nmax;
    int32_t* qbase = scr.queues + (int64_t)blockIdx.x * 2 * scr.nmax;
    for (int qi = blockIdx.x; qi < dem.Q; qi += gridDim.x) {
        if (!fl.absorb_q[qi]) continue;
        const int inst = dem.dest_inst[qi];
        if (!inst_live(st, inst)) continue;
        const InstDev I = net.inst[inst];
        const int n = I.n, node0 = I.node0;
        const float* lab = labels + dem.dest_lab[qi];
        const int sb = dem.sb;
        const int q = dem.dest_node[qi];
        for (int v = threadIdx.x; v < n; v += kWG) hop[v] = -1;
        if (threadIdx.x == 0) { s_cnt[0] = 1; s_cnt[1] = 0; }
        __syncthreads();
        if (threadIdx.x == 0) { hop[q - node0] = 0; qbase[0] = q - node0; }
        __syncthreads();
        int cur = 0;
        for (int level = 0;; ++level) {
            const int cnt = s_cnt[cur];
            if (cnt == 0) break;
            const int32_t* qc = qbase + (int64_t)cur * scr.nmax;
            int32_t* qn = qbase + (int64_t)(cur ^ 1) * scr.nmax;
            for (int i = threadIdx.x; i < cnt; i += kWG) {
                const int u = qc[i];
                const float du = lab[(int64_t)u * sb];
                for (int e = net.rptr[node0 + u]; e < net.rptr[node0 + u + 1]; ++e) {
                    const int v = net.rsrc[e] - node0;
                    const int link = net.rlink[e];
                    const float dv = lab[(int64_t)v * sb];
                    if (dv <= 3.4028234663852886e38f && du + tree_cost[link] == dv) {
                        if (atomicCAS(&hop[v], -1, level + 1) == -1) {
                            int pos = atomicAdd(&s_cnt[cur ^ 1], 1);
                            qn[pos] = v;
                        }
                    }
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) s_cnt[cur] = 0;
            cur ^= 1;
            __syncthreads();
        }
        // successor with the hop rule where no strict tight link exists
        auto succ_full = [&](int u, float du) -> int {
            int e = succ_strict(net, lab, sb, node0, u, du, tree_cost);
            if (e >= 0) return e;
            const int hu = ld_coherent(&hop[u - node0]);
            for (int k = net.row_ptr[u]; k < net.row_ptr[u + 1]; ++k) {
                const int w = net.col[k];
                const float dw = lab[(int64_t)(w - node0) * sb];
                if (dw + tree_cost[k] == du && ld_coherent(&hop[w - node0]) == hu - 1) return k;
            }
            return -1;
        };
        if (trees_mode) {
            const int t = qi;
            for (int v = threadIdx.x; v < n; v += kWG) {
                const int g = node0 + v;
                const float dv = lab[(int64_t)v * sb];
                if (g == q || !(dv <= 3.4028234663852886e38f)) continue;
                if (succ_out[(int64_t)t * n_out + v] >= 0) continue;
                const int e = succ_full(g, dv);
                succ_out[(int64_t)t * n_out + v] = e >= 0 ? e - I.link0 : -1;
            }
        } else {
            for (int l = dem.qptr[qi] + threadIdx.x; l < dem.qptr[qi + 1]; l += kWG) {
                int u = fl.int_node[l];
                if (u < 0) continue;
                float tau = fl.int_tau[l];
                float du = lab[(int64_t)(u - node0) * sb];
                const int64_t d = dem.leg_dfx[l];
                for (int hops = 0; u != q && hops <= n; ++hops) {
                    if (I.rule == RULE_CEIL && tau >= I.dt32) break;
                    const int e = succ_full(u, du);
                    if (e < 0) break;
                    const float nt = tau + time_cost[e];
                    if (I.rule == RULE_FLOOR && nt > I.dt32) break;
                    if (!o.residual_mode) atomicAdd((unsigned long long*)&o.y[e], (unsigned long long)d);
                    tau = nt;
                    u = net.col[e];
                    du = lab[(int64_t)(u - node0) * sb];
                }
                fl.int_node[l] = -1;
                finish_leg(o, l, u, q, qi, inst, node0, d);
            }
        }
        __syncthreads();
    }
}

hipError_t launch_fallback(hipStream_t s, const NetDev& net, const DemDev& dem, const float* labels,
                           const float* tree_cost, const float* time_cost, int64_t* y, int32_t* stop,
                           const InstState* st, const FlagsDev& fl, const Scratch& scr, int slots,
                           int residual_mode, const double* lambda, int32_t* r_orig, int32_t* r_dest, int64_t* r_w,
                           unsigned long long* r_count, unsigned long long* done_fx, int trees_mode,
                           int32_t* succ_out, int32_t n_out) {
    if (dem.Q == 0) return hipSuccess;
    WalkOut o{y, stop, residual_mode, lambda, r_orig, r_dest, r_w, r_count, done_fx};
    hipLaunchKernelGGL(k_fallback, dim3(slots), dim3(kWG), 0, s, net, dem, labels, tree_cost, time_cost, st, fl, scr,
                       o, trees_mode, succ_out, n_out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Parity output of trees: dist[t][v], succ[t][v] (local uid)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_trees_out(NetDev net, DemDev dem, const float* __restrict__ labels,
                                                   const float* __restrict__ cost, int32_t inst, float* dist,
                                                   int32_t* succ, int32_t* absorb_q) {
    const InstDev I = net.inst[inst];
    const int n = I.n;
    const int64_t total = (int64_t)dem.Q * n;
    for (int64_t i = blockIdx.x * (int64_t)kWG + threadIdx.x; i < total; i += (int64_t)gridDim.x * kWG) {
        const int t = (int)(i / n);
        const int v = (int)(i - (int64_t)t * n);
        const float* lab = labels + dem.dest_lab[t];
        const float dv = lab[(int64_t)v * dem.sb];
        dist[i] = dv;
        const int g = I.node0 + v;
        int e = -1;
        if (g != dem.dest_node[t] && dv <= 3.4028234663852886e38f) {
            e = succ_strict(net, lab, dem.sb, I.node0, g, dv, cost);   // cost: global link order
            if (e < 0) absorb_q[t] = 1;
        }
        succ[i] = e >= 0 ? e - I.link0 : -1;
    }
}

hipError_t launch_trees_out(hipStream_t s, const NetDev& net, const DemDev& dem, const float* labels,
                            const float* cost, int32_t inst, float* dist, int32_t* succ, int32_t* absorb_q) {
    if (dem.Q == 0) return hipSuccess;
    hipLaunchKernelGGL(k_trees_out, dim3(2048), dim3(kWG), 0, s, net, dem, labels, cost, inst, dist, succ, absorb_q);
    return hipGetLastError();
}

}  // namespace qdta
