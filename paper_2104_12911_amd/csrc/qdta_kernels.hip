// qdta_kernels.hip -- gfx950 kernels of the QDTA hot path.
//
// One Frank-Wolfe iteration of the link-flow form (Alg. 6, section 5.1):
//   k_bpr        link costs by the BPR curve (Eq. 1)
//   k_sssp_wg    destination-rooted FP32 shortest-path trees, delta-stepping
//   k_sssp_ds    (Get_shortest_path of Alg. 3 / Alg. 7), one workgroup or one
//                wavefront per tree
//   k_walk       route truncation (Eq. 2) and loading along the successor
//                links (Eq. 5, Alg. 3), int64 fixed-point atomics
//   k_gap_sums   exact sums for the relative gap / stop test
//   k_ls_*       line search on the Beckmann objective (Eq. 6, Eq. 8-10,
//                Alg. 8-9), K step sizes per pass over the links
//   k_fw_update  f <- f + rint(alpha (y - f))
// plus the tie-rule fallback under FP32 absorption, the residual-demand
// walk of Alg. 4 and the compaction of its accumulator, and the frozen-path
// model of an interval's iterations with its reverse pass (k_path_*,
// k_adj_*: derivatives for OD calibration, not part of the paper).
//
// Numeric contract: FP64 per-link arithmetic with no fused multiply-add (the
// library is compiled with -ffp-contract=off), power by repeated
// multiplication, FP32 min-plus with IEEE round-to-nearest adds, int64 flows
// in units of 2^-20 vehicle, decision sums exact as int128 multiples of 2^-16.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <type_traits>

#include "qdta_internal.h"

namespace qdta {

typedef __int128 i128;

#define RULE_NONE 0
#define RULE_CEIL 1
#define RULE_FLOOR 2
#define RULE_PROGRESS 3

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

// BPR curve (Eq. 1): c0 (1 + alpha (kappa F / C)^beta) in FP64; with
// `marginal` the marginal cost d(F c)/dF = c0 (1 + (alpha (beta+1)) p).
__device__ __forceinline__ double bpr64(double F, float c0, float cap, double alpha, int beta, double kappa,
                                        int marginal = 0) {
    double r = (F * kappa) / (double)cap;
    double p = r;
    for (int k = 1; k < beta; ++k) p = p * r;
    const double g = marginal ? alpha * (double)(beta + 1) : alpha;
    return (double)c0 * (1.0 + g * p);
}

// Objective term and its derivative along the FW direction at step alpha:
// the Beckmann integral (Eq. 6), or under the system optimum the total
// travel time v c(v) with derivative t c0 (1 + (ab (beta+1)) p).
__device__ __forceinline__ void ls_terms(double F, double Y, float c0, float cap, double ab, int beta, double kappa,
                                         double alpha, int so, double& obj, double& der) {
    double t = Y - F;
    double v = F + alpha * t;
    double r = (v * kappa) / (double)cap;
    double p = r;
    for (int k = 1; k < beta; ++k) p = p * r;
    double cost = (double)c0 * (1.0 + ab * p);
    if (so) {
        const double mc = (double)c0 * (1.0 + (ab * (double)(beta + 1)) * p);
        obj = v * cost;
        der = t * mc;
        return;
    }
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
                                             float* __restrict__ cost, uint2* __restrict__ radj,
                                             const InstState* st, int only_active, int* err,
                                             float* __restrict__ tcost) {
    const int b = blockIdx.x;
    const int inst = net.blk_inst[b];
    if (only_active && !inst_live(st, inst)) return;
    const InstDev I = net.inst[inst];
    const int a0 = net.blk_start[b];
    const int a1 = min(a0 + kChunk, I.link0 + I.m);
    int bad = 0;
    for (int a = a0 + threadIdx.x; a < a1; a += kWG) {
        const double F = (double)f[a] * kFxInv;
        double c = bpr64(F, net.c0[a], net.cap[a], alpha, beta, I.kappa, net.objective);
        float c32 = (float)c;
        if (!(c32 <= 3.4028234663852886e38f)) bad = 1;
        cost[a] = c32;
        if (tcost) {
            const float t32 = net.objective ? (float)bpr64(F, net.c0[a], net.cap[a], alpha, beta, I.kappa) : c32;
            if (!(t32 <= 3.4028234663852886e38f)) bad = 1;
            tcost[a] = t32;
        }
        if (radj) {
            radj[net.revpos[a]].y = __float_as_uint(c32);
            net.fadj[a].y = __float_as_uint(c32);
            if (net.cbuf) {
                const int2 w = net.cslot[a];
                if (w.x >= 0) net.cbuf[w.x] = __float_as_uint(c32);
                if (w.y >= 0) net.cbuf[w.y] = __float_as_uint(c32);
            }
        }
    }
    if (bad) atomicOr(err, 1);
}

hipError_t launch_bpr(hipStream_t s, const NetDev& net, const int64_t* f, double alpha, int beta, float* cost,
                      uint2* radj, const InstState* st, int only_active, int* err, float* tcost) {
    if (net.nblk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bpr, dim3(net.nblk), dim3(kWG), 0, s, net, f, alpha, beta, cost, radj, st, only_active,
                       err, tcost);
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
// Also advances the iteration index j of each live instance, so a captured
// iteration replays with the right j.
__global__ void k_gap_decide(int ninst, const long long* acc, InstState* st, int stop_rule, double tol,
                             int fixed_iters, int cap_iter) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst) return;
    InstState& S = st[i];
    if (!S.active || S.converged) return;
    S.iter += 1;
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
                             double tol, int fixed_iters, int cap_iter) {
    hipLaunchKernelGGL(k_gap_decide, dim3((ninst + 63) / 64), dim3(64), 0, s, ninst, acc, st, stop_rule, tol,
                       fixed_iters, cap_iter);
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
                                                 const InstState* st, int only_pending, int* err, int k0, int kstride) {
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
    const double alpha = live ? alphas[(long long)inst * kstride + k0 + k] : 0.0;
    i128 sc = 0, sd = 0;
    int bad = 0;
    if (live) {
        for (int a = a0 + g; a < a1; a += LPB) {
            double obj, der;
            ls_terms((double)f[a] * kFxInv, (double)y[a] * kFxInv, net.c0[a], net.cap[a], alpha_b, beta, I.kappa,
                     alpha, net.objective, obj, der);
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
        long long* acc = ls_acc + ((long long)inst * kstride + k0 + k) * 6;
        if (ldsC[threadIdx.x] != 0) acc3_add(acc, ldsC[threadIdx.x]);
        if (ldsD[threadIdx.x] != 0) acc3_add(acc + 3, ldsD[threadIdx.x]);
    }
}

hipError_t launch_ls_eval(hipStream_t s, const NetDev& net, const int64_t* f, const int64_t* y, double alpha_b,
                          int beta, int K, const double* alphas, long long* ls_acc, const InstState* st,
                          int only_pending, int* err, int k0, int kstride) {
    if (net.nblk == 0) return hipSuccess;
    if (kstride <= 0) kstride = K;
    dim3 g(net.nblk), blk(kWG);
    if (K <= 1)
        hipLaunchKernelGGL(k_ls_eval<1>, g, blk, 0, s, net, f, y, alpha_b, beta, K, alphas, ls_acc, st, only_pending,
                           err, k0, kstride);
    else if (K <= 4)
        hipLaunchKernelGGL(k_ls_eval<4>, g, blk, 0, s, net, f, y, alpha_b, beta, K, alphas, ls_acc, st, only_pending,
                           err, k0, kstride);
    else if (K <= 8)
        hipLaunchKernelGGL(k_ls_eval<8>, g, blk, 0, s, net, f, y, alpha_b, beta, K, alphas, ls_acc, st, only_pending,
                           err, k0, kstride);
    else if (K <= 16)
        hipLaunchKernelGGL(k_ls_eval<16>, g, blk, 0, s, net, f, y, alpha_b, beta, K, alphas, ls_acc, st,
                           only_pending, err, k0, kstride);
    else if (K <= 32)
        hipLaunchKernelGGL(k_ls_eval<32>, g, blk, 0, s, net, f, y, alpha_b, beta, K, alphas, ls_acc, st,
                           only_pending, err, k0, kstride);
    else
        hipLaunchKernelGGL(k_ls_eval<64>, g, blk, 0, s, net, f, y, alpha_b, beta, K, alphas, ls_acc, st,
                           only_pending, err, k0, kstride);
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

// A zero step leaves f unchanged, so the next iteration would repeat this
// one: stop there unless a fixed iteration count was asked for.
__global__ void k_stall_check(int ninst, InstState* st, int fixed_iters) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst || fixed_iters > 0) return;
    InstState& S = st[i];
    if (!S.active || S.converged) return;
    if (S.alpha == 0.0) { S.converged = 1; S.stopped_by = 3; }
}

hipError_t launch_stall_check(hipStream_t s, int ninst, InstState* st, int fixed_iters) {
    hipLaunchKernelGGL(k_stall_check, dim3((ninst + 63) / 64), dim3(64), 0, s, ninst, st, fixed_iters);
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

// Scratch of the allocation-free line-search entry point: error flags and the
// exact chunk accumulators, in a static array every device holds once for
// the process (kNoAllocWords 64-bit words, 196,736 bytes).  Host code never
// passes the array's name to a kernel: on the host it is not a device
// address.  noalloc_scratch() looks the device address up once per device
// (with that device current) and the kernels receive that pointer.
static __device__ __align__(256) long long scratch[kNoAllocWords];

hipError_t noalloc_scratch(int device, long long** out) {
    static std::mutex mu;
    static std::map<int, long long*> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(device);
    if (it != addr.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = static_cast<long long*>(p);
    *out = static_cast<long long*>(p);
    return hipSuccess;
}

// Objective (Beckmann, or total travel time under the system optimum) of f
// (slot 0) and of the would-be update f + rint(alpha (y - f)) (slot 1),
// exact -- the Converged test of Eq. 7.
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
        ls_terms(F, F, net.c0[a], net.cap[a], alpha_b, beta, I.kappa, 0.0, net.objective, obj, der);
        s0 += quant(obj, bad);
        if (use_alpha) {
            int64_t fn = f[a] + (int64_t)__builtin_rint(alpha * (double)(y[a] - f[a]));
            double Fn = (double)fn * kFxInv;
            ls_terms(Fn, Fn, net.c0[a], net.cap[a], alpha_b, beta, I.kappa, 0.0, net.objective, obj, der);
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

// Costs into the link records: the reverse records (source node, cost) read
// by the shortest-path kernels, one 8-byte record per in-link, and the
// forward records (head node, cost) read by the walks.
__global__ __launch_bounds__(kWG) void k_scatter_rcost(NetDev net, const float* __restrict__ cost,
                                                       uint2* __restrict__ radj) {
    for (int64_t a = blockIdx.x * (int64_t)kWG + threadIdx.x; a < net.M; a += (int64_t)gridDim.x * kWG) {
        radj[net.revpos[a]].y = __float_as_uint(cost[a]);
        net.fadj[a].y = __float_as_uint(cost[a]);
        if (net.cbuf) {
            const int2 w = net.cslot[a];
            if (w.x >= 0) net.cbuf[w.x] = __float_as_uint(cost[a]);
            if (w.y >= 0) net.cbuf[w.y] = __float_as_uint(cost[a]);
        }
    }
}

hipError_t launch_scatter_rcost(hipStream_t s, const NetDev& net, const float* cost, uint2* radj) {
    if (net.M == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_rcost, dim3(grid_for(net.M)), dim3(kWG), 0, s, net, cost, radj);
    return hipGetLastError();
}

__global__ __launch_bounds__(kWG) void k_cslot_init(NetDev net) {
    for (int64_t a = blockIdx.x * (int64_t)kWG + threadIdx.x; a < net.M; a += (int64_t)gridDim.x * kWG) {
        const int2 w = net.cslot[a];
        if (w.x >= 0) net.cbuf[w.x] = net.fadj[a].y;
        if (w.y >= 0) net.cbuf[w.y] = net.fadj[a].y;
    }
}

hipError_t launch_cslot_init(hipStream_t s, const NetDev& net) {
    if (net.M == 0 || !net.cbuf) return hipSuccess;
    hipLaunchKernelGGL(k_cslot_init, dim3(grid_for(net.M)), dim3(kWG), 0, s, net);
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
// A2: shortest-path trees, one wavefront per destination (delta-stepping)
// ---------------------------------------------------------------------------
// A tree's label of node v is one 32-bit word, tree t's at
// labels[dest_lab[t] + v]:
//     (f << 31) | FP32 bits of D(v),   f = 1 when v is NOT queued.
// D >= 0, so the value bits order like the value.  Among queued words
// (f = 0) unsigned order is value order, so an atomicMin of a queued
// candidate both lowers the value and marks the node queued -- provided the
// candidate is below the current value, which the relaxation checks first
// with a coherent read (only the tree's own wavefront writes its labels, and
// lanes of one instruction only write queued words, which keeps that check
// valid).  The word it replaced tells whether this relaxation queued the
// node.  An atomicOr of the flag takes a node off the queue and returns its
// label.  A tree starts from +inf, not queued, on every node.
constexpr uint32_t kNotQueued = 0x80000000u;
constexpr uint32_t kValueBits = 0x7fffffffu;
__device__ __forceinline__ const label_t* tree_labels(const label_t* labels, const DemDev& dem, int t) {
    return labels + dem.dest_lab[t];
}
__device__ __forceinline__ float lab_val(const label_t* lab, int64_t v) {
    return __uint_as_float(lab[v] & kValueBits);
}

__device__ __forceinline__ unsigned long long lanes_below(int lane) {
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ float wave_min(float x) {
    for (int o = 32; o > 0; o >>= 1) x = fminf(x, __shfl_xor(x, o));
    return x;
}

// Each wavefront owns one destination tree at a time (a work counter hands
// out trees) and runs delta-stepping on the reverse graph: D[q] = 0, and the
// nodes taken from the near queue relax their in-links (u, w):
// D[u] = min(D[u], fl32(D[w] + c)).
//   - Up to 64 nodes are popped per step (FIFO ring); their in-links are
//     flattened across the lanes with a prefix sum of the in-degrees, so each
//     step relaxes 64 links whatever the degree mix.
//   - A relaxation that lowers a label and finds the node's queued bit clear
//     sets it and puts the node in the near queue when its label is below the
//     bucket bound thr, else in the far queue together with that label.  A
//     node is in at most one queue.  A pop clears the bit first, then reads
//     the label, so an improvement after the read queues the node again.
//   - A tree starts by writing +inf over its labels and clearing the wave's
//     bitmap (128-byte aligned streaming stores).
//   - When the near queue empties, thr moves to delta above the smallest far
//     label (kept as a running minimum) and one pass moves the far entries
//     below thr to the near queue.
// Queue counters are wave-uniform values updated from ballots, so a tree
// needs no barrier and no shared-memory atomics.  Whatever the order, the
// labels reach the least fixed point of D(v) = min_e fl32(D(head e) + c_e),
// the FP32 min-plus distance.

// U: nodes popped per lane per step (up to 64 U per step); V: in-links each
// lane relaxes per chunk, their loads, label checks and atomics issued back
// to back.
// early: stop a tree once every origin of its legs is settled (AON and
// residual walks read nothing beyond); 0 builds complete trees.
template <int U, int V>
__global__ __launch_bounds__(kWG) void k_sssp_ds(NetDev net, DemDev dem, const uint2* __restrict__ radj,
                                                 label_t* labels, Scratch scr, const InstState* st,
                                                 const float* __restrict__ delta_inst, int early, int t_begin,
                                                 int t_end) {
    constexpr int W = kWG / 64;
    constexpr int NP = 64 * U;                    // nodes per step
    __shared__ int s_pre[W][NP + 1];
    __shared__ float s_dw[W][NP];
    __shared__ int s_e0[W][NP];
    // near queue as 64 rings, one per node-id range (lane r keeps range r's
    // head and count): take offsets / heads for pops, tails / push counts
    __shared__ int s_tpre[W][64], s_rh[W][64], s_tail[W][64], s_push[W][64];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t slot = (int64_t)blockIdx.x * W + wv;
    const unsigned long long below = lanes_below(lane);
    int32_t* nearq = scr.nearq + slot * scr.nmax;
    uint2* farq = reinterpret_cast<uint2*>(scr.farq) + slot * scr.nmax;
    int* pre = s_pre[wv];
    float* sdw = s_dw[wv];
    int* se0 = s_e0[wv];
    int* tpre = s_tpre[wv];
    int* rhd = s_rh[wv];
    int* rtail = s_tail[wv];
    int* rpush = s_push[wv];

    for (;;) {
        int t = 0;
        if (lane == 0) t = t_begin + atomicAdd(scr.work, 1);
        t = __shfl(t, 0);
        if (t >= t_end) break;
        const int inst = dem.dest_inst[t];
        if (!inst_live(st, inst)) continue;
        const InstDev I = net.inst[inst];
        const int n = I.n, node0 = I.node0;
        const int* __restrict__ rptr = net.rptr + node0;
        label_t* D = labels + dem.dest_lab[t];
        const int root = dem.dest_node[t] - node0;
        const float delta = delta_inst[inst];
        // reset the tree's labels to +inf, not queued (the region is 128-byte
        // aligned and padded to a multiple of 32 words)
        {
            uint4* D4 = reinterpret_cast<uint4*>(D);
            const uint32_t w0 = kNotQueued | kInfBits;
            const uint4 inf4 = make_uint4(w0, w0, w0, w0);
            const int n4 = (n + 31) / 32 * 8;
            for (int i = lane; i < n4; i += 64) D4[i] = inf4;
        }
        __threadfence_block();
        // ranges of 2^rsh node ids (at most 64); ring r holds at most the
        // range's nodes (each node is queued once): capacity size + 1, so the
        // rings take n + 64 entries
        int rsh = 0;
        while (((n - 1) >> rsh) >= 64) ++rsh;
        const int rs = 1 << rsh;
        const int nranges = ((n - 1) >> rsh) + 1;
        const bool rvalid = lane < nranges;
        const int rcap = rvalid ? min(rs, n - lane * rs) + 1 : 1;
        if (lane == 0) {
            D[root] = 0u;                         // value 0, queued
            nearq[(root >> rsh) * (rs + 1)] = root;
        }
        __threadfence_block();
        int rh = 0, rc = (lane == (root >> rsh)) ? 1 : 0;
        // ring slot of range r at position pos (r < nranges)
        auto ring_at = [&](int r, int pos) -> int32_t* {
            const int cap = min(rs, n - r * rs) + 1;
            if (pos >= cap) pos -= cap;
            return nearq + (int64_t)r * (rs + 1) + pos;
        };
        // before a phase that pushes to near: tails after the pops, counters at 0
        auto open_push = [&]() {
            int tl = rh + rc;
            if (tl >= rcap) tl -= rcap;
            rtail[lane] = tl;
            rpush[lane] = 0;
            __builtin_amdgcn_wave_barrier();
        };
        auto push_near = [&](int v) {
            const int r = v >> rsh;
            *ring_at(r, rtail[r] + atomicAdd(&rpush[r], 1)) = v;
        };
        // after it: the ring counts take in what was pushed
        auto close_push = [&]() {
            __builtin_amdgcn_wave_barrier();
            if (rvalid) rc += rpush[lane];
        };
        const int l0 = early ? dem.qptr[t] : 0, l1 = early ? dem.qptr[t + 1] : 0;
        int ncnt = 1;                             // queued in near (sum of the ring counts)
        int fcnt = 0;
        float thr = delta;
        float fmin = __uint_as_float(kInfBits);   // smallest label pushed to far
        for (;;) {
            while (ncnt > 0) {
                const int k = ncnt < NP ? ncnt : NP;
                // pop from the lowest non-empty ranges first: nodes close in id
                // (and, in Hilbert order, in space) are handled together, so
                // their label lines are reused before they leave the cache
                int incl = rc;
                for (int o = 1; o < 64; o <<= 1) {
                    const int x = __shfl_up(incl, o);
                    if (lane >= o) incl += x;
                }
                const int excl = incl - rc;
                const int take = max(0, min(rc, NP - excl));
                tpre[lane] = min(excl, NP);
                rhd[lane] = rh;
                __builtin_amdgcn_wave_barrier();
                // pop: slot j = u * 64 + lane, from the largest range r with tpre[r] <= j
                int deg[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int j = u * 64 + lane;
                    deg[u] = 0;
                    if (j < k) {
                        int lo = 0, hi = 64;
                        while (hi - lo > 1) {
                            const int mid = (lo + hi) >> 1;
                            if (tpre[mid] <= j) lo = mid; else hi = mid;
                        }
                        const int w = *ring_at(lo, rhd[lo] + (j - tpre[lo]));
                        const uint32_t lw = atomicOr(&D[w], kNotQueued);   // dequeue, read the label
                        const int e0 = rptr[w];
                        deg[u] = rptr[w + 1] - e0;
                        se0[j] = e0;
                        sdw[j] = __uint_as_float(lw & kValueBits);
                    }
                }
                rh += take;
                if (rh >= rcap) rh -= rcap;
                rc -= take;
                ncnt -= k;
                open_push();
                // exclusive prefix of in-degrees in slot order
                int base = 0;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    int incl = deg[u];
                    for (int o = 1; o < 64; o <<= 1) {
                        const int x = __shfl_up(incl, o);
                        if (lane >= o) incl += x;
                    }
                    pre[u * 64 + lane] = base + incl - deg[u];
                    base += __shfl(incl, 63);
                }
                if (lane == 0) pre[k] = base;
                const int total = base;
                __builtin_amdgcn_wave_barrier();
                for (int g0 = 0; g0 < total; g0 += 64 * V) {
                    int vv[V];
                    float cd[V];
                    bool ok[V];
#pragma unroll
                    for (int x = 0; x < V; ++x) {
                        const int g = g0 + x * 64 + lane;
                        ok[x] = g < total;
                        vv[x] = 0;
                        cd[x] = 0.0f;
                        if (ok[x]) {
                            int lo = 0, hi = k;   // owner slot: pre[lo] <= g < pre[lo + 1]
                            while (hi - lo > 1) {
                                const int mid = (lo + hi) >> 1;
                                if (pre[mid] <= g) lo = mid; else hi = mid;
                            }
                            const int e = se0[lo] + (g - pre[lo]);
                            const uint2 r = radj[e];
                            vv[x] = (int)r.x - node0;
                            cd[x] = sdw[lo] + __uint_as_float(r.y);
                        }
                    }
                    uint32_t cur[V];               // current value bits (coherent: see the word layout)
#pragma unroll
                    for (int x = 0; x < V; ++x) cur[x] = ok[x] ? (ld_coherent(&D[vv[x]]) & kValueBits) : 0u;
                    bool pn[V], pf[V];
#pragma unroll
                    for (int x = 0; x < V; ++x) {
                        pn[x] = pf[x] = false;
                        const uint32_t cb = __float_as_uint(cd[x]);
                        // cb is a queued word below the value: the min lowers the value;
                        // a replaced word that was not queued means this relaxation queued v
                        if (ok[x] && cb < cur[x] && (atomicMin(&D[vv[x]], cb) & kNotQueued)) {
                            pn[x] = cd[x] < thr;
                            pf[x] = !pn[x];
                        }
                    }
                    float fm = __uint_as_float(kInfBits);
#pragma unroll
                    for (int x = 0; x < V; ++x) {
                        const unsigned long long bn = __ballot(pn[x]), bf = __ballot(pf[x]);
                        if (pn[x]) push_near(vv[x]);
                        if (pf[x]) {
                            farq[fcnt + __popcll(bf & below)] = make_uint2((uint32_t)vv[x], __float_as_uint(cd[x]));
                            fm = fminf(fm, cd[x]);
                        }
                        ncnt += __popcll(bn);
                        fcnt += __popcll(bf);
                    }
                    fmin = fminf(fmin, wave_min(fm));
                }
                close_push();
                __threadfence_block();
            }
            // Bucket [.., thr) is drained.  Far entries carry the label they had
            // when queued; one improved since may now lie below thr.
            if (early) {
                // all origins below thr?  (cheap test before the exact one)
                bool pend = false;
                for (int l = l0 + lane; l < l1; l += 64) {
                    const int o = dem.leg_orig[l] - node0;
                    if (!(__uint_as_float(ld_coherent(&D[o]) & kValueBits) < thr)) pend = true;
                }
                if (__ballot(pend) == 0ull) {
                    // exact: move far entries whose current label is below thr
                    int moved = 0;
                    open_push();
                    for (int i0 = 0; i0 < fcnt; i0 += 64) {
                        const int i = i0 + lane;
                        const bool h = i < fcnt;
                        const uint2 ent = h ? farq[i] : make_uint2(0u, kInfBits);
                        const float dv = h ? __uint_as_float(ld_coherent(&D[ent.x]) & kValueBits) : 0.0f;
                        const bool late = h && dv < thr;
                        const unsigned long long bl = __ballot(late);
                        if (late) push_near((int)ent.x);
                        // keep the rest, in order
                        const unsigned long long bk = __ballot(h && !late);
                        if (h && !late) farq[i0 - moved + __popcll(bk & below)] = ent;
                        ncnt += __popcll(bl);
                        moved += __popcll(bl);
                    }
                    fcnt -= moved;
                    close_push();
                    __threadfence_block();
                    if (moved == 0) break;            // every node below thr is settled
                    if (fcnt > 0) {
                        float km = __uint_as_float(kInfBits);
                        for (int i = lane; i < fcnt; i += 64) km = fminf(km, __uint_as_float(farq[i].y));
                        fmin = wave_min(km);
                    } else {
                        fmin = __uint_as_float(kInfBits);
                    }
                    continue;
                }
            }
            if (fcnt == 0) break;
            // next bucket: delta above the smallest far label
            thr = fmaxf(thr, fmin) + delta;
            // FP32 absorption can make fmin + delta == fmin: always admit the minimum
            if (!(thr > fmin)) thr = __uint_as_float(__float_as_uint(fmin) + 1u);
            int keep = 0;
            float kmin = __uint_as_float(kInfBits);
            open_push();
            for (int i0 = 0; i0 < fcnt; i0 += 64) {
                const int i = i0 + lane;
                const bool h = i < fcnt;
                uint2 ent = h ? farq[i] : make_uint2(0u, kInfBits);
                if (h) ent.y = ld_coherent(&D[ent.x]) & kValueBits;   // the label now (see k_sssp_wg)
                const float dv = __uint_as_float(ent.y);
                const bool ton = h && dv < thr;
                const bool tok = h && !ton;
                const unsigned long long bn = __ballot(ton), bk = __ballot(tok);
                if (ton) push_near((int)ent.x);
                if (tok) farq[keep + __popcll(bk & below)] = ent;
                ncnt += __popcll(bn);
                keep += __popcll(bk);
                kmin = fminf(kmin, tok ? dv : __uint_as_float(kInfBits));
            }
            fcnt = keep;
            fmin = wave_min(kmin);
            close_push();
            __threadfence_block();
        }
    }
}

// Candidate label of a shortcut's source: the target's label plus each cost
// of the chain in turn (blk[0] = number of costs, then the costs), rounded to
// FP32 after every addition as the link-by-link relaxations would be.
__device__ __forceinline__ float chain_fold(const uint32_t* __restrict__ blk, float d) {
    const uint4 h = *reinterpret_cast<const uint4*>(blk);
    const int len = (int)h.x;
    d = d + __uint_as_float(h.y);
    if (len > 1) d = d + __uint_as_float(h.z);
    if (len > 2) d = d + __uint_as_float(h.w);
    for (int i = 3; i < len; i += 4) {
        const uint4 g = *reinterpret_cast<const uint4*>(blk + 1 + i);
        d = d + __uint_as_float(g.x);
        if (i + 1 < len) d = d + __uint_as_float(g.y);
        if (i + 2 < len) d = d + __uint_as_float(g.z);
        if (i + 3 < len) d = d + __uint_as_float(g.w);
    }
    return d;
}

// Workgroup-per-tree form of the same delta-stepping: the four wavefronts of
// a workgroup grow one tree together, popping up to 256 U nodes per step
// from the lowest node-id ranges, so a quarter as many trees are in flight
// for the same number of wavefronts and each keeps four times as many of its
// label lines in the L2.  Queue state (range heads and counts, near / far
// counts) is in LDS; a step is: wavefront 0 takes the pops from the lowest
// ranges; every thread pops; a workgroup prefix sum of the in-degrees;
// every thread relaxes V in-links per chunk; the counts are folded in.
//
// CT: the chain-contracted search.  Nodes left out by the contraction are
// never queued; the kept nodes' in-links come from the contracted records
// (a chain's record adds its link costs one at a time); a leg whose origin
// is left out waits for the kept nodes its label depends on; the chain
// nodes' labels are filled from their chains' ends afterwards (k_chain_fill).
//
// W: wavefronts per SIMD the register allocation leaves room for (1: the
// compiler's choice).  The contracted <2, 4> form fits 7 in 72 VGPRs with no
// spill, one more than the 6 the compiler's own choice of 74 allows.
template <int U, int V, bool CT, int W = 1>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(W))) void k_sssp_wg(NetDev net, DemDev dem, const uint2* __restrict__ radj,
                                                 label_t* labels, Scratch scr, const InstState* st,
                                                 const float* __restrict__ delta_inst, int early, int t_begin,
                                                 int t_end) {
    constexpr int NT = kWG;
    constexpr int NW = NT / 64;
    constexpr int NP = NT * U;                    // nodes per step
    __shared__ int s_pre[NP + 1];
    __shared__ float s_dw[NP];
    __shared__ int s_e0[NP];
    __shared__ int s_rh[64], s_rc[64], s_rhp[64], s_tail[64], s_push[64], s_tpre[64];
    __shared__ int s_wsum[NW];
    __shared__ int s_t, s_nn, s_fn;
    __shared__ uint32_t s_fm;
    __shared__ uint32_t s_row[CT ? NT * V : 1];   // each relaxation's source row, kept out of registers
    // queue entries: the node (near) and (node, label) (far); the contracted
    // search's also carry the node's packed row (kNoRow: read the row pointers)
    using NearE = typename std::conditional<CT, uint2, int32_t>::type;
    using FarE = typename std::conditional<CT, uint4, uint2>::type;
    // The near entries one pushing phase makes go to an LDS buffer first (the
    // next step pops them all, before the rings), and to the rings in HBM
    // once it is full: s_bp counts the pushes since the last pop.
    constexpr int NB = NP;
    __shared__ NearE s_buf[NB];
    __shared__ int s_bp;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    NearE* nearq = reinterpret_cast<NearE*>(scr.nearq) + (int64_t)blockIdx.x * scr.nmax;
    FarE* farq = reinterpret_cast<FarE*>(scr.farq) + (int64_t)blockIdx.x * scr.nmax;
    auto near_entry = [](int v, uint32_t row) -> NearE {
        if constexpr (CT) return make_uint2((uint32_t)v, row);
        else return v;
    };
    auto far_entry = [](uint32_t v, uint32_t lab, uint32_t row) -> FarE {
        if constexpr (CT) return make_uint4(v, lab, row, 0u);
        else return make_uint2(v, lab);
    };
    auto far_row = [](const FarE& e) -> uint32_t {
        if constexpr (CT) return e.z;
        else return kNoRow;
    };
    unsigned long long n_taken = 0, n_relaxed = 0;    // counted by every thread alike (uniform values)
    for (;;) {
        if (tid == 0) s_t = t_begin + atomicAdd(scr.work, 1);
        __syncthreads();
        const int t = s_t;
        __syncthreads();
        if (t >= t_end) break;
        const int inst = dem.dest_inst[t];
        if (!inst_live(st, inst)) continue;
        const InstDev I = net.inst[inst];
        const int n = I.n, node0 = I.node0;
        const int* __restrict__ rptr = (CT ? net.crptr : net.rptr) + node0;
        const uint2* __restrict__ recs = radj;
        const uint4* __restrict__ crec = reinterpret_cast<const uint4*>(net.cbuf);
        label_t* D = labels + dem.dest_lab[t];
        const int root = dem.dest_node[t] - node0;
        const float delta = delta_inst[inst];
        {
            uint4* D4 = reinterpret_cast<uint4*>(D);
            const uint32_t w0 = kNotQueued | kInfBits;
            const uint4 inf4 = make_uint4(w0, w0, w0, w0);
            const int n4 = (n + 31) / 32 * 8;
            for (int i = tid; i < n4; i += NT) D4[i] = inf4;
        }
        int rsh = 0;
        while (((n - 1) >> rsh) >= 64) ++rsh;
        const int rs = 1 << rsh;
        const int nranges = ((n - 1) >> rsh) + 1;
        if (tid < 64) {
            s_rh[tid] = 0;
            s_rc[tid] = (tid == (root >> rsh)) ? 1 : 0;
            s_push[tid] = 0;
        }
        if (tid == 0) {
            s_nn = 0;
            s_fn = 0;
            s_fm = kInfBits;
            s_bp = 0;
        }
        __threadfence_block();
        __syncthreads();
        if (tid == 0) {
            D[root] = 0u;                         // value 0, queued
            nearq[(root >> rsh) * (rs + 1)] = near_entry(root, pack_row(rptr[root], rptr[root + 1] - rptr[root]));
        }
        __threadfence_block();
        __syncthreads();
        auto ring_at = [&](int r, int pos) -> NearE* {
            const int cap = min(rs, n - r * rs) + 1;
            if (pos >= cap) pos -= cap;
            return nearq + (int64_t)r * (rs + 1) + pos;
        };
        auto push_near = [&](int v, uint32_t row) {
            const int b = atomicAdd(&s_bp, 1);
            if (b < NB) {
                s_buf[b] = near_entry(v, row);
            } else {
                const int r = v >> rsh;
                *ring_at(r, s_tail[r] + atomicAdd(&s_push[r], 1)) = near_entry(v, row);
            }
            atomicAdd(&s_nn, 1);
        };
        // wavefront 0: tails of the rings for the pushes to come
        auto open_push = [&]() {
            if (wv == 0) {
                const int cap = lane < nranges ? min(rs, n - lane * rs) + 1 : 1;
                int tl = s_rh[lane] + s_rc[lane];
                if (tl >= cap) tl -= cap;
                s_tail[lane] = tl;
                s_push[lane] = 0;
            }
        };
        // after a pushing phase (all threads past a barrier): counts folded in
        int ncnt = 1, fcnt = 0;
        float thr = delta, fmin = __uint_as_float(kInfBits);
        auto fold = [&]() -> int {
            __threadfence_block();
            __syncthreads();
            const int nn = s_nn, fn = s_fn;
            const float fm = __uint_as_float(s_fm);
            __syncthreads();
            if (wv == 0) {
                if (lane < nranges) s_rc[lane] += s_push[lane];
                s_push[lane] = 0;
            }
            if (tid == 0) {
                s_nn = 0;
                s_fn = 0;
                s_fm = kInfBits;
            }
            ncnt += nn;
            fcnt += fn;
            fmin = fminf(fmin, fm);
            return nn;
        };
        int lcur = early ? dem.qptr[t] : 0;
        const int lend = early ? dem.qptr[t + 1] : 0;
        for (;;) {
            while (ncnt > 0) {
                const int k = ncnt < NP ? ncnt : NP;
                // the buffer's entries first (all of them: kb <= k), then the
                // lowest ranges' rings
                const int kb = min(s_bp, NB);
                if (wv == 0) {
                    const int rc = s_rc[lane], rh = s_rh[lane];
                    int incl = rc;
                    for (int o = 1; o < 64; o <<= 1) {
                        const int x = __shfl_up(incl, o);
                        if (lane >= o) incl += x;
                    }
                    const int excl = incl - rc;
                    const int take = max(0, min(rc, NP - kb - excl));
                    const int cap = lane < nranges ? min(rs, n - lane * rs) + 1 : 1;
                    s_tpre[lane] = min(excl, NP - kb);
                    s_rhp[lane] = rh;
                    int nh = rh + take;
                    if (nh >= cap) nh -= cap;
                    s_rh[lane] = nh;
                    s_rc[lane] = rc - take;
                    int tl = nh + rc - take;
                    if (tl >= cap) tl -= cap;
                    s_tail[lane] = tl;
                    s_push[lane] = 0;
                }
                __syncthreads();
                if (tid == 0) s_bp = 0;               // every thread has read it; pushes come after barriers
                int deg[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int j = u * NT + tid;
                    deg[u] = 0;
                    if (j < k) {
                        NearE qe;
                        if (j < kb) {
                            qe = s_buf[j];
                        } else {
                            const int jr = j - kb;
                            int lo = 0, hi = 64;
                            while (hi - lo > 1) {
                                const int mid = (lo + hi) >> 1;
                                if (s_tpre[mid] <= jr) lo = mid; else hi = mid;
                            }
                            qe = *ring_at(lo, s_rhp[lo] + (jr - s_tpre[lo]));
                        }
                        int w, e0;
                        if constexpr (CT) {
                            w = (int)qe.x;
                            if (qe.y != kNoRow) {
                                e0 = (int)(qe.y >> kRowCountBits);
                                deg[u] = (int)(qe.y & ((1u << kRowCountBits) - 1u));
                            } else {
                                e0 = rptr[w];
                                deg[u] = rptr[w + 1] - e0;
                            }
                        } else {
                            w = qe;
                            e0 = rptr[w];
                            deg[u] = rptr[w + 1] - e0;
                        }
                        const uint32_t lw = atomicOr(&D[w], kNotQueued);   // dequeue, read the label
                        s_e0[j] = e0;
                        s_dw[j] = __uint_as_float(lw & kValueBits);
                    }
                }
                // exclusive prefix of the in-degrees in slot order (workgroup-wide)
                int base = 0;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    int incl = deg[u];
                    for (int o = 1; o < 64; o <<= 1) {
                        const int x = __shfl_up(incl, o);
                        if (lane >= o) incl += x;
                    }
                    if (lane == 63) s_wsum[wv] = incl;
                    __syncthreads();
                    int before = 0, all = 0;
                    for (int q = 0; q < NW; ++q) {
                        if (q < wv) before += s_wsum[q];
                        all += s_wsum[q];
                    }
                    s_pre[u * NT + tid] = base + before + incl - deg[u];
                    base += all;
                    __syncthreads();
                }
                if (tid == 0) s_pre[NP] = base;
                if (k < NP && tid == 0) s_pre[k] = base;
                __syncthreads();
                const int total = base;
                ncnt -= k;
                n_taken += (unsigned)k;
                n_relaxed += (unsigned)total;
                for (int g0 = 0; g0 < total; g0 += NT * V) {
                    int vv[V];
                    float cd[V];
                    bool ok[V];
#pragma unroll
                    for (int x = 0; x < V; ++x) {
                        const int g = g0 + x * NT + tid;
                        ok[x] = g < total;
                        vv[x] = 0;
                        cd[x] = 0.0f;
                        if (ok[x]) {
                            int lo = 0, hi = k;   // owner slot: pre[lo] <= g < pre[lo + 1]
                            while (hi - lo > 1) {
                                const int mid = (lo + hi) >> 1;
                                if (s_pre[mid] <= g) lo = mid; else hi = mid;
                            }
                            const int e = s_e0[lo] + (g - s_pre[lo]);
                            if (CT) {
                                // form 0: a link; 1, 2: a chain's two or three
                                // costs inline; 3: a longer chain's cost block
                                const uint4 r = crec[e];
                                const uint32_t form = r.x >> 30;
                                vv[x] = (int)(r.x & 0x3fffffffu) - node0;
                                s_row[x * NT + tid] = form != 2u ? r.w : kNoRow;   // the source's packed row
                                if (form == 3u) {
                                    cd[x] = chain_fold(net.cbuf + r.y, s_dw[lo]);
                                } else {
                                    float d = s_dw[lo] + __uint_as_float(r.y);
                                    if (form >= 1u) d = d + __uint_as_float(r.z);
                                    if (form >= 2u) d = d + __uint_as_float(r.w);
                                    cd[x] = d;
                                }
                            } else {
                                const uint2 r = recs[e];
                                vv[x] = (int)r.x - node0;
                                cd[x] = s_dw[lo] + __uint_as_float(r.y);
                            }
                        }
                    }
                    uint32_t cur[V];
#pragma unroll
                    for (int x = 0; x < V; ++x) cur[x] = ok[x] ? (ld_coherent(&D[vv[x]]) & kValueBits) : 0u;
#pragma unroll
                    for (int x = 0; x < V; ++x) {
                        const uint32_t cb = __float_as_uint(cd[x]);
                        if (ok[x] && cb < cur[x] && (atomicMin(&D[vv[x]], cb) & kNotQueued)) {
                            const uint32_t row = CT ? s_row[x * NT + tid] : kNoRow;
                            if (cd[x] < thr) {
                                push_near(vv[x], row);
                            } else {
                                farq[fcnt + atomicAdd(&s_fn, 1)] = far_entry((uint32_t)vv[x], cb, row);
                                atomicMin(&s_fm, cb);
                            }
                        }
                    }
                }
                fold();
            }
            if (early) {
                bool pend = false;
                while (lcur < lend) {
                    const int l = lcur + tid;
                    bool p = false;
                    if (l < lend) {
                        if (CT) {
                            const uint2 an = net.anc[dem.leg_orig[l]];
                            p = !(__uint_as_float(ld_coherent(&D[(int)an.x - node0]) & kValueBits) < thr &&
                                  __uint_as_float(ld_coherent(&D[(int)an.y - node0]) & kValueBits) < thr);
                        } else {
                            const int o = dem.leg_orig[l] - node0;
                            p = !(__uint_as_float(ld_coherent(&D[o]) & kValueBits) < thr);
                        }
                    }
                    if (__syncthreads_or(p)) { pend = true; break; }
                    lcur += NT;
                }
                if (!pend) {
                    // exact: queue the far nodes whose current label is below thr
                    int moved = 0, keep = 0;
                    float km = __uint_as_float(kInfBits);
                    open_push();
                    __syncthreads();
                    for (int i0 = 0; i0 < fcnt; i0 += NT) {
                        const int i = i0 + tid;
                        const bool h = i < fcnt;
                        FarE ent = h ? farq[i] : far_entry(0u, kInfBits, kNoRow);
                        if (h) ent.y = ld_coherent(&D[ent.x]) & kValueBits;   // the label now
                        const bool late = h && __uint_as_float(ent.y) < thr;
                        __syncthreads();                  // the chunk is read before it is overwritten
                        if (late) {
                            push_near((int)ent.x, far_row(ent));
                        } else if (h) {
                            farq[keep + atomicAdd(&s_fn, 1)] = ent;
                            atomicMin(&s_fm, ent.y);
                        }
                        __threadfence_block();
                        __syncthreads();
                        const int nn = s_nn, fn = s_fn;
                        const float fm = __uint_as_float(s_fm);
                        __syncthreads();
                        if (tid == 0) {
                            s_nn = 0;
                            s_fn = 0;
                            s_fm = kInfBits;
                        }
                        ncnt += nn;
                        moved += nn;
                        keep += fn;
                        km = fminf(km, fm);
                    }
                    if (wv == 0) {
                        if (lane < nranges) s_rc[lane] += s_push[lane];
                        s_push[lane] = 0;
                    }
                    __syncthreads();
                    fcnt = keep;
                    fmin = km;
                    if (moved == 0) break;                // every label below thr is final
                    continue;
                }
            }
            if (fcnt == 0) break;
            thr = fmaxf(thr, fmin) + delta;
            if (!(thr > fmin)) thr = __uint_as_float(__float_as_uint(fmin) + 1u);
            int keep = 0;
            float km = __uint_as_float(kInfBits);
            open_push();
            __syncthreads();
            for (int i0 = 0; i0 < fcnt; i0 += NT) {
                const int i = i0 + tid;
                const bool h = i < fcnt;
                FarE ent = h ? farq[i] : far_entry(0u, kInfBits, kNoRow);
                // key by the label now: a far node improved since its push keeps
                // its queued flag and is not pushed again, and waiting for the
                // threshold to pass its old label would make every node it
                // reaches meanwhile be popped again
                if (h) ent.y = ld_coherent(&D[ent.x]) & kValueBits;
                __syncthreads();
                if (h && __uint_as_float(ent.y) < thr) {
                    push_near((int)ent.x, far_row(ent));
                } else if (h) {
                    farq[keep + atomicAdd(&s_fn, 1)] = ent;
                    atomicMin(&s_fm, ent.y);
                }
                __threadfence_block();
                __syncthreads();
                const int nn = s_nn, fn = s_fn;
                const float fm = __uint_as_float(s_fm);
                __syncthreads();
                if (tid == 0) {
                    s_nn = 0;
                    s_fn = 0;
                    s_fm = kInfBits;
                }
                ncnt += nn;
                keep += fn;
                km = fminf(km, fm);
            }
            if (wv == 0) {
                if (lane < nranges) s_rc[lane] += s_push[lane];
                s_push[lane] = 0;
            }
            __syncthreads();
            fcnt = keep;
            fmin = km;
        }
        __syncthreads();
    }
    if (scr.stats && tid == 0) {
        atomicAdd(&scr.stats[0], n_taken);
        atomicAdd(&scr.stats[1], n_relaxed);
    }
}

template <int U, int V>
__global__ __launch_bounds__(kWG) void k_sssp_wn(NetDev net, DemDev dem, const uint2* __restrict__ radj,
                                                 label_t* labels, Scratch scr, const InstState* st,
                                                 const float* __restrict__ delta_inst, int early, int t_begin,
                                                 int t_end) {
    constexpr int NT = kWG;
    constexpr int NW = NT / 64;
    constexpr int NP = NT * U;                    // nodes per step
    __shared__ int s_pre[NP + 1];
    __shared__ float s_dw[NP];
    __shared__ int s_e0[NP];
    __shared__ int s_rh[64], s_rc[64], s_rhp[64], s_tail[64], s_push[64], s_tpre[64];
    __shared__ int s_wsum[NW];
    __shared__ int s_t, s_nn, s_fn;
    __shared__ uint32_t s_fm;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    int32_t* nearq = scr.nearq + (int64_t)blockIdx.x * scr.nmax;
    uint2* farq = reinterpret_cast<uint2*>(scr.farq) + (int64_t)blockIdx.x * scr.nmax;
    unsigned long long n_taken = 0, n_relaxed = 0;    // counted by every thread alike (uniform values)
    for (;;) {
        if (tid == 0) s_t = t_begin + atomicAdd(scr.work, 1);
        __syncthreads();
        const int t = s_t;
        __syncthreads();
        if (t >= t_end) break;
        const int inst = dem.dest_inst[t];
        if (!inst_live(st, inst)) continue;
        const InstDev I = net.inst[inst];
        const int n = I.n, node0 = I.node0;
        const int* __restrict__ rptr = net.rptr + node0;
        label_t* D = labels + dem.dest_lab[t];
        const int root = dem.dest_node[t] - node0;
        const float delta = delta_inst[inst];
        {
            uint4* D4 = reinterpret_cast<uint4*>(D);
            const uint32_t w0 = kNotQueued | kInfBits;
            const uint4 inf4 = make_uint4(w0, w0, w0, w0);
            const int n4 = (n + 31) / 32 * 8;
            for (int i = tid; i < n4; i += NT) D4[i] = inf4;
        }
        int rsh = 0;
        while (((n - 1) >> rsh) >= 64) ++rsh;
        const int rs = 1 << rsh;
        const int nranges = ((n - 1) >> rsh) + 1;
        if (tid < 64) {
            s_rh[tid] = 0;
            s_rc[tid] = (tid == (root >> rsh)) ? 1 : 0;
            s_push[tid] = 0;
        }
        if (tid == 0) {
            s_nn = 0;
            s_fn = 0;
            s_fm = kInfBits;
        }
        __threadfence_block();
        __syncthreads();
        if (tid == 0) {
            D[root] = 0u;                         // value 0, queued
            nearq[(root >> rsh) * (rs + 1)] = root;
        }
        __threadfence_block();
        __syncthreads();
        auto ring_at = [&](int r, int pos) -> int32_t* {
            const int cap = min(rs, n - r * rs) + 1;
            if (pos >= cap) pos -= cap;
            return nearq + (int64_t)r * (rs + 1) + pos;
        };
        auto push_near = [&](int v) {
            const int r = v >> rsh;
            *ring_at(r, s_tail[r] + atomicAdd(&s_push[r], 1)) = v;
            atomicAdd(&s_nn, 1);
        };
        // wavefront 0: tails of the rings for the pushes to come
        auto open_push = [&]() {
            if (wv == 0) {
                const int cap = lane < nranges ? min(rs, n - lane * rs) + 1 : 1;
                int tl = s_rh[lane] + s_rc[lane];
                if (tl >= cap) tl -= cap;
                s_tail[lane] = tl;
                s_push[lane] = 0;
            }
        };
        // after a pushing phase (all threads past a barrier): counts folded in
        int ncnt = 1, fcnt = 0;
        float thr = delta, fmin = __uint_as_float(kInfBits);
        auto fold = [&]() -> int {
            __threadfence_block();
            __syncthreads();
            const int nn = s_nn, fn = s_fn;
            const float fm = __uint_as_float(s_fm);
            __syncthreads();
            if (wv == 0) {
                if (lane < nranges) s_rc[lane] += s_push[lane];
                s_push[lane] = 0;
            }
            if (tid == 0) {
                s_nn = 0;
                s_fn = 0;
                s_fm = kInfBits;
            }
            ncnt += nn;
            fcnt += fn;
            fmin = fminf(fmin, fm);
            return nn;
        };
        int lcur = early ? dem.qptr[t] : 0;
        const int lend = early ? dem.qptr[t + 1] : 0;
        for (;;) {
            while (ncnt > 0) {
                const int k = ncnt < NP ? ncnt : NP;
                if (wv == 0) {
                    const int rc = s_rc[lane], rh = s_rh[lane];
                    int incl = rc;
                    for (int o = 1; o < 64; o <<= 1) {
                        const int x = __shfl_up(incl, o);
                        if (lane >= o) incl += x;
                    }
                    const int excl = incl - rc;
                    const int take = max(0, min(rc, NP - excl));
                    const int cap = lane < nranges ? min(rs, n - lane * rs) + 1 : 1;
                    s_tpre[lane] = min(excl, NP);
                    s_rhp[lane] = rh;
                    int nh = rh + take;
                    if (nh >= cap) nh -= cap;
                    s_rh[lane] = nh;
                    s_rc[lane] = rc - take;
                    int tl = nh + rc - take;
                    if (tl >= cap) tl -= cap;
                    s_tail[lane] = tl;
                    s_push[lane] = 0;
                }
                __syncthreads();
                // every thread takes up to U nodes and relaxes all their in-links
                // itself: in-degrees of road networks are small, so the owner
                // search and the degree prefix sum of k_sssp_wg are left out
                int wn_[U], e0_[U], e1_[U];
                float dw_[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int j = u * NT + tid;
                    wn_[u] = -1;
                    e0_[u] = e1_[u] = 0;
                    dw_[u] = 0.0f;
                    if (j < k) {
                        int lo = 0, hi = 64;
                        while (hi - lo > 1) {
                            const int mid = (lo + hi) >> 1;
                            if (s_tpre[mid] <= j) lo = mid; else hi = mid;
                        }
                        wn_[u] = *ring_at(lo, s_rhp[lo] + (j - s_tpre[lo]));
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (wn_[u] < 0) continue;
                    const uint32_t lw = atomicOr(&D[wn_[u]], kNotQueued);   // dequeue, read the label
                    e0_[u] = rptr[wn_[u]];
                    e1_[u] = rptr[wn_[u] + 1];
                    dw_[u] = __uint_as_float(lw & kValueBits);
                }
                ncnt -= k;
                n_taken += (unsigned)k;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    for (int e = e0_[u]; e < e1_[u]; e += V) {
                        int vv[V];
                        float cd[V];
                        bool ok[V];
#pragma unroll
                        for (int x = 0; x < V; ++x) {
                            ok[x] = e + x < e1_[u];
                            vv[x] = 0;
                            cd[x] = 0.0f;
                            if (ok[x]) {
                                const uint2 r = radj[e + x];
                                vv[x] = (int)r.x - node0;
                                cd[x] = dw_[u] + __uint_as_float(r.y);
                            }
                        }
                        uint32_t cur[V];
#pragma unroll
                        for (int x = 0; x < V; ++x) cur[x] = ok[x] ? (ld_coherent(&D[vv[x]]) & kValueBits) : 0u;
#pragma unroll
                        for (int x = 0; x < V; ++x) {
                            const uint32_t cb = __float_as_uint(cd[x]);
                            if (ok[x] && cb < cur[x] && (atomicMin(&D[vv[x]], cb) & kNotQueued)) {
                                if (cd[x] < thr) {
                                    push_near(vv[x]);
                                } else {
                                    farq[fcnt + atomicAdd(&s_fn, 1)] = make_uint2((uint32_t)vv[x], cb);
                                    atomicMin(&s_fm, cb);
                                }
                            }
                        }
                    }
                    n_relaxed += (unsigned)(e1_[u] - e0_[u]);
                }
                fold();
            }
            if (early) {
                bool pend = false;
                while (lcur < lend) {
                    const int l = lcur + tid;
                    bool p = false;
                    if (l < lend) {
                        const int o = dem.leg_orig[l] - node0;
                        p = !(__uint_as_float(ld_coherent(&D[o]) & kValueBits) < thr);
                    }
                    if (__syncthreads_or(p)) { pend = true; break; }
                    lcur += NT;
                }
                if (!pend) {
                    // exact: queue the far nodes whose current label is below thr
                    int moved = 0, keep = 0;
                    float km = __uint_as_float(kInfBits);
                    open_push();
                    __syncthreads();
                    for (int i0 = 0; i0 < fcnt; i0 += NT) {
                        const int i = i0 + tid;
                        const bool h = i < fcnt;
                        uint2 ent = h ? farq[i] : make_uint2(0u, kInfBits);
                        if (h) ent.y = ld_coherent(&D[ent.x]) & kValueBits;   // the label now
                        const bool late = h && __uint_as_float(ent.y) < thr;
                        __syncthreads();                  // the chunk is read before it is overwritten
                        if (late) {
                            push_near((int)ent.x);
                        } else if (h) {
                            farq[keep + atomicAdd(&s_fn, 1)] = ent;
                            atomicMin(&s_fm, ent.y);
                        }
                        __threadfence_block();
                        __syncthreads();
                        const int nn = s_nn, fn = s_fn;
                        const float fm = __uint_as_float(s_fm);
                        __syncthreads();
                        if (tid == 0) {
                            s_nn = 0;
                            s_fn = 0;
                            s_fm = kInfBits;
                        }
                        ncnt += nn;
                        moved += nn;
                        keep += fn;
                        km = fminf(km, fm);
                    }
                    if (wv == 0) {
                        if (lane < nranges) s_rc[lane] += s_push[lane];
                        s_push[lane] = 0;
                    }
                    __syncthreads();
                    fcnt = keep;
                    fmin = km;
                    if (moved == 0) break;                // every label below thr is final
                    continue;
                }
            }
            if (fcnt == 0) break;
            thr = fmaxf(thr, fmin) + delta;
            if (!(thr > fmin)) thr = __uint_as_float(__float_as_uint(fmin) + 1u);
            int keep = 0;
            float km = __uint_as_float(kInfBits);
            open_push();
            __syncthreads();
            for (int i0 = 0; i0 < fcnt; i0 += NT) {
                const int i = i0 + tid;
                const bool h = i < fcnt;
                uint2 ent = h ? farq[i] : make_uint2(0u, kInfBits);
                // key by the label now: a far node improved since its push keeps
                // its queued flag and is not pushed again, and waiting for the
                // threshold to pass its old label would make every node it
                // reaches meanwhile be popped again
                if (h) ent.y = ld_coherent(&D[ent.x]) & kValueBits;
                __syncthreads();
                if (h && __uint_as_float(ent.y) < thr) {
                    push_near((int)ent.x);
                } else if (h) {
                    farq[keep + atomicAdd(&s_fn, 1)] = ent;
                    atomicMin(&s_fm, ent.y);
                }
                __threadfence_block();
                __syncthreads();
                const int nn = s_nn, fn = s_fn;
                const float fm = __uint_as_float(s_fm);
                __syncthreads();
                if (tid == 0) {
                    s_nn = 0;
                    s_fn = 0;
                    s_fm = kInfBits;
                }
                ncnt += nn;
                keep += fn;
                km = fminf(km, fm);
            }
            if (wv == 0) {
                if (lane < nranges) s_rc[lane] += s_push[lane];
                s_push[lane] = 0;
            }
            __syncthreads();
            fcnt = keep;
            fmin = km;
        }
        __syncthreads();
    }
    if (scr.stats) {
        for (int o = 32; o > 0; o >>= 1) n_relaxed += __shfl_xor(n_relaxed, o);
        if (tid == 0) atomicAdd(&scr.stats[0], n_taken);
        if (lane == 0) atomicAdd(&scr.stats[1], n_relaxed);
    }
}

// Block-local form of the same delta-stepping.  The node ids of an instance
// are cut into blocks of B consecutive ids (in Hilbert order a block is a
// compact patch of the network).  The near queue holds blocks, not nodes: a
// block is queued (once: a bit per block in LDS) while it holds a queued node
// whose label is below the bucket bound thr.  A step takes up to NW * KB
// blocks off the queue; each wavefront, for each of its blocks,
//   - loads the block's label words and in-link offsets (coalesced) and its
//     in-link records into LDS;
//   - relaxes inside the block to closure: every queued node below thr is
//     taken (flag set with an LDS atomicOr that returns its label) and its
//     in-links relaxed, those from inside the block by an LDS atomicMin on the
//     staged word, those from other blocks into a mailbox; repeated until no
//     queued node below thr is left -- many hops for one load of the block;
//   - writes the changed words back; a node first queued in this visit at or
//     above thr goes to the far queue.
// Then the whole workgroup applies the mailboxes to the labels in memory (a
// coherent read, then an atomicMin where the candidate is lower), queueing the
// block of every node it improves below thr and sending to the far queue the
// nodes it queues at or above thr.  Only one workgroup touches a tree, and
// the two phases are separated by barriers, so the words a phase-1 wavefront
// stages are not changed under it.  Whatever the order, the labels reach the
// least fixed point of D(v) = min_e fl32(D(head e) + c_e), as in k_sssp_wg.
//   A node is sent to the far queue at most once per tree: it is queued at or
// above thr only before it is first taken (afterwards its label stays below
// the thr of that moment), so the far queue holds at most n entries.
// B: nodes per block (a multiple of 64); KB: blocks per wavefront per step.
// kBlkMaxBits (qdta_internal.h): blocks per tree the LDS bitmap covers.
template <int B, int KB>
__global__ __launch_bounds__(kWG) void k_sssp_blk(NetDev net, DemDev dem, const uint2* __restrict__ radj,
                                                  label_t* labels, Scratch scr, const InstState* st,
                                                  const float* __restrict__ delta_inst, int early, int t_begin,
                                                  int t_end) {
    constexpr int NT = kWG;
    constexpr int NW = NT / 64;
    constexpr int R = B / 64;                   // nodes per lane in a block
    constexpr int KMAX = NW * KB;               // blocks per step
    constexpr int kBlkEmax = 3 * B;             // in-link records staged per block (the rest are read in place)
    constexpr int kBlkMbx = 2 * B;              // mailbox entries (target, candidate) per wavefront and step
    constexpr int kBig = 8;                     // per wavefront and step: nodes whose cross-block in-links
                                                // are too many for the mailbox, relaxed in phase 2 by all threads
    __shared__ uint32_t s_bits[kBlkMaxBits / 32];
    __shared__ uint32_t s_lab[NW][B];
    __shared__ int s_rp[NW][B + 1];
    __shared__ uint2 s_adj[NW][kBlkEmax];
    // one mailbox and one big-node list per (wavefront, block of the step), so
    // every block visit starts with room for any one node: each visit takes
    // at least one node
    __shared__ uint2 s_mb[NW * KB][kBlkMbx];
    __shared__ int s_mc[NW * KB];
    __shared__ uint2 s_big[NW * KB][kBig];
    __shared__ int s_nbig[NW * KB];
    __shared__ int s_blk[KMAX];
    __shared__ int s_t, s_qh, s_qn, s_qt, s_fn;
    __shared__ uint32_t s_fm;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const unsigned long long below = lanes_below(lane);
    int32_t* ring = scr.nearq + (int64_t)blockIdx.x * scr.nmax;
    uint2* farq = reinterpret_cast<uint2*>(scr.farq) + (int64_t)blockIdx.x * scr.nmax;
    uint32_t* L = s_lab[wv];
    int* RP = s_rp[wv];
    uint2* A = s_adj[wv];
    unsigned long long n_taken = 0, n_relaxed = 0;    // this lane's work, for the counters
    for (;;) {
        if (tid == 0) s_t = t_begin + atomicAdd(scr.work, 1);
        __syncthreads();
        const int t = s_t;
        __syncthreads();
        if (t >= t_end) break;
        const int inst = dem.dest_inst[t];
        if (!inst_live(st, inst)) continue;
        const InstDev I = net.inst[inst];
        const int n = I.n, node0 = I.node0;
        const int* __restrict__ rptr = net.rptr + node0;
        label_t* D = labels + dem.dest_lab[t];
        const int root = dem.dest_node[t] - node0;
        const float delta = delta_inst[inst];
        const int nb = (n + B - 1) / B;
        const int qcap = nb + 1;                // ring of block ids; at most nb are queued
        {
            uint4* D4 = reinterpret_cast<uint4*>(D);
            const uint32_t w0 = kNotQueued | kInfBits;
            const uint4 inf4 = make_uint4(w0, w0, w0, w0);
            const int n4 = (n + 31) / 32 * 8;
            for (int i = tid; i < n4; i += NT) D4[i] = inf4;
        }
        for (int i = tid; i < (nb + 31) / 32; i += NT) s_bits[i] = 0u;
        if (tid == 0) {
            s_qh = 0;
            s_qn = 0;
            s_qt = 0;
            s_fn = 0;
            s_fm = kInfBits;
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0) {
            D[root] = 0u;                       // value 0, queued
            const int b = root / B;
            s_bits[b >> 5] |= 1u << (b & 31);
            ring[0] = b;
            s_qt = 1;
            s_qn = 1;
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        // queue block b unless it is queued (LDS bit); safe from any thread
        auto push_block = [&](int b) {
            const uint32_t bit = 1u << (b & 31);
            if (atomicOr(&s_bits[b >> 5], bit) & bit) return;
            int pos = atomicAdd(&s_qt, 1);
            pos = pos % qcap;
            ring[pos] = b;
            atomicAdd(&s_qn, 1);
        };
        float thr = delta;
        int fcnt = 0;
        float fmin = __uint_as_float(kInfBits);
        int lcur = early ? dem.qptr[t] : 0;
        const int lend = early ? dem.qptr[t + 1] : 0;
        for (;;) {
            for (;;) {
                const int qn = s_qn;
                if (qn == 0) break;
                const int k = qn < KMAX ? qn : KMAX;
                const int qh = s_qh;
                __syncthreads();                // every thread has read the counters
                if (tid < k) {
                    const int b = ring[(qh + tid) % qcap];
                    s_blk[tid] = b;
                    atomicAnd(&s_bits[b >> 5], ~(1u << (b & 31)));
                }
                if (tid == 0) {
                    s_qh = (qh + k) % qcap;
                    s_qn = qn - k;
                }
                if (tid < KMAX) {
                    s_mc[tid] = 0;
                    s_nbig[tid] = 0;
                }
                __syncthreads();
                // ---- phase 1: each wavefront relaxes its blocks to closure
                for (int kb = 0; kb < KB; ++kb) {
                    const int j = kb * NW + wv;
                    if (j >= k) break;
                    const int b = s_blk[j];
                    uint2* MB = s_mb[j];
                    uint2* BG = s_big[j];
                    int mcnt = 0, nbig = 0;
                    const int v0 = b * B;
                    const int nv = min(B, n - v0);
                    uint32_t w0[R];
                    bool q0[R];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int i = lane + 64 * r;
                        w0[r] = i < nv ? ld_coherent(&D[v0 + i]) : (kNotQueued | kInfBits);
                        q0[r] = !(w0[r] & kNotQueued);
                        L[i] = w0[r];
                        RP[i] = i < nv ? rptr[v0 + i] : 0;
                    }
                    if (lane == 0) RP[nv] = rptr[v0 + nv];
                    __builtin_amdgcn_wave_barrier();
                    const int e_lo = RP[0];
                    const int E = RP[nv] - e_lo;
                    for (int x = lane; x < E && x < kBlkEmax; x += 64) A[x] = radj[e_lo + x];
                    __builtin_amdgcn_wave_barrier();
                    bool skipped = false;
                    for (;;) {
                        bool act[R];
                        int cc[R];
                        bool any = false;
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const int i = lane + 64 * r;
                            const uint32_t w = i < nv ? L[i] : kNotQueued;
                            act[r] = !(w & kNotQueued) && __uint_as_float(w) < thr;
                            cc[r] = 0;
                            if (act[r]) {
                                any = true;
                                for (int e = RP[i]; e < RP[i + 1]; ++e) {
                                    const int x = e - e_lo;
                                    const uint32_t src = x < kBlkEmax ? A[x].x : radj[e].x;
                                    if ((unsigned)((int)src - node0 - v0) >= (unsigned)nv) ++cc[r];
                                }
                            }
                        }
                        if (__ballot(any) == 0ull) break;
                        // mailbox room: nodes in (r, lane) order take their cross-block
                        // in-links while they fit; the rest stay queued for a later visit.
                        // A node with more than half a mailbox of them ("big") takes one
                        // of kBig slots instead and is relaxed in phase 2.
                        bool big[R];
                        int excl[R], bex[R];
                        int base = 0, bbase = 0;
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            big[r] = act[r] && cc[r] > kBlkMbx / 2;
                            const int c1 = big[r] ? 0 : cc[r];
                            int incl = c1;
                            for (int o = 1; o < 64; o <<= 1) {
                                const int y = __shfl_up(incl, o);
                                if (lane >= o) incl += y;
                            }
                            excl[r] = base + incl - c1;
                            base += __shfl(incl, 63);
                            const unsigned long long bb = __ballot(big[r]);
                            bex[r] = bbase + __popcll(bb & below);
                            bbase += __popcll(bb);
                        }
                        bool fit[R];
                        bool anyfit = false, anyskip = false;
                        int used = 0, bused = 0;
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            fit[r] = act[r] && (big[r] ? nbig + bex[r] < kBig : mcnt + excl[r] + cc[r] <= kBlkMbx);
                            anyfit |= fit[r];
                            anyskip |= act[r] && !fit[r];
                            if (fit[r] && !big[r]) used = max(used, excl[r] + cc[r]);
                            if (fit[r] && big[r]) bused = max(bused, bex[r] + 1);
                        }
                        for (int o = 32; o > 0; o >>= 1) {
                            used = max(used, __shfl_xor(used, o));
                            bused = max(bused, __shfl_xor(bused, o));
                        }
                        if (__ballot(anyskip) != 0ull) skipped = true;
                        if (__ballot(anyfit) == 0ull) break;
                        float du[R];
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            du[r] = 0.0f;
                            if (fit[r]) {
                                const int i = lane + 64 * r;
                                du[r] = __uint_as_float(atomicOr(&L[i], kNotQueued) & kValueBits);
                                n_taken += 1;
                                n_relaxed += (unsigned)(RP[i + 1] - RP[i]);
                            }
                        }
                        __builtin_amdgcn_wave_barrier();
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            if (!fit[r]) continue;
                            const int i = lane + 64 * r;
                            if (big[r]) BG[nbig + bex[r]] = make_uint2((uint32_t)(v0 + i), __float_as_uint(du[r]));
                            int slot = mcnt + excl[r];
                            for (int e = RP[i]; e < RP[i + 1]; ++e) {
                                const int x = e - e_lo;
                                const uint2 rec = x < kBlkEmax ? A[x] : radj[e];
                                const int sv = (int)rec.x - node0;
                                const float cd = du[r] + __uint_as_float(rec.y);
                                const uint32_t cb = __float_as_uint(cd);
                                const int jj = sv - v0;
                                if ((unsigned)jj < (unsigned)nv) {
                                    if (cb < (L[jj] & kValueBits)) atomicMin(&L[jj], cb);
                                } else if (!big[r]) {
                                    MB[slot++] = make_uint2((uint32_t)sv, cb);
                                }
                            }
                        }
                        mcnt += used;
                        nbig += bused;
                        __builtin_amdgcn_wave_barrier();
                    }
                    // write the changed words back; a node first queued in this visit
                    // at or above thr goes to the far queue
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int i = lane + 64 * r;
                        const uint32_t w = i < nv ? L[i] : w0[r];
                        if (w != w0[r]) D[v0 + i] = w;
                        const bool far = i < nv && !(w & kNotQueued) && !(__uint_as_float(w) < thr);
                        const bool tofar = far && !q0[r];
                        if (far && w != w0[r]) atomicMin(&s_fm, w);
                        const unsigned long long bf = __ballot(tofar);
                        if (bf) {
                            int fb = 0;
                            if (lane == 0) fb = atomicAdd(&s_fn, __popcll(bf));
                            fb = __shfl(fb, 0);
                            if (tofar) farq[fcnt + fb + __popcll(bf & below)] = make_uint2((uint32_t)(v0 + i), w);
                        }
                    }
                    if (skipped && lane == 0) push_block(b);
                    if (lane == 0) {
                        s_mc[j] = mcnt;
                        s_nbig[j] = nbig;
                    }
                    __builtin_amdgcn_wave_barrier();
                }
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                // ---- phase 2: the mailboxes into the labels in memory
                auto apply = [&](int sv, uint32_t cb) {
                    const uint32_t cur = ld_coherent(&D[sv]);
                    if (cb < (cur & kValueBits)) {
                        const uint32_t old = atomicMin(&D[sv], cb);
                        const bool below_thr = __uint_as_float(cb) < thr;
                        if (old & kNotQueued) {
                            // this relaxation queued the node
                            if (below_thr) {
                                push_block(sv / B);
                            } else {
                                const int fp = atomicAdd(&s_fn, 1);
                                farq[fcnt + fp] = make_uint2((uint32_t)sv, cb);
                                atomicMin(&s_fm, cb);
                            }
                        } else if (!(__uint_as_float(old & kValueBits) < thr)) {
                            if (below_thr) push_block(sv / B);   // a far node now below thr
                            else atomicMin(&s_fm, cb);           // a far node improved
                        }
                    }
                };
                int mtot = 0, moff[KMAX];
#pragma unroll
                for (int w = 0; w < KMAX; ++w) {
                    moff[w] = mtot;
                    mtot += s_mc[w];
                }
                for (int g = tid; g < mtot; g += NT) {
                    int w = 0;
#pragma unroll
                    for (int x = 1; x < KMAX; ++x)
                        if (g >= moff[x]) w = x;
                    const uint2 m = s_mb[w][g - moff[w]];
                    apply((int)m.x, m.y);
                }
                // the big nodes' cross-block in-links, spread over the workgroup
                for (int w = 0; w < KMAX; ++w) {
                    for (int x = 0; x < s_nbig[w]; ++x) {
                        const uint2 bg = s_big[w][x];
                        const int u = (int)bg.x, ub = u / B;
                        const float du = __uint_as_float(bg.y);
                        for (int e = rptr[u] + tid; e < rptr[u + 1]; e += NT) {
                            const uint2 rec = radj[e];
                            const int sv = (int)rec.x - node0;
                            if (sv / B != ub) apply(sv, __float_as_uint(du + __uint_as_float(rec.y)));
                        }
                    }
                }
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                fcnt += s_fn;
                fmin = fminf(fmin, __uint_as_float(s_fm));
                __syncthreads();
                if (tid == 0) {
                    s_fn = 0;
                    s_fm = kInfBits;
                }
                __syncthreads();
            }
            // bucket [.., thr) drained: every label below thr is final
            if (early) {
                bool pend = false;
                while (lcur < lend) {
                    const int l = lcur + tid;
                    bool p = false;
                    if (l < lend) {
                        const int o = dem.leg_orig[l] - node0;
                        p = !(__uint_as_float(ld_coherent(&D[o]) & kValueBits) < thr);
                    }
                    if (__syncthreads_or(p)) { pend = true; break; }
                    lcur += NT;
                }
                if (!pend) break;               // every origin is settled
            }
            if (fcnt == 0) break;
            thr = fmaxf(thr, fmin) + delta;
            if (!(thr > fmin)) thr = __uint_as_float(__float_as_uint(fmin) + 1u);
            // move the far nodes below thr (keyed by their labels now) to the
            // near queue; drop those taken since (flag set)
            int keep = 0;
            float km = __uint_as_float(kInfBits);
            for (int i0 = 0; i0 < fcnt; i0 += NT) {
                const int i = i0 + tid;
                const bool h = i < fcnt;
                uint2 ent = h ? farq[i] : make_uint2(0u, kInfBits);
                uint32_t cur = h ? ld_coherent(&D[ent.x]) : kNotQueued;
                __syncthreads();                // the chunk is read before it is overwritten
                const bool live = h && !(cur & kNotQueued);
                ent.y = cur & kValueBits;
                if (live && __uint_as_float(ent.y) < thr) {
                    push_block((int)ent.x / B);
                } else if (live) {
                    farq[keep + atomicAdd(&s_fn, 1)] = ent;
                    atomicMin(&s_fm, ent.y);
                }
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                const int fn = s_fn;
                const float fm = __uint_as_float(s_fm);
                __syncthreads();
                if (tid == 0) {
                    s_fn = 0;
                    s_fm = kInfBits;
                }
                keep += fn;
                km = fminf(km, fm);
            }
            __syncthreads();
            fcnt = keep;
            fmin = km;
        }
        __syncthreads();
    }
    if (scr.stats) {
        for (int o = 32; o > 0; o >>= 1) {
            n_taken += __shfl_xor(n_taken, o);
            n_relaxed += __shfl_xor(n_relaxed, o);
        }
        if (lane == 0) {
            atomicAdd(&scr.stats[0], n_taken);
            atomicAdd(&scr.stats[1], n_relaxed);
        }
    }
}

// Bucket width per instance: delta = scale * (geometric mean link cost of the
// instance).  The geometric mean follows the typical link; the arithmetic
// mean is dominated by the few links that congestion makes very slow.
// Partial sums of log(cost) per link chunk, then one division per instance.
__global__ __launch_bounds__(kWG) void k_logcost(NetDev net, const float* __restrict__ cost, double* logsum) {
    __shared__ double part[kWG];
    const int b = blockIdx.x;
    const int inst = net.blk_inst[b];
    const InstDev I = net.inst[inst];
    const int a0 = net.blk_start[b];
    const int a1 = min(a0 + kChunk, I.link0 + I.m);
    double s = 0.0;
    for (int a = a0 + threadIdx.x; a < a1; a += kWG) s += log((double)cost[a]);
    part[threadIdx.x] = s;
    __syncthreads();
    for (int k = kWG / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) part[threadIdx.x] += part[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(&logsum[inst], part[0]);
}

__global__ void k_delta(NetDev net, const double* logsum, double scale, float* delta_inst) {
    const int inst = blockIdx.x * blockDim.x + threadIdx.x;
    if (inst >= net.ninst) return;
    const InstDev I = net.inst[inst];
    double d = I.m > 0 ? scale * exp(logsum[inst] / (double)I.m) : 1.0;
    if (!(d > 0.0) || !(d < 3.0e38)) d = 3.0e38;
    delta_inst[inst] = (float)d;
}

hipError_t launch_delta(hipStream_t s, const NetDev& net, const float* cost, double delta_scale, float* delta_inst,
                        double* logsum) {
    hipError_t e0 = launch_fill_i64(s, reinterpret_cast<int64_t*>(logsum), 0, net.ninst);
    if (e0 != hipSuccess) return e0;
    if (net.nblk > 0) hipLaunchKernelGGL(k_logcost, dim3(net.nblk), dim3(kWG), 0, s, net, cost, logsum);
    hipLaunchKernelGGL(k_delta, dim3((net.ninst + 63) / 64), dim3(64), 0, s, net, logsum, delta_scale, delta_inst);
    return hipGetLastError();
}

// Labels of the chain nodes left out of the contracted search, from their
// chains' ends: for chain node x_j, the FP32 fold from v through x_k..x_j
// and the fold from u through x_1..x_j (each over links that exist: a
// missing link's +inf cost stops the fold), and the lesser of the two.
// Turning back inside a chain never beats this, since each addition of a
// non-negative cost keeps or raises a value.  Work item (r, t): chunk r of
// kFillChunk chains of tree t's instance, kFillPer per thread with their
// header and end-label loads in flight together; items run chunk by chunk,
// so the trees in flight share the chunk's headers and blocks in the cache.
constexpr int kFillPer = kFillChunk / kWG;
__global__ __launch_bounds__(kWG) void k_chain_fill(NetDev net, DemDev dem, label_t* labels, const InstState* st,
                                                    int t_begin, int t_end) {
    const int64_t nq = t_end - t_begin;
    const int64_t items = (int64_t)net.fill_chunks * nq;
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int r = (int)(it / nq);
        const int t = t_begin + (int)(it - (int64_t)r * nq);
        const int inst = dem.dest_inst[t];
        if (!inst_live(st, inst)) continue;
        const int cb = net.inst_chain[inst] + r * kFillChunk;
        const int ce = min(net.inst_chain[inst + 1], cb + kFillChunk);
        if (cb >= ce) continue;
        label_t* D = labels + dem.dest_lab[t];
        const int node0 = net.inst[inst].node0;
        // loads with in-range indices whether or not the slot has a chain, so
        // that none of them waits on a branch
        int4 h[kFillPer];
        bool ok[kFillPer];
#pragma unroll
        for (int q = 0; q < kFillPer; ++q) {
            const int ch = cb + q * kWG + (int)threadIdx.x;
            ok[q] = ch < ce;
            h[q] = net.ch_hdr[min(ch, ce - 1)];
        }
        uint32_t wu[kFillPer], wv[kFillPer];
#pragma unroll
        for (int q = 0; q < kFillPer; ++q) {
            wu[q] = D[h[q].x - node0];
            wv[q] = D[h[q].y - node0];
        }
#pragma unroll
        for (int q = 0; q < kFillPer; ++q) {
            const float du = __uint_as_float(wu[q] & kValueBits), dv = __uint_as_float(wv[q] & kValueBits);
            if (!ok[q] || (!(du < __uint_as_float(kInfBits)) && !(dv < __uint_as_float(kInfBits)))) continue;
            const uint32_t* blk = net.cbuf + h[q].w;
            const int k = h[q].z;
            float lv[kChainMax];
            float l = du;
#pragma unroll
            for (int j = 0; j < kChainMax; ++j) {
                if (j < k) {
                    l = l + __uint_as_float(blk[3 * j + 2]);
                    lv[j] = l;
                }
            }
            float rv = dv;
#pragma unroll
            for (int j = kChainMax - 1; j >= 0; --j) {
                if (j < k) {
                    rv = rv + __uint_as_float(blk[3 * j + 1]);
                    D[(int)blk[3 * j] - node0] = kNotQueued | __float_as_uint(fminf(lv[j], rv));
                }
            }
        }
    }
}

hipError_t launch_chain_fill(hipStream_t s, const NetDev& net, const DemDev& dem, label_t* labels,
                             const InstState* st, int t_begin, int t_end) {
    const int64_t items = (int64_t)net.fill_chunks * (t_end - t_begin);
    if (items <= 0 || !net.cbuf) return hipSuccess;
    hipLaunchKernelGGL(k_chain_fill, dim3((unsigned)std::min<int64_t>(items, 4096)), dim3(kWG), 0, s, net, dem, labels,
                       st, t_begin, t_end);
    return hipGetLastError();
}

hipError_t launch_trees(hipStream_t s, const NetDev& net, const DemDev& dem, const uint2* radj, label_t* labels,
                        const Scratch& scr, int slots, const InstState* st, const float* delta_inst, int variant,
                        int early, int t_begin, int t_end, bool fill) {
    if (t_end <= t_begin) return hipSuccess;
    hipError_t e = launch_fill_u32(s, reinterpret_cast<uint32_t*>(scr.work), 0u, 1);
    if (e != hipSuccess) return e;
    int blocks = (slots + (kWG / 64) - 1) / (kWG / 64);
    if (variant >= 32) {
        // chain-contracted search, one workgroup per tree (scratch slot = workgroup)
        if (!net.cbuf) return hipErrorInvalidValue;
        blocks = min(blocks, scr.nslots);
        if (blocks <= 0) return hipErrorInvalidValue;
        dim3 g(blocks), b(kWG);
#define QDTA_SSSP_CT(U, V) \
    hipLaunchKernelGGL((k_sssp_wg<U, V, true>), g, b, 0, s, net, dem, radj, labels, scr, st, delta_inst, early, \
                       t_begin, t_end)
        switch (variant - 32) {
            case 0: QDTA_SSSP_CT(1, 2); break;
            case 1: QDTA_SSSP_CT(1, 4); break;
            case 2:
                hipLaunchKernelGGL((k_sssp_wg<2, 4, true, 7>), g, b, 0, s, net, dem, radj, labels, scr, st, delta_inst,
                                   early, t_begin, t_end);
                break;
            case 3: QDTA_SSSP_CT(4, 4); break;
            case 4: QDTA_SSSP_CT(2, 2); break;
            default: QDTA_SSSP_CT(4, 2); break;
        }
#undef QDTA_SSSP_CT
        e = hipGetLastError();
        if (e != hipSuccess || !fill) return e;
        return launch_chain_fill(s, net, dem, labels, st, t_begin, t_end);   // the left-out chain nodes
    }
    if (variant >= 24) {
        // one workgroup per tree, every thread relaxing its own nodes' in-links
        blocks = min(blocks, scr.nslots);
        if (blocks <= 0) return hipErrorInvalidValue;
        dim3 g(blocks), b(kWG);
#define QDTA_SSSP_WN(U, V) \
    hipLaunchKernelGGL((k_sssp_wn<U, V>), g, b, 0, s, net, dem, radj, labels, scr, st, delta_inst, early, t_begin, \
                       t_end)
        switch (variant - 24) {
            case 0: QDTA_SSSP_WN(1, 4); break;
            case 1: QDTA_SSSP_WN(2, 4); break;
            case 2: QDTA_SSSP_WN(2, 2); break;
            default: QDTA_SSSP_WN(1, 2); break;
        }
#undef QDTA_SSSP_WN
        return hipGetLastError();
    }
    if (variant >= 16) {
        // block-local trees, one workgroup per tree (scratch slot = workgroup)
        blocks = min(blocks, scr.nslots);
        if (blocks <= 0) return hipErrorInvalidValue;
        dim3 g(blocks), b(kWG);
#define QDTA_SSSP_BLK(B, KB) \
    hipLaunchKernelGGL((k_sssp_blk<B, KB>), g, b, 0, s, net, dem, radj, labels, scr, st, delta_inst, early, t_begin, \
                       t_end)
        switch (variant - 16) {
            case 0: QDTA_SSSP_BLK(128, 1); break;
            case 1: QDTA_SSSP_BLK(128, 2); break;
            case 2: QDTA_SSSP_BLK(64, 2); break;
            default: QDTA_SSSP_BLK(256, 1); break;
        }
#undef QDTA_SSSP_BLK
        return hipGetLastError();
    }
    if (variant >= 8) {
        // one workgroup per tree (scratch slot = workgroup)
        blocks = min(blocks, scr.nslots);
        if (blocks <= 0) return hipErrorInvalidValue;
        dim3 g(blocks), b(kWG);
#define QDTA_SSSP_WG(U, V) \
    hipLaunchKernelGGL((k_sssp_wg<U, V, false>), g, b, 0, s, net, dem, radj, labels, scr, st, delta_inst, early, \
                       t_begin, t_end)
        switch (variant - 8) {
            case 0: QDTA_SSSP_WG(1, 2); break;
            case 1: QDTA_SSSP_WG(1, 4); break;
            case 2: QDTA_SSSP_WG(2, 4); break;
            case 3: QDTA_SSSP_WG(4, 4); break;
            case 4: QDTA_SSSP_WG(2, 2); break;
            default: QDTA_SSSP_WG(4, 2); break;
        }
#undef QDTA_SSSP_WG
        return hipGetLastError();
    }
    // one wavefront per tree (scratch slot = wavefront)
    blocks = min(blocks, scr.nslots / (kWG / 64));
    if (blocks <= 0) return hipErrorInvalidValue;
    dim3 g(blocks), b(kWG);
#define QDTA_SSSP(U, V) \
    hipLaunchKernelGGL((k_sssp_ds<U, V>), g, b, 0, s, net, dem, radj, labels, scr, st, delta_inst, early, \
                       t_begin, t_end)
    switch (variant) {
        case 0: QDTA_SSSP(1, 4); break;
        case 1: QDTA_SSSP(2, 4); break;
        case 2: QDTA_SSSP(4, 4); break;
        case 3: QDTA_SSSP(4, 8); break;
        case 4: QDTA_SSSP(8, 8); break;
        default: QDTA_SSSP(1, 1); break;
    }
#undef QDTA_SSSP
    return hipGetLastError();
}

hipError_t launch_sssp(hipStream_t s, const NetDev& net, const DemDev& dem, const float* cost, const uint2* radj,
                       label_t* labels, const Scratch& scr, int slots, const InstState* st, double delta_scale,
                       float* delta_inst, double* logsum, int variant, int early, bool fill) {
    if (dem.Q == 0) return hipSuccess;
    hipError_t e = launch_delta(s, net, cost, delta_scale, delta_inst, logsum);
    if (e != hipSuccess) return e;
    return launch_trees(s, net, dem, radj, labels, scr, slots, st, delta_inst, variant, early, 0, dem.Q, fill);
}

// ---------------------------------------------------------------------------
// A3: truncation + loading, and the residual walk of Alg. 4
// ---------------------------------------------------------------------------
// Successor of u on the tree whose labels are lab[node - node0]: the
// lowest-uid out-link (u, w) that is tight, fl32(D(w) + c) == D(u), and
// strict, D(w) < D(u).  -1 when FP32 absorption leaves none.
__device__ __forceinline__ int succ_strict(const NetDev& net, const label_t* lab, int node0, int u, float du,
                                          const float* tree_cost) {
    const int e1 = net.row_ptr[u + 1];
    for (int e = net.row_ptr[u]; e < e1; ++e) {
        const float dw = lab_val(lab, net.col[e] - node0);
        if (dw < du && dw + tree_cost[e] == du) return e;
    }
    return -1;
}

// The same successor, reading (head, cost) from the forward link records,
// whose costs are the ones the trees were grown with: one line per link
// instead of the head and cost arrays.  Also returns the head and the cost.
__device__ __forceinline__ int succ_rec(const NetDev& net, const label_t* lab, int node0, int u, float du, int& head,
                                       float& cost) {
    const int e1 = net.row_ptr[u + 1];
    for (int e = net.row_ptr[u]; e < e1; ++e) {
        const uint2 r = net.fadj[e];
        const float dw = lab_val(lab, (int)r.x - node0);
        const float c = __uint_as_float(r.y);
        if (dw < du && dw + c == du) {
            head = (int)r.x;
            cost = c;
            return e;
        }
    }
    return -1;
}

// The same successor as succ_rec, for a walk that carries u's forward row
// packed (kNoRow: read the row pointers): the row's records with their
// heads' packed rows, then the heads' labels, are loaded four at a time
// together (indices past the row's end repeat its last link), and the
// lowest tight strict link wins as before.  Also returns the head's packed
// row and label for the next hop.
__device__ __forceinline__ int succ_row(const NetDev& net, const label_t* lab, int node0, int u, uint32_t row,
                                        float du, int& head, float& cost, uint32_t& head_row, float& head_lab) {
    int e0, deg;
    if (row != kNoRow) {
        e0 = (int)(row >> kRowCountBits);
        deg = (int)(row & ((1u << kRowCountBits) - 1u));
    } else {
        e0 = net.row_ptr[u];
        deg = net.row_ptr[u + 1] - e0;
    }
    const int last = e0 + deg - 1;
    for (int b = 0; b < deg; b += 4) {
        uint2 r[4];
        uint32_t fr[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int e = min(e0 + b + j, last);
            r[j] = net.fadj[e];
            fr[j] = net.frow[e];
        }
        float dw[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) dw[j] = lab_val(lab, (int)r[j].x - node0);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float c = __uint_as_float(r[j].y);
            if (b + j < deg && dw[j] < du && dw[j] + c == du) {
                head = (int)r[j].x;
                cost = c;
                head_row = fr[j];
                head_lab = dw[j];
                return e0 + b + j;
            }
        }
    }
    return -1;
}

struct WalkOut {
    int64_t* y;
    int32_t* stop;
    float* stop_delay;           // AON mode, may be NULL: the delay a leg stops with (link-progress rule)
    int residual_mode;
    const double* lambda;        // per instance (residual mode)
    int64_t* r_dense;            // residual accumulator, indexed like the labels
    unsigned long long* done_fx;
    TransitOut tr;               // residual mode, link-progress rule: legs left on a link
    int* err;                    // set when the transit list overflows
};

// Residual mode adds rint(lambda d) of a leg that stops at s short of q to
// the accumulator word of (tree qi, node s), whose label offset is lab0 --
// or, when it stops on a link with a delay, appends it to the transit list
// -- and counts the completed weight otherwise.
__device__ __forceinline__ void finish_leg(const WalkOut& o, int l, int s, int q, int qi, int64_t lab0, int inst,
                                           int node0, int64_t d, float delay) {
    if (!o.residual_mode) {
        if (o.stop) o.stop[l] = s - node0;
        if (o.stop_delay) o.stop_delay[l] = delay;
        return;
    }
    const int64_t w = (int64_t)__builtin_rint(o.lambda[inst] * (double)d);
    if (s == q) {
        if (w) atomicAdd(&o.done_fx[inst], (unsigned long long)w);
        return;
    }
    if (w == 0) return;
    if (delay > 0.0f) {
        const unsigned int k = atomicAdd(o.tr.n, 1u);
        if (k < o.tr.cap) {
            o.tr.q[k] = qi;
            o.tr.node[k] = s - node0;
            o.tr.delay[k] = delay;
            o.tr.w[k] = w;
        } else {
            atomicOr(o.err, 1);
        }
        return;
    }
    atomicAdd(reinterpret_cast<unsigned long long*>(&o.r_dense[lab0 + (s - node0)]), (unsigned long long)w);
}

// One step of the truncated walk (Eq. 2 read as CEIL / FLOOR / NONE, or the
// link-progress rule): whether a leg at a node at time tau stops there, and
// after entering a link (new time nt) whether it stops on it.  PROGRESS loads
// as CEIL; a trip still on a link at dt stops at its head with delay
// nt - dt (a trip on its last link completes), and a leg that starts with
// its delay at or above dt is still on its way to its origin.
// A delay a leg leaves the interval with, rounded up to a whole multiple of
// pq seconds in FP64 when pq > 0 (legs stopped on the same link for the
// same destination then merge).
__device__ __forceinline__ float progress_delay(float x, double pq) {
    return pq > 0.0 ? (float)(pq * ceil((double)x / pq)) : x;
}

__device__ __forceinline__ bool stop_at_node(int rule, float tau, float dt) {
    return (rule == RULE_CEIL || rule == RULE_PROGRESS) && tau >= dt;
}

// time_cost: the costs that clock the truncation (Eq. 2); NULL = the trees'
// own costs (the forward records), as in the AON of an iteration.
// Legs per thread of the walk: the threads of a wavefront walk legs of
// different lengths, so each takes several (a workgroup walks a contiguous
// run of kWG * kWalkLegsPerThread legs, a wavefront 64 consecutive legs at a
// time) and the sums of their lengths vary less than single lengths do.
constexpr int kWalkLegsPerThread = 4;
// Loads of a workgroup's legs are summed per link in an LDS table first
// (legs of one destination share links); the table is added to y when the
// workgroup is done, and a load whose probes find no slot goes to y directly.
// Integer sums: the order does not change them.  4,096 slots (48 KB, three
// workgroups per CU): a workgroup's 1,024 legs load more distinct links than
// 2,048 slots hold, and 8,192 leave one workgroup per CU.
constexpr int kWalkSlots = 4096;

__global__ __launch_bounds__(kWG) void k_walk(NetDev net, DemDev dem, const label_t* __restrict__ labels,
                                              const float* __restrict__ time_cost, const InstState* st,
                                              FlagsDev fl, WalkOut o, int l_begin, int l_end) {
    __shared__ int s_key[kWalkSlots];
    __shared__ unsigned long long s_sum[kWalkSlots];
    for (int x = threadIdx.x; x < kWalkSlots; x += kWG) {
        s_key[x] = -1;
        s_sum[x] = 0ull;
    }
    __syncthreads();
    auto load = [&](int e, int64_t d) {
        int h = (int)(((unsigned)e * 2654435761u) >> 20) & (kWalkSlots - 1);
        for (int probe = 0; probe < 4; ++probe) {
            int k = s_key[h];
            if (k == -1) k = atomicCAS(&s_key[h], -1, e);
            if (k == -1 || k == e) {
                atomicAdd(&s_sum[h], (unsigned long long)d);
                return;
            }
            h = (h + 1) & (kWalkSlots - 1);
        }
        atomicAdd(reinterpret_cast<unsigned long long*>(&o.y[e]), (unsigned long long)d);
    };
    const int base = l_begin + blockIdx.x * kWG * kWalkLegsPerThread;
    const int lim = min(l_end, base + kWG * kWalkLegsPerThread);
    for (int l = base + threadIdx.x; l < lim; l += kWG) {
        const int qi = dem.leg_q[l];
        const int inst = dem.dest_inst[qi];
        if (!inst_live(st, inst)) continue;
        const InstDev I = net.inst[inst];
        const int node0 = I.node0;
        const int q = dem.dest_node[qi];
        const label_t* lab = tree_labels(labels, dem, qi);
        const int64_t d = dem.leg_dfx[l];
        int u = dem.leg_orig[l];
        float du = lab_val(lab, u - node0);
        fl.int_node[l] = -1;
        if (!(du <= 3.4028234663852886e38f)) {       // origin cannot reach q
            atomicOr(fl.err_unreach, 1);
            if (o.stop) o.stop[l] = -1;
            continue;
        }
        float tau = dem.leg_delay ? dem.leg_delay[l] : 0.0f;
        float delay = 0.0f;
        bool absorbed = false;
        if (I.rule == RULE_PROGRESS && tau >= I.dt32) {
            delay = progress_delay(tau - I.dt32, I.pq);   // still on its way to its origin
        } else {
            uint32_t urow = kNoRow;                   // u's forward row, carried from the link into u
            for (int hops = 0; u != q; ++hops) {
                if (stop_at_node(I.rule, tau, I.dt32)) break;
                int head = 0;
                float ce = 0.0f, hlab = 0.0f;
                uint32_t hrow = kNoRow;
                const int e = succ_row(net, lab, node0, u, urow, du, head, ce, hrow, hlab);
                if (e < 0 || hops > I.n) {            // absorption: finish in the fallback
                    fl.int_node[l] = u;
                    fl.int_tau[l] = tau;
                    fl.absorb_q[qi] = 1;
                    atomicAdd(fl.absorb_count, 1);
                    absorbed = true;
                    break;
                }
                const float nt = tau + (time_cost ? time_cost[e] : ce);
                if (I.rule == RULE_FLOOR && nt > I.dt32) break;
                if (!o.residual_mode) load(e, d);
                tau = nt;
                u = head;
                urow = hrow;
                du = hlab;
                if (I.rule == RULE_PROGRESS && tau > I.dt32) {
                    if (u != q) delay = progress_delay(tau - I.dt32, I.pq);
                    break;
                }
            }
        }
        if (!absorbed) finish_leg(o, l, u, q, qi, dem.dest_lab[qi], inst, node0, d, delay);
    }
    __syncthreads();
    for (int x = threadIdx.x; x < kWalkSlots; x += kWG)
        if (s_key[x] >= 0) atomicAdd(reinterpret_cast<unsigned long long*>(&o.y[s_key[x]]), s_sum[x]);
}

hipError_t launch_walk(hipStream_t s, const NetDev& net, const DemDev& dem, const label_t* labels,
                       const float* time_cost, int64_t* y, int32_t* stop,
                       const InstState* st, const FlagsDev& fl, int residual_mode, const double* lambda,
                       int64_t* r_dense, unsigned long long* done_fx,
                       int l_begin, int l_end, float* stop_delay, const TransitOut* tr) {
    if (l_end < 0) l_end = dem.P;
    if (l_end <= l_begin) return hipSuccess;
    WalkOut o{y, stop, stop_delay, residual_mode, lambda, r_dense, done_fx,
              tr ? *tr : TransitOut{nullptr, nullptr, nullptr, nullptr, nullptr, 0u}, fl.err_overflow};
    const int64_t per = (int64_t)kWG * kWalkLegsPerThread;
    hipLaunchKernelGGL(k_walk, dim3((unsigned)((l_end - l_begin + per - 1) / per)), dim3(kWG), 0, s, net, dem, labels,
                       time_cost, st, fl, o, l_begin, l_end);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// A3, plain intervals: loading by children-before-parent accumulation
// ---------------------------------------------------------------------------
// Without truncation every leg of tree q loads its whole path to q, so the
// flow on the successor link of v is the demand of all legs whose paths pass
// through v.  Instead of walking every leg to q, the legs' paths are merged:
//   pass 1 (k_sweep_count): each leg walks from its origin; at every node it
//     reaches it adds 1 to the node's arrival count and goes on only if it
//     was the first to arrive -- so each node's count is the number of legs
//     and path branches that will bring demand into it;
//   pass 2 (k_sweep_push): each leg starts again with its demand; at a node
//     it adds what it carries to the node's accumulator and takes one off
//     the count; the arrival that takes the count to zero is the last, takes
//     the whole accumulated demand, loads the successor link with it and goes
//     on to the parent.
// Every link is loaded once per tree with the integer sum of the demand of
// the legs that use it: the same int64 y as the walk.  Both scratch arrays
// (indexed like the labels) are back at zero afterwards.  A tree where a
// walker meets FP32 absorption is flagged; pass 2 walks its legs as k_walk
// does (clearing the counts pass 1 left on their paths) and the tie
// fallback finishes them.  Used only when every instance is plain.
__device__ __forceinline__ void wait_memory() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

__global__ __launch_bounds__(kWG) void k_sweep_count(NetDev net, DemDev dem, const label_t* __restrict__ labels,
                                                     const InstState* st, FlagsDev fl, uint32_t* cnt) {
    const int l = blockIdx.x * kWG + threadIdx.x;
    if (l >= dem.P) return;
    const int qi = dem.leg_q[l];
    const int inst = dem.dest_inst[qi];
    if (!inst_live(st, inst)) return;
    const InstDev I = net.inst[inst];
    if (I.rule != RULE_NONE) return;
    const int node0 = I.node0, q = dem.dest_node[qi];
    const label_t* lab = tree_labels(labels, dem, qi);
    uint32_t* C = cnt + dem.dest_lab[qi] - node0;       // indexed by global node id
    int u = dem.leg_orig[l];
    float du = lab_val(lab, u - node0);
    if (!(du <= 3.4028234663852886e38f)) return;        // unreachable: reported by pass 2
    for (int hops = 0; u != q; ++hops) {
        if (atomicAdd(&C[u], 1u) != 0u) return;         // another arrival goes on from here
        int head = 0;
        float ce = 0.0f;
        const int e = succ_rec(net, lab, node0, u, du, head, ce);
        if (e < 0 || hops > I.n) {                      // absorption: this tree is walked
            fl.absorb_q[qi] = 1;
            return;
        }
        u = head;
        du = lab_val(lab, u - node0);
    }
}

__global__ __launch_bounds__(kWG) void k_sweep_push(NetDev net, DemDev dem, const label_t* __restrict__ labels,
                                                    const InstState* st, FlagsDev fl, WalkOut o, uint32_t* cnt,
                                                    int64_t* acc) {
    const int l = blockIdx.x * kWG + threadIdx.x;
    if (l >= dem.P) return;
    const int qi = dem.leg_q[l];
    const int inst = dem.dest_inst[qi];
    if (!inst_live(st, inst)) return;
    const InstDev I = net.inst[inst];
    const int node0 = I.node0, q = dem.dest_node[qi];
    const label_t* lab = tree_labels(labels, dem, qi);
    uint32_t* C = cnt + dem.dest_lab[qi] - node0;
    int64_t* A = acc + dem.dest_lab[qi] - node0;
    int u = dem.leg_orig[l];
    float du = lab_val(lab, u - node0);
    fl.int_node[l] = -1;
    if (!(du <= 3.4028234663852886e38f)) {
        atomicOr(fl.err_unreach, 1);
        if (o.stop) o.stop[l] = -1;
        return;
    }
    if (o.stop) o.stop[l] = q - node0;                  // without truncation every leg completes
    if (o.stop_delay) o.stop_delay[l] = 0.0f;
    const bool sweep = !ld_coherent(&fl.absorb_q[qi]);
    int64_t carry = dem.leg_dfx[l];
    for (int hops = 0; u != q; ++hops) {
        if (sweep) {
            atomicAdd(reinterpret_cast<unsigned long long*>(&A[u]), (unsigned long long)carry);
            wait_memory();                              // the demand is in before the count drops
            if (atomicSub(&C[u], 1u) != 1u) return;     // not the last arrival: done
            carry = (int64_t)atomicExch(reinterpret_cast<unsigned long long*>(&A[u]), 0ull);
        } else {
            C[u] = 0u;                                  // a flagged tree: clear what pass 1 counted
        }
        int head = 0;
        float ce = 0.0f;
        const int e = succ_rec(net, lab, node0, u, du, head, ce);
        if (e < 0 || hops > I.n) {                      // absorption (flagged trees only): the fallback
            fl.int_node[l] = u;                         // finishes the leg
            fl.int_tau[l] = 0.0f;
            fl.absorb_q[qi] = 1;
            atomicAdd(fl.absorb_count, 1);
            return;
        }
        atomicAdd((unsigned long long*)&o.y[e], (unsigned long long)carry);
        u = head;
        du = lab_val(lab, u - node0);
    }
}

hipError_t launch_sweep(hipStream_t s, const NetDev& net, const DemDev& dem, const label_t* labels,
                        int64_t* y, int32_t* stop, float* stop_delay, const InstState* st, const FlagsDev& fl,
                        uint32_t* cnt, int64_t* acc) {
    if (dem.P == 0) return hipSuccess;
    const dim3 g((dem.P + kWG - 1) / kWG), b(kWG);
    hipLaunchKernelGGL(k_sweep_count, g, b, 0, s, net, dem, labels, st, fl, cnt);
    WalkOut o{y, stop, stop_delay, 0, nullptr, nullptr, nullptr,
              TransitOut{nullptr, nullptr, nullptr, nullptr, nullptr, 0u}, fl.err_overflow};
    hipLaunchKernelGGL(k_sweep_push, g, b, 0, s, net, dem, labels, st, fl, o, cnt, acc);
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
__global__ __launch_bounds__(kWG) void k_fallback(NetDev net, DemDev dem, const label_t* __restrict__ labels,
                                                  const float* __restrict__ tree_cost,
                                                  const float* __restrict__ time_cost, const InstState* st,
                                                  FlagsDev fl, Scratch scr, WalkOut o, int trees_mode,
                                                  int32_t* succ_out, int32_t n_out) {
    __shared__ int s_cnt[2];
    int32_t* hop = scr.farq + (int64_t)blockIdx.x * scr.nmax;
    int32_t* qbase = scr.nearq + (int64_t)blockIdx.x * scr.nmax;
    for (int qi = blockIdx.x; qi < dem.Q; qi += gridDim.x) {
        if (!fl.absorb_q[qi]) continue;
        const int inst = dem.dest_inst[qi];
        if (!inst_live(st, inst)) continue;
        const InstDev I = net.inst[inst];
        const int n = I.n, node0 = I.node0;
        const label_t* lab = tree_labels(labels, dem, qi);
        const int q = dem.dest_node[qi];
        // breadth-first levels in one FIFO: level L occupies [s_cnt[0], s_cnt[1])
        for (int v = threadIdx.x; v < n; v += kWG) hop[v] = -1;
        if (threadIdx.x == 0) { s_cnt[0] = 0; s_cnt[1] = 1; }
        __syncthreads();
        if (threadIdx.x == 0) { hop[q - node0] = 0; qbase[0] = q - node0; }
        __syncthreads();
        for (int level = 0;; ++level) {
            const int lo = s_cnt[0], hi = s_cnt[1];
            if (lo == hi) break;
            __syncthreads();
            for (int i = lo + threadIdx.x; i < hi; i += kWG) {
                const int u = qbase[i];
                const float du = lab_val(lab, u);
                for (int e = net.rptr[node0 + u]; e < net.rptr[node0 + u + 1]; ++e) {
                    const int v = net.rsrc[e] - node0;
                    const int link = net.rlink[e];
                    const float dv = lab_val(lab, v);
                    if (dv <= 3.4028234663852886e38f && du + tree_cost[link] == dv) {
                        if (atomicCAS(&hop[v], -1, level + 1) == -1) {
                            int pos = atomicAdd(&s_cnt[1], 1);
                            qbase[pos] = v;
                        }
                    }
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) s_cnt[0] = hi;
            __syncthreads();
        }
        // successor with the hop rule where no strict tight link exists
        auto succ_full = [&](int u, float du) -> int {
            int e = succ_strict(net, lab, node0, u, du, tree_cost);
            if (e >= 0) return e;
            const int hu = ld_coherent(&hop[u - node0]);
            for (int k = net.row_ptr[u]; k < net.row_ptr[u + 1]; ++k) {
                const int w = net.col[k];
                const float dw = lab_val(lab, w - node0);
                if (dw + tree_cost[k] == du && ld_coherent(&hop[w - node0]) == hu - 1) return k;
            }
            return -1;
        };
        if (trees_mode) {
            const int t = qi;
            for (int v = threadIdx.x; v < n; v += kWG) {
                const int g = node0 + v;
                const float dv = lab_val(lab, v);
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
                float du = lab_val(lab, u - node0);
                const int64_t d = dem.leg_dfx[l];
                float delay = 0.0f;
                for (int hops = 0; u != q && hops <= n; ++hops) {
                    if (stop_at_node(I.rule, tau, I.dt32)) break;
                    const int e = succ_full(u, du);
                    if (e < 0) break;
                    const float nt = tau + time_cost[e];
                    if (I.rule == RULE_FLOOR && nt > I.dt32) break;
                    if (!o.residual_mode) atomicAdd((unsigned long long*)&o.y[e], (unsigned long long)d);
                    tau = nt;
                    u = net.col[e];
                    du = lab_val(lab, u - node0);
                    if (I.rule == RULE_PROGRESS && tau > I.dt32) {
                        if (u != q) delay = progress_delay(tau - I.dt32, I.pq);
                        break;
                    }
                }
                fl.int_node[l] = -1;
                finish_leg(o, l, u, q, qi, dem.dest_lab[qi], inst, node0, d, delay);
            }
        }
        __syncthreads();
    }
}

hipError_t launch_fallback(hipStream_t s, const NetDev& net, const DemDev& dem, const label_t* labels,
                           const float* tree_cost, const float* time_cost, int64_t* y, int32_t* stop,
                           const InstState* st, const FlagsDev& fl, const Scratch& scr, int slots,
                           int residual_mode, const double* lambda, int64_t* r_dense,
                           unsigned long long* done_fx, int trees_mode,
                           int32_t* succ_out, int32_t n_out, float* stop_delay, const TransitOut* tr) {
    if (dem.Q == 0) return hipSuccess;
    WalkOut o{y, stop, stop_delay, residual_mode, lambda, r_dense, done_fx,
              tr ? *tr : TransitOut{nullptr, nullptr, nullptr, nullptr, nullptr, 0u}, fl.err_overflow};
    hipLaunchKernelGGL(k_fallback, dim3(slots), dim3(kWG), 0, s, net, dem, labels, tree_cost, time_cost, st, fl, scr,
                       o, trees_mode, succ_out, n_out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// A8: compaction of the residual accumulator
// ---------------------------------------------------------------------------
// Tree t's residual legs are the non-zero words of its row (n words at
// dest_lab[t]); rows are taken in tree order and nodes in ascending order,
// which is (destination, origin) order.  The write pass clears what it
// reads, so the accumulator is all zero again afterwards.
__device__ __forceinline__ int block_excl_scan(int x, int* tot, int* s_w) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int incl = x;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == 63) s_w[wv] = incl;
    __syncthreads();
    int before = 0, all = 0;
    for (int k = 0; k < kWG / 64; ++k) {
        if (k < wv) before += s_w[k];
        all += s_w[k];
    }
    __syncthreads();
    *tot = all;
    return before + incl - x;
}

__global__ __launch_bounds__(kWG) void k_resid_count(NetDev net, DemDev dem, const int64_t* __restrict__ r_dense,
                                                     int64_t* cnt) {
    __shared__ int s_w[kWG / 64];
    const int t = blockIdx.x;
    const int n = net.inst[dem.dest_inst[t]].n;
    const int64_t* row = r_dense + dem.dest_lab[t];
    int c = 0;
    for (int v = threadIdx.x; v < n; v += kWG) c += row[v] != 0;
    int tot = 0;
    block_excl_scan(c, &tot, s_w);
    if (threadIdx.x == 0) cnt[t] = tot;
}

__global__ __launch_bounds__(kWG) void k_resid_write(NetDev net, DemDev dem, int64_t* r_dense, const int64_t* off,
                                                     int32_t* r_orig, int32_t* r_q, int64_t* r_w) {
    __shared__ int s_w[kWG / 64];
    const int t = blockIdx.x;
    const int n = net.inst[dem.dest_inst[t]].n;
    int64_t* row = r_dense + dem.dest_lab[t];
    int64_t base = off[t];
    for (int v0 = 0; v0 < n; v0 += kWG) {
        const int v = v0 + threadIdx.x;
        const int64_t x = v < n ? row[v] : 0;
        int tot = 0;
        const int pos = block_excl_scan(x != 0 ? 1 : 0, &tot, s_w);
        if (x != 0) {
            r_orig[base + pos] = v;
            r_q[base + pos] = t;
            r_w[base + pos] = x;
            row[v] = 0;
        }
        base += tot;
    }
}

hipError_t launch_resid_count(hipStream_t s, const NetDev& net, const DemDev& dem, const int64_t* r_dense,
                              int64_t* cnt) {
    if (dem.Q == 0) return hipSuccess;
    hipLaunchKernelGGL(k_resid_count, dim3(dem.Q), dim3(kWG), 0, s, net, dem, r_dense, cnt);
    return hipGetLastError();
}

hipError_t launch_resid_write(hipStream_t s, const NetDev& net, const DemDev& dem, int64_t* r_dense,
                              const int64_t* off, int32_t* r_orig, int32_t* r_q, int64_t* r_w) {
    if (dem.Q == 0) return hipSuccess;
    hipLaunchKernelGGL(k_resid_write, dim3(dem.Q), dim3(kWG), 0, s, net, dem, r_dense, off, r_orig, r_q, r_w);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Parity output of trees: dist[t][v], succ[t][v] (local uid)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_trees_out(NetDev net, DemDev dem, const label_t* __restrict__ labels,
                                                   const float* __restrict__ cost, int32_t inst, float* dist,
                                                   int32_t* succ, int32_t* absorb_q) {
    const InstDev I = net.inst[inst];
    const int n = I.n;
    const int64_t total = (int64_t)dem.Q * n;
    for (int64_t i = blockIdx.x * (int64_t)kWG + threadIdx.x; i < total; i += (int64_t)gridDim.x * kWG) {
        const int t = (int)(i / n);
        const int v = (int)(i - (int64_t)t * n);
        const label_t* lab = tree_labels(labels, dem, t);
        const float dv = lab_val(lab, v);
        dist[i] = dv;
        const int g = I.node0 + v;
        int e = -1;
        if (g != dem.dest_node[t] && dv <= 3.4028234663852886e38f) {
            e = succ_strict(net, lab, I.node0, g, dv, cost);   // cost: global link order
            if (e < 0) absorb_q[t] = 1;
        }
        succ[i] = e >= 0 ? e - I.link0 : -1;
    }
}

hipError_t launch_trees_out(hipStream_t s, const NetDev& net, const DemDev& dem, const label_t* labels,
                            const float* cost, int32_t inst, float* dist, int32_t* succ, int32_t* absorb_q) {
    if (dem.Q == 0) return hipSuccess;
    hipLaunchKernelGGL(k_trees_out, dim3(2048), dim3(kWG), 0, s, net, dem, labels, cost, inst, dist, succ, absorb_q);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Frozen-path model and its reverse pass (OD calibration)
// ---------------------------------------------------------------------------
// The truncated path of every leg under one iterate's trees: the links the
// walk of that iterate loads (same successor rule, same clock), in walk
// order.  ptr == NULL counts them into len[l]; otherwise they are written at
// links[ptr[l]] (and the leg index at leg_of[ptr[l]]), never past ptr[l + 1].  bad: 1 an origin cannot reach its
// destination, 2 FP32 absorption (the tie fallback's paths are not
// recorded), 4 a path longer than counted.
__global__ __launch_bounds__(kWG) void k_path_walk(NetDev net, DemDev dem, const label_t* __restrict__ labels,
                                                   const int64_t* __restrict__ ptr, int32_t* __restrict__ links,
                                                   int32_t* __restrict__ leg_of, int64_t* __restrict__ len,
                                                   int* bad) {
    const int l = blockIdx.x * kWG + threadIdx.x;
    if (l >= dem.P) return;
    const int qi = dem.leg_q[l];
    const InstDev I = net.inst[dem.dest_inst[qi]];
    const int node0 = I.node0;
    const int q = dem.dest_node[qi];
    const label_t* lab = tree_labels(labels, dem, qi);
    int u = dem.leg_orig[l];
    float du = lab_val(lab, u - node0);
    const int64_t at = ptr ? ptr[l] : 0, end = ptr ? ptr[l + 1] : 0;
    int64_t k = 0;
    if (!(du <= 3.4028234663852886e38f)) {
        atomicOr(bad, 1);
        if (len) len[l] = 0;
        return;
    }
    float tau = 0.0f;
    for (int hops = 0; u != q; ++hops) {
        if (I.rule == RULE_CEIL && tau >= I.dt32) break;
        int head = 0;
        float ce = 0.0f;
        const int e = succ_rec(net, lab, node0, u, du, head, ce);
        if (e < 0 || hops > I.n) {
            atomicOr(bad, 2);
            break;
        }
        const float nt = tau + ce;
        if (I.rule == RULE_FLOOR && nt > I.dt32) break;
        if (ptr) {
            if (at + k >= end) {
                atomicOr(bad, 4);
                break;
            }
            links[at + k] = e;
            leg_of[at + k] = l;
        }
        ++k;
        tau = nt;
        u = head;
        du = lab_val(lab, u - node0);
    }
    if (len) len[l] = k;
}

hipError_t launch_path_walk(hipStream_t s, const NetDev& net, const DemDev& dem, const label_t* labels,
                            const int64_t* ptr, int32_t* links, int32_t* leg_of, int64_t* len, int* bad) {
    if (dem.P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_path_walk, dim3((dem.P + kWG - 1) / kWG), dim3(kWG), 0, s, net, dem, labels, ptr, links,
                       leg_of, len, bad);
    return hipGetLastError();
}

// y += rint(d 2^20) along every leg's path: the loading of Eq. 5 for a
// real-valued demand, exact in int64 whatever the order of the atomics.
// One lane per (leg, link) entry of the flattened paths, so the link ids
// and leg indices are read coalesced and long paths spread over lanes.
__global__ __launch_bounds__(kWG) void k_path_load(int64_t total, const int32_t* __restrict__ links,
                                                   const int32_t* __restrict__ leg_of, const double* __restrict__ d,
                                                   int64_t* y, int* err) {
    for (int64_t i = blockIdx.x * (int64_t)kWG + threadIdx.x; i < total; i += (int64_t)gridDim.x * kWG) {
        const double x = d[leg_of[i]] * 1048576.0;
        if (!(x > -9.0e18 && x < 9.0e18)) {
            atomicOr(err, 1);
            continue;
        }
        const int64_t w = (int64_t)__builtin_rint(x);
        if (w != 0) atomicAdd(reinterpret_cast<unsigned long long*>(&y[links[i]]), (unsigned long long)w);
    }
}

hipError_t launch_path_load(hipStream_t s, int64_t total, const int32_t* links, const int32_t* leg_of,
                            const double* d, int64_t* y, int* err) {
    if (total == 0) return hipSuccess;
    const int64_t b = (total + kWG - 1) / kWG;
    hipLaunchKernelGGL(k_path_load, dim3((unsigned)(b < 8192 ? b : 8192)), dim3(kWG), 0, s, total, links, leg_of, d,
                       y, err);
    return hipGetLastError();
}

// dbar[l] (+)= the sum of g over leg l's path: the transpose of the
// loading.  A group of 16 lanes per leg reads the link ids coalesced; each
// lane sums every 16th entry in walk order, then the group adds its 16
// partial sums by a fixed butterfly, so the result does not vary run to run.
constexpr int kGatherLanes = 16;

__global__ __launch_bounds__(kWG) void k_path_gather(int P, const int64_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ links,
                                                     const double* __restrict__ g, double* dbar, int accumulate) {
    const int64_t gid = (blockIdx.x * (int64_t)kWG + threadIdx.x) / kGatherLanes;
    const int sub = threadIdx.x % kGatherLanes;
    const bool live = gid < P;
    double acc = 0.0;
    if (live) {
        const int l = (int)gid;
        for (int64_t k = ptr[l] + sub; k < ptr[l + 1]; k += kGatherLanes) acc += g[links[k]];
    }
    for (int o = kGatherLanes / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kGatherLanes);
    if (live && sub == 0) {
        const int l = (int)gid;
        dbar[l] = accumulate ? dbar[l] + acc : acc;
    }
}

hipError_t launch_path_gather(hipStream_t s, int P, const int64_t* ptr, const int32_t* links, const double* g,
                              double* dbar, int accumulate) {
    if (P == 0) return hipSuccess;
    const int64_t threads = (int64_t)P * kGatherLanes;
    hipLaunchKernelGGL(k_path_gather, dim3((unsigned)((threads + kWG - 1) / kWG)), dim3(kWG), 0, s, P, ptr, links, g,
                       dbar, accumulate);
    return hipGetLastError();
}

// BPR cost, dc/dv and dc/dC at v (veh) in FP64, products left to right.
__device__ __forceinline__ void bpr_terms(double v, float c0f, float capf, double ab, int beta, double kappa,
                                          double& cost, double& dcdv, double& dcdcap) {
    const double c0 = (double)c0f, cap = (double)capf;
    const double r = (v * kappa) / cap;
    double p1 = 1.0;
    for (int k = 1; k < beta; ++k) p1 = p1 * r;
    const double p = p1 * r;
    cost = c0 * (1.0 + ab * p);
    dcdv = c0 * ab * (double)beta * p1 * kappa / cap;
    dcdcap = -c0 * ab * (double)beta * p / cap;
}

// Reverse step of one FW update f' = f + alpha (y - f), where alpha is the
// root of F(a) = sum_a t_a c_a(f_a + a t_a) (t = y - f): per-workgroup
// partial sums of abar = fbar . t and dF/dalpha = sum t^2 c'(v).
__global__ __launch_bounds__(kWG) void k_adj_sums(NetDev net, const int64_t* __restrict__ f,
                                                  const int64_t* __restrict__ y, const double* __restrict__ alpha,
                                                  const double* __restrict__ fbar, double ab, int beta,
                                                  double* part) {
    __shared__ double s0[kWG], s1[kWG];
    const double al = *alpha, kappa = net.inst[0].kappa;
    double a0 = 0.0, a1 = 0.0;
    for (int64_t a = blockIdx.x * (int64_t)kWG + threadIdx.x; a < net.M; a += (int64_t)gridDim.x * kWG) {
        const double F = (double)f[a] * kFxInv, t = (double)y[a] * kFxInv - F;
        double cost, dcdv, dcdcap;
        bpr_terms(F + al * t, net.c0[a], net.cap[a], ab, beta, kappa, cost, dcdv, dcdcap);
        a0 += fbar[a] * t;
        a1 += t * t * dcdv;
    }
    s0[threadIdx.x] = a0;
    s1[threadIdx.x] = a1;
    __syncthreads();
    for (int k = kWG / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            s0[threadIdx.x] += s0[threadIdx.x + k];
            s1[threadIdx.x] += s1[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s0[0];
        part[2 * blockIdx.x + 1] = s1[0];
    }
}

// s = -abar / (dF/dalpha) for a step size strictly inside (0, 1) that is a
// root (not the fixed MSA sequence); 0 otherwise.  One workgroup, partials
// summed in a fixed order.
__global__ __launch_bounds__(kWG) void k_adj_scale(const double* __restrict__ part, int nb,
                                                   const double* __restrict__ alpha, int is_root, double* s_out) {
    __shared__ double s0[kWG], s1[kWG];
    double a0 = 0.0, a1 = 0.0;
    for (int b = threadIdx.x; b < nb; b += kWG) {
        a0 += part[2 * b];
        a1 += part[2 * b + 1];
    }
    s0[threadIdx.x] = a0;
    s1[threadIdx.x] = a1;
    __syncthreads();
    for (int k = kWG / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            s0[threadIdx.x] += s0[threadIdx.x + k];
            s1[threadIdx.x] += s1[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double al = *alpha;
        *s_out = (is_root && al > 0.0 && al < 1.0 && s1[0] != 0.0) ? -s0[0] / s1[0] : 0.0;
    }
}

// Per link: ybar, and fbar and capbar carried back through the update and
// through alpha's dependence on (f, y, C) (implicit-function theorem).
__global__ __launch_bounds__(kWG) void k_adj_links(NetDev net, const int64_t* __restrict__ f,
                                                   const int64_t* __restrict__ y, const double* __restrict__ alpha,
                                                   const double* __restrict__ sp, double ab, int beta, double* fbar,
                                                   double* __restrict__ ybar, double* capbar) {
    const double al = *alpha, s = *sp, kappa = net.inst[0].kappa;
    for (int64_t a = blockIdx.x * (int64_t)kWG + threadIdx.x; a < net.M; a += (int64_t)gridDim.x * kWG) {
        const double F = (double)f[a] * kFxInv, t = (double)y[a] * kFxInv - F;
        double cost, dcdv, dcdcap;
        bpr_terms(F + al * t, net.c0[a], net.cap[a], ab, beta, kappa, cost, dcdv, dcdcap);
        const double g = fbar[a];
        ybar[a] = al * g + s * (cost + al * t * dcdv);
        fbar[a] = (1.0 - al) * g + s * (-cost + (1.0 - al) * t * dcdv);
        capbar[a] = capbar[a] + s * t * dcdcap;
    }
}

static int adj_blocks(int64_t M) {
    const int64_t b = (M + kWG - 1) / kWG;
    return b < 1 ? 1 : (b > 1024 ? 1024 : (int)b);
}

hipError_t launch_adj_step(hipStream_t s, const NetDev& net, const int64_t* f, const int64_t* y,
                           const double* alpha, int is_root, double ab, int beta, double* fbar, double* ybar,
                           double* capbar, double* part /*[2 x 1024]*/, double* sbuf) {
    if (net.M == 0) return hipSuccess;
    const int nb = adj_blocks(net.M);
    hipLaunchKernelGGL(k_adj_sums, dim3(nb), dim3(kWG), 0, s, net, f, y, alpha, fbar, ab, beta, part);
    hipLaunchKernelGGL(k_adj_scale, dim3(1), dim3(kWG), 0, s, part, nb, alpha, is_root, sbuf);
    hipLaunchKernelGGL(k_adj_links, dim3(nb), dim3(kWG), 0, s, net, f, y, alpha, sbuf, ab, beta, fbar, ybar, capbar);
    return hipGetLastError();
}

// flows in veh from fixed point
__global__ void k_fx_to_veh(int64_t M, const int64_t* __restrict__ f, double* out) {
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < M; a += (int64_t)gridDim.x * blockDim.x)
        out[a] = (double)f[a] * kFxInv;
}

hipError_t launch_fx_to_veh(hipStream_t s, int64_t M, const int64_t* f, double* out) {
    if (M == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fx_to_veh, dim3(adj_blocks(M)), dim3(kWG), 0, s, M, f, out);
    return hipGetLastError();
}

}  // namespace qdta
