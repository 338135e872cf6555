"""CPU oracle for the QDTA hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps `qdta_oracle.c` (FP64 contract mode, OpenMP
over destinations) through ctypes, and adds the interval chain of Alg. 1 in
plain numpy.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qdta_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libqdta_oracle.so")

RULE_NONE, RULE_CEIL, RULE_FLOOR, RULE_PROGRESS = 0, 1, 2, 3
LS_KSECTION, LS_QN, LS_MSA = 0, 1, 2
STOP_GAP, STOP_OBJ = 0, 1
OBJ_UE, OBJ_SO = 0, 1
WARN_ABSORB = 1
FX = 1 << 20
SUM_Q = 1 << 16


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, IEEE semantics)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-std=gnu11", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _LsOpts(C.Structure):
    _fields_ = [("ls_mode", C.c_int32), ("K", C.c_int32), ("passes", C.c_int32),
                ("max_ls", C.c_int32), ("T1", C.c_double), ("T2", C.c_double), ("dx", C.c_double),
                ("objective", C.c_int32)]


class _LsInfo(C.Structure):
    _fields_ = [("alpha", C.c_double), ("evals", C.c_int32), ("qn_iters", C.c_int32)]


class _FwOpts(C.Structure):
    _fields_ = [("alpha_b", C.c_double), ("beta", C.c_int32), ("rule", C.c_int32),
                ("dt_s", C.c_double), ("stop_rule", C.c_int32), ("tol", C.c_double),
                ("max_iter", C.c_int32), ("fixed_iters", C.c_int32), ("ls", _LsOpts),
                ("nthreads", C.c_int32)]


class _FwStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("ls_evals", C.c_int32), ("qn_iters", C.c_int32),
                ("absorb", C.c_int32), ("stopped_by", C.c_int32), ("gap", C.c_double),
                ("objective", C.c_double), ("last_alpha", C.c_double), ("gap_fp64", C.c_double),
                ("objective_fp64", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = C.CDLL(_LIB_PATH)
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def i128(limbs) -> int:
    """Python int of an int128 stored as (low, high) int64 limbs."""
    lo = int(limbs[0]) & ((1 << 64) - 1)
    return (int(limbs[1]) << 64) | lo


# ---------------------------------------------------------------------------
# thin wrappers
# ---------------------------------------------------------------------------
def trips_to_fx(trips) -> np.ndarray:
    """Trips -> int64 units of 2^-20 vehicle, round half to even (the C
    routine orc_trips_to_fx, one call per value)."""
    L = lib()
    L.orc_trips_to_fx.restype = C.c_int64
    L.orc_trips_to_fx.argtypes = [C.c_double]
    return np.array([L.orc_trips_to_fx(float(t)) for t in np.asarray(trips, dtype=np.float64)],
                    dtype=np.int64)


def trips_to_fx_array(trips) -> np.ndarray:
    """The same conversion for large arrays: trips * 2^20 is exact (a power of
    two), and numpy's rint rounds half to even."""
    return np.rint(np.asarray(trips, dtype=np.float64) * FX).astype(np.int64)


def demand_legs(orig, dest, trips):
    """The legs an interval's demand becomes (the problem statement of section
    3.1 with the conventions of the fixed-point contract): trips quantised to
    2^-20 vehicle, legs with equal (origin, destination) summed, legs with
    origin == destination or no trips dropped, sorted by (destination,
    origin)."""
    o, d, w = merge_legs(orig, dest, trips_to_fx_array(trips))
    keep = (w > 0) & (o != d)
    return o[keep], d[keep], w[keep]


def kappa(dt_s: float) -> float:
    return 3600.0 / dt_s if math.isfinite(dt_s) else 1.0


def bpr(f_fx, c0, cap, alpha, beta, dt_s, marginal=False):
    """BPR costs (Eq. 1), or with `marginal` the system optimum's marginal
    costs c + F dc/dF."""
    f_fx, c0, cap = _i64(f_fx), _f32(c0), _f32(cap)
    out = np.empty(c0.shape[0], dtype=np.float32)
    L = lib()
    L.orc_bpr_obj.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32,
                              C.c_double, C.c_int32, C.c_void_p]
    rc = L.orc_bpr_obj(c0.shape[0], _p(f_fx), _p(c0), _p(cap), alpha, beta, kappa(dt_s), int(bool(marginal)),
                       _p(out))
    return out, rc


def sum_cx(c, x_fx) -> int:
    c, x_fx = _f32(c), _i64(x_fx)
    out = np.zeros(2, dtype=np.int64)
    L = lib()
    L.orc_sum_cx.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_sum_cx(c.shape[0], _p(c), _p(x_fx), _p(out))
    return i128(out)


def ref_fp64(f_fx, y_fx, c0, cap, alpha_b, beta, dt_s, objective=OBJ_UE):
    """FP64 reference (long double, no FP32 costs, no quantised terms) of the
    relative gap and the objective of flows f with direction y: a dict with
    scf, scy, gap, objective."""
    f_fx, y_fx, c0, cap = _i64(f_fx), _i64(y_fx), _f32(c0), _f32(cap)
    out = np.zeros(4, dtype=np.float64)
    L = lib()
    L.orc_ref_fp64.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32,
                               C.c_double, C.c_int32, C.c_void_p]
    L.orc_ref_fp64(c0.shape[0], _p(f_fx), _p(y_fx), _p(c0), _p(cap), alpha_b, beta, kappa(dt_s), int(objective),
                   _p(out))
    return {"scf": out[0], "scy": out[1], "gap": out[2], "objective": out[3]}


def tree(net, cost, q):
    rp, col, cost = _i32(net.row_ptr), _i32(net.col), _f32(cost)
    D = np.empty(net.n, dtype=np.float32)
    succ = np.empty(net.n, dtype=np.int32)
    L = lib()
    L.orc_tree.argtypes = [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                           C.c_void_p, C.c_void_p]
    rc = L.orc_tree(net.n, col.shape[0], _p(rp), _p(col), _p(cost), int(q), _p(D), _p(succ))
    if rc < 0:
        raise RuntimeError(f"orc_tree failed {rc}")
    return D, succ, rc


def aon(net, cost, orig, dest, d_fx, dt_s, rule=RULE_CEIL, nthreads=0, delay=None, want_delay=False, pq=0.0):
    """All-or-nothing loading; delay (float32[P] or None): each leg's carried
    time to its origin (PROGRESS rule); pq > 0: stop delays rounded up to
    multiples of pq seconds.  Returns (y, stop, rc), plus the stop delays
    when want_delay."""
    rp, col, cost = _i32(net.row_ptr), _i32(net.col), _f32(cost)
    orig, dest, d_fx = _i32(orig), _i32(dest), _i64(d_fx)
    tau0 = None if delay is None else _f32(delay)
    y = np.zeros(col.shape[0], dtype=np.int64)
    stop = np.empty(orig.shape[0], dtype=np.int32)
    sdl = np.zeros(orig.shape[0], dtype=np.float32)
    L = lib()
    L.orc_aon_d.argtypes = [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                            C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32, C.c_void_p,
                            C.c_void_p, C.c_void_p, C.c_double, C.c_int32]
    rc = L.orc_aon_d(net.n, col.shape[0], _p(rp), _p(col), _p(cost), None, orig.shape[0], _p(orig), _p(dest),
                     _p(d_fx), _p(tau0) if tau0 is not None else None, float(dt_s), rule, _p(y), _p(stop), _p(sdl),
                     float(pq), nthreads)
    if rc < 0:
        raise RuntimeError(f"orc_aon failed {rc}")
    if want_delay:
        return y, stop, sdl, rc
    return y, stop, rc


def ls_eval(f, y, c0, cap, alpha_b, beta, dt_s, alphas, objective=0):
    f, y, c0, cap, alphas = _i64(f), _i64(y), _f32(c0), _f32(cap), _f64(alphas)
    K = alphas.shape[0]
    Cs = np.zeros(2 * K, dtype=np.int64)
    Ds = np.zeros(2 * K, dtype=np.int64)
    L = lib()
    L.orc_ls_eval.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                              C.c_int32, C.c_double, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]
    rc = L.orc_ls_eval(f.shape[0], _p(f), _p(y), _p(c0), _p(cap), alpha_b, beta, kappa(dt_s), K,
                       _p(alphas), _p(Cs), _p(Ds), objective)
    return [i128(Cs[2 * k:2 * k + 2]) for k in range(K)], [i128(Ds[2 * k:2 * k + 2]) for k in range(K)], rc


def ls_options(ls_mode=LS_KSECTION, K=32, passes=3, max_ls=20, T1=1e-4, T2=1e-4, dx=1e-4, objective=OBJ_UE):
    return _LsOpts(ls_mode, K, passes, max_ls, T1, T2, dx, objective)


def line_search(f, y, c0, cap, alpha_b, beta, dt_s, j, **kw):
    f, y, c0, cap = _i64(f), _i64(y), _f32(c0), _f32(cap)
    o = ls_options(**kw)
    info = _LsInfo()
    L = lib()
    L.orc_line_search.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                  C.c_int32, C.c_double, C.c_int32, C.c_void_p, C.c_void_p]
    rc = L.orc_line_search(f.shape[0], _p(f), _p(y), _p(c0), _p(cap), alpha_b, beta, kappa(dt_s), j,
                           C.byref(o), C.byref(info))
    if rc < 0:
        raise RuntimeError(f"orc_line_search failed {rc}")
    return info.alpha, info.evals, info.qn_iters


def fw_update(f, y, alpha):
    f = _i64(f).copy()
    y = _i64(y)
    L = lib()
    L.orc_fw_update.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_double]
    L.orc_fw_update(f.shape[0], _p(f), _p(y), float(alpha))
    return f


def i128_to_double(v: int) -> float:
    limbs = np.array([v & ((1 << 64) - 1), v >> 64], dtype=np.uint64).view(np.int64) if v >= 0 else \
        np.array([(v % (1 << 128)) & ((1 << 64) - 1), ((v % (1 << 128)) >> 64)], dtype=np.uint64).view(np.int64)
    L = lib()
    L.orc_i128_to_double.restype = C.c_double
    L.orc_i128_to_double.argtypes = [C.c_void_p]
    return L.orc_i128_to_double(_p(limbs))


class FwResult:
    def __init__(self, f, stats, hist_alpha, hist_cost, gaps):
        self.f = f
        self.iters = stats.iters
        self.ls_evals = stats.ls_evals
        self.qn_iters = stats.qn_iters
        self.absorb = bool(stats.absorb)
        self.stopped_by = stats.stopped_by
        self.gap = stats.gap
        self.objective = stats.objective
        self.last_alpha = stats.last_alpha
        self.gap_fp64 = stats.gap_fp64
        self.objective_fp64 = stats.objective_fp64
        self.hist_alpha = hist_alpha[: stats.iters + 1]
        self.hist_cost = hist_cost[: stats.iters + 1] if hist_cost is not None else None
        self.gaps = gaps[: stats.iters + 1]


def fw_solve(net, orig, dest, d_fx, *, alpha_b=0.15, beta=4, dt_s=float("inf"), rule=RULE_CEIL,
             stop_rule=STOP_GAP, tol=1e-4, max_iter=1000, fixed_iters=0, keep_history=True,
             nthreads=0, delay=None, **ls_kw) -> FwResult:
    rp, col = _i32(net.row_ptr), _i32(net.col)
    c0, cap = _f32(net.fftt), _f32(net.cap)
    orig, dest, d_fx = _i32(orig), _i32(dest), _i64(d_fx)
    tau0 = None if delay is None else _f32(delay)
    m = col.shape[0]
    cap_iter = fixed_iters if fixed_iters > 0 else max_iter
    o = _FwOpts(alpha_b, beta, rule, float(dt_s), stop_rule, tol, max_iter, fixed_iters,
                ls_options(**ls_kw), nthreads)
    st = _FwStats()
    f = np.zeros(m, dtype=np.int64)
    ha = np.zeros(cap_iter + 2, dtype=np.float64)
    hc = np.zeros((cap_iter + 2, m), dtype=np.float32) if keep_history else None
    gaps = np.zeros(cap_iter + 2, dtype=np.float64)
    L = lib()
    L.orc_fw_solve.argtypes = [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    rc = L.orc_fw_solve(net.n, m, _p(rp), _p(col), _p(c0), _p(cap), orig.shape[0], _p(orig), _p(dest),
                        _p(d_fx), _p(tau0) if tau0 is not None else None, C.byref(o), _p(f), C.byref(st), _p(ha),
                        _p(hc) if hc is not None else None, _p(gaps))
    if rc < 0:
        raise RuntimeError(f"orc_fw_solve failed {rc}")
    return FwResult(f, st, ha, hc, gaps)


def residual(net, f, hist_alpha, hist_cost, orig, dest, d_fx, *, alpha_b=0.15, beta=4, dt_s=900.0,
             rule=RULE_CEIL, delay=None, want_delay=False, pq=0.0):
    rp, col = _i32(net.row_ptr), _i32(net.col)
    c0, cap = _f32(net.fftt), _f32(net.cap)
    orig, dest, d_fx = _i32(orig), _i32(dest), _i64(d_fx)
    tau0 = None if delay is None else _f32(delay)
    J = len(hist_alpha) - 1
    P = orig.shape[0]
    cap_out = (J + 1) * max(P, 1)
    ro = np.empty(cap_out, np.int32)
    rd = np.empty(cap_out, np.int32)
    rw = np.empty(cap_out, np.int64)
    rdl = np.zeros(cap_out, np.float32)
    cnt = C.c_int64(0)
    done = C.c_int64(0)
    lam = np.empty(J + 1, np.float64)
    hc = np.ascontiguousarray(hist_cost, dtype=np.float32)
    ha = _f64(hist_alpha)
    L = lib()
    L.orc_residual.argtypes = [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_double, C.c_int32, C.c_double, C.c_int32, C.c_void_p, C.c_int32,
                               C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_void_p]
    rc = L.orc_residual(net.n, col.shape[0], _p(rp), _p(col), _p(c0), _p(cap), alpha_b, beta, float(dt_s),
                        rule, _p(_i64(f)), J, _p(ha), _p(hc), P, _p(orig), _p(dest), _p(d_fx),
                        _p(tau0) if tau0 is not None else None, float(pq), _p(ro), _p(rd), _p(rw), _p(rdl),
                        C.byref(cnt), C.byref(done), _p(lam))
    if rc < 0:
        raise RuntimeError(f"orc_residual failed {rc}")
    k = cnt.value
    if want_delay:
        return ro[:k].copy(), rd[:k].copy(), rw[:k].copy(), done.value, lam, rdl[:k].copy()
    return ro[:k].copy(), rd[:k].copy(), rw[:k].copy(), done.value, lam


def merge_legs(orig, dest, w_fx, delay=None):
    """Sum fixed-point legs with equal (origin, destination) -- and equal
    carried delay when `delay` is given (then a fourth array is returned);
    sorted by (dest, orig, delay)."""
    orig, dest, w_fx = _i32(orig), _i32(dest), _i64(w_fx)
    if delay is None:
        if orig.size == 0:
            return orig, dest, w_fx
        key = dest.astype(np.int64) * (1 << 31) + orig.astype(np.int64)
        u, inv = np.unique(key, return_inverse=True)
        w = np.zeros(u.shape[0], dtype=np.int64)
        np.add.at(w, inv, w_fx)
        return (u % (1 << 31)).astype(np.int32), (u // (1 << 31)).astype(np.int32), w
    dl = _f32(delay)
    if orig.size == 0:
        return orig, dest, w_fx, dl
    bits = dl.view(np.uint32).astype(np.int64)           # non-negative floats order like their bits
    keys = np.stack([bits, orig.astype(np.int64), dest.astype(np.int64)])
    order = np.lexsort(keys)
    k = keys[:, order]
    new = np.ones(order.size, bool)
    new[1:] = np.any(k[:, 1:] != k[:, :-1], axis=0)
    grp = np.cumsum(new) - 1
    w = np.zeros(int(grp[-1]) + 1, dtype=np.int64)
    np.add.at(w, grp, w_fx[order])
    first = order[new]
    return orig[first].copy(), dest[first].copy(), w, dl[first].copy()


def qdta_day(net, days, *, alpha_b=0.15, beta=4, rule=RULE_CEIL, tol=1e-4, max_iter=1000,
             stop_rule=STOP_GAP, nthreads=0, pq=0.0, **ls_kw):
    """Alg. 1: for each interval, d(i) = d^o(i) + d^r(i), Frank-Wolfe, then
    Alg. 4 for d^r(i+1).  d^r(0) is empty.  Returns per-interval records and
    the residual left after the last interval (reported, not assigned).
    Under RULE_PROGRESS the residual legs carry their delays (time still
    needed to reach their origin node; rounded up to multiples of pq seconds
    when pq > 0), legs are merged by (destination, origin, delay), and the
    records' "res" hold four arrays."""
    prog = rule == RULE_PROGRESS
    res_o = np.zeros(0, np.int32)
    res_d = np.zeros(0, np.int32)
    res_w = np.zeros(0, np.int64)
    res_t = np.zeros(0, np.float32)
    out = []
    for i, dem in enumerate(days):
        o_fx = np.array([int(np.rint(t * FX)) for t in dem.trips], dtype=np.int64) if dem.P else \
            np.zeros(0, np.int64)
        if prog:
            o, d, w, t = merge_legs(np.concatenate([dem.orig, res_o]), np.concatenate([dem.dest, res_d]),
                                    np.concatenate([o_fx, res_w]),
                                    np.concatenate([np.zeros(dem.P, np.float32), res_t]))
        else:
            o, d, w = merge_legs(np.concatenate([dem.orig, res_o]), np.concatenate([dem.dest, res_d]),
                                 np.concatenate([o_fx, res_w]))
            t = np.zeros(o.size, np.float32)
        keep = (w > 0) & (o != d)
        o, d, w, t = o[keep], d[keep], w[keep], t[keep]
        if o.size == 0:
            f = np.zeros(net.m, np.int64)
            res = (res_o[:0], res_d[:0], res_w[:0]) + ((res_t[:0],) if prog else ())
            out.append({"interval": i, "f": f, "iters": 0, "gap": 0.0, "legs": 0,
                        "res": res, "done_fx": 0, "in_fx": 0})
            res_o, res_d, res_w, res_t = res_o[:0], res_d[:0], res_w[:0], res_t[:0]
            continue
        fw = fw_solve(net, o, d, w, alpha_b=alpha_b, beta=beta, dt_s=dem.dt_s, rule=rule, tol=tol,
                      max_iter=max_iter, stop_rule=stop_rule, nthreads=nthreads, delay=t if prog else None,
                      **ls_kw)
        ro, rd, rw, done, lam, rt = residual(net, fw.f, fw.hist_alpha, fw.hist_cost, o, d, w, alpha_b=alpha_b,
                                             beta=beta, dt_s=dem.dt_s, rule=rule, delay=t if prog else None,
                                             want_delay=True, pq=pq)
        if prog:
            res_o, res_d, res_w, res_t = merge_legs(ro, rd, rw, rt)
            res = (res_o, res_d, res_w, res_t)
        else:
            res_o, res_d, res_w = merge_legs(ro, rd, rw)
            res = (res_o, res_d, res_w)
        out.append({"interval": i, "f": fw.f, "iters": fw.iters, "gap": fw.gap, "legs": int(o.size),
                    "res": res, "done_fx": done, "in_fx": int(w.sum()),
                    "hist_alpha": fw.hist_alpha, "lambda": lam})
    return out, ((res_o, res_d, res_w, res_t) if prog else (res_o, res_d, res_w))
