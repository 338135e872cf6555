"""Reverse-mode derivative of the Frank-Wolfe flows at frozen paths, for OD
calibration against link counts -- TEST INFRASTRUCTURE ONLY (oracle).

The model.  An interval was solved (Alg. 6) with J applied updates; iterate
j's trees (grown under its costs c_j, Eq. 1) and the truncation they implied
(Eq. 2, Eq. 5) are frozen into a link incidence L_j (legs x links).  For a
demand vector d (veh per leg) and capacities C:

    f <- L_0 d                                         (initial AON, Alg. 6)
    for j = 1..J:
        y_j     = L_j d
        alpha_j = root in [0, 1] of C'(a) = sum_a t_a c_a(f_a + a t_a; C_a),
                  t = y_j - f                          (line search, Eq. 6)
        f       <- f + alpha_j (y_j - f)               (FW update, Alg. 6)

with c_a the BPR cost of Eq. 1 (kappa = 3600/dt).  The paper has no
calibration; this is the model the derivative is taken of.  alpha_j depends
on (f, y_j, C) through C'(alpha_j) = 0, so by the implicit-function theorem
d alpha_j = -(dF)/(dF/d alpha) with F = C':

    dF/d alpha = sum t^2 c'(v),   dF/df_a = -c_a + (1 - alpha) t_a c'_a,
    dF/dy_a = c_a + alpha t_a c'_a,   dF/dC_a = t_a dc_a/dC_a,

(v = f + alpha t, c' = dc/dv); a step size at 0 or 1 (bracket end), or
one of the fixed MSA sequence, has zero derivative.  Two forward forms:

  * contract: the library's own arithmetic -- demand in fixed point
    (rint(d 2^20)), integer loading, the K-section line search with exact
    sums, f += rint(alpha (y - f)).  Its states are bit-identical to the GPU
    solve, so GPU and oracle backward passes see the same inputs.
  * exact: FP64 throughout, alpha_j the root of C' to full precision; smooth
    in (d, C), so central finite differences check the backward pass.

Plain numpy; the incidence is a scipy sparse matrix.  Shares no code with the
GPU library.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import scipy.sparse as sp

from . import (FX, RULE_CEIL, _f32, _i32, _i64, _p, fw_update, kappa, lib, line_search, trips_to_fx)


def paths(net, cost, orig, dest, d_fx, dt_s, rule=RULE_CEIL):
    """Truncated path of every leg under the trees of `cost` (walk order):
    offsets ptr (int64[P+1]) and link ids (int32[ptr[-1]])."""
    rp, col, cost = _i32(net.row_ptr), _i32(net.col), _f32(cost)
    orig, dest, d_fx = _i32(orig), _i32(dest), _i64(d_fx)
    P = orig.shape[0]
    ptr = np.zeros(P + 1, dtype=np.int64)
    L = lib()
    L.orc_paths.argtypes = [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                            C.c_void_p, C.c_void_p, C.c_double, C.c_int32, C.c_void_p, C.c_void_p]
    args = (net.n, col.shape[0], _p(rp), _p(col), _p(cost), P, _p(orig), _p(dest), _p(d_fx), float(dt_s), rule)
    rc = L.orc_paths(*args, _p(ptr), None)
    if rc < 0:
        raise RuntimeError(f"orc_paths failed {rc}")
    links = np.zeros(int(ptr[-1]), dtype=np.int32)
    rc = L.orc_paths(*args, _p(ptr), _p(links))
    if rc < 0:
        raise RuntimeError(f"orc_paths failed {rc}")
    return ptr, links


def incidence(ptr, links, m, dtype=np.float64):
    """L (legs x links): L[p, a] = 1 when leg p's truncated path loads a."""
    P = ptr.shape[0] - 1
    rows = np.repeat(np.arange(P, dtype=np.int64), np.diff(ptr))
    return sp.csr_matrix((np.ones(links.shape[0], dtype=dtype), (rows, links.astype(np.int64))), shape=(P, m))


def frozen_paths(net, orig, dest, d_fx, hist_cost, dt_s, rule=RULE_CEIL):
    """Paths of iterates j = 0..J under the recorded costs c_j."""
    return [paths(net, hist_cost[j], orig, dest, d_fx, dt_s, rule) for j in range(len(hist_cost))]


def bpr_terms(v, c0, cap, alpha_b, beta, kap):
    """c(v), dc/dv and dc/dC of Eq. 1 in FP64 (v in veh, r = kappa v / C)."""
    c0 = np.asarray(c0, dtype=np.float64)
    cap = np.asarray(cap, dtype=np.float64)
    r = (v * kap) / cap
    p1 = np.ones_like(r)
    for _ in range(beta - 1):
        p1 = p1 * r
    p = p1 * r
    cost = c0 * (1.0 + alpha_b * p)
    dcdv = c0 * alpha_b * beta * p1 * kap / cap
    dcdcap = -c0 * alpha_b * beta * p / cap
    return cost, dcdv, dcdcap


def forward_contract(path_list, m, d, c0, cap, alpha_b, beta, dt_s, **ls_kw):
    """The library's arithmetic at frozen paths.  Returns f_fx (int64[m]) and
    the states [(f_j before update j, y_j, alpha_j)], j = 0..J (j = 0 holds
    (None, y_0, 1.0))."""
    d_fx = trips_to_fx(d)
    ys = []
    for ptr, links in path_list:
        Lj = incidence(ptr, links, m, dtype=np.int64)
        ys.append(np.asarray(Lj.T @ d_fx, dtype=np.int64))
    f = ys[0].copy()
    states = [(None, ys[0], 1.0)]
    for j in range(1, len(ys)):
        a, _, _ = line_search(f, ys[j], c0, cap, alpha_b, beta, dt_s, j, **ls_kw)
        states.append((f.copy(), ys[j], a))
        f = fw_update(f, ys[j], a)
    return f, states


def exact_root(F, Y, c0, cap, alpha_b, beta, kap):
    """Root of C'(a) = sum t c(F + a t) on [0, 1] by bisection to adjacent
    doubles; 0 when C'(0) >= 0, 1 when C'(1) < 0 (the bracket ends of the
    K-section rule)."""
    t = Y - F

    def g(a):
        return float(np.sum(t * bpr_terms(F + a * t, c0, cap, alpha_b, beta, kap)[0]))

    if g(0.0) >= 0.0:
        return 0.0
    if g(1.0) < 0.0:
        return 1.0
    lo, hi = 0.0, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if g(mid) >= 0.0:
            hi = mid
        else:
            lo = mid
    return lo if abs(g(lo)) <= abs(g(hi)) else hi


def forward_exact(path_list, m, d, c0, cap, alpha_b, beta, dt_s):
    """FP64 model (no fixed point, exact step sizes): f (veh) and states."""
    kap = kappa(dt_s)
    d = np.asarray(d, dtype=np.float64)
    ys = [np.asarray(incidence(ptr, links, m).T @ d) for ptr, links in path_list]
    f = ys[0].copy()
    states = [(None, ys[0], 1.0)]
    for j in range(1, len(ys)):
        a = exact_root(f, ys[j], c0, cap, alpha_b, beta, kap)
        states.append((f.copy(), ys[j], a))
        f = f + a * (ys[j] - f)
    return f, states


def backward(states, fbar, path_list, c0, cap, alpha_b, beta, dt_s, fixed_point=True, fixed_steps=False):
    """Reverse pass: given dL/df (per link, per veh), returns dL/dd (per leg,
    per veh) and dL/dC (per link).  `fixed_point` states hold int64 flows in
    units of 2^-20 veh (forward_contract), else FP64 veh (forward_exact).
    `fixed_steps`: the step sizes are a fixed sequence (MSA), not roots, so
    they carry no derivative."""
    kap = kappa(dt_s)
    m = np.asarray(c0).shape[0]
    fbar = np.array(fbar, dtype=np.float64)
    capbar = np.zeros(m, dtype=np.float64)
    P = path_list[0][0].shape[0] - 1
    dbar = np.zeros(P, dtype=np.float64)
    scale = 1.0 / FX if fixed_point else 1.0
    for j in range(len(states) - 1, 0, -1):
        fj, yj, a = states[j]
        F = np.asarray(fj, dtype=np.float64) * scale
        Y = np.asarray(yj, dtype=np.float64) * scale
        t = Y - F
        cost, dcdv, dcdcap = bpr_terms(F + a * t, c0, cap, alpha_b, beta, kap)
        abar = float(np.sum(fbar * t))
        s = 0.0
        if not fixed_steps and 0.0 < a < 1.0:
            Fa = float(np.sum(t * t * dcdv))
            if Fa != 0.0:
                s = -abar / Fa
        ybar = a * fbar + s * (cost + a * t * dcdv)
        fbar = (1.0 - a) * fbar + s * (-cost + (1.0 - a) * t * dcdv)
        capbar = capbar + s * t * dcdcap
        dbar = dbar + np.asarray(incidence(*path_list[j], m) @ ybar)
    dbar = dbar + np.asarray(incidence(*path_list[0], m) @ fbar)
    return dbar, capbar
