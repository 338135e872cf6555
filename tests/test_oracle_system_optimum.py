"""Pins of the oracle's system-optimum objective (the second of Wardrop's
principles, named in section 3 next to the user equilibrium the paper
adopts): the routing cost is the marginal cost d(F c(F))/dF, the objective
the total travel time sum F c(F).  Each pin checks the oracle against a
definition it does not use: numerical derivatives of the total cost,
direct minimisation of the total travel time, and the ordering of the two
equilibria's total travel times."""
from __future__ import annotations

import numpy as np
import pytest
from scipy.optimize import minimize, minimize_scalar

import synth
from synth.networks import Network

FX = 1 << 20


def _tt(x, c0, cap, ab, beta, kap=1.0):
    """Total travel time of flows x (veh): sum x c(x), c by Eq. 1, FP64."""
    x = np.asarray(x, np.float64)
    return float(np.sum(x * c0 * (1.0 + ab * (kap * x / cap) ** beta)))


def test_marginal_cost_is_derivative_of_total_cost(orc):
    rng = np.random.default_rng(3)
    m = 200
    c0 = rng.uniform(30, 120, m).astype(np.float32)
    cap = rng.choice([900.0, 1800.0, 3600.0], m).astype(np.float32)
    F = rng.uniform(0, 4000, m)
    f_fx = np.rint(F * FX).astype(np.int64)
    F = f_fx / FX
    for beta, dt in [(4, float("inf")), (1, 900.0), (3, 600.0)]:
        kap = 3600.0 / dt if np.isfinite(dt) else 1.0
        mc, rc = orc.bpr(f_fx, c0, cap, 0.15, beta, dt, marginal=True)
        assert rc == 0
        c64, c064 = cap.astype(np.longdouble), c0.astype(np.longdouble)
        h = np.longdouble(1e-3)
        Fl = F.astype(np.longdouble)

        def total(x):
            return x * c064 * (1 + np.longdouble(0.15) * (np.longdouble(kap) * x / c64) ** beta)

        num = (total(Fl + h) - total(Fl - h)) / (2 * h)
        assert np.allclose(mc.astype(np.float64), num.astype(np.float64), rtol=2e-7, atol=0)
        zero, _ = orc.bpr(np.zeros(m, np.int64), c0, cap, 0.15, beta, dt, marginal=True)
        assert np.array_equal(zero, c0)


def test_system_optimum_two_parallel_links(orc):
    """0 -> 1 by two parallel links: the FW system optimum equals the
    minimiser of x c1(x) + (D - x) c2(D - x) found by bounded scalar search,
    and its total travel time is below the user equilibrium's."""
    net = Network(2, np.array([0, 2, 2], np.int32), np.array([1, 1], np.int32),
                  np.array([60.0, 75.0], np.float32), np.array([900.0, 1800.0], np.float32))
    D, ab, beta = 2500.0, 0.15, 4
    c0, cap = net.fftt.astype(np.float64), net.cap.astype(np.float64)
    r = minimize_scalar(lambda x: _tt([x, D - x], c0, cap, ab, beta), bounds=(0, D), method="bounded",
                        options={"xatol": 1e-9})
    args = (net, np.array([0], np.int32), np.array([1], np.int32), np.array([int(D * FX)]))
    so = orc.fw_solve(*args, dt_s=float("inf"), tol=1e-8, max_iter=400, objective=orc.OBJ_SO)
    ue = orc.fw_solve(*args, dt_s=float("inf"), tol=1e-8, max_iter=400)
    assert abs(so.f[0] / FX - r.x) < 1e-3 * D
    assert abs(ue.f[0] / FX - r.x) > 1e-2 * D              # the two principles differ here
    tt_so = _tt(so.f / FX, c0, cap, ab, beta)
    tt_ue = _tt(ue.f / FX, c0, cap, ab, beta)
    assert tt_so < tt_ue
    assert so.objective == pytest.approx(tt_so, rel=1e-9)


def test_system_optimum_braess(orc):
    """Braess network with beta = 1 (affine costs): the system optimum's link
    flows against a direct constrained minimisation of the total travel
    time over the three path flows."""
    rp = np.array([0, 2, 4, 5, 5], np.int32)
    col = np.array([1, 2, 2, 3, 3], np.int32)
    c0 = np.array([1.0, 50.0, 10.0, 50.0, 1.0], np.float32)
    cap = np.array([0.1, 50.0, 10.0, 50.0, 0.1], np.float32)
    net = Network(4, rp, col, c0, cap)
    D = 6.0
    inc = np.array([[1, 0, 1], [0, 1, 0], [0, 0, 1], [1, 0, 0], [0, 1, 1]], np.float64)  # links x paths
    c064, cap64 = c0.astype(np.float64), cap.astype(np.float64)

    def tt(h):
        return _tt(inc @ h, c064, cap64, 1.0, 1)

    r = minimize(tt, np.full(3, D / 3), method="SLSQP", bounds=[(0, D)] * 3,
                 constraints=[{"type": "eq", "fun": lambda h: h.sum() - D}], options={"ftol": 1e-14})
    xstar = inc @ r.x
    fw = orc.fw_solve(net, np.array([0], np.int32), np.array([3], np.int32), np.array([int(D * FX)]),
                      alpha_b=1.0, beta=1, dt_s=float("inf"), tol=1e-9, max_iter=3000, objective=orc.OBJ_SO)
    assert np.allclose(fw.f / FX, xstar, rtol=0, atol=5e-3 * D)
    ue = orc.fw_solve(net, np.array([0], np.int32), np.array([3], np.int32), np.array([int(D * FX)]),
                      alpha_b=1.0, beta=1, dt_s=float("inf"), tol=1e-9, max_iter=3000)
    assert tt(np.linalg.lstsq(inc, fw.f / FX, rcond=None)[0]) <= tt(np.linalg.lstsq(inc, ue.f / FX, rcond=None)[0])


def test_system_optimum_total_time_below_equilibrium_grid(orc):
    """Config 1: the system optimum's total travel time is below the user
    equilibrium's, and the reported objective is the total travel time."""
    w = synth.config1()
    d_fx = orc.trips_to_fx(w.demand.trips)
    args = (w.net, w.demand.orig, w.demand.dest, d_fx)
    so = orc.fw_solve(*args, fixed_iters=60, objective=orc.OBJ_SO, keep_history=False)
    ue = orc.fw_solve(*args, fixed_iters=60, keep_history=False)
    c0, cap = w.net.fftt.astype(np.float64), w.net.cap.astype(np.float64)
    tt_so, tt_ue = _tt(so.f / FX, c0, cap, 0.15, 4), _tt(ue.f / FX, c0, cap, 0.15, 4)
    assert tt_so < tt_ue
    assert so.objective == pytest.approx(tt_so, rel=1e-9)
    assert 0 <= so.gap < 1e-2


def _tt_root(f, y, c0, cap, ab, beta, kappa):
    """Root in [0, 1] of d/dalpha sum v c(v), v = F + alpha t, from the
    polynomial v (c0 + c0 ab (kappa v / C)^beta) expanded in alpha and
    differentiated by numpy (no marginal-cost formula involved)."""
    poly = np.poly1d([0.0])
    for a in range(f.size):
        F, t = f[a] / FX, (y[a] - f[a]) / FX
        v = np.poly1d([t, F])
        base = np.poly1d([kappa * t / cap[a], kappa * F / cap[a]])
        poly = poly + v * float(c0[a]) + v * float(c0[a]) * ab * base ** beta
    d = poly.deriv()
    real = [r.real for r in d.roots if abs(r.imag) < 1e-9 and -1e-9 <= r.real <= 1 + 1e-9]
    return min(real) if real else None


@pytest.mark.parametrize("seed", [0, 1, 4, 7])       # instances whose root lies inside (0, 1)
def test_system_optimum_line_search_root(orc, seed):
    rng = np.random.default_rng(700 + seed)
    m = 5
    c0 = rng.uniform(10, 100, m).astype(np.float32)
    cap = rng.choice([900.0, 1800.0], m).astype(np.float32)
    f = rng.integers(100 * FX, 900 * FX, m).astype(np.int64)
    y = rng.integers(0, 300 * FX, m).astype(np.int64)
    y[0] = 2000 * FX
    root = _tt_root(f, y, c0, cap, 0.15, 4, 4.0)
    assert root is not None and 0.0 < root < 1.0
    a_ks, _, _ = orc.line_search(f, y, c0, cap, 0.15, 4, 900.0, 3, objective=orc.OBJ_SO)
    assert abs(a_ks - root) < 1e-4
    a_qn, _, _ = orc.line_search(f, y, c0, cap, 0.15, 4, 900.0, 3, ls_mode=orc.LS_QN, objective=orc.OBJ_SO)
    assert abs(a_qn - root) < 2e-4
    ue, _, _ = orc.line_search(f, y, c0, cap, 0.15, 4, 900.0, 3)
    assert abs(ue - a_ks) > 1e-3          # a different objective, a different step


def test_system_optimum_day_trip_conservation(orc):
    """Under the system optimum too, demand entering an interval = demand
    completing in it + residual carried out (travel times clock the walk),
    to within one fixed-point unit per (iterate, leg)."""
    w = synth.config1()
    rng = np.random.default_rng(19)
    days = []
    for i in range(3):
        sel = rng.random(w.demand.P) < 0.4
        days.append(synth.demand.Demand(w.demand.orig[sel], w.demand.dest[sel], w.demand.trips[sel] / 3, 600.0))
    out, left = orc.qdta_day(w.net, days, tol=1e-3, max_iter=20, objective=orc.OBJ_SO)
    carried = 0
    for r in out:
        res = int(r["res"][2].sum())
        assert abs(r["in_fx"] - (r["done_fx"] + res)) <= (r["iters"] + 1) * r["legs"]
        carried += res
    assert carried > 0
