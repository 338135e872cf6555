"""Pins of the oracle's FP64 references and of its stop branches.

- orc_ref_fp64 (the long-double gap and objective of an iterate) against
  exact rational arithmetic and quadrature;
- the contract's exact-sum gap and objective within 1e-6 of that reference;
- the pure-FP64 Frank-Wolfe (oracle/pure.py) against the two-link and Braess
  closed forms, and the contract mode against it through the Frank-Wolfe
  duality bound;
- the objective-change stop of Eq. 7 on a two-link instance whose relative
  change is computed by hand in exact arithmetic;
- the stall stop (alpha* = 0) on an instance built so that the truncated
  all-or-nothing direction is uphill;
- the rounding of the flow update (Alg. 6), hand-computed halves.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.integrate import quad

import synth
from oracle import pure
from synth.networks import Network

FX = 1 << 20


def _frac_cost(F, c0, cap, ab, beta, kappa, so=False):
    p = (Fraction(kappa) * F / Fraction(float(cap))) ** beta
    if so:
        return Fraction(float(c0)) * (1 + Fraction(ab) * (beta + 1) * p)
    return Fraction(float(c0)) * (1 + Fraction(ab) * p)


@pytest.mark.parametrize("so", [False, True])
@pytest.mark.parametrize("dt", [float("inf"), 900.0])
def test_ref_fp64_against_exact_rationals(orc, so, dt):
    """Sums of costs times flows in exact rational arithmetic (every input is
    a binary fraction, so the sums have an exact value); the Beckmann integral
    by adaptive quadrature of the cost curve."""
    rng = np.random.default_rng(31)
    m = 40
    c0 = rng.uniform(10, 200, m).astype(np.float32)
    cap = rng.choice([900.0, 1800.0, 3600.0], m).astype(np.float32)
    f = rng.integers(0, 400 * FX, m).astype(np.int64)
    y = rng.integers(0, 800 * FX, m).astype(np.int64)
    ab, beta = 0.15, 4
    kappa = 3600.0 / dt if math.isfinite(dt) else 1.0
    r = orc.ref_fp64(f, y, c0, cap, ab, beta, dt, objective=1 if so else 0)
    scf = sum(_frac_cost(Fraction(int(f[a]), FX), c0[a], cap[a], ab, beta, kappa, so) * Fraction(int(f[a]), FX)
              for a in range(m))
    scy = sum(_frac_cost(Fraction(int(f[a]), FX), c0[a], cap[a], ab, beta, kappa, so) * Fraction(int(y[a]), FX)
              for a in range(m))
    assert abs(r["scf"] - float(scf)) <= 1e-14 * float(scf)
    assert abs(r["scy"] - float(scy)) <= 1e-14 * float(scy)
    assert abs(r["gap"] - float((scf - scy) / scf)) <= 1e-13 * abs(float((scf - scy) / scf))
    if so:
        obj = sum(Fraction(int(f[a]), FX) * _frac_cost(Fraction(int(f[a]), FX), c0[a], cap[a], ab, beta, kappa)
                  for a in range(m))
        assert abs(r["objective"] - float(obj)) <= 1e-14 * float(obj)
    else:
        obj = 0.0
        for a in range(m):
            F = f[a] / FX
            obj += quad(lambda s: float(c0[a]) * (1 + ab * (kappa * s / float(cap[a])) ** beta), 0.0, F,
                        epsabs=0, epsrel=1e-13)[0]
        assert abs(r["objective"] - obj) <= 1e-11 * obj


@pytest.mark.parametrize("case", ["config1", "config1_trunc", "config1_so"])
def test_contract_gap_and_objective_within_1e6_of_fp64(orc, case):
    """Per reported result: the relative gap and the objective the contract
    computes (FP32 routing costs, terms quantised to 2^-16 and summed exactly)
    agree with the long-double reference of the same iterate to 1e-6 (the gap,
    itself a relative quantity, in absolute terms; the objective relatively)."""
    w = synth.config1()
    o, d, wfx = orc.merge_legs(w.demand.orig, w.demand.dest, orc.trips_to_fx(w.demand.trips))
    kw = dict(fixed_iters=20, keep_history=False)
    if case == "config1_trunc":
        kw.update(dt_s=900.0)
    if case == "config1_so":
        kw.update(objective=orc.OBJ_SO)
    for fixed in (1, 5, 20):
        kw["fixed_iters"] = fixed
        r = orc.fw_solve(w.net, o, d, wfx, **kw)
        assert abs(r.gap - r.gap_fp64) <= 1e-6, (fixed, r.gap, r.gap_fp64)
        assert abs(r.objective - r.objective_fp64) <= 1e-6 * abs(r.objective_fp64), fixed
        # and the reference is not the same computation: the FP32 routing costs
        # move the gap by a few 1e-8 at most, but not by nothing
        assert r.gap_fp64 != 0.0


# ---------------------------------------------------------------------------
# pure-FP64 Frank-Wolfe
# ---------------------------------------------------------------------------
def test_pure_fw_two_parallel_links():
    net = Network(2, np.array([0, 2, 2], np.int32), np.array([1, 1], np.int32),
                  np.array([60.0, 75.0], np.float32), np.array([900.0, 1800.0], np.float32))
    D, ab, beta = 2500.0, 0.15, 4

    def c(k, x):
        return float(net.fftt[k]) * (1 + ab * (x / float(net.cap[k])) ** beta)

    lo, hi = 0.0, D
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if c(0, mid) < c(1, D - mid):
            lo = mid
        else:
            hi = mid
    r = pure.fw(net, [0], [1], [D], iters=60)
    assert abs(r.f[0] - 0.5 * (lo + hi)) < 1e-6 * D
    assert abs(r.gaps[-1]) < 1e-9


def test_pure_fw_braess_affine():
    rp = np.array([0, 2, 4, 5, 5], np.int32)
    col = np.array([1, 2, 2, 3, 3], np.int32)
    c0 = np.array([1.0, 50.0, 10.0, 50.0, 1.0], np.float32)
    cap = np.array([0.1, 50.0, 10.0, 50.0, 0.1], np.float32)
    net = Network(4, rp, col, c0, cap)
    D = 6.0
    slope = c0.astype(np.float64) / cap.astype(np.float64)
    inc = np.array([[1, 0, 1], [0, 1, 0], [0, 0, 1], [1, 0, 0], [0, 1, 1]], np.float64)
    Cm = inc.T @ np.diag(slope) @ inc
    c0p = inc.T @ c0.astype(np.float64)
    A = np.array([Cm[0] - Cm[1], Cm[0] - Cm[2], [1.0, 1.0, 1.0]])
    b = np.array([c0p[1] - c0p[0], c0p[2] - c0p[0], D])
    xstar = inc @ np.linalg.solve(A, b)
    r = pure.fw(net, [0], [3], [D], alpha_b=1.0, beta=1, iters=3000)
    assert np.allclose(r.f, xstar, rtol=0, atol=2e-3 * D)


def test_contract_and_pure_objectives_bracket_the_optimum(orc):
    """Config 1, 50 updates of each mode.  For plain static assignment every
    iterate f with direction y bounds the optimum from below,
    B* >= B(f) - sum c(f) (f - y), and from above by B(f).  The lower bound of
    either run must lie below the objective of both (a wrong objective or a
    wrong direction in either mode breaks this), and both runs end within
    their own bound of the optimum."""
    w = synth.config1()
    o, d, wfx = orc.merge_legs(w.demand.orig, w.demand.dest, orc.trips_to_fx(w.demand.trips))
    c = orc.fw_solve(w.net, o, d, wfx, fixed_iters=50, keep_history=False)
    cost, _ = orc.bpr(c.f, w.net.fftt, w.net.cap, 0.15, 4, float("inf"))
    y, _, _ = orc.aon(w.net, cost, o, d, wfx, float("inf"))
    rr = orc.ref_fp64(c.f, y, w.net.fftt, w.net.cap, 0.15, 4, float("inf"))
    lb_c = rr["objective"] - (rr["scf"] - rr["scy"])
    p = pure.fw(w.net, o, d, wfx / FX, iters=50)
    lb = max(lb_c, p.lower_bound)
    ub = min(c.objective, p.objectives[-1])
    assert lb <= ub * (1 + 1e-12)
    assert c.objective - lb <= 5e-3 * c.objective
    assert p.objectives[-1] - lb <= 5e-3 * p.objectives[-1]
    assert abs(c.objective - rr["objective"]) <= 1e-6 * rr["objective"]


# ---------------------------------------------------------------------------
# stop branches
# ---------------------------------------------------------------------------
def _two_links():
    # 0 -> 1 by two parallel links: c0 = 10 s and 12 s, capacity 1000 veh/h
    return Network(2, np.array([0, 2, 2], np.int32), np.array([1, 1], np.int32),
                   np.array([10.0, 12.0], np.float32), np.array([1000.0, 1000.0], np.float32))


def _beckmann_exact(fx, net, ab, beta):
    """Eq. 6 by hand for plain static assignment, exact rationals:
    sum c0 F (1 + ab (F / C)^beta / (beta + 1))."""
    s = Fraction(0)
    for a in range(net.m):
        F = Fraction(int(fx[a]), FX)
        s += Fraction(float(net.fftt[a])) * F * (1 + Fraction(ab) * (F / Fraction(float(net.cap[a]))) ** beta /
                                                  (beta + 1))
    return s


def test_objective_change_stop_eq7(orc):
    """Free flow puts all 2,000 veh/h on link 0 (10 s < 12 s); under BPR link 0
    costs 34 s, so the first direction moves everything to link 1.  The step
    alpha* balances the two costs.  The relative objective change of Eq. 7,
    |B(f) - B(f_new)| / B(f), is computed here by hand in exact arithmetic
    from the closed form; the oracle must stop at the first test (returning the
    free-flow iterate, Alg. 2 breaks before updating) exactly when T0 exceeds
    that change."""
    net = _two_links()
    ab, beta, D = 0.15, 4, 2000.0
    dfx = np.array([int(D * FX)], np.int64)
    f0 = np.array([int(D * FX), 0], np.int64)
    y1 = np.array([0, int(D * FX)], np.int64)
    alpha, _, _ = orc.line_search(f0, y1, net.fftt, net.cap, ab, beta, float("inf"), 1)
    # the step is the balance point of the two BPR curves (pinned, not assumed)
    lo, hi = 0.0, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        xa, xb = D * (1 - mid), D * mid
        if 10 * (1 + ab * (xa / 1000) ** 4) > 12 * (1 + ab * (xb / 1000) ** 4):
            lo = mid
        else:
            hi = mid
    assert abs(alpha - 0.5 * (lo + hi)) < 1e-4
    f1 = f0 + np.array([int(np.rint(alpha * (y1[a] - f0[a]))) for a in range(2)], np.int64)
    b0, b1 = _beckmann_exact(f0, net, ab, beta), _beckmann_exact(f1, net, ab, beta)
    change = float(abs(b0 - b1) / b0)
    assert 0.05 < change < 0.9
    for tol, stops in ((change * (1 + 1e-6), True), (change * (1 - 1e-6), False)):
        r = orc.fw_solve(net, [0], [1], dfx, alpha_b=ab, beta=beta, stop_rule=orc.STOP_OBJ, tol=tol, max_iter=1,
                         keep_history=False)
        if stops:
            assert r.stopped_by == 2 and r.iters == 0
            assert np.array_equal(r.f, f0)
        else:
            assert r.stopped_by != 2 and r.iters == 1
            assert np.array_equal(r.f, f1)


def _uphill_net():
    # node 0 (origin) -> 1 -> 3 (route A: 12 s + 1 s) and 0 -> 2 -> 3 (route B:
    # 2 s + 12 s); CSR order: 0->1, 0->2, 1->3, 2->3; capacities 3,600 veh/h
    return Network(4, np.array([0, 2, 3, 4, 4], np.int32), np.array([1, 2, 3, 3], np.int32),
                   np.array([12.0, 2.0, 1.0, 12.0], np.float32), np.full(4, 3600.0, np.float32))


@pytest.mark.parametrize("mode", ["ksection", "qn"])
def test_stall_stop_on_uphill_truncated_direction(orc, mode):
    """A 10 s interval, one leg of 9.5 trips from 0 to 3.  At free flow route A
    (13 s) wins; under CEIL the leg enters link 0->1 at 0 s and is cut at node 1
    (12 s >= 10 s), so f loads 0->1 only.  Under BPR(f) with kappa = 360,
    0->1 costs 12 (1 + 0.15 * 0.95^4) = 13.47 s, so route B (14 s) is now
    shorter, and the leg enters both of its links before 10 s: y loads 0->2
    and 2->3.  sum c(f) y = 14 * 9.5 > sum c(f) f = 13.47 * 9.5, so the
    direction is uphill, C'(alpha) > 0 on [0, 1], alpha* = 0, and the oracle
    must stop on the stall rule with the free-flow iterate."""
    net = _uphill_net()
    dfx = np.array([int(9.5 * FX)], np.int64)
    ls_mode = {"ksection": 0, "qn": 1}[mode]
    r = orc.fw_solve(net, [0], [3], dfx, dt_s=10.0, rule=orc.RULE_CEIL, tol=1e-4, max_iter=50, ls_mode=ls_mode,
                     keep_history=False)
    assert r.stopped_by == 3 and r.iters == 0
    assert r.f.tolist() == [int(9.5 * FX), 0, 0, 0]
    c13 = 12.0 * (1 + 0.15 * 0.95 ** 4)
    assert abs(r.gap - (c13 - 14.0) / c13) < 1e-6
    # MSA has no line search to stall: it takes alpha = 1/2
    rm = orc.fw_solve(net, [0], [3], dfx, dt_s=10.0, rule=orc.RULE_CEIL, fixed_iters=1, ls_mode=2,
                      keep_history=False)
    assert rm.iters == 1 and rm.f.tolist() == [int(4.75 * FX), int(4.75 * FX), 0, int(4.75 * FX)]


def test_fw_update_rounds_half_to_even(orc):
    """f + rint(alpha (y - f)) with ties to even, hand-computed: a floor, a
    truncation or a round-half-away rule each fails one of these."""
    f = np.zeros(9, np.int64)
    y = np.array([3, 5, -3, -5, 1, 7, 2, 6, -1], np.int64)
    assert orc.fw_update(f, y, 0.5).tolist() == [2, 2, -2, -2, 0, 4, 1, 3, 0]
    y = np.array([2, 6, 10, -2, -6, -10, 1, 3], np.int64)
    assert orc.fw_update(f[:8], y, 0.25).tolist() == [0, 2, 2, 0, -2, -2, 0, 1]
    f = np.array([100, 100, 100], np.int64)
    y = np.array([103, 97, 105], np.int64)
    assert orc.fw_update(f, y, 0.5).tolist() == [102, 98, 102]


def test_demand_legs_quantise_and_merge(orc):
    """The vectorised quantisation equals the C routine on halves of a unit
    (ties to even), and demand_legs sums equal pairs, drops self and empty
    legs, and sorts by (destination, origin)."""
    u = 2.0 ** -20
    trips = np.array([0.5 * u, 1.5 * u, 2.5 * u, 3.0, 1e-9, 7.25, 0.0, 12345.678], np.float64)
    assert np.array_equal(orc.trips_to_fx_array(trips), orc.trips_to_fx(trips))
    assert orc.trips_to_fx_array(trips)[:3].tolist() == [0, 2, 2]
    o, d, w = orc.demand_legs([3, 1, 3, 2, 2, 0], [5, 5, 5, 2, 4, 5], [1.0, 2.0, 0.5, 9.0, 0.0, 4.0])
    assert o.tolist() == [0, 1, 3] and d.tolist() == [5, 5, 5]
    assert w.tolist() == [4 * FX, 2 * FX, int(1.5 * FX)]
