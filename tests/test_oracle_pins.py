"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every test here checks the oracle against something other than itself:
values printed in the paper's worked example (section 6), brute-force path
enumeration, a library Dijkstra on integer costs, closed-form equilibria,
quadrature, exact Python integers, and structural invariants.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import dijkstra

import synth
from synth.networks import Network
from tests import bruteforce as bf

GOLD = os.path.join(os.path.dirname(__file__), "golden")
FX = 1 << 20


def _example():
    with open(os.path.join(GOLD, "paper_example.json")) as fh:
        return json.load(fh)


# ---------------------------------------------------------------------------
# BPR (Eq. 1) -- worked example, section 6
# ---------------------------------------------------------------------------
def test_bpr_worked_example(orc):
    g = _example()
    w = synth.paper_example()
    net = w.net
    # t2: 225 veh/h on l34 over a 15-min interval = 56.25 vehicles
    f = np.array([0, 0, int(56.25 * FX), 0], dtype=np.int64)
    c, rc = orc.bpr(f, net.fftt, net.cap, g["bpr"]["alpha"], g["bpr"]["beta"], 900.0)
    assert rc == 0
    assert abs(c[2] / 60.0 - g["printed"]["t2_time_l34_min"]["value"]) < 0.05
    # t1: 175 veh/h on l23; printed 6.3, truncated to one decimal
    f = np.array([int(43.75 * FX), int(43.75 * FX), 0, 0], dtype=np.int64)
    c, rc = orc.bpr(f, net.fftt, net.cap, 0.15, 4, 900.0)
    assert 6.3 <= c[1] / 60.0 < 6.4
    # zero flow: exactly the free-flow time
    c, _ = orc.bpr(np.zeros(4, np.int64), net.fftt, net.cap, 0.15, 4, 900.0)
    assert np.array_equal(c, net.fftt)


def test_bpr_special_points(orc):
    # at flow rate == capacity the curve is c0 (1 + alpha): kappa = 1 (plain)
    c0 = np.array([30.0, 45.5, 119.0], np.float32)
    cap = np.array([900.0, 1800.0, 3600.0], np.float32)
    f = (cap.astype(np.float64) * FX).astype(np.int64)
    c, _ = orc.bpr(f, c0, cap, 0.15, 4, float("inf"))
    assert np.array_equal(c, (c0.astype(np.float64) * 1.15).astype(np.float32))
    # 15-min interval: a quarter of capacity in vehicles is a rate equal to capacity
    f = (cap.astype(np.float64) / 4 * FX).astype(np.int64)
    c, _ = orc.bpr(f, c0, cap, 0.15, 4, 900.0)
    assert np.array_equal(c, (c0.astype(np.float64) * 1.15).astype(np.float32))
    # beta = 1 is affine: twice capacity gives c0 (1 + 2 alpha)
    c, _ = orc.bpr(2 * (cap.astype(np.float64) * FX).astype(np.int64), c0, cap, 0.5, 1, float("inf"))
    assert np.array_equal(c, (c0.astype(np.float64) * 2.0).astype(np.float32))


# ---------------------------------------------------------------------------
# QDTA on the worked example (Alg. 1, Alg. 4; Eq. 2 under the CEIL reading)
# ---------------------------------------------------------------------------
def test_qdta_worked_example_ceil(orc):
    g = _example()
    w = synth.paper_example()
    out, left = orc.qdta_day(w.net, w.demand, alpha_b=0.15, beta=4, rule=orc.RULE_CEIL)
    r1 = out[0]
    # t1: l12 and l23 are loaded with the whole 175 veh/h, nothing beyond
    assert np.array_equal(r1["f"], np.array([int(43.75 * FX), int(43.75 * FX), 0, 0]))
    ro, rd, rw = r1["res"]
    # the residual sits at paper node 3 (index 2), bound for node 4 (index 3)
    assert ro.tolist() == [g["printed"]["t1_residual"]["node"] - 1]
    assert rd.tolist() == [3]
    assert rw.tolist() == [int(g["printed"]["t1_residual"]["vph"] / 4 * FX)]
    # t2: residual + new demand traverse l34 (225 veh/h), d35 continues on l45
    r2 = out[1]
    assert r2["f"][2] == int(g["printed"]["t2_flow_l34_vph"]["value"] / 4 * FX)
    assert r2["f"][3] == int(50 / 4 * FX)
    assert r2["res"][0].size == 0          # all demand arrives in t2
    assert left[0].size == 0
    for r in out[2:]:
        assert r["legs"] == 0


def test_qdta_worked_example_floor_contradicts_paper(orc):
    """The FLOOR reading of Eq. 2 puts the t1 residual at node 2 and leaves
    d35 unfinished in t2 -- both contradict the narrative, which is why CEIL
    is the default reading."""
    w = synth.paper_example()
    out, left = orc.qdta_day(w.net, w.demand, alpha_b=0.15, beta=4, rule=orc.RULE_FLOOR)
    assert out[0]["res"][0].tolist() == [1]
    assert out[1]["res"][0].size > 0


def test_sta_worked_example(orc):
    """STA over the whole hour (section 6, STA figure): flows 43.75, 43.75,
    56.25, 12.5 veh/h, printed as 44/44/57/13; times printed 10/5/10/10."""
    g = _example()
    w = synth.paper_example()
    orig = np.array([0, 2], np.int32)
    dest = np.array([3, 4], np.int32)
    d = np.array([int(43.75 * FX), int(12.5 * FX)], np.int64)
    fw = orc.fw_solve(w.net, orig, dest, d, dt_s=3600.0, rule=orc.RULE_NONE)
    flows = fw.f / FX
    printed = g["printed"]["sta_flows_vph"]
    for k, name in enumerate(["l12", "l23", "l34", "l45"]):
        assert abs(flows[k] - printed[name]) <= 1.0
    c, _ = orc.bpr(fw.f, w.net.fftt, w.net.cap, 0.15, 4, 3600.0)
    times = g["printed"]["sta_times_min"]
    for k, name in enumerate(["l12", "l23", "l34", "l45"]):
        assert round(c[k] / 60.0) == times[name]


def test_plain_interval_equals_sta(orc):
    """dt = inf turns truncation off: QDTA of one interval is STA."""
    w = synth.paper_example()
    out, left = orc.qdta_day(w.net, [synth.demand.Demand(np.array([0], np.int32), np.array([4], np.int32),
                                                          np.array([43.75]), float("inf"))])
    assert out[0]["res"][0].size == 0
    assert np.array_equal(out[0]["f"], np.full(4, int(43.75 * FX)))


def test_free_flow_residual_by_hand(orc):
    """alpha_b = 0: costs stay at free flow (10, 5, 10, 10 min).  d14 reaches
    node 3 at exactly 15 min; CEIL stops there (15 >= 15) without entering l34."""
    w = synth.paper_example()
    out, left = orc.qdta_day(w.net, w.demand[:1], alpha_b=0.0, beta=4)
    assert out[0]["res"][0].tolist() == [2]
    assert out[0]["f"].tolist() == [int(43.75 * FX), int(43.75 * FX), 0, 0]


# ---------------------------------------------------------------------------
# Shortest-path trees: brute force, library special case, invariants
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("costs", ["float", "int", "huge"])
@pytest.mark.parametrize("seed", range(6))
def test_tree_vs_bruteforce(orc, costs, seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(4, 9))
    net = synth.tiny_network(n, int(rng.integers(2, 8)), rng, costs=costs)
    for q in range(n):
        D, succ, rc = orc.tree(net, net.fftt, q)
        Dbf = bf.bf_distances(net, net.fftt, q)
        assert np.array_equal(D, Dbf), (costs, seed, q)
        sbf, absorbed = bf.rule_successors(net, net.fftt, q, Dbf)
        assert np.array_equal(succ.astype(np.int64), sbf), (costs, seed, q)
        assert (rc == orc.WARN_ABSORB) == absorbed


def test_absorption_fallback_is_acyclic(orc):
    """Costs 1e8 next to O(1) costs make fl32(D + c) == D; the fallback must
    still give every node a path to q."""
    found = 0
    for seed in range(40):
        rng = np.random.default_rng(seed)
        net = synth.tiny_network(8, 10, rng, costs="huge")
        for q in range(net.n):
            D, succ, rc = orc.tree(net, net.fftt, q)
            if rc == orc.WARN_ABSORB:
                found += 1
            for v in range(net.n):
                u, steps = v, 0
                while u != q:
                    u = int(net.col[succ[u]])
                    steps += 1
                    assert steps <= net.n
    assert found > 0


def test_tree_integer_costs_match_library_dijkstra(orc):
    """Integer costs with sums below 2^24 make FP32 min-plus exact, so the
    distances must equal SciPy's float64 Dijkstra exactly."""
    rng = np.random.default_rng(7)
    net = synth.grid_network(15, rng)
    cost = np.floor(net.fftt).astype(np.float32)
    g = csr_matrix((cost.astype(np.float64), net.col, net.row_ptr), shape=(net.n, net.n))
    for q in [0, 17, 112, 224]:
        D, succ, _ = orc.tree(net, cost, q)
        ref = dijkstra(g.T.tocsr(), indices=q)
        assert np.array_equal(D.astype(np.float64), ref)
        # invariants: each successor is tight and strictly closer
        for v in range(net.n):
            if v == q:
                assert succ[v] == -1
                continue
            e = succ[v]
            assert net.row_ptr[v] <= e < net.row_ptr[v + 1]
            w = net.col[e]
            assert np.float32(D[w] + cost[e]) == D[v] and D[w] < D[v]


# ---------------------------------------------------------------------------
# Loading with truncation (Alg. 3, Eq. 2, Eq. 5)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("rule,name", [(1, "ceil"), (2, "floor"), (0, "none")])
def test_aon_vs_bruteforce(orc, rule, name):
    for seed in range(5):
        rng = np.random.default_rng(50 + seed)
        net = synth.tiny_network(7, 6, rng, costs="float")
        P = 25
        orig = rng.integers(0, 7, P).astype(np.int32)
        dest = rng.integers(0, 7, P).astype(np.int32)
        d = rng.integers(1, 5 * FX, P).astype(np.int64)
        dt = float(rng.uniform(20, 120))
        y, stop, rc = orc.aon(net, net.fftt, orig, dest, d, dt, rule)
        yb = np.zeros(net.m, np.int64)
        for p in range(P):
            if orig[p] == dest[p]:
                assert stop[p] == -1
                continue
            Dq = bf.bf_distances(net, net.fftt, int(dest[p]))
            sq, _ = bf.rule_successors(net, net.fftt, int(dest[p]), Dq)
            links, s = bf.walk(net, sq, net.fftt, int(orig[p]), int(dest[p]), dt, name)
            for e in links:
                yb[e] += d[p]
            assert stop[p] == s
        assert np.array_equal(y, yb)


def test_aon_node_conservation(orc):
    """At every node: inflow - outflow = -(legs starting there) + (legs that
    complete or stop there)."""
    w = synth.config1()
    net = w.net
    rng = np.random.default_rng(3)
    d = np.array([int(np.rint(t * FX)) for t in w.demand.trips], np.int64)
    y, stop, rc = orc.aon(net, net.fftt * rng.uniform(1, 3, net.m).astype(np.float32), w.demand.orig,
                          w.demand.dest, d, 240.0, orc.RULE_CEIL)
    tails = net.tails()
    bal = np.zeros(net.n, dtype=object)
    np.add.at(bal, net.col, y.astype(object))
    np.subtract.at(bal, tails, y.astype(object))
    exp = np.zeros(net.n, dtype=object)
    np.subtract.at(exp, w.demand.orig, d.astype(object))
    np.add.at(exp, stop, d.astype(object))
    assert (bal == exp).all()
    assert (stop != w.demand.dest).any()      # the 240 s horizon truncates legs


def test_aon_untruncated_hop_sum(orc):
    """Without truncation, sum_a y_a = sum_legs d * hops(path)."""
    w = synth.config1()
    net = w.net
    d = np.array([int(np.rint(t * FX)) for t in w.demand.trips], np.int64)
    y, stop, _ = orc.aon(net, net.fftt, w.demand.orig, w.demand.dest, d, float("inf"))
    total = 0
    for q in np.unique(w.demand.dest):
        D, succ, _ = orc.tree(net, net.fftt, int(q))
        for p in np.nonzero(w.demand.dest == q)[0]:
            u, hops = int(w.demand.orig[p]), 0
            while u != q:
                u = int(net.col[succ[u]])
                hops += 1
            total += int(d[p]) * hops
    assert int(y.sum()) == total
    assert (stop == w.demand.dest).all()


# ---------------------------------------------------------------------------
# Exact sums and conversions
# ---------------------------------------------------------------------------
def test_exact_sum_matches_python_integers(orc):
    rng = np.random.default_rng(11)
    m = 5000
    c = rng.uniform(1, 5000, m).astype(np.float32)
    x = rng.integers(0, 3000 * FX, m).astype(np.int64)
    x[::7] = 0
    s = orc.sum_cx(c, x)
    terms = [float(c[a]) * (float(x[a]) / FX) for a in range(m)]
    assert s == bf.exact_q_sum(terms)


def test_int128_to_double_correctly_rounded(orc):
    rng = np.random.default_rng(5)
    vals = [0, 1, -1, (1 << 53) + 1, (1 << 64) + 12345, -(1 << 90) - 7, (1 << 100) + (1 << 47)]
    vals += [int(v) for v in rng.integers(-(1 << 62), 1 << 62, 50)]
    vals += [int(a) << 40 | int(b) for a, b in zip(rng.integers(0, 1 << 60, 20), rng.integers(0, 1 << 40, 20))]
    for v in vals:
        assert orc.i128_to_double(v) == float(v), v


def test_trips_fixed_point_half_even(orc):
    half = 0.5 / FX
    t = np.array([1.0, 2.5, 3.0 + half, 4.0 + 3 * half, 0.0, 1e-9], np.float64)
    fx = orc.trips_to_fx(t)
    assert fx.tolist() == [FX, int(2.5 * FX), 3 * FX, 4 * FX + 2, 0, 0]


# ---------------------------------------------------------------------------
# Objective (Eq. 6) and its derivative along the direction (Eq. 8-9)
# ---------------------------------------------------------------------------
def _objective_quad(f, y, c0, cap, ab, beta, kappa, alpha):
    tot = 0.0
    for a in range(f.size):
        v = f[a] / FX + alpha * (y[a] / FX - f[a] / FX)
        val, _ = quad(lambda s: float(c0[a]) * (1 + ab * (kappa * s / float(cap[a])) ** beta), 0.0, v,
                      epsabs=0, epsrel=1e-13, limit=200)
        tot += val
    return tot


def test_objective_closed_form_vs_quadrature(orc):
    rng = np.random.default_rng(21)
    m = 60
    c0 = rng.uniform(10, 100, m).astype(np.float32)
    cap = rng.choice([900.0, 1800.0, 3600.0], m).astype(np.float32)
    f = rng.integers(0, 500 * FX, m).astype(np.int64)
    y = rng.integers(0, 800 * FX, m).astype(np.int64)
    alphas = np.array([0.0, 0.25, 0.5, 1.0])
    Cs, Ds, rc = orc.ls_eval(f, y, c0, cap, 0.15, 4, 900.0, alphas)
    for k, a in enumerate(alphas):
        ref = _objective_quad(f, y, c0, cap, 0.15, 4, 4.0, a)
        assert abs(Cs[k] / 65536.0 - ref) <= 1e-9 * ref + m * 2.0 ** -16
    # C'(alpha) is the derivative of C: central difference of the quadrature
    h = 1e-4
    for a in (0.3, 0.7):
        num = (_objective_quad(f, y, c0, cap, 0.15, 4, 4.0, a + h) -
               _objective_quad(f, y, c0, cap, 0.15, 4, 4.0, a - h)) / (2 * h)
        _, Ds1, _ = orc.ls_eval(f, y, c0, cap, 0.15, 4, 900.0, np.array([a]))
        assert abs(Ds1[0] / 65536.0 - num) <= 1e-5 * abs(num)


def test_objective_endpoints(orc):
    """C(0) is the Beckmann objective of f and C(1) that of y."""
    rng = np.random.default_rng(22)
    m = 100
    c0 = rng.uniform(10, 100, m).astype(np.float32)
    cap = rng.choice([900.0, 1800.0], m).astype(np.float32)
    f = rng.integers(0, 500 * FX, m).astype(np.int64)
    y = rng.integers(0, 500 * FX, m).astype(np.int64)
    C01, _, _ = orc.ls_eval(f, y, c0, cap, 0.15, 4, 900.0, np.array([0.0, 1.0]))
    Cf, _, _ = orc.ls_eval(f, f, c0, cap, 0.15, 4, 900.0, np.array([0.0]))
    Cy, _, _ = orc.ls_eval(y, y, c0, cap, 0.15, 4, 900.0, np.array([0.0]))
    assert C01[0] == Cf[0] and C01[1] == Cy[0]


# ---------------------------------------------------------------------------
# Line search (Alg. 8-9) against the polynomial root of C'
# ---------------------------------------------------------------------------
def _cprime_root(f, y, c0, cap, ab, beta, kappa):
    """Root in [0,1] of C'(alpha) = sum_a t_a c0_a (1 + ab (kappa (F + alpha t)/C)^beta),
    expanded as a polynomial in alpha."""
    poly = np.zeros(beta + 1)
    for a in range(f.size):
        F, t = f[a] / FX, (y[a] - f[a]) / FX
        base = np.poly1d([kappa * t / cap[a], kappa * F / cap[a]])
        p = np.poly1d([0.0])
        p = p + t * float(c0[a])
        p = p + t * float(c0[a]) * ab * base ** beta
        poly = np.polyadd(poly, p.coeffs)
    roots = np.roots(poly)
    real = [r.real for r in roots if abs(r.imag) < 1e-9 and -1e-9 <= r.real <= 1 + 1e-9]
    return min(real) if real else None


@pytest.mark.parametrize("seed", range(4))
def test_line_search_root(orc, seed):
    rng = np.random.default_rng(300 + seed)
    m = 5
    c0 = rng.uniform(10, 100, m).astype(np.float32)
    cap = rng.choice([900.0, 1800.0], m).astype(np.float32)
    f = rng.integers(100 * FX, 900 * FX, m).astype(np.int64)
    y = rng.integers(0, 300 * FX, m).astype(np.int64)
    y[0] = 2000 * FX          # make the descent direction cross the root
    root = _cprime_root(f, y, c0, cap, 0.15, 4, 4.0)
    assert root is not None
    a_ks, evals, _ = orc.line_search(f, y, c0, cap, 0.15, 4, 900.0, 3)
    assert evals == 3
    assert abs(a_ks - root) < 1e-4
    a_qn, evals, it = orc.line_search(f, y, c0, cap, 0.15, 4, 900.0, 3, ls_mode=orc.LS_QN)
    assert abs(a_qn - root) < 2e-4
    assert it <= 20
    a_msa, _, _ = orc.line_search(f, y, c0, cap, 0.15, 4, 900.0, 3, ls_mode=orc.LS_MSA)
    assert a_msa == 0.25


def test_line_search_edge_cases(orc):
    c0 = np.array([10.0, 20.0], np.float32)
    cap = np.array([900.0, 900.0], np.float32)
    f = np.array([100 * FX, 100 * FX], np.int64)
    # y == f: C' == 0 everywhere -> the first point already has C' >= 0
    a, _, _ = orc.line_search(f, f, c0, cap, 0.15, 4, 900.0, 1)
    assert a == 0.0
    # y strictly better everywhere (less flow, nothing added): C' < 0 on [0,1]
    a, _, _ = orc.line_search(f, np.zeros(2, np.int64), c0, cap, 0.15, 4, 900.0, 1)
    assert a == 1.0


# ---------------------------------------------------------------------------
# Frank-Wolfe equilibria (Alg. 2 / Alg. 6)
# ---------------------------------------------------------------------------
def _two_link_net():
    # 0 -> 1 by two parallel links
    return Network(2, np.array([0, 2, 2], np.int32), np.array([1, 1], np.int32),
                   np.array([60.0, 75.0], np.float32), np.array([900.0, 1800.0], np.float32))


def test_fw_two_parallel_links(orc):
    net = _two_link_net()
    D = 2500.0
    ab, beta = 0.15, 4

    def c(k, x):
        return float(net.fftt[k]) * (1 + ab * (x / float(net.cap[k])) ** beta)

    lo, hi = 0.0, D
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if c(0, mid) < c(1, D - mid):
            lo = mid
        else:
            hi = mid
    xstar = 0.5 * (lo + hi)
    fw = orc.fw_solve(net, np.array([0], np.int32), np.array([1], np.int32), np.array([int(D * FX)]),
                      dt_s=float("inf"), tol=1e-7, max_iter=200)
    assert abs(fw.f[0] / FX - xstar) < 1e-3 * D
    assert 0 <= fw.gap < 1e-5
    # MSA converges to the same point, more slowly
    fwm = orc.fw_solve(net, np.array([0], np.int32), np.array([1], np.int32), np.array([int(D * FX)]),
                       dt_s=float("inf"), fixed_iters=400, ls_mode=orc.LS_MSA)
    assert abs(fwm.f[0] / FX - xstar) < 2e-2 * D


def test_fw_braess_affine(orc):
    """Braess network with beta = 1 (affine costs, positive intercepts).
    Nodes s=0, a=1, b=2, t=3; links s-a, s-b, a-b, a-t, b-t.  Equilibrium
    path flows solve a 3x3 linear system."""
    # CSR order (tail, head): (0,1) (0,2) (1,2) (1,3) (2,3)
    rp = np.array([0, 2, 4, 5, 5], np.int32)
    col = np.array([1, 2, 2, 3, 3], np.int32)
    # intercepts (c0) 1, 50, 10, 50, 1 and slopes (c0/cap) 10, 1, 1, 1, 10
    c0 = np.array([1.0, 50.0, 10.0, 50.0, 1.0], np.float32)
    cap = np.array([0.1, 50.0, 10.0, 50.0, 0.1], np.float32)
    net = Network(4, rp, col, c0, cap)
    D = 6.0
    # link cost c = c0 + (c0/cap) x; paths P1 = s-a-t (0,3), P2 = s-b-t (1,4), P3 = s-a-b-t (0,2,4)
    slope = c0.astype(np.float64) / cap.astype(np.float64)
    inc = np.array([[1, 0, 1], [0, 1, 0], [0, 0, 1], [1, 0, 0], [0, 1, 1]], np.float64)  # links x paths
    Cmat = inc.T @ np.diag(slope) @ inc
    c0p = inc.T @ c0.astype(np.float64)
    A = np.zeros((3, 3))
    b = np.zeros(3)
    A[0] = Cmat[0] - Cmat[1]
    b[0] = c0p[1] - c0p[0]
    A[1] = Cmat[0] - Cmat[2]
    b[1] = c0p[2] - c0p[0]
    A[2] = 1.0
    b[2] = D
    h = np.linalg.solve(A, b)
    assert (h > 0).all()
    xstar = inc @ h
    fw = orc.fw_solve(net, np.array([0], np.int32), np.array([3], np.int32), np.array([int(D * FX)]),
                      alpha_b=1.0, beta=1, dt_s=float("inf"), tol=1e-9, max_iter=3000)
    assert np.allclose(fw.f / FX, xstar, rtol=0, atol=5e-3 * D)


def test_fw_wardrop_and_flow_reconstruction(orc):
    """Config-1 static assignment: (i) the returned f equals sum_j lambda_j y_j
    rebuilt from the iteration history (Eq. 8-9) to within the rounding of the
    fixed-point updates; (ii) at the end, the paths that carry the most weight
    cost at most 1% above the shortest (Wardrop)."""
    w = synth.config1()
    net = w.net
    d = np.array([int(np.rint(t * FX)) for t in w.demand.trips], np.int64)
    fw = orc.fw_solve(net, w.demand.orig, w.demand.dest, d, fixed_iters=50)
    J = fw.iters
    assert J == 50
    lam = np.empty(J + 1)
    for j in range(J + 1):
        lam[j] = (1.0 if j == 0 else fw.hist_alpha[j]) * np.prod(1 - fw.hist_alpha[j + 1:J + 1])
    assert abs(lam.sum() - 1.0) < 1e-12
    rebuilt = np.zeros(net.m)
    ys = []
    for j in range(J + 1):
        y, _, _ = orc.aon(net, fw.hist_cost[j], w.demand.orig, w.demand.dest, d, float("inf"))
        ys.append(y)
        rebuilt += lam[j] * y
    assert np.abs(rebuilt - fw.f).max() <= J + 1
    cfin, _ = orc.bpr(fw.f, net.fftt, net.cap, 0.15, 4, float("inf"))
    heavy = int(np.argmax(lam))
    worst = 0.0
    for q in np.unique(w.demand.dest)[:10]:
        Dfin, _, _ = orc.tree(net, cfin, int(q))
        _, sj, _ = orc.tree(net, fw.hist_cost[heavy], int(q))
        for p in np.nonzero(w.demand.dest == q)[0][:10]:
            u, t = int(w.demand.orig[p]), 0.0
            while u != q:
                e = sj[u]
                t += float(cfin[e])
                u = int(net.col[e])
            worst = max(worst, t / float(Dfin[w.demand.orig[p]]) - 1)
    assert worst < 0.01
    assert 0 <= fw.gap < 0.01


def test_fw_gap_nonnegative_plain(orc):
    """Without truncation, y minimises sum c y over feasible loadings, so the
    relative gap is a true duality gap: >= 0 at every iteration."""
    w = synth.config1()
    d = np.array([int(np.rint(t * FX)) for t in w.demand.trips], np.int64)
    fw = orc.fw_solve(w.net, w.demand.orig, w.demand.dest, d, fixed_iters=20)
    assert (fw.gaps[:20] >= 0).all()
    assert fw.gaps[19] < fw.gaps[0]


# ---------------------------------------------------------------------------
# Interval chain: conservation (Alg. 1, Alg. 4)
# ---------------------------------------------------------------------------
def test_day_trip_conservation(orc):
    """Demand entering an interval = demand completing in it + residual
    carried out, to within one fixed-point unit per (iterate, leg)."""
    w = synth.config1()
    rng = np.random.default_rng(9)
    days = []
    for i in range(4):
        sel = rng.random(w.demand.P) < 0.3
        days.append(synth.demand.Demand(w.demand.orig[sel], w.demand.dest[sel],
                                        w.demand.trips[sel] / 4, 300.0))
    out, left = orc.qdta_day(w.net, days, tol=1e-3, max_iter=30)
    carried = 0
    for r in out:
        res = int(r["res"][2].sum())
        slack = (r["iters"] + 1) * r["legs"]
        assert abs(r["in_fx"] - (r["done_fx"] + res)) <= slack
        carried += res
    assert carried > 0
    assert out[1]["in_fx"] > int(sum(np.rint(days[1].trips * FX)))   # residual joined interval 1
