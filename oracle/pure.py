"""Pure-FP64 Frank-Wolfe -- TEST INFRASTRUCTURE ONLY.

The oracle's second mode: the same method (BPR costs of Eq. 1, all-or-nothing
assignment of Alg. 3 with the truncation of Eq. 2 and Eq. 5, the Beckmann
objective of Eq. 6, the link-flow Frank-Wolfe loop of Alg. 6) with every
quantity in FP64 and nothing rounded: costs stay FP64, shortest paths come
from SciPy's FP64 Dijkstra, flows are real numbers (no fixed point), and the
step size is the root of C'(alpha) found by bisection to adjacent doubles.

It does not follow the numeric contract (FP32 min-plus distances, lowest-id
tie rule, int64 flows), so near-tied routes can differ from the contract
mode.  It is compared through quantities that do not depend on which of
several equally short routes is taken: the objective of the iterates and the
Frank-Wolfe duality bound.  For plain static assignment (dt = inf) the
Beckmann objective is convex and, for every iterate f with all-or-nothing
direction y, B* >= B(f) - sum_a c_a(f) (f_a - y_a) (the linearisation bound
of a convex function at f, minimised over the feasible set by y).  So every
iterate of every run gives a lower bound on the optimum B*, and its own
objective an upper bound.

Only the test suite may import this module.  It shares no code with the GPU
library.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import dijkstra

RULE_NONE, RULE_CEIL, RULE_FLOOR = 0, 1, 2


def _kappa(dt_s):
    return 3600.0 / dt_s if math.isfinite(dt_s) else 1.0


class PureResult:
    def __init__(self, f, objectives, gaps, lower_bounds, alphas):
        self.f = f                      # veh per link (FP64)
        self.objectives = objectives    # B(f_j), j = 0..J
        self.gaps = gaps                # relative gap at the test of iteration j (1-based)
        self.lower_bounds = lower_bounds  # B(f_j) - sum c(f_j) (f_j - y_j) per iteration
        self.alphas = alphas

    @property
    def lower_bound(self):
        return max(self.lower_bounds) if self.lower_bounds else -math.inf


def _reverse_graph(net, cost):
    """Reverse graph for FP64 Dijkstra towards a destination: entry (head, tail)
    with the cheapest parallel link's cost; also that link's id per pair."""
    n = net.n
    rp = np.asarray(net.row_ptr, np.int64)
    tail = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    head = np.asarray(net.col, np.int64)
    order = np.lexsort((cost, tail, head))       # by head, then tail, then cost
    h, t = head[order], tail[order]
    first = np.ones(order.size, bool)
    first[1:] = (h[1:] != h[:-1]) | (t[1:] != t[:-1])
    keep = order[first]
    G = csr_matrix((cost[keep], (head[keep], tail[keep])), shape=(n, n))
    link_of = {(int(tail[a]), int(head[a])): int(a) for a in keep}
    return G, link_of


def aon(net, cost, orig, dest, trips, dt_s=math.inf, rule=RULE_CEIL):
    """All-or-nothing loading in FP64: every leg follows an FP64 shortest path
    to its destination, with the elapsed time accumulated in FP64 and the
    truncation rule applied to it (CEIL: a link entered before dt is loaded;
    FLOOR: only a link left by dt).  Returns link flows (veh)."""
    cost = np.asarray(cost, np.float64)
    G, link_of = _reverse_graph(net, cost)
    y = np.zeros(net.m, np.float64)
    eff = rule if math.isfinite(dt_s) else RULE_NONE
    orig, dest, trips = np.asarray(orig), np.asarray(dest), np.asarray(trips, np.float64)
    for q in np.unique(dest):
        _, pred = dijkstra(G, directed=True, indices=int(q), return_predecessors=True)
        for k in np.nonzero(dest == q)[0]:
            v, tau = int(orig[k]), 0.0
            while v != q:
                w = int(pred[v])
                if w < 0:
                    raise ValueError("destination unreachable")
                e = link_of[(v, w)]
                if eff == RULE_CEIL and not tau < dt_s:
                    break
                if eff == RULE_FLOOR and tau + cost[e] > dt_s:
                    break
                y[e] += trips[k]
                tau += cost[e]
                v = w
    return y


def bpr(F, c0, cap, alpha_b, beta, kappa):
    return c0 * (1.0 + alpha_b * (kappa * F / cap) ** beta)


def beckmann(F, c0, cap, alpha_b, beta, kappa):
    """Eq. 6 in closed form: sum of int_0^F c0 (1 + alpha_b (kappa s / C)^beta) ds."""
    return float(np.sum(c0 * F * (1.0 + alpha_b * (kappa * F / cap) ** beta / (beta + 1))))


def step_size(F, Y, c0, cap, alpha_b, beta, kappa):
    """alpha* in [0, 1] minimising B(F + alpha (Y - F)): the root of the
    increasing C'(alpha) = sum t c(F + alpha t), by bisection to adjacent doubles."""
    t = Y - F

    def d(a):
        return float(np.sum(t * bpr(F + a * t, c0, cap, alpha_b, beta, kappa)))

    if d(0.0) >= 0.0:
        return 0.0
    if d(1.0) <= 0.0:
        return 1.0
    lo, hi = 0.0, 1.0
    while True:
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            return lo if abs(d(lo)) <= abs(d(hi)) else hi
        if d(mid) < 0.0:
            lo = mid
        else:
            hi = mid


def fw(net, orig, dest, trips, *, alpha_b=0.15, beta=4, dt_s=math.inf, rule=RULE_CEIL, iters=50):
    """Frank-Wolfe (Alg. 6) for `iters` updates from the free-flow AON, all in
    FP64.  Records B(f_j), the gap of each test and the duality lower bound."""
    c0 = np.asarray(net.fftt, np.float64)
    cap = np.asarray(net.cap, np.float64)
    kappa = _kappa(dt_s)
    f = aon(net, c0, orig, dest, trips, dt_s, rule)
    objectives = [beckmann(f, c0, cap, alpha_b, beta, kappa)]
    gaps, lbs, alphas = [], [], []
    for _ in range(iters):
        c = bpr(f, c0, cap, alpha_b, beta, kappa)
        y = aon(net, c, orig, dest, trips, dt_s, rule)
        scf, scy = float(np.sum(c * f)), float(np.sum(c * y))
        gaps.append((scf - scy) / scf)
        lbs.append(objectives[-1] - (scf - scy))
        a = step_size(f, y, c0, cap, alpha_b, beta, kappa)
        alphas.append(a)
        f = f + a * (y - f)
        objectives.append(beckmann(f, c0, cap, alpha_b, beta, kappa))
    return PureResult(f, objectives, gaps, lbs, alphas)
