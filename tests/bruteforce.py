"""Brute-force and closed-form references used to pin the oracle.

These are deliberately different algorithms from the oracle's: exhaustive
simple-path enumeration instead of Dijkstra, per-leg path walks in Python
float32, exact Python integers for sums, quadrature for the objective.
"""
from __future__ import annotations

import numpy as np

f32 = np.float32


def simple_paths_to(net, q, max_paths=200_000):
    """All simple paths (as link lists) from every node to q, by DFS over
    out-links.  Only for tiny graphs."""
    n = net.n
    rp, col = net.row_ptr, net.col
    paths = {v: [] for v in range(n)}
    count = 0
    for s in range(n):
        if s == q:
            continue
        stack = [(s, [], {s})]
        while stack:
            u, links, seen = stack.pop()
            for e in range(rp[u], rp[u + 1]):
                w = int(col[e])
                if w in seen:
                    continue
                nl = links + [e]
                if w == q:
                    paths[s].append(nl)
                    count += 1
                    if count > max_paths:
                        raise RuntimeError("too many paths")
                else:
                    stack.append((w, nl, seen | {w}))
    return paths


def fold_time(links, cost):
    """Right fold from the destination: t = fl32(c_e + t) starting at 0,
    i.e. the FP32 time-to-go of the path's first node."""
    t = f32(0.0)
    for e in reversed(links):
        t = f32(t + f32(cost[e]))
    return t


def bf_distances(net, cost, q):
    paths = simple_paths_to(net, q)
    D = np.full(net.n, np.inf, dtype=np.float32)
    D[q] = 0.0
    for v, ps in paths.items():
        for p in ps:
            t = fold_time(p, cost)
            if t < D[v]:
                D[v] = t
    return D


def rule_successors(net, cost, q, D):
    """Successor links by the tie rule, from given distances: lowest-id
    out-link that is tight and strict; otherwise (FP32 absorption) the
    lowest-id tight link to a node one breadth-first hop closer to q inside
    the tight subgraph."""
    n = net.n
    rp, col = net.row_ptr, net.col
    tails = np.repeat(np.arange(n), np.diff(rp))
    succ = np.full(n, -1, dtype=np.int64)
    tight = np.array([f32(D[col[e]] + f32(cost[e])) == D[tails[e]] for e in range(col.size)])
    for v in range(n):
        if v == q or not np.isfinite(D[v]):
            continue
        for e in range(rp[v], rp[v + 1]):
            if tight[e] and D[col[e]] < D[v]:
                succ[v] = e
                break
    if (succ[[v for v in range(n) if v != q and np.isfinite(D[v])]] >= 0).all():
        return succ, False
    hop = np.full(n, -1)
    hop[q] = 0
    frontier = [q]
    while frontier:
        nxt = []
        for u in frontier:
            for e in np.nonzero((col == u) & tight)[0]:
                v = tails[e]
                if hop[v] < 0:
                    hop[v] = hop[u] + 1
                    nxt.append(v)
        frontier = sorted(set(nxt))
    for v in range(n):
        if v == q or not np.isfinite(D[v]) or succ[v] >= 0:
            continue
        for e in range(rp[v], rp[v + 1]):
            if tight[e] and hop[col[e]] == hop[v] - 1:
                succ[v] = e
                break
    return succ, True


def walk(net, succ, tcost, s0, q, dt, rule):
    """Truncated walk in Python float32.  rule: 'none', 'ceil', 'floor'.
    Returns (loaded links, stop node)."""
    u, tau, out = s0, f32(0.0), []
    dt32 = f32(dt)
    for _ in range(net.n + 1):
        if u == q:
            return out, q
        if rule == "ceil" and tau >= dt32:
            return out, u
        e = int(succ[u])
        nt = f32(tau + f32(tcost[e]))
        if rule == "floor" and nt > dt32:
            return out, u
        out.append(e)
        tau = nt
        u = int(net.col[e])
    raise RuntimeError("successor cycle")


def exact_q_sum(values):
    """Sum of round-half-even(x * 2^16) in exact Python integers (x * 2^16 is
    exact in binary64, and Python's round() on a float is half-even)."""
    return sum(int(round(float(x) * 65536.0)) for x in values)
