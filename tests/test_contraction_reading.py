"""CPU check of the reading behind the chain-contracted shortest-path search.

Leaving out of the search every node that has exactly two neighbours and is
no tree's root, relaxing each run of such nodes as one record whose link
costs are added one at a time in FP32, and labelling the left-out nodes
afterwards with the lesser of the two FP32 folds from the run's ends must
give every node exactly the label of the least fixed point
D(v) = min over out-links (v, w) of fl32(D(w) + c(v, w)), D(root) = 0,
that the oracle's trees compute over the whole network (Alg. 3, the
shortest paths of each destination tree).

The contraction rules, the search over the kept nodes and the fill are a
plain Python restatement written for this check (heap-ordered label
correction, numpy float32 additions); nothing here calls the library.  They
are compared with the oracle bit for bit on hand-made chains (two-way,
one-way, broken in either direction, a loop back to one node, a run longer
than one chain, a ring with no kept node, a pendant node), random sparse
graphs with ties and FP32 absorption, and the 20 x 20 grid.
"""
from __future__ import annotations

import heapq

import numpy as np
import pytest

import synth
from synth.networks import Network, _csr_from_edges

F32 = np.float32
INF = F32(np.inf)
CHAIN_MAX = 8          # most left-out nodes in one chain; longer runs keep a node


def _net(n, edges, rng, costs):
    tail = np.array([e[0] for e in edges], np.int64)
    head = np.array([e[1] for e in edges], np.int64)
    m = tail.size
    if costs == "float":
        c = rng.uniform(1.0, 100.0, m)
    elif costs == "int":
        c = rng.integers(1, 4, m).astype(np.float64)
    else:       # half the links so costly that the others are absorbed
        c = np.where(rng.random(m) < 0.5, rng.uniform(1e8, 4e8, m), rng.uniform(0.5, 8.0, m))
    row_ptr, col, c = _csr_from_edges(n, tail, head, c)
    return Network(n, row_ptr, col, c.astype(np.float32), np.full(m, 1800.0, np.float32))


def _chains(rng, costs):
    """Hubs 0-3 linked both ways, and runs hung between them: 4-6 two-way
    0..1; 7-8 one-way 0->2; 9-12 broken (9-10 both ways, 10->11 and 12->11
    only) 1..3; 13-15 a loop 2..2; 16-35 a two-way run of 20 nodes 3..0;
    36-40 a one-way ring with no hub; 41 a pendant node on 1."""
    edges = []
    for a, b in [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2)]:
        edges += [(a, b), (b, a)]

    def two_way(path):
        for a, b in zip(path, path[1:]):
            edges.extend([(a, b), (b, a)])

    two_way([0, 4, 5, 6, 1])
    edges += [(0, 7), (7, 8), (8, 2)]
    edges += [(1, 9), (9, 1), (9, 10), (10, 9), (10, 11), (12, 11), (3, 12), (12, 3)]
    two_way([2, 13, 14, 15, 2])
    two_way([3] + list(range(16, 36)) + [0])
    edges += [(36, 37), (37, 38), (38, 39), (39, 40), (40, 36)]
    edges += [(1, 41), (41, 1)]
    return _net(42, edges, rng, costs)


def _link(net, x, y):
    """Lowest id of a link x -> y, -1 if there is none."""
    for a in range(net.row_ptr[x], net.row_ptr[x + 1]):
        if net.col[a] == y:
            return a
    return -1


def contract(net, roots):
    """Left-out nodes, chains (u, v, nodes u-side first, link toward v and
    link toward u of each node) and the records of the kept nodes: per head
    a list of (source, links whose costs are added in this order)."""
    n = net.n
    ins = [[] for _ in range(n)]
    for x in range(n):
        for a in range(net.row_ptr[x], net.row_ptr[x + 1]):
            ins[net.col[a]].append(x)
    left = np.zeros(n, bool)
    nbrs = {}
    for x in range(n):
        outs = list(net.col[net.row_ptr[x]:net.row_ptr[x + 1]])
        if x in roots or not (1 <= len(outs) <= 2 and 1 <= len(ins[x]) <= 2):
            continue
        if len(outs) != len(set(outs)) or len(ins[x]) != len(set(ins[x])):
            continue        # parallel links
        around = set(outs) | set(ins[x])
        if x in around or len(around) != 2:
            continue        # a self-loop, or not exactly two neighbours
        left[x] = True
        nbrs[x] = sorted(around)

    def step(x, came_from):
        a, b = nbrs[x]
        return b if a == came_from else a

    seen = np.zeros(n, bool)
    chains = []
    for s in range(n):
        if not left[s] or seen[s]:
            continue
        # walk both ways from s through left-out nodes to the kept ends
        side, prev, cur, ring = [], s, nbrs[s][0], False
        while left[cur]:
            if cur == s:
                ring = True
                break
            side.append(cur)
            prev, cur = cur, step(cur, prev)
        if ring:            # no kept node on the ring: keep all of it
            for x in [s] + side:
                seen[x] = True
                left[x] = False
            continue
        u = cur
        other, prev, cur = [], s, nbrs[s][1]
        while left[cur]:
            other.append(cur)
            prev, cur = cur, step(cur, prev)
        v = cur
        run = side[::-1] + [s] + other
        for x in run:
            seen[x] = True
        a_end, p = u, 0
        while p < len(run):
            q = min(len(run), p + CHAIN_MAX)
            b_end = run[q] if q < len(run) else v
            if q < len(run):
                left[run[q]] = False            # the cut node is kept
            piece = run[p:q]
            toward_v = [_link(net, x, piece[j + 1] if j + 1 < len(piece) else b_end) for j, x in enumerate(piece)]
            toward_u = [_link(net, x, piece[j - 1] if j > 0 else a_end) for j, x in enumerate(piece)]
            chains.append((a_end, b_end, piece, toward_v, toward_u))
            a_end = b_end
            p = q + (1 if q < len(run) else 0)
    records = [[] for _ in range(n)]
    for x in range(n):
        if left[x]:
            continue
        for a in range(net.row_ptr[x], net.row_ptr[x + 1]):
            if not left[net.col[a]]:
                records[net.col[a]].append((x, [a]))
    for u, v, piece, toward_v, toward_u in chains:
        if u == v:
            continue        # a loop back to one node is no shortcut
        k = len(piece)
        into_first, into_last = _link(net, u, piece[0]), _link(net, v, piece[-1])
        if into_first >= 0 and all(a >= 0 for a in toward_v):
            # u -> x1 -> ... -> xk -> v, held at v: costs from v's side first
            records[v].append((u, [toward_v[j] for j in range(k - 1, -1, -1)] + [into_first]))
        if into_last >= 0 and all(a >= 0 for a in toward_u):
            records[u].append((v, list(toward_u) + [into_last]))
    return left, chains, records


def labels(net, cost, root, chains, records):
    """Least fixed point over the kept nodes by heap-ordered label
    correction, then the left-out nodes from their chains' ends."""
    D = np.full(net.n, INF, F32)
    D[root] = F32(0.0)
    heap = [(0.0, root)]
    while heap:
        d, v = heapq.heappop(heap)
        if d > D[v]:
            continue
        for src, links in records[v]:
            cand = D[v]
            for a in links:
                cand = F32(cand + cost[a])
            if cand < D[src]:
                D[src] = cand
                heapq.heappush(heap, (float(cand), src))
    for u, v, piece, toward_v, toward_u in chains:
        k = len(piece)
        from_u, acc = [None] * k, D[u]
        for j in range(k):
            acc = F32(acc + cost[toward_u[j]]) if toward_u[j] >= 0 else INF
            from_u[j] = acc
        acc = D[v]
        for j in range(k - 1, -1, -1):
            acc = F32(acc + cost[toward_v[j]]) if toward_v[j] >= 0 else INF
            D[piece[j]] = min(from_u[j], acc)
    return D


def _check(orc, net, roots):
    left, chains, records = contract(net, set(roots))
    for q in roots:
        D = labels(net, net.fftt, q, chains, records)
        Do, _, _ = orc.tree(net, net.fftt, int(q))
        assert np.array_equal(D.view(np.uint32), Do.view(np.uint32)), (q, np.nonzero(D != Do)[0][:8])
    return int(left.sum()), len(chains)


@pytest.mark.parametrize("costs", ["float", "int", "huge"])
def test_contraction_reading_hand_made_chains(orc, costs):
    for seed in range(4):
        net = _chains(np.random.default_rng(900 + seed), costs)
        for roots in ([0], [2, 3], [5, 30], [8, 11, 14, 38]):
            n_left, n_chains = _check(orc, net, roots)
            assert n_left > 0 and n_chains > 0


@pytest.mark.parametrize("costs", ["float", "int", "huge"])
def test_contraction_reading_sparse_random(orc, costs):
    for seed in range(30):
        rng = np.random.default_rng(700 + seed)
        n = int(rng.integers(6, 60))
        net = synth.tiny_network(n, int(rng.integers(0, n // 2 + 1)), rng, costs=costs)
        roots = sorted(set(rng.integers(0, n, 3).tolist()))
        _check(orc, net, roots)


def test_contraction_reading_grid(orc):
    net = synth.config1().net
    n_left, _ = _check(orc, net, list(range(0, net.n, 37)))
    assert n_left > 0       # the grid's corners have two neighbours


def test_contraction_cuts_long_runs_and_keeps_rings():
    net = _chains(np.random.default_rng(1), "float")
    left, chains, _ = contract(net, {0})
    assert all(len(piece) <= CHAIN_MAX for _, _, piece, _, _ in chains)
    run = [c for c in chains if set(c[2]) <= set(range(16, 36))]
    assert len(run) == 3 and sum(len(c[2]) for c in run) == 18          # 20 nodes, two cut and kept
    assert not left[36:41].any()                                        # the ring with no hub stays whole
    assert not left[[0, 1, 2, 3]].any() and not left[41]                # hubs kept; a pendant has one neighbour


def test_contraction_reading_detects_a_reversed_fold(orc):
    """The check is sensitive to the order of the FP32 additions: the same
    records with each shortcut's costs added from the far end first (a
    plausible slip) disagree with the oracle on some tree."""
    wrong = 0
    for seed in range(4):
        net = _chains(np.random.default_rng(900 + seed), "float")
        _, chains, records = contract(net, {0})
        flipped = [[(src, links[::-1]) for src, links in recs] for recs in records]
        D = labels(net, net.fftt, 0, chains, flipped)
        Do, _, _ = orc.tree(net, net.fftt, 0)
        wrong += int(not np.array_equal(D.view(np.uint32), Do.view(np.uint32)))
    assert wrong > 0
