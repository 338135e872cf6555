"""GPU parity of the chain-contracted shortest-path search (opts.sssp_kernel =
4) against the oracle.  The search leaves out nodes with two neighbours that
are no tree's root and fills their labels from the chain ends afterwards, so
everything the oracle computes over the whole network -- FP32 distances and
successor links of every node, loads, stop nodes, flows -- must come out bit
for bit: on hand-made chains (two-way, one-way, broken in either direction,
loops back to one node, runs longer than one chain, rings with no kept
node), a hub whose record row is too long to pack into its queue entries
and whose pop queues more near entries than the LDS buffer holds, random
sparse graphs with ties and FP32 absorption, the grid, the metro networks
and the 1.0M-link peak interval; with legs starting on left-out nodes; and
after the destinations change."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from synth.networks import Network, _csr_from_edges

pytestmark = pytest.mark.gpu

FX = 1 << 20
KERNEL = 4


@pytest.fixture(scope="module")
def q():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    from paper_2104_12911_amd import qdta
    qdta.lib()
    return qdta


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _net(n, edges, rng, costs="float"):
    tail = np.array([e[0] for e in edges], np.int64)
    head = np.array([e[1] for e in edges], np.int64)
    m = tail.size
    if costs == "float":
        c = rng.uniform(1.0, 100.0, m)
    elif costs == "int":
        c = rng.integers(1, 4, m).astype(np.float64)
    else:
        c = np.where(rng.random(m) < 0.5, rng.uniform(1e8, 4e8, m), rng.uniform(0.5, 8.0, m))
    row_ptr, col, c = _csr_from_edges(n, tail, head, c)
    return Network(n, row_ptr, col, c.astype(np.float32), np.full(m, 1800.0, np.float32))


def _chains_net(rng, costs="float"):
    """Hubs 0-3 linked both ways, and chains hung between them:
    4-6 two-way 0..1; 7-8 one-way 0->2; 9-12 mixed (9-10 both ways,
    10->11 only, 12->11 only) 1..3; 13-15 a loop 2..2; 16-35 a two-way run
    of 20 nodes 3..0 (cut into chains of at most 8); 36-40 a one-way ring
    with no hub; 41 a pendant node on 1."""
    E = []
    hubs = [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2)]
    for a, b in hubs:
        E += [(a, b), (b, a)]

    def two_way(path):
        for a, b in zip(path, path[1:]):
            E.extend([(a, b), (b, a)])

    two_way([0, 4, 5, 6, 1])
    E += [(0, 7), (7, 8), (8, 2)]
    E += [(1, 9), (9, 1), (9, 10), (10, 9), (10, 11), (12, 11), (3, 12), (12, 3)]
    two_way([2, 13, 14, 15, 2])
    two_way([3] + list(range(16, 36)) + [0])
    E += [(36, 37), (37, 38), (38, 39), (39, 40), (40, 36)]
    E += [(1, 41), (41, 1)]
    return _net(42, E, rng, costs)


def _trees(q, net, cost, dests, ds=0.0, kernel=KERNEL):
    import torch
    with q.Context() as ctx:
        ctx.add(net)
        nq = len(dests)
        dist = torch.empty(nq * net.n, dtype=torch.float32, device="cuda")
        succ = torch.empty(nq * net.n, dtype=torch.int32, device="cuda")
        rc = ctx.trees(q.default_opts(delta_scale=ds, sssp_kernel=kernel), 0, _dev(cost.astype(np.float32)),
                       _dev(np.asarray(dests, np.int32)), dist, succ)
        return _host(dist).reshape(nq, net.n), _host(succ).reshape(nq, net.n), rc


def _check(orc, net, cost, dests, D, S):
    for k, t in enumerate(dests):
        Do, So, _ = orc.tree(net, cost, int(t))
        assert np.array_equal(D[k].view(np.uint32), Do.view(np.uint32)), t
        assert np.array_equal(S[k], So), t


@pytest.mark.parametrize("costs", ["float", "int", "huge"])
@pytest.mark.parametrize("ds", [0.3, 3.0, 1e30])
def test_contract_trees_hand_made_chains(q, orc, costs, ds):
    for seed in range(4):
        rng = np.random.default_rng(900 + seed)
        net = _chains_net(rng, costs)
        for dests in ([0], [2, 3], [5, 30], [8, 11, 14, 38]):
            D, S, _ = _trees(q, net, net.fftt, dests, ds=ds)
            _check(orc, net, net.fftt, dests, D, S)


@pytest.mark.parametrize("costs", ["float", "int", "huge"])
def test_contract_trees_sparse_random(q, orc, costs):
    """A random Hamiltonian cycle plus a few links: most nodes have two
    neighbours; a handful of destinations."""
    for seed in range(10):
        rng = np.random.default_rng(700 + seed)
        n = int(rng.integers(6, 60))
        net = synth.tiny_network(n, int(rng.integers(0, n // 2 + 1)), rng, costs=costs)
        dests = sorted(set(rng.integers(0, n, 3).tolist()))
        D, S, _ = _trees(q, net, net.fftt, dests, ds=0.7)
        _check(orc, net, net.fftt, dests, D, S)


def _hub_net(rng, k, costs):
    """Hub 0 linked both ways to spokes 1..k, the spokes in a two-way ring
    (three neighbours each, so all are kept), and every seventh spoke with a
    two-way run of three two-neighbour nodes to the next spoke: the hub's
    row holds k records (too many to pack, so its pops read the row
    pointers), and popping it queues k spokes in one step (more than the
    LDS buffer of near entries holds when the bucket takes them all)."""
    edges = []
    for i in range(1, k + 1):
        edges += [(0, i), (i, 0)]
        j = i % k + 1
        edges += [(i, j), (j, i)]
    n = k + 1
    for i in range(1, k + 1, 7):
        a, b, c = n, n + 1, n + 2
        n += 3
        j = i % k + 1
        edges += [(i, a), (a, i), (a, b), (b, a), (b, c), (c, b), (c, j), (j, c)]
    return _net(n, edges, rng, costs)


@pytest.mark.parametrize("costs", ["float", "int"])
@pytest.mark.parametrize("ds", [0.3, 1e30])
def test_contract_trees_hub_unpacked_row_and_buffer_overflow(q, orc, costs, ds):
    rng = np.random.default_rng(4242)
    k = 700
    net = _hub_net(rng, k, costs)
    dests = [5, 0, 350, k + 2]          # spokes, the hub, a run node (kept as a root)
    D, S, _ = _trees(q, net, net.fftt, dests, ds=ds)
    _check(orc, net, net.fftt, dests, D, S)


@pytest.mark.parametrize("ds", [0.05, 1.0, 40.0])
def test_contract_trees_grid_and_metro(q, orc, ds):
    w = synth.config1()
    rng = np.random.default_rng(7)
    cost = (w.net.fftt * rng.uniform(1, 4, w.net.m)).astype(np.float32)
    dests = list(range(0, w.net.n, 37))
    D, S, _ = _trees(q, w.net, cost, dests, ds=ds)
    _check(orc, w.net, cost, dests, D, S)
    w2 = synth.config2()
    f = rng.integers(0, 300 * FX, w2.net.m).astype(np.int64)
    cost2, _ = orc.bpr(f, w2.net.fftt, w2.net.cap, 0.15, 4, 900.0)
    dests2 = list(w2.extra["zones"][rng.choice(len(w2.extra["zones"]), 6, replace=False)])
    D, S, _ = _trees(q, w2.net, cost2, dests2, ds=ds)
    _check(orc, w2.net, cost2, dests2, D, S)


def _aon(q, net, cost, orig, dest, trips, dt, rule, res=None, kernel=KERNEL):
    import torch
    with q.Context() as ctx:
        ctx.add(net)
        if res is not None:
            ctx.set_residual(0, *res)
        ctx.set_demand(0, orig, dest, trips, dt)
        o, d, w = ctx.legs()
        y = torch.empty(net.m, dtype=torch.int64, device="cuda")
        stop = torch.empty(max(len(o), 1), dtype=torch.int32, device="cuda")
        ctx.aon(q.default_opts(trunc_rule=rule, sssp_kernel=kernel), _dev(cost.astype(np.float32)), y, stop)
        return (o, d, w), _host(y), _host(stop)[:len(o)]


@pytest.mark.parametrize("rule", [0, 1, 2])
def test_contract_aon_legs_from_left_out_nodes(q, orc, rule):
    """Legs whose origins are chain nodes (left out of the search; the tree
    stops only once both ends that can reach them are final): loads and stop
    nodes against the oracle, truncated and not."""
    for seed in range(4):
        rng = np.random.default_rng(950 + seed)
        net = _chains_net(rng)
        # every node that reaches the hubs: not the ring, not node 11 (links in only)
        nodes = np.array([v for v in range(net.n) if not 36 <= v <= 40 and v != 11])
        dests = np.array([0, 3], np.int32)
        orig = rng.choice(nodes, 40)
        dest = rng.choice(dests, 40)
        keep = orig != dest
        orig, dest = orig[keep].astype(np.int32), dest[keep]
        trips = rng.uniform(0.5, 3.0, orig.size)
        dt = 150.0 if rule else float("inf")
        (o, d, wfx), y, stop = _aon(q, net, net.fftt, orig, dest, trips, dt, rule)
        yo, so, _ = orc.aon(net, net.fftt, o, d, wfx, dt, rule)
        assert np.array_equal(y, yo) and np.array_equal(stop, so), seed


def test_contract_aon_residual_legs_metro(q, orc):
    """Config 2, congested, 900 s: the interval's legs plus residual legs
    starting at random nodes (many of them left out of the search)."""
    w = synth.config2()
    rng = np.random.default_rng(8)
    f = rng.integers(0, 400 * FX, w.net.m).astype(np.int64)
    cost, _ = orc.bpr(f, w.net.fftt, w.net.cap, 0.15, 4, 900.0)
    dq = np.unique(w.demand.dest)
    ro = rng.integers(0, w.net.n, 20_000).astype(np.int32)
    rd = rng.choice(dq, 20_000).astype(np.int32)
    keep = ro != rd
    ro, rd = ro[keep], rd[keep]
    rw = rng.integers(1, 4 * FX, ro.size).astype(np.int64)
    ro, rd, rw = orc.merge_legs(ro, rd, rw)
    (o, d, wfx), y, stop = _aon(q, w.net, cost, w.demand.orig, w.demand.dest, w.demand.trips, 900.0, 1,
                                res=(ro, rd, rw))
    yo, so, _ = orc.aon(w.net, cost, o, d, wfx, 900.0, 1)
    assert np.array_equal(y, yo)
    assert np.array_equal(stop, so)


def test_contract_fw_config1_and_config2(q, orc):
    import torch
    for w, opts_kw, it in ((synth.config1(), {}, 30), (synth.config2(), {}, 3)):
        opts = q.default_opts(fixed_iters=it, sssp_kernel=KERNEL, **opts_kw)
        with q.Context() as ctx:
            ctx.add(w.net)
            ctx.set_demand(0, w.demand.orig, w.demand.dest, w.demand.trips, w.demand.dt_s)
            st, rc = ctx.solve(opts)
            f = torch.empty(w.net.m, dtype=torch.int64, device="cuda")
            ctx.get_flows(f)
        o, d, wfx = orc.demand_legs(w.demand.orig, w.demand.dest, w.demand.trips)
        ref = orc.fw_solve(w.net, o, d, wfx, fixed_iters=it, keep_history=False, dt_s=w.demand.dt_s)
        assert np.array_equal(_host(f), ref.f)
        assert st[0]["gap"] == ref.gap


def test_contract_destinations_change(q, orc):
    """One context, three intervals whose destinations differ (the later ones
    are nodes the first interval's search left out): flows of each interval
    against the oracle."""
    import torch
    rng = np.random.default_rng(31)
    net = _chains_net(rng)
    nodes = np.array([v for v in range(net.n) if not 36 <= v <= 40 and v != 11])
    with q.Context() as ctx:
        ctx.add(net)
        for dests in ([0, 1], [5, 20, 1], [9, 14, 27, 8]):
            orig = rng.choice(nodes, 30).astype(np.int32)
            dest = rng.choice(np.asarray(dests, np.int32), 30)
            keep = orig != dest
            orig, dest = orig[keep], dest[keep]
            trips = rng.uniform(0.5, 3.0, orig.size)
            ctx.set_demand(0, orig, dest, trips, float("inf"))
            o, d, wfx = ctx.legs()
            y = torch.empty(net.m, dtype=torch.int64, device="cuda")
            ctx.aon(q.default_opts(sssp_kernel=KERNEL), _dev(net.fftt), y)
            yo, _, _ = orc.aon(net, net.fftt, o, d, wfx, float("inf"), 0)
            assert np.array_equal(_host(y), yo), dests


def test_contract_peak_interval_full_network(q, orc):
    """The 1.0M-link network under congested costs, the legs of 40 of the
    peak interval's destinations: loading and stop nodes bit for bit."""
    w = synth.config3()
    rng = np.random.default_rng(12)
    f = rng.integers(0, 120 * FX, w.net.m).astype(np.int64)
    cost, _ = orc.bpr(f, w.net.fftt, w.net.cap, w.alpha, w.beta, 900.0)
    dq = np.unique(w.demand.dest)
    sel = np.isin(w.demand.dest, dq[rng.choice(dq.size, 40, replace=False)])
    o, d, wfx = orc.demand_legs(w.demand.orig[sel], w.demand.dest[sel], w.demand.trips[sel])
    _, y, stop = _aon(q, w.net, cost, w.demand.orig[sel], w.demand.dest[sel], w.demand.trips[sel], 900.0, 1)
    yo, so, _ = orc.aon(w.net, cost, o, d, wfx, 900.0, 1)
    assert np.array_equal(y, yo)
    assert np.array_equal(stop, so)
