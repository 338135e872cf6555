"""GPU parity of the alternative shortest-path kernels against the oracle:
the block-local kernel (opts.sssp_kernel = 2; blocks of 64, 128, 128 with two
blocks per wavefront and step, 256 nodes) and the node-per-thread queue
kernel (opts.sssp_kernel = 3; 1 or 2 nodes and 2 or 4 links per thread).
FP32 distances and successor links bit for bit, loading and stop nodes bit
for bit, in every shape, at bucket widths from near-Dijkstra to one bucket,
on tiny graphs with ties, dense in-links and FP32 absorption, the grid, the
metro networks and the 1.0M-link peak interval."""
from __future__ import annotations

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

FX = 1 << 20
SHAPES = [1, 2, 3, 4]
KERNELS = [2, 3]


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


def _trees(q, net, cost, dests, shape, ds=0.0, kernel=2):
    import torch
    with q.Context() as ctx:
        ctx.add(net)
        nq = len(dests)
        dist = torch.empty(nq * net.n, dtype=torch.float32, device="cuda")
        succ = torch.empty(nq * net.n, dtype=torch.int32, device="cuda")
        rc = ctx.trees(q.default_opts(delta_scale=ds, sssp_kernel=kernel, sssp_shape=shape), 0,
                       _dev(cost.astype(np.float32)), _dev(np.asarray(dests, np.int32)), dist, succ)
        return _host(dist).reshape(nq, net.n), _host(succ).reshape(nq, net.n), rc


def _check(orc, net, cost, dests, D, S):
    for k, t in enumerate(dests):
        Do, So, _ = orc.tree(net, cost, int(t))
        assert np.array_equal(D[k].view(np.uint32), Do.view(np.uint32)), t
        assert np.array_equal(S[k], So), t


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("costs", ["float", "int", "huge"])
def test_blk_trees_tiny_all_destinations(q, orc, costs, shape, kernel):
    for seed in range(8):
        rng = np.random.default_rng(500 + seed)
        n = int(rng.integers(3, 12))
        net = synth.tiny_network(n, int(rng.integers(2, 14)), rng, costs=costs)
        D, S, rc = _trees(q, net, net.fftt, list(range(n)), shape, ds=0.7, kernel=kernel)
        _check(orc, net, net.fftt, range(n), D, S)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("shape", SHAPES)
def test_blk_trees_high_in_degree(q, orc, shape, kernel):
    """In-degrees above what a block stages (the rest read in place) and many
    cross-block links per node (mailbox pressure) on a 700-node graph."""
    rng = np.random.default_rng(77)
    net = synth.tiny_network(700, 60_000, rng, costs="float")
    assert np.bincount(net.col, minlength=net.n).max() > 100
    dests = [0, 13, 350, 699]
    D, S, _ = _trees(q, net, net.fftt, dests, shape, ds=0.5, kernel=kernel)
    _check(orc, net, net.fftt, dests, D, S)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("shape", [1, 2])
@pytest.mark.parametrize("ds", [0.05, 1.0, 3.0, 40.0, 1e30])
def test_blk_trees_grid_every_bucket_width(q, orc, ds, shape, kernel):
    w = synth.config1()
    rng = np.random.default_rng(7)
    cost = (w.net.fftt * rng.uniform(1, 4, w.net.m)).astype(np.float32)
    dests = list(range(0, w.net.n, 7))
    D, S, _ = _trees(q, w.net, cost, dests, shape, ds=ds, kernel=kernel)
    _check(orc, w.net, cost, dests, D, S)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("shape", SHAPES)
def test_blk_trees_metro_network_sample(q, orc, shape, kernel):
    w = synth.config2()
    rng = np.random.default_rng(4)
    f = rng.integers(0, 300 * FX, w.net.m).astype(np.int64)
    cost, _ = orc.bpr(f, w.net.fftt, w.net.cap, 0.15, 4, 900.0)
    dests = list(w.extra["zones"][rng.choice(len(w.extra["zones"]), 12, replace=False)])
    D, S, _ = _trees(q, w.net, cost, dests, shape, kernel=kernel)
    _check(orc, w.net, cost, dests, D, S)


def _aon(q, net, cost, orig, dest, trips, dt, rule, shape, kernel=2):
    import torch
    with q.Context() as ctx:
        ctx.add(net)
        ctx.set_demand(0, orig, dest, trips, dt)
        o, d, w = ctx.legs()
        y = torch.empty(net.m, dtype=torch.int64, device="cuda")
        stop = torch.empty(max(len(o), 1), dtype=torch.int32, device="cuda")
        ctx.aon(q.default_opts(trunc_rule=rule, sssp_kernel=kernel, sssp_shape=shape), _dev(cost.astype(np.float32)), y,
                stop)
        return _host(y), _host(stop)[:len(o)]


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("shape", [1, 2, 4])
def test_blk_aon_config2_truncated(q, orc, shape, kernel):
    w = synth.config2()
    rng = np.random.default_rng(8)
    f = rng.integers(0, 400 * FX, w.net.m).astype(np.int64)
    cost, _ = orc.bpr(f, w.net.fftt, w.net.cap, 0.15, 4, 900.0)
    o, d, wfx = orc.demand_legs(w.demand.orig, w.demand.dest, w.demand.trips)
    y, stop = _aon(q, w.net, cost, w.demand.orig, w.demand.dest, w.demand.trips, 900.0, 1, shape, kernel)
    yo, so, _ = orc.aon(w.net, cost, o, d, wfx, 900.0, 1)
    assert np.array_equal(y, yo)
    assert np.array_equal(stop, so)


@pytest.mark.parametrize("kernel", KERNELS)
def test_blk_fw_config1_fixed50(q, orc, kernel):
    import torch
    w = synth.config1()
    opts = q.default_opts(fixed_iters=50, sssp_kernel=kernel, sssp_shape=2)
    with q.Context() as ctx:
        ctx.add(w.net)
        ctx.set_demand(0, w.demand.orig, w.demand.dest, w.demand.trips, w.demand.dt_s)
        st, rc = ctx.solve(opts)
        f = torch.empty(w.net.m, dtype=torch.int64, device="cuda")
        ctx.get_flows(f)
    o, d, wfx = orc.demand_legs(w.demand.orig, w.demand.dest, w.demand.trips)
    ref = orc.fw_solve(w.net, o, d, wfx, fixed_iters=50, keep_history=False)
    assert np.array_equal(_host(f), ref.f)
    assert st[0]["gap"] == ref.gap


@pytest.mark.parametrize("kernel,shape", [(2, 2), (2, 4), (3, 1), (3, 2)])
def test_blk_aon_peak_interval_full_network(q, orc, shape, kernel):
    """The 1.0M-link network under congested costs, the legs of 40 of the
    peak interval's destinations (trees grown over the full network, early
    exit at their origins), loading and stop nodes bit for bit."""
    w = synth.config3()
    rng = np.random.default_rng(12)
    f = rng.integers(0, 120 * FX, w.net.m).astype(np.int64)
    cost, _ = orc.bpr(f, w.net.fftt, w.net.cap, w.alpha, w.beta, 900.0)
    dq = np.unique(w.demand.dest)
    sel = np.isin(w.demand.dest, dq[rng.choice(dq.size, 40, replace=False)])
    o, d, wfx = orc.demand_legs(w.demand.orig[sel], w.demand.dest[sel], w.demand.trips[sel])
    y, stop = _aon(q, w.net, cost, w.demand.orig[sel], w.demand.dest[sel], w.demand.trips[sel], 900.0, 1, shape,
                   kernel)
    yo, so, _ = orc.aon(w.net, cost, o, d, wfx, 900.0, 1)
    assert np.array_equal(y, yo)
    assert np.array_equal(stop, so)
