"""GPU parity of the plain-interval loading by merged paths (opts.load_form
= 2): link flows and stop nodes equal the oracle's walk-per-leg loading bit
for bit -- on the grid, with FP32 absorption (trees the sweep hands to the
walk and the tie fallback), over 50 Frank-Wolfe iterations, for uneven
instances loaded together, and for all 64 grids of the batched workload;
repeated launches leave the scratch clean."""
from __future__ import annotations

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

FX = 1 << 20


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


def _aon(q, net, cost, orig, dest, trips, repeat=1):
    import torch
    with q.Context() as ctx:
        ctx.add(net)
        ctx.set_demand(0, orig, dest, trips, float("inf"))
        o, d, w = ctx.legs()
        y = torch.empty(net.m, dtype=torch.int64, device="cuda")
        stop = torch.empty(max(len(o), 1), dtype=torch.int32, device="cuda")
        out = []
        for _ in range(repeat):
            rc = ctx.aon(q.default_opts(load_form=2, delta_scale=0.5), _dev(cost.astype(np.float32)), y, stop)
            out.append((_host(y).copy(), _host(stop)[:len(o)].copy(), rc))
        return out


def test_sweep_grid_plain(q, orc):
    w = synth.config1()
    o, d, wfx = orc.demand_legs(w.demand.orig, w.demand.dest, w.demand.trips)
    rng = np.random.default_rng(2)
    cost = (w.net.fftt * rng.uniform(1, 5, w.net.m)).astype(np.float32)
    res = _aon(q, w.net, cost, w.demand.orig, w.demand.dest, w.demand.trips, repeat=3)
    yo, so, _ = orc.aon(w.net, cost, o, d, wfx, float("inf"), orc.RULE_NONE)
    for y, stop, _ in res:
        assert np.array_equal(y, yo) and np.array_equal(stop, so)


def test_sweep_with_absorption(q, orc):
    hits = 0
    for seed in range(30):
        rng = np.random.default_rng(seed)
        net = synth.tiny_network(8, 10, rng, costs="huge")
        orig = rng.integers(0, 8, 30)
        dest = rng.integers(0, 8, 30)
        trips = rng.uniform(1, 10, 30)
        o, d, wfx = orc.demand_legs(orig, dest, trips)
        res = _aon(q, net, net.fftt, orig, dest, trips, repeat=2)
        yo, so, rco = orc.aon(net, net.fftt, o, d, wfx, float("inf"), orc.RULE_NONE)
        for y, stop, rc in res:
            assert np.array_equal(y, yo) and np.array_equal(stop, so), seed
        hits += res[0][2] == q.WABSORB
    assert hits > 0


def test_sweep_fw_config1_fixed50(q, orc):
    import torch
    w = synth.config1()
    with q.Context() as ctx:
        ctx.add(w.net)
        ctx.set_demand(0, w.demand.orig, w.demand.dest, w.demand.trips, w.demand.dt_s)
        st, _ = ctx.solve(q.default_opts(fixed_iters=50, load_form=2))
        f = torch.empty(w.net.m, dtype=torch.int64, device="cuda")
        ctx.get_flows(f)
    o, d, wfx = orc.demand_legs(w.demand.orig, w.demand.dest, w.demand.trips)
    ref = orc.fw_solve(w.net, o, d, wfx, fixed_iters=50, keep_history=False)
    assert np.array_equal(_host(f), ref.f) and st[0]["gap"] == ref.gap


@pytest.mark.parametrize("full", [False, True])
def test_sweep_batched_grids(q, orc, full):
    """Uneven grids in one context (all 64 of the batched workload when
    `full`; three of them checked against the oracle), two iterations."""
    import torch
    insts = synth.config4() if full else synth.config4(count=6, k_lo=20, k_hi=60, z_lo=20, z_hi=80)
    with q.Context() as ctx:
        for x in insts:
            i = ctx.add(x.net)
            ctx.set_demand(i, x.demand.orig, x.demand.dest, x.demand.trips, x.demand.dt_s)
        st, _ = ctx.solve(q.default_opts(fixed_iters=2, load_form=2))
        li = ctx.layout()
        f = torch.empty(li.total_links, dtype=torch.int64, device="cuda")
        ctx.get_flows(f)
        off = ctx.offsets()
    fh = _host(f)
    pick = [int(np.argmax([x.net.m for x in insts])), 3, len(insts) - 1] if full else range(len(insts))
    for i in pick:
        x = insts[i]
        o, d, wfx = orc.demand_legs(x.demand.orig, x.demand.dest, x.demand.trips)
        ref = orc.fw_solve(x.net, o, d, wfx, fixed_iters=2, keep_history=False)
        assert np.array_equal(fh[off["link"][i]:off["link"][i + 1]], ref.f), i
        assert st[i]["gap"] == ref.gap
