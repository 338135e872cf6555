"""GPU parity of the link-progress truncation (QDTA_RULE_PROGRESS) against the
oracle: loading, stop nodes and stop delays bit for bit; Frank-Wolfe and the
interval chain with residual legs carrying their delays, bit for bit; the
long-link example of the oracle's pins; checkpoint and resume with delays.
With exact delays (progress_quantum_s = 0) and with delays rounded up to a
quantum (the library's default of 60 s, and others)."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from synth.demand import Demand
from synth.networks import Network

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


@pytest.mark.parametrize("pq", [0.0, 60.0, 7.5])
def test_progress_aon_with_carried_delays(q, orc, pq):
    """Legs carrying delays (set as residual, merged by set_demand) on tiny
    graphs and on the metro network: loading, stop nodes and delays equal the
    oracle's."""
    import torch
    cases = []
    for seed in range(5):
        rng = np.random.default_rng(60 + seed)
        cases.append((synth.tiny_network(9, 14, rng, costs="float"), rng, 60.0))
    w2 = synth.config2()
    cases.append((w2.net, np.random.default_rng(5), 240.0))
    for net, rng, dt in cases:
        P = min(400, net.n * 4)
        o = rng.integers(0, net.n, P).astype(np.int32)
        d = rng.integers(0, net.n, P).astype(np.int32)
        keep = o != d
        o, d = o[keep], d[keep]
        w = rng.integers(1, 50 * FX, o.size).astype(np.int64)
        t = rng.uniform(0, 1.5 * dt, o.size).astype(np.float32)
        t[::4] = 0.0
        o, d, w, t = orc.merge_legs(o, d, w, t)
        cost = (net.fftt * rng.uniform(1, 3, net.m)).astype(np.float32)
        with q.Context() as ctx:
            ctx.add(net)
            ctx.set_residual(0, o, d, w, t)
            ctx.set_demand(0, [], [], [], dt)
            lo, ld, lw, lt = ctx.legs(with_delay=True)
            assert np.array_equal(lo, o) and np.array_equal(lt, t) and np.array_equal(lw, w)
            y = torch.empty(net.m, dtype=torch.int64, device="cuda")
            stop = torch.empty(o.size, dtype=torch.int32, device="cuda")
            sd = torch.empty(o.size, dtype=torch.float32, device="cuda")
            ctx.aon(q.default_opts(trunc_rule=q.RULE_PROGRESS, delta_scale=0.5, progress_quantum_s=pq), _dev(cost),
                    y, stop, sd)
            yo, so, sdo, _ = orc.aon(net, cost, o, d, w, dt, orc.RULE_PROGRESS, delay=t, want_delay=True, pq=pq)
            assert np.array_equal(_host(y), yo)
            assert np.array_equal(_host(stop), so)
            assert np.array_equal(_host(sd).view(np.uint32), sdo.view(np.uint32))
            assert (sdo > 0).any()


def _day(q, torch, net, days, opts):
    out = []
    with q.Context() as ctx:
        ctx.add(net)
        for dem in days:
            ctx.set_demand(0, dem.orig, dem.dest, dem.trips, dem.dt_s)
            if ctx.layout().total_legs == 0:
                out.append(None)
                continue
            st, rc = ctx.solve(opts)
            f = torch.empty(net.m, dtype=torch.int64, device="cuda")
            ctx.get_flows(f)
            ctx.advance_interval(opts)
            ro, rd, rw, rt, done = ctx.residual(0, with_delay=True)
            out.append({"f": _host(f), "res": (ro, rd, rw, rt), "iters": st[0]["iters"], "done": done})
    return out


@pytest.mark.parametrize("pq", [0.0, 60.0])
def test_progress_long_link_by_hand(q, orc, pq):
    """The oracle pin's 12-minute link under 5-minute intervals: the trip is
    carried 420 s, then 120 s short of node 1, and completes in interval 2
    (both delays are whole minutes, so rounding to 60 s keeps them)."""
    import torch
    net = Network(3, np.array([0, 1, 2, 2], np.int32), np.array([1, 2], np.int32),
                  np.array([720.0, 60.0], np.float32), np.array([1e6, 1e6], np.float32))
    one = Demand(np.array([0], np.int32), np.array([2], np.int32), np.array([1.0]), 300.0)
    empty = Demand(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0), 300.0)
    opts = q.default_opts(alpha=0.0, trunc_rule=q.RULE_PROGRESS, keep_history=1, progress_quantum_s=pq)
    g = _day(q, torch, net, [one, empty, empty, empty], opts)
    assert g[0]["f"].tolist() == [FX, 0] and g[0]["res"][3].tolist() == [420.0]
    assert g[1]["f"].tolist() == [0, 0] and g[1]["res"][3].tolist() == [120.0]
    assert g[2]["f"].tolist() == [0, FX] and g[2]["res"][0].size == 0
    ref, _ = orc.qdta_day(net, [one, empty, empty, empty], alpha_b=0.0, rule=orc.RULE_PROGRESS, pq=pq)
    for a, b in zip(g, ref):
        if a is None:
            continue
        assert np.array_equal(a["f"], b["f"])
        for x, y in zip(a["res"], b["res"]):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("scale,pq", [("grid", 0.0), ("grid", 30.0), ("metro", 0.0), ("metro", 60.0)])
def test_progress_day_chain(q, orc, scale, pq):
    """A chain of short intervals (90 s on the grid; 120 s on the 1/20-scale
    metro network's morning): flows, iterations and the residual legs with
    their delays equal the oracle's, interval by interval."""
    import torch
    if scale == "grid":
        w = synth.config1()
        rng = np.random.default_rng(9)
        days = []
        for i in range(4):
            sel = rng.random(w.demand.P) < 0.3
            days.append(Demand(w.demand.orig[sel], w.demand.dest[sel], w.demand.trips[sel] / 4, 90.0))
        net = w.net
    else:
        w = synth.config3_day(0.05)
        net = w.net
        days = [Demand(x.orig, x.dest, x.trips, 120.0) for x in w.demand[30:33]]
    opts = q.default_opts(keep_history=1, tol=1e-3, max_iter=30, trunc_rule=q.RULE_PROGRESS, progress_quantum_s=pq)
    g = _day(q, torch, net, days, opts)
    ref, _ = orc.qdta_day(net, days, tol=1e-3, max_iter=30, rule=orc.RULE_PROGRESS, pq=pq)
    carried = 0
    for a, b in zip(g, ref):
        assert a["iters"] == b["iters"]
        assert np.array_equal(a["f"], b["f"])
        for x, y in zip(a["res"], b["res"]):
            assert np.array_equal(x, y)
        assert a["done"] == b["done_fx"]
        carried += int((a["res"][3] > 0).sum())
    assert carried > 0


def test_progress_resume_with_delays(q, orc):
    """Checkpoint and resume carry the delays: a chain cut after interval 1
    and resumed through set_residual equals the uninterrupted chain."""
    import torch
    w = synth.config1()
    rng = np.random.default_rng(17)
    days = []
    for i in range(3):
        sel = rng.random(w.demand.P) < 0.4
        days.append(Demand(w.demand.orig[sel], w.demand.dest[sel], w.demand.trips[sel] / 3, 100.0))
    opts = q.default_opts(keep_history=1, tol=1e-3, max_iter=20, trunc_rule=q.RULE_PROGRESS)
    whole = _day(q, torch, w.net, days, opts)
    head = _day(q, torch, w.net, days[:2], opts)
    with q.Context() as ctx:
        ctx.add(w.net)
        ctx.set_residual(0, *head[-1]["res"])
        dem = days[2]
        ctx.set_demand(0, dem.orig, dem.dest, dem.trips, dem.dt_s)
        st, rc = ctx.solve(opts)
        f = torch.empty(w.net.m, dtype=torch.int64, device="cuda")
        ctx.get_flows(f)
        assert np.array_equal(_host(f), whole[2]["f"])
    assert (head[-1]["res"][3] > 0).any()
