"""GPU tests of the caller-owned workspace (qdta_workspace_query /
qdta_bind_workspace): with a workspace bound the library makes no hipMalloc
call, gives the same bits as with its own allocations, and refuses a
workspace that is too small or bound too late."""
from __future__ import annotations

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

FX = 1 << 20


@pytest.fixture(scope="module")
def q():
    from paper_2104_12911_amd import qdta
    qdta.lib()
    return qdta


def _run(torch, q, net, days, opts, ws_bytes=None, max_legs=0, max_dests=0):
    """Solve and advance each interval; returns flows and residuals per
    interval, and (hipMalloc calls, workspace bytes) of the context."""
    out = []
    with q.Context() as ctx:
        ctx.add(net)
        ctx.set_demand(0, days[0].orig, days[0].dest, days[0].trips, days[0].dt_s)
        if ws_bytes is not None:
            need = ctx.workspace_query(opts, max_legs, max_dests)
            ws = torch.empty(need + ws_bytes, dtype=torch.uint8, device="cuda")
            ctx.bind_workspace(ws)
        for i, dem in enumerate(days):
            if i:
                ctx.set_demand(0, dem.orig, dem.dest, dem.trips, dem.dt_s)
            st, rc = ctx.solve(opts)
            f = torch.empty(net.m, dtype=torch.int64, device="cuda")
            ctx.get_flows(f)
            ctx.advance_interval(opts)
            ro, rd, rw, done = ctx.residual(0)
            torch.cuda.synchronize()
            out.append((f.cpu().numpy(), ro, rd, rw, st[0]["iters"], st[0]["gap"]))
        counts = ctx.alloc_count()
    return out, counts


def test_workspace_day_no_allocation_same_bits(q):
    """Four morning intervals of the 1/20-scale metro day, solved and carried
    over with the residual step: once bound, the context makes no hipMalloc
    call, and flows, residual legs, iterations and gaps equal those of a
    context that allocates its own memory."""
    import torch
    w = synth.config3_day(0.05)
    days = w.demand[30:34]
    opts = q.default_opts(tol=1e-4, max_iter=30, keep_history=1, history_mib=64)
    ref, (nm_ref, _) = _run(torch, q, w.net, days, opts)
    assert nm_ref > 0
    # maxima: the largest interval's legs (original + residual) and all zones
    max_legs = 4 * max(int(d.P) for d in days) + 200_000
    dests = len(np.unique(np.concatenate([d.dest for d in days])))
    got, (nm, used) = _run(torch, q, w.net, days, opts, ws_bytes=0, max_legs=max_legs, max_dests=dests)
    assert nm == 0 and used > 0
    for a, b in zip(got, ref):
        assert np.array_equal(a[0], b[0])
        for x, y in zip(a[1:4], b[1:4]):
            assert np.array_equal(x, y)
        assert a[4] == b[4] and a[5] == b[5]


def test_workspace_config2_interval_and_too_small(q):
    """Config 2 (255,754 links, 1,000 destinations): a workspace of exactly
    the queried size solves and advances the interval with no hipMalloc and
    the same bits; one 1 MiB short is refused with QDTA_ENOMEM."""
    import torch
    w = synth.config2()
    opts = q.default_opts(fixed_iters=3, keep_history=1, history_mib=-1)
    ref, _ = _run(torch, q, w.net, [w.demand], opts)
    # residual legs: at most one per (iterate, leg) before merging, 4 iterates here
    got, (nm, used) = _run(torch, q, w.net, [w.demand], opts, ws_bytes=0, max_legs=4 * w.demand.P)
    assert nm == 0
    assert np.array_equal(got[0][0], ref[0][0])
    for x, y in zip(got[0][1:4], ref[0][1:4]):
        assert np.array_equal(x, y)
    with q.Context() as ctx:
        ctx.add(w.net)
        ctx.set_demand(0, w.demand.orig, w.demand.dest, w.demand.trips, w.demand.dt_s)
        need = ctx.workspace_query(opts, 4 * w.demand.P)
        ws = torch.empty(need - (1 << 20), dtype=torch.uint8, device="cuda")
        ctx.bind_workspace(ws)
        with pytest.raises(q.QdtaError) as e:
            ctx.solve(opts)
            ctx.advance_interval(opts)
        assert e.value.code == q.ENOMEM
        assert ctx.alloc_count()[0] == 0


def test_workspace_bind_rules(q):
    import torch
    w = synth.config1()
    with q.Context() as ctx:
        ctx.add(w.net)
        ctx.set_demand(0, w.demand.orig, w.demand.dest, w.demand.trips, w.demand.dt_s)
        ctx.layout()                                  # lays the network out in device memory
        ws = torch.empty(1 << 24, dtype=torch.uint8, device="cuda")
        with pytest.raises(q.QdtaError) as e:
            ctx.bind_workspace(ws)
        assert e.value.code == q.ESTATE
    with q.Context() as ctx:
        ctx.add(w.net)
        ctx.set_demand(0, w.demand.orig, w.demand.dest, w.demand.trips, w.demand.dt_s)
        ws = torch.empty(1 << 24, dtype=torch.uint8, device="cuda")
        import ctypes
        assert q.lib().qdta_bind_workspace(ctx._h, ctypes.c_void_p(ws.data_ptr() + 4), 1 << 20) == q.EARG
        ctx.bind_workspace(ws)
        with pytest.raises(q.QdtaError) as e:               # twice
            ctx.bind_workspace(ws)
        assert e.value.code == q.ESTATE
        st, rc = ctx.solve(q.default_opts(fixed_iters=5))
        assert st[0]["iters"] == 5 and ctx.alloc_count()[0] == 0
