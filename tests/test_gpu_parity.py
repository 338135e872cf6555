"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on
the same seeded inputs.  Integer results (fixed-point flows, successor links,
stop nodes, exact int128 sums) and the FP32 distances must be bit-exact; the
step sizes and relative gaps too, since they are computed from exact sums by
the same IEEE operations.  Objectives are compared to 1e-12 relative."""
from __future__ import annotations

import math

import numpy as np
import pytest

import synth
from synth.networks import Network

pytestmark = pytest.mark.gpu

FX = 1 << 20


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    return torch


@pytest.fixture(scope="module")
def q():
    from paper_2104_12911_amd import qdta
    qdta.lib()
    return qdta


def dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def fx_of(trips):
    return np.array([int(np.rint(t * FX)) for t in np.asarray(trips, np.float64)], np.int64)


def i128(lo, hi):
    return (int(hi) << 64) | (int(lo) & ((1 << 64) - 1))


def orc_legs(orc, ctx, dems):
    """The oracle's own quantisation and merge of each instance's demand;
    asserts that the library holds exactly these legs, and returns the
    oracle's copy (concatenated over instances) for the oracle to use."""
    parts = [orc.demand_legs(dm.orig, dm.dest, dm.trips) for dm in dems]
    o = np.concatenate([p[0] for p in parts]) if parts else np.zeros(0, np.int32)
    d = np.concatenate([p[1] for p in parts]) if parts else np.zeros(0, np.int32)
    w = np.concatenate([p[2] for p in parts]) if parts else np.zeros(0, np.int64)
    lo, ld, lw = ctx.legs()
    assert np.array_equal(lo, o) and np.array_equal(ld, d) and np.array_equal(lw, w)
    return o, d, w


class _Dem:
    def __init__(self, orig, dest, trips):
        self.orig, self.dest, self.trips = np.asarray(orig), np.asarray(dest), np.asarray(trips, np.float64)


def fp64_check(st, ref):
    """The reported gap and objective against the oracle's FP64 reference of
    the same iterate (long double, no FP32 costs, no quantised terms): within
    1e-6 (the gap in absolute terms, being relative already; the objective
    relatively)."""
    dg = abs(st["gap"] - ref.gap_fp64)
    do = abs(st["objective"] - ref.objective_fp64) / abs(ref.objective_fp64)
    assert dg <= 1e-6 and do <= 1e-6, (dg, do)
    return dg, do


# ---------------------------------------------------------------------------
# A1 -- BPR
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dt", [float("inf"), 900.0, 300.0])
def test_bpr_bit_exact(torch_dev, q, orc, dt):
    torch = torch_dev
    w = synth.config2()
    net = w.net
    rng = np.random.default_rng(1)
    f = rng.integers(0, 5000 * FX, net.m).astype(np.int64)
    f[::11] = 0
    ref, _ = orc.bpr(f, net.fftt, net.cap, 0.15, 4, dt)
    with q.Context() as ctx:
        ctx.add(net)
        ctx.set_demand(0, [], [], [], dt)
        c = torch.empty(net.m, dtype=torch.float32, device="cuda")
        ctx.bpr(q.default_opts(), dev(torch, f), c)
        assert np.array_equal(host(c).view(np.uint32), ref.view(np.uint32))


def test_bpr_worked_example(torch_dev, q, orc):
    torch = torch_dev
    w = synth.paper_example()
    f = np.array([int(43.75 * FX), int(43.75 * FX), int(56.25 * FX), int(12.5 * FX)], np.int64)
    ref, _ = orc.bpr(f, w.net.fftt, w.net.cap, 0.15, 4, 900.0)
    with q.Context() as ctx:
        ctx.add(w.net)
        ctx.set_demand(0, [], [], [], 900.0)
        c = torch.empty(4, dtype=torch.float32, device="cuda")
        ctx.bpr(q.default_opts(), dev(torch, f), c)
        got = host(c)
    assert np.array_equal(got, ref)
    assert abs(got[2] / 60 - 12.4) < 0.05 and 6.3 <= got[1] / 60 < 6.4


# ---------------------------------------------------------------------------
# A2 -- trees
# ---------------------------------------------------------------------------
def _trees(torch, q, net, cost, dests, ds=0.0, waves=1):
    with q.Context() as ctx:
        ctx.add(net)
        nq = len(dests)
        dist = torch.empty(nq * net.n, dtype=torch.float32, device="cuda")
        succ = torch.empty(nq * net.n, dtype=torch.int32, device="cuda")
        rc = ctx.trees(q.default_opts(delta_scale=ds, tree_waves=waves), 0, dev(torch, cost.astype(np.float32)),
                       dev(torch, np.asarray(dests, np.int32)), dist, succ)
        return host(dist).reshape(nq, net.n), host(succ).reshape(nq, net.n), rc


@pytest.mark.parametrize("costs", ["float", "int", "huge"])
def test_trees_tiny_all_destinations(torch_dev, q, orc, costs):
    for seed in range(8):
        rng = np.random.default_rng(500 + seed)
        n = int(rng.integers(3, 12))
        net = synth.tiny_network(n, int(rng.integers(2, 14)), rng, costs=costs)
        D, S, rc = _trees(torch_dev, q, net, net.fftt, list(range(n)), ds=0.7)
        absorbed = False
        for t in range(n):
            Do, So, rco = orc.tree(net, net.fftt, t)
            assert np.array_equal(D[t].view(np.uint32), Do.view(np.uint32)), (costs, seed, t)
            assert np.array_equal(S[t], So), (costs, seed, t)
            absorbed |= rco == orc.WARN_ABSORB
        assert (rc == q.WABSORB) == absorbed


@pytest.mark.parametrize("waves", [1, 4])
@pytest.mark.parametrize("costs", ["float", "int"])
def test_trees_high_in_degree(torch_dev, q, orc, costs, waves):
    """Dense tiny graphs (in-degrees up to about 15, parallel links) put most
    in-links in the overflow run of the node records."""
    for seed in range(4):
        rng = np.random.default_rng(900 + seed)
        net = synth.tiny_network(12, 90, rng, costs=costs)
        indeg = np.bincount(net.col, minlength=net.n)
        assert indeg.max() > 8
        D, S, rc = _trees(torch_dev, q, net, net.fftt, list(range(net.n)), ds=0.5, waves=waves)
        for t in range(net.n):
            Do, So, _ = orc.tree(net, net.fftt, t)
            assert np.array_equal(D[t].view(np.uint32), Do.view(np.uint32)), (costs, seed, t)
            assert np.array_equal(S[t], So), (costs, seed, t)


@pytest.mark.parametrize("waves", [1, 4])
@pytest.mark.parametrize("ds", [0.05, 1.0, 3.0, 40.0, 1e30])
def test_trees_grid_every_bucket_width(torch_dev, q, orc, ds, waves):
    """Any bucket width gives the same least fixed point: tiny buckets (near
    Dijkstra), the default, and one bucket (Bellman-Ford); one wavefront or
    one workgroup per tree."""
    w = synth.config1()
    rng = np.random.default_rng(7)
    cost = (w.net.fftt * rng.uniform(1, 4, w.net.m)).astype(np.float32)
    dests = list(range(0, w.net.n, 7))          # 58 trees
    D, S, _ = _trees(torch_dev, q, w.net, cost, dests, ds=ds, waves=waves)
    for k, t in enumerate(dests):
        Do, So, _ = orc.tree(w.net, cost, t)
        assert np.array_equal(D[k].view(np.uint32), Do.view(np.uint32))
        assert np.array_equal(S[k], So)


def test_trees_metro_network_sample(torch_dev, q, orc):
    w = synth.config2()
    rng = np.random.default_rng(4)
    f = rng.integers(0, 300 * FX, w.net.m).astype(np.int64)
    cost, _ = orc.bpr(f, w.net.fftt, w.net.cap, 0.15, 4, 900.0)
    dests = list(w.extra["zones"][rng.choice(len(w.extra["zones"]), 20, replace=False)])
    D, S, _ = _trees(torch_dev, q, w.net, cost, dests)
    for k, t in enumerate(dests):
        Do, So, _ = orc.tree(w.net, cost, int(t))
        assert np.array_equal(D[k].view(np.uint32), Do.view(np.uint32))
        assert np.array_equal(S[k], So)


# ---------------------------------------------------------------------------
# A2 + A3 -- all-or-nothing with truncation
# ---------------------------------------------------------------------------
def _orc():
    import oracle
    return oracle


def _aon(torch, q, net, cost, orig, dest, trips, dt, rule, ds=0.0):
    with q.Context() as ctx:
        ctx.add(net)
        ctx.set_demand(0, orig, dest, trips, dt)
        o, d, wfx = orc_legs(_orc(), ctx, [_Dem(orig, dest, trips)])
        y = torch.empty(net.m, dtype=torch.int64, device="cuda")
        stop = torch.empty(max(len(o), 1), dtype=torch.int32, device="cuda")
        rc = ctx.aon(q.default_opts(trunc_rule=rule, delta_scale=ds), dev(torch, cost.astype(np.float32)), y,
                     stop)
        return host(y), host(stop)[:len(o)], (o, d, wfx), rc


@pytest.mark.parametrize("rule", [0, 1, 2])
def test_aon_tiny(torch_dev, q, orc, rule):
    for seed in range(6):
        rng = np.random.default_rng(700 + seed)
        n = int(rng.integers(4, 10))
        net = synth.tiny_network(n, int(rng.integers(3, 12)), rng, costs="float")
        P = 40
        orig = rng.integers(0, n, P)
        dest = rng.integers(0, n, P)
        trips = rng.uniform(0.1, 30, P)
        dt = float(rng.uniform(30, 150))
        y, stop, (o, d, wfx), rc = _aon(torch_dev, q, net, net.fftt, orig, dest, trips, dt, rule, ds=0.5)
        yo, so, _ = orc.aon(net, net.fftt, o, d, wfx, dt, rule)
        assert np.array_equal(y, yo), seed
        assert np.array_equal(stop, so), seed


def test_aon_absorption_fallback(torch_dev, q, orc):
    hits = 0
    for seed in range(30):
        rng = np.random.default_rng(seed)
        net = synth.tiny_network(8, 10, rng, costs="huge")
        orig = rng.integers(0, 8, 30)
        dest = rng.integers(0, 8, 30)
        trips = rng.uniform(1, 10, 30)
        y, stop, (o, d, wfx), rc = _aon(torch_dev, q, net, net.fftt, orig, dest, trips, float("inf"), 1, ds=0.5)
        yo, so, rco = orc.aon(net, net.fftt, o, d, wfx, float("inf"), 1)
        assert np.array_equal(y, yo) and np.array_equal(stop, so), seed
        hits += rc == q.WABSORB
    assert hits > 0


def test_aon_config1_plain(torch_dev, q, orc):
    w = synth.config1()
    y, stop, (o, d, wfx), _ = _aon(torch_dev, q, w.net, w.net.fftt, w.demand.orig, w.demand.dest, w.demand.trips,
                                   float("inf"), 1)
    yo, so, _ = orc.aon(w.net, w.net.fftt, o, d, wfx, float("inf"), 1)
    assert np.array_equal(y, yo) and np.array_equal(stop, so)


def test_aon_config2_truncated(torch_dev, q, orc):
    w = synth.config2()
    rng = np.random.default_rng(8)
    f = rng.integers(0, 400 * FX, w.net.m).astype(np.int64)
    cost, _ = orc.bpr(f, w.net.fftt, w.net.cap, 0.15, 4, 900.0)
    y, stop, (o, d, wfx), _ = _aon(torch_dev, q, w.net, cost, w.demand.orig, w.demand.dest, w.demand.trips, 900.0, 1)
    yo, so, _ = orc.aon(w.net, cost, o, d, wfx, 900.0, 1)
    assert np.array_equal(y, yo)
    assert np.array_equal(stop, so)
    assert (so != d).mean() > 0.05           # truncation is active


def test_aon_edge_cases(torch_dev, q, orc):
    torch = torch_dev
    w = synth.paper_example()
    # orig == dest and zero-trip legs are dropped; one real leg remains
    y, stop, (o, d, wfx), _ = _aon(torch, q, w.net, w.net.fftt, [0, 2, 1], [3, 2, 4], [43.75, 5.0, 0.0], 900.0, 1)
    assert o.tolist() == [0] and d.tolist() == [3]
    assert y.tolist() == [int(43.75 * FX), int(43.75 * FX), 0, 0] and stop.tolist() == [2]
    # no legs at all
    y, stop, (o, d, wfx), _ = _aon(torch, q, w.net, w.net.fftt, [], [], [], 900.0, 1)
    assert (y == 0).all() and len(o) == 0
    # unreachable destination (the serial network has no way back)
    with pytest.raises(q.QdtaError) as ei:
        _aon(torch, q, w.net, w.net.fftt, [3], [0], [1.0], 900.0, 1)
    assert ei.value.code == q.EUNREACH


def test_bad_inputs_rejected(torch_dev, q):
    with q.Context() as ctx:
        with pytest.raises(q.QdtaError) as ei:
            ctx.add_network(3, [0, 1, 1, 2], [1, 5], [1.0, 1.0], [1.0, 1.0])
        assert ei.value.code == q.ECSR
        with pytest.raises(q.QdtaError) as ei:
            ctx.add_network(3, [0, 1, 1, 2], [1, 0], [1.0, -1.0], [1.0, 1.0])
        assert ei.value.code == q.EVAL
        with pytest.raises(q.QdtaError) as ei:
            ctx.add_network(3, [0, 2, 1, 2], [1, 0], [1.0, 1.0], [1.0, 1.0])
        assert ei.value.code == q.ECSR
        ctx.add_network(3, [0, 1, 2, 3], [1, 2, 0], [1.0, 1.0, 1.0], [1.0, 1.0, 1.0])
        with pytest.raises(q.QdtaError) as ei:
            ctx.set_demand(0, [0], [7], [1.0], 900.0)
        assert ei.value.code == q.EARG
        with pytest.raises(q.QdtaError) as ei:
            ctx.solve(q.default_opts(beta=0))
        assert ei.value.code == q.EARG
        for tw in (2, 3, 8, -1):
            with pytest.raises(q.QdtaError) as ei:
                ctx.solve(q.default_opts(tree_waves=tw))
            assert ei.value.code == q.EARG


# ---------------------------------------------------------------------------
# A5 / A6 -- line search and update
# ---------------------------------------------------------------------------
def _flows_pair(w, seed):
    rng = np.random.default_rng(seed)
    f = rng.integers(0, 800 * FX, w.net.m).astype(np.int64)
    y = rng.integers(0, 1600 * FX, w.net.m).astype(np.int64)
    y[rng.random(w.net.m) < 0.3] = 0
    return f, y


@pytest.mark.parametrize("dt", [float("inf"), 900.0])
def test_ls_eval_exact_sums(torch_dev, q, orc, dt):
    torch = torch_dev
    w = synth.config2()
    f, y = _flows_pair(w, 3)
    alphas = np.linspace(0.0, 1.0, 32)
    alphas[5] = 0.123456789
    Co, Do, _ = orc.ls_eval(f, y, w.net.fftt, w.net.cap, 0.15, 4, dt, alphas)
    with q.Context() as ctx:
        ctx.add(w.net)
        ctx.set_demand(0, [], [], [], dt)
        sums = torch.zeros(32 * 4, dtype=torch.int64, device="cuda")
        ctx.ls_eval(q.default_opts(), dev(torch, f), dev(torch, y), dev(torch, alphas), sums)
        s = host(sums).reshape(32, 2, 2)
    for k in range(32):
        assert i128(*s[k, 0]) == Co[k]
        assert i128(*s[k, 1]) == Do[k]


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_line_search_bit_exact(torch_dev, q, orc, mode):
    torch = torch_dev
    w = synth.config1()
    rng = np.random.default_rng(12)
    for j in (1, 4, 17):
        f = rng.integers(0, 300 * FX, w.net.m).astype(np.int64)
        y = rng.integers(0, 600 * FX, w.net.m).astype(np.int64)
        ao, _, _ = orc.line_search(f, y, w.net.fftt, w.net.cap, 0.15, 4, float("inf"), j, ls_mode=mode)
        with q.Context() as ctx:
            ctx.add(w.net)
            ctx.set_demand(0, [], [], [], float("inf"))
            a = torch.zeros(1, dtype=torch.float64, device="cuda")
            ctx.line_search(q.default_opts(ls_mode=mode), dev(torch, f), dev(torch, y), j, a)
            assert host(a)[0] == ao, (mode, j)


def test_fw_update_bit_exact(torch_dev, q, orc):
    torch = torch_dev
    w = synth.config2()
    f, y = _flows_pair(w, 5)
    for alpha in (0.0, 1.0, 0.3141592653589793, 1e-7):
        ref = orc.fw_update(f, y, alpha)
        with q.Context() as ctx:
            ctx.add(w.net)
            ft = dev(torch, f)
            ctx.fw_update(ft, dev(torch, y), dev(torch, np.array([alpha])))
            assert np.array_equal(host(ft), ref)


# ---------------------------------------------------------------------------
# A1-A7 -- full Frank-Wolfe
# ---------------------------------------------------------------------------
def _solve(torch, q, nets_dems, opts):
    with q.Context() as ctx:
        for net, dem in nets_dems:
            i = ctx.add(net)
            ctx.set_demand(i, dem.orig, dem.dest, dem.trips, dem.dt_s)
        st, rc = ctx.solve(opts)
        li = ctx.layout()
        f = torch.empty(li.total_links, dtype=torch.int64, device="cuda")
        ctx.get_flows(f)
        off = ctx.offsets()
        legs = orc_legs(_orc(), ctx, [dem for _, dem in nets_dems])
        return st, host(f), off, legs, rc


def _cmp_fw(st, fo, gpu_f, ref):
    assert st["iters"] == ref.iters
    assert np.array_equal(gpu_f, ref.f)
    assert st["gap"] == ref.gap
    assert abs(st["objective"] - ref.objective) <= 1e-12 * abs(ref.objective)
    assert st["ls_evals"] == ref.ls_evals
    fp64_check(st, ref)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_fw_config1_fixed50(torch_dev, q, orc, mode):
    w = synth.config1()
    st, f, off, (o, d, wfx), rc = _solve(torch_dev, q, [(w.net, w.demand)],
                                         q.default_opts(fixed_iters=50, ls_mode=mode))
    ref = orc.fw_solve(w.net, o, d, wfx, fixed_iters=50, ls_mode=mode)
    _cmp_fw(st[0], None, f, ref)


def test_fw_config2_truncated(torch_dev, q, orc):
    w = synth.config2()
    opts = q.default_opts(fixed_iters=4)
    st, f, off, (o, d, wfx), rc = _solve(torch_dev, q, [(w.net, w.demand)], opts)
    ref = orc.fw_solve(w.net, o, d, wfx, dt_s=900.0, fixed_iters=4, keep_history=False)
    _cmp_fw(st[0], None, f, ref)


def test_fw_objective_stop_rule(torch_dev, q, orc):
    w = synth.config1()
    opts = q.default_opts(stop_rule=q.STOP_OBJ, tol=1e-4, max_iter=200)
    st, f, off, (o, d, wfx), rc = _solve(torch_dev, q, [(w.net, w.demand)], opts)
    ref = orc.fw_solve(w.net, o, d, wfx, stop_rule=orc.STOP_OBJ, tol=1e-4, max_iter=200)
    _cmp_fw(st[0], None, f, ref)
    assert st[0]["stopped_by"] == 2


def test_config3_peak_full_size(torch_dev, q, orc):
    """The benchmark workload at full size (550k nodes, 1.0M links, 5,000
    trees, 261k legs, dt = 900 s) in the configuration bench.py times (one
    FW iteration replayed as a HIP graph, default kernel and bucket width):
    the initial AON and two FW iterations equal the oracle bit for bit."""
    w = synth.config3()
    opts = q.default_opts(alpha=w.alpha, beta=w.beta, fixed_iters=2)
    st, f, off, (o, d, wfx), rc = _solve(torch_dev, q, [(w.net, w.demand)], opts)
    ref = orc.fw_solve(w.net, o, d, wfx, alpha_b=w.alpha, beta=w.beta, dt_s=w.demand.dt_s, fixed_iters=2,
                       keep_history=False)
    assert np.array_equal(f, ref.f)
    assert st[0]["gap"] == ref.gap
    assert st[0]["iters"] == ref.iters
    fp64_check(st[0], ref)


def test_config3_peak_interior_steps_and_residual_full_size(torch_dev, q, orc):
    """The 1.0M-link network with the 08:00 legs plus those of the three
    intervals before it carried in as residual demand (synthetic legs set
    with qdta_set_residual; congested), dt = 900 s, CEIL.  For each of three
    Frank-Wolfe updates, the direction y_j (the GPU's own BPR and AON on the
    GPU's previous iterate, in a second context), the step size alpha_j and
    the flows f_j equal the oracle's element by element, at least two steps
    lying inside (0, 1); then the residual demand of Alg. 4 after those
    updates equals the oracle's leg for leg."""
    torch = torch_dev

    def say(msg):                                  # the oracle's full-size legs take minutes: show progress
        print(f"[interior full size] {msg}", flush=True)

    w = synth.config3_window(29)
    say("inputs generated")
    net, peak, carried = w.net, w.demand[-1], w.demand[:-1]
    co = np.concatenate([x.orig for x in carried])
    cd = np.concatenate([x.dest for x in carried])
    ct = np.concatenate([x.trips for x in carried])
    ro_in, rd_in, rw_in = orc.demand_legs(co, cd, ct)
    o, d, wfx = orc.merge_legs(np.concatenate([peak.orig, ro_in]), np.concatenate([peak.dest, rd_in]),
                               np.concatenate([orc.trips_to_fx_array(peak.trips), rw_in]))
    keep = (wfx > 0) & (o != d)
    o, d, wfx = o[keep], d[keep], wfx[keep]
    opts = q.default_opts(alpha=w.alpha, beta=w.beta, fixed_iters=3, keep_history=1)

    def ctx_for():
        c = q.Context()
        c.add(net)
        c.set_residual(0, ro_in, rd_in, rw_in)
        c.set_demand(0, peak.orig, peak.dest, peak.trips, peak.dt_s)
        return c

    ctx, side = ctx_for(), ctx_for()
    try:
        lo, ld, lw = ctx.legs()
        assert np.array_equal(lo, o) and np.array_equal(ld, d) and np.array_equal(lw, wfx)
        f = torch.empty(net.m, dtype=torch.int64, device="cuda")
        cost = torch.empty(net.m, dtype=torch.float32, device="cuda")
        y = torch.empty(net.m, dtype=torch.int64, device="cuda")
        ctx.fw_begin(opts)
        ctx.get_flows(f)
        fo, _, _ = orc.aon(net, net.fftt, o, d, wfx, 900.0)
        assert np.array_equal(host(f), fo)
        say("initial AON equal")
        hist_alpha, hist_cost, interior = [1.0], [net.fftt.astype(np.float32)], 0
        for j in (1, 2, 3):
            f_prev = host(f).copy()
            co_j, _ = orc.bpr(fo, net.fftt, net.cap, w.alpha, w.beta, 900.0)
            yo, _, _ = orc.aon(net, co_j, o, d, wfx, 900.0)
            ao, _, _ = orc.line_search(fo, yo, net.fftt, net.cap, w.alpha, w.beta, 900.0, j)
            fo = orc.fw_update(fo, yo, ao)
            # the GPU's direction from its own costs of its own previous iterate
            side.bpr(opts, dev(torch, f_prev), cost)
            side.aon(opts, cost, y)
            assert np.array_equal(host(cost).view(np.uint32), co_j.view(np.uint32)), j
            assert np.array_equal(host(y), yo), j
            st, _ = ctx.fw_step(opts)
            ctx.get_flows(f)
            assert st[0]["last_alpha"] == ao, j
            assert np.array_equal(host(f), fo), j
            interior += 0.0 < ao < 1.0
            say(f"update {j} equal, alpha {ao}")
            hist_alpha.append(ao)
            hist_cost.append(co_j)
        assert interior >= 2
        st, live = ctx.fw_step(opts)                 # the final test; the interval is solved
        assert not live and st[0]["iters"] == 3
        ctx.advance_interval(opts)
        g_o, g_d, g_w, g_done = ctx.residual(0)
        # the oracle's residual pass by groups of destinations (residual legs of
        # different destinations never merge), reporting progress in between
        parts, done = [], 0
        dq = np.unique(d)
        for k, grp in enumerate(np.array_split(dq, 8)):
            sel = np.isin(d, grp)
            p_o, p_d, p_w, p_done, _ = orc.residual(net, fo, np.array(hist_alpha), np.stack(hist_cost), o[sel],
                                                    d[sel], wfx[sel], alpha_b=w.alpha, beta=w.beta, dt_s=900.0)
            parts.append((p_o, p_d, p_w))
            done += p_done
            say(f"oracle residual, destination group {k + 1} of 8")
        r_o, r_d, r_w = orc.merge_legs(*(np.concatenate(x) for x in zip(*parts)))
        say(f"residual: {r_o.size} legs")
        assert np.array_equal(g_o, r_o) and np.array_equal(g_d, r_d) and np.array_equal(g_w, r_w)
        assert g_done == done and r_o.size > 100_000
    finally:
        ctx.close()
        side.close()


def test_config4_full_batch_sampled(torch_dev, q, orc):
    """All 64 uneven networks at full size in one context (4.7M links,
    33,840 trees; one launch sequence per FW iteration, replayed as a HIP
    graph): three sampled instances, the largest among them, equal the
    single-instance oracle bit for bit after two iterations."""
    insts = synth.config4()
    opts = q.default_opts(fixed_iters=2)
    st, f, off, (o, d, wfx), rc = _solve(torch_dev, q, [(x.net, x.demand) for x in insts], opts)
    big = int(np.argmax([x.net.m for x in insts]))
    for i in (big, 7, 40):
        x = insts[i]
        a, b = off["leg"][i], off["leg"][i + 1]
        ref = orc.fw_solve(x.net, o[a:b], d[a:b], wfx[a:b], fixed_iters=2, keep_history=False)
        _cmp_fw(st[i], None, f[off["link"][i]:off["link"][i + 1]], ref)


def test_fw_batched_instances_match_single(torch_dev, q, orc):
    """Several uneven grids in one context (one launch sequence per FW
    iteration) give, per instance, exactly the single-instance oracle result."""
    insts = synth.config4(count=5, k_lo=8, k_hi=18, z_lo=10, z_hi=40)
    opts = q.default_opts(tol=1e-3, max_iter=40)
    st, f, off, (o, d, wfx), rc = _solve(torch_dev, q, [(x.net, x.demand) for x in insts], opts)
    for i, x in enumerate(insts):
        a, b = off["leg"][i], off["leg"][i + 1]
        ref = orc.fw_solve(x.net, o[a:b], d[a:b], wfx[a:b], tol=1e-3, max_iter=40, keep_history=False)
        _cmp_fw(st[i], None, f[off["link"][i]:off["link"][i + 1]], ref)


# ---------------------------------------------------------------------------
# A8 -- residual demand and the interval chain
# ---------------------------------------------------------------------------
def _day_gpu(torch, q, net, days, opts):
    out = []
    with q.Context() as ctx:
        ctx.add(net)
        for dem in days:
            ctx.set_demand(0, dem.orig, dem.dest, dem.trips, dem.dt_s)
            li = ctx.layout()
            if li.total_legs == 0:
                out.append({"f": np.zeros(net.m, np.int64), "res": (np.zeros(0, np.int32),) * 2 +
                            (np.zeros(0, np.int64),), "iters": 0})
                continue
            st, rc = ctx.solve(opts)
            f = torch.empty(net.m, dtype=torch.int64, device="cuda")
            ctx.get_flows(f)
            ctx.advance_interval(opts)
            ro, rd, rw, done = ctx.residual(0)
            out.append({"f": host(f), "res": (ro, rd, rw), "iters": st[0]["iters"], "done": done})
    return out


def test_day_worked_example(torch_dev, q, orc):
    w = synth.paper_example()
    opts = q.default_opts(keep_history=1)
    g = _day_gpu(torch_dev, q, w.net, w.demand, opts)
    ref, _ = orc.qdta_day(w.net, w.demand)
    for a, b in zip(g, ref):
        assert np.array_equal(a["f"], b["f"])
        for x, y in zip(a["res"], b["res"]):
            assert np.array_equal(x, y)
    assert g[0]["res"][0].tolist() == [2]


def test_day_small_network_chain(torch_dev, q, orc):
    w = synth.config1()
    rng = np.random.default_rng(9)
    days = []
    for i in range(4):
        sel = rng.random(w.demand.P) < 0.3
        days.append(synth.demand.Demand(w.demand.orig[sel], w.demand.dest[sel], w.demand.trips[sel] / 4, 300.0))
    opts = q.default_opts(keep_history=1, tol=1e-3, max_iter=30)
    g = _day_gpu(torch_dev, q, w.net, days, opts)
    ref, _ = orc.qdta_day(w.net, days, tol=1e-3, max_iter=30)
    for a, b in zip(g, ref):
        assert a["iters"] == b["iters"]
        assert np.array_equal(a["f"], b["f"])
        for x, y in zip(a["res"], b["res"]):
            assert np.array_equal(x, y)
        assert a["done"] == b["done_fx"]


def test_day_chain_workgroup_trees(torch_dev, q, orc):
    """The interval chain with one workgroup per tree (early exit, residual
    walks on stored labels) equals the oracle."""
    w = synth.config1()
    rng = np.random.default_rng(23)
    days = []
    for frac in (0.6, 0.3, 0.5):
        sel = rng.random(w.demand.P) < frac
        days.append(synth.demand.Demand(w.demand.orig[sel], w.demand.dest[sel], w.demand.trips[sel] / 2, 600.0))
    opts = q.default_opts(keep_history=1, tol=1e-3, max_iter=20, tree_waves=4)
    g = _day_gpu(torch_dev, q, w.net, days, opts)
    ref, _ = orc.qdta_day(w.net, days, tol=1e-3, max_iter=20)
    for a, b in zip(g, ref):
        assert a["iters"] == b["iters"]
        assert np.array_equal(a["f"], b["f"])
        for x, y in zip(a["res"], b["res"]):
            assert np.array_equal(x, y)


def test_day_peak_scaled_network(torch_dev, q, orc):
    """Six morning-peak intervals of the 1/20-scale day (27,500 nodes, 250
    zones, up to 14 iterates and 28k residual legs per interval), chained
    from a cold start under the objective rule of Eq. 7: flows, iteration
    counts and residual legs equal the oracle with the label history on
    (every iterate stored), capped at 100 MiB (three stored, the rest grown
    again) and off."""
    w = synth.config3_day(0.05)
    days = w.demand[28:34]
    ref, _ = orc.qdta_day(w.net, days, stop_rule=orc.STOP_OBJ, tol=1e-4, max_iter=100)
    assert max(r["iters"] for r in ref) >= 10
    for hist in (0, 100, -1):
        opts = q.default_opts(stop_rule=q.STOP_OBJ, tol=1e-4, max_iter=100, keep_history=1, history_mib=hist)
        g = _day_gpu(torch_dev, q, w.net, days, opts)
        for a, b in zip(g, ref):
            assert a["iters"] == b["iters"], hist
            assert np.array_equal(a["f"], b["f"]), hist
            for x, y in zip(a["res"], b["res"]):
                assert np.array_equal(x, y), hist
            assert a["done"] == b["done_fx"], hist


def test_day_resume_from_saved_residual(torch_dev, q, orc):
    """Checkpoint and resume: a day stopped after interval 2 (its residual
    legs read back to the host, the context destroyed) and continued in a
    fresh context from qdta_set_residual gives the flows and residual legs
    of the uninterrupted run bit for bit."""
    w = synth.config1()
    rng = np.random.default_rng(31)
    days = []
    for frac in (0.7, 0.4, 0.6, 0.3, 0.5):
        sel = rng.random(w.demand.P) < frac
        days.append(synth.demand.Demand(w.demand.orig[sel], w.demand.dest[sel], w.demand.trips[sel] / 2, 450.0))
    opts = q.default_opts(keep_history=1, tol=1e-3, max_iter=25)
    whole = _day_gpu(torch_dev, q, w.net, days, opts)
    head = _day_gpu(torch_dev, q, w.net, days[:3], opts)
    saved = head[-1]["res"]
    assert len(saved[0]) > 0
    tail = []
    with q.Context() as ctx:
        ctx.add(w.net)
        ctx.set_residual(0, *saved)
        o, d, wt, _ = ctx.residual(0)
        assert all(np.array_equal(x, y) for x, y in zip((o, d, wt), saved))
        for dem in days[3:]:
            ctx.set_demand(0, dem.orig, dem.dest, dem.trips, dem.dt_s)
            st, rc = ctx.solve(opts)
            f = torch_dev.empty(w.net.m, dtype=torch_dev.int64, device="cuda")
            ctx.get_flows(f)
            ctx.advance_interval(opts)
            ro, rd, rw, done = ctx.residual(0)
            tail.append({"f": host(f), "res": (ro, rd, rw), "iters": st[0]["iters"]})
    for a_, b_ in zip(head + tail, whole):
        assert a_["iters"] == b_["iters"]
        assert np.array_equal(a_["f"], b_["f"])
        for x, y in zip(a_["res"], b_["res"]):
            assert np.array_equal(x, y)
    ref, _ = orc.qdta_day(w.net, days, tol=1e-3, max_iter=25)
    for a_, b_ in zip(whole, ref):
        assert np.array_equal(a_["f"], b_["f"])


def test_set_residual_rejects_bad_legs(torch_dev, q):
    w = synth.config1()
    n = w.net.n
    bad = [([1, 2], [5, 5], [3, 0]),            # weight 0
           ([2, 1], [5, 5], [3, 3]),            # origins out of order
           ([1, 1], [5, 5], [3, 3]),            # repeated leg
           ([1, 2], [7, 5], [3, 3]),            # destinations out of order
           ([5], [5], [3]),                     # origin == destination
           ([n], [0], [3]),                     # node out of range
           ([0], [-1], [3])]
    with q.Context() as ctx:
        ctx.add(w.net)
        for o, d, wt in bad:
            with pytest.raises(q.QdtaError) as e:
                ctx.set_residual(0, np.array(o), np.array(d), np.array(wt))
            assert e.value.code == q.EARG
        with pytest.raises(q.QdtaError):
            ctx.set_residual(1, np.array([1]), np.array([2]), np.array([3]))
        ctx.set_residual(0, np.array([1, 3, 0]), np.array([2, 2, 4]), np.array([5, 6, 7]))
        assert ctx.residual(0)[0].tolist() == [1, 3, 0]
        ctx.set_residual(0, np.zeros(0), np.zeros(0), np.zeros(0))
        assert ctx.residual(0)[0].size == 0


def test_day_demand_shrinks_and_regrows(torch_dev, q, orc):
    """Intervals whose leg and destination counts fall and then rise again
    within the buffers of the largest one: every interval is re-captured
    for its own sizes, so each still matches the oracle exactly."""
    w = synth.config1()
    rng = np.random.default_rng(17)
    days = []
    for frac in (0.8, 0.1, 0.45, 0.05, 0.5):
        sel = rng.random(w.demand.P) < frac
        days.append(synth.demand.Demand(w.demand.orig[sel], w.demand.dest[sel], w.demand.trips[sel] / 3, 900.0))
    opts = q.default_opts(keep_history=1, tol=1e-3, max_iter=25)
    g = _day_gpu(torch_dev, q, w.net, days, opts)
    ref, _ = orc.qdta_day(w.net, days, tol=1e-3, max_iter=25)
    legs = [b["legs"] for b in ref]
    assert legs[1] < legs[0] and legs[3] < legs[4] < legs[0]
    for a, b in zip(g, ref):
        assert a["iters"] == b["iters"]
        assert np.array_equal(a["f"], b["f"])
        for x, y in zip(a["res"], b["res"]):
            assert np.array_equal(x, y)


# ---------------------------------------------------------------------------
# A9 -- launch structure: graph replay, plain form, kernel shapes
# ---------------------------------------------------------------------------
def _step_flows(torch, q, nets_dems, opts, steps):
    """Flows and stats after each FW step (one entry per replayed iteration)."""
    out = []
    with q.Context() as ctx:
        for net, dem in nets_dems:
            i = ctx.add(net)
            ctx.set_demand(i, dem.orig, dem.dest, dem.trips, dem.dt_s)
        ctx.fw_begin(opts)
        li = ctx.layout()
        f = torch.empty(li.total_links, dtype=torch.int64, device="cuda")
        for _ in range(steps):
            st, live = ctx.fw_step(opts)
            ctx.get_flows(f)
            out.append((host(f).copy(), [(s["iters"], s["gap"], s["last_alpha"]) for s in st]))
    return out


def test_graph_replay_matches_direct_launches(torch_dev, q):
    """One FW iteration captured as a HIP graph and replayed (with the host's
    state copy and synchronisation between replays) gives, after every
    replay, exactly what direct launches give."""
    insts = synth.config4(count=3, k_lo=10, k_hi=16, z_lo=12, z_hi=30)
    nd = [(x.net, x.demand) for x in insts]
    for mode in (q.LS_KSECTION, q.LS_MSA):
        g = _step_flows(torch_dev, q, nd, q.default_opts(fixed_iters=1000, ls_mode=mode, launch_form=0), 12)
        d = _step_flows(torch_dev, q, nd, q.default_opts(fixed_iters=1000, ls_mode=mode, launch_form=1), 12)
        for (fg, sg), (fd, sd) in zip(g, d):
            assert np.array_equal(fg, fd)
            assert sg == sd


def test_plain_form_matches_batched(torch_dev, q, orc):
    w = synth.config1()
    for mode in (q.LS_KSECTION, q.LS_QN):
        st_p, f_p, _, (o, d, wfx), _ = _solve(torch_dev, q, [(w.net, w.demand)],
                                              q.default_opts(fixed_iters=8, ls_mode=mode, launch_form=2))
        st_b, f_b, _, _, _ = _solve(torch_dev, q, [(w.net, w.demand)],
                                    q.default_opts(fixed_iters=8, ls_mode=mode, launch_form=0))
        assert np.array_equal(f_p, f_b) and st_p[0]["gap"] == st_b[0]["gap"]
        ref = orc.fw_solve(w.net, o, d, wfx, fixed_iters=8, ls_mode=mode, keep_history=False)
        assert np.array_equal(f_p, ref.f)


def test_autotune_picks_valid_options_and_results_do_not_move(torch_dev, q, orc):
    """The autotuner only chooses kernel shape, bucket width and wavefronts
    per tree; a solve with its choice equals the oracle bit for bit."""
    w = synth.config2()
    sel = np.isin(w.demand.dest, w.extra["zones"][:40])
    dem = synth.demand.Demand(w.demand.orig[sel], w.demand.dest[sel], w.demand.trips[sel], 900.0)
    with q.Context() as ctx:
        ctx.add(w.net)
        ctx.set_demand(0, dem.orig, dem.dest, dem.trips, dem.dt_s)
        opts, best = ctx.autotune(q.default_opts(fixed_iters=3), 300.0)
        assert 1 <= opts.sssp_shape <= 6 and opts.delta_scale > 0 and opts.tree_waves in (1, 4)
        assert best > 0
        st, rc = ctx.solve(opts)
        f = torch_dev.empty(w.net.m, dtype=torch_dev.int64, device="cuda")
        ctx.get_flows(f)
        o, d, wfx = orc_legs(orc, ctx, [dem])
    ref = orc.fw_solve(w.net, o, d, wfx, fixed_iters=3, dt_s=900.0, keep_history=False)
    assert np.array_equal(host(f), ref.f)


def test_autotune_inside_a_running_solve_and_load_form(torch_dev, q, orc):
    """Tuned after two iterations of a running solve (its trials overwrite
    the costs, trees and direction, which the next step recomputes), the
    solve goes on to the same flows as an untuned one and as the oracle.  On
    a plain interval the tuner also picks the loading form (walks or merged
    paths), which changes no bit either."""
    w = synth.config1()
    o, d, wfx = orc.demand_legs(w.demand.orig, w.demand.dest, w.demand.trips)
    ref = orc.fw_solve(w.net, o, d, wfx, fixed_iters=6, keep_history=False)
    with q.Context() as ctx:
        ctx.add(w.net)
        ctx.set_demand(0, w.demand.orig, w.demand.dest, w.demand.trips, w.demand.dt_s)
        opts = q.default_opts(fixed_iters=6)
        ctx.fw_begin(opts)
        for _ in range(2):
            ctx.fw_step(opts)
        tuned, best = ctx.autotune(opts, 200.0)
        assert tuned.load_form in (1, 2) and best > 0
        live = True
        while live:
            st, live = ctx.fw_step(tuned)
        f = torch_dev.empty(w.net.m, dtype=torch_dev.int64, device="cuda")
        ctx.get_flows(f)
        assert np.array_equal(host(f), ref.f)
        assert st[0]["iters"] == 6 and st[0]["gap"] == ref.gap
        for form in (1, 2):
            st2, _ = ctx.solve(q.default_opts(fixed_iters=6, load_form=form))
            ctx.get_flows(f)
            assert np.array_equal(host(f), ref.f), form


@pytest.mark.parametrize("waves", [1, 4])
@pytest.mark.parametrize("shape", [1, 2, 3, 4, 5, 6])
def test_sssp_shapes_identical(torch_dev, q, orc, shape, waves):
    w = synth.config2()
    rng = np.random.default_rng(40 + shape)
    f = rng.integers(0, 600 * FX, w.net.m).astype(np.int64)
    cost, _ = orc.bpr(f, w.net.fftt, w.net.cap, 0.15, 4, 900.0)
    sel = np.isin(w.demand.dest, w.extra["zones"][:25])
    y, stop, (o, d, wfx), _ = _aon(torch_dev, q, w.net, cost, w.demand.orig[sel], w.demand.dest[sel],
                                   w.demand.trips[sel], 900.0, 1)
    with q.Context() as ctx:
        ctx.add(w.net)
        ctx.set_demand(0, w.demand.orig[sel], w.demand.dest[sel], w.demand.trips[sel], 900.0)
        yy = torch_dev.empty(w.net.m, dtype=torch_dev.int64, device="cuda")
        ctx.aon(q.default_opts(sssp_shape=shape, tree_waves=waves), dev(torch_dev, cost), yy)
        assert np.array_equal(host(yy), y)
    yo, so, _ = orc.aon(w.net, cost, o, d, wfx, 900.0, 1)
    assert np.array_equal(y, yo)


# ---------------------------------------------------------------------------
# Derivatives of the frozen-path model (OD calibration)
# ---------------------------------------------------------------------------
def _adj_case(name):
    if name == "grid":
        w = synth.config1()
        return w.net, w.demand, 5
    if name == "grid_trunc":
        w = synth.config1()
        rng = np.random.default_rng(5)
        sel = rng.random(w.demand.P) < 0.35
        dem = synth.demand.Demand(w.demand.orig[sel], w.demand.dest[sel], w.demand.trips[sel] * 0.5, 1800.0)
        return w.net, dem, 4
    # 1/20-scale metro network, a morning interval with doubled trips and a
    # 30-minute horizon (congested, truncated, step sizes inside (0, 1))
    w = synth.config3_day(0.05)
    x = w.demand[34]
    return w.net, synth.demand.Demand(x.orig, x.dest, x.trips * 2.0, 1800.0), 3


def _adj_setup(q, orc, net, dem, iters):
    from oracle import adjoint as adj
    ctx = q.Context()
    ctx.add(net)
    ctx.set_demand(0, dem.orig, dem.dest, dem.trips, dem.dt_s)
    opts = q.default_opts(fixed_iters=iters, keep_history=1)
    ctx.solve(opts)
    ctx.adjoint_record(opts)
    o, d, wfx = orc_legs(orc, ctx, [dem])
    res = orc.fw_solve(net, o, d, wfx, dt_s=dem.dt_s, fixed_iters=iters, keep_history=True)
    pl = adj.frozen_paths(net, o, d, wfx, res.hist_cost, dem.dt_s)
    return ctx, opts, (o, d, wfx), res, pl


def _perturbed(net, wfx, seed):
    rng = np.random.default_rng(seed)
    d2 = (wfx / FX) * (1.0 + 0.3 * rng.uniform(-1.0, 1.0, wfx.shape[0]))
    cap2 = (net.cap.astype(np.float64) * (1.0 + 0.2 * rng.uniform(-1.0, 1.0, net.m))).astype(np.float32)
    return d2, cap2


@pytest.mark.parametrize("case", ["grid", "grid_trunc", "metro_scaled"])
def test_model_forward_bit_exact(torch_dev, q, orc, case):
    """The frozen-path replay at the solve's own demand gives the solve's
    flows; at another demand and other capacities it equals the oracle's
    contract replay bit for bit."""
    from oracle import adjoint as adj
    torch = torch_dev
    net, dem, iters = _adj_case(case)
    ctx, opts, (o, d, wfx), res, pl = _adj_setup(q, orc, net, dem, iters)
    try:
        f_solve = torch.empty(net.m, dtype=torch.int64, device="cuda")
        ctx.get_flows(f_solve)
        fo = torch.empty(net.m, dtype=torch.float64, device="cuda")
        ctx.model_forward(opts, dev(torch, wfx / FX), None, fo)
        assert np.array_equal(host(fo), host(f_solve) / FX)
        assert np.array_equal(host(fo), res.f / FX)
        d2, cap2 = _perturbed(net, wfx, 3)
        ctx.model_forward(opts, dev(torch, d2), dev(torch, cap2), fo)
        f2, st2 = adj.forward_contract(pl, net.m, d2, net.fftt, cap2, 0.15, 4, dem.dt_s)
        assert np.array_equal(host(fo) * FX, f2.astype(np.float64))
    finally:
        ctx.close()


@pytest.mark.parametrize("case", ["grid", "grid_trunc", "metro_scaled"])
def test_model_backward_matches_oracle(torch_dev, q, orc, case):
    """Reverse pass at a perturbed demand and capacities: dL/dd per leg and
    dL/dC per link against the oracle's FP64 reverse pass on the same
    (bit-identical) iterates.  Only the order of the FP64 reductions over the
    links differs: agreement to 1e-9 of the largest component."""
    from oracle import adjoint as adj
    torch = torch_dev
    net, dem, iters = _adj_case(case)
    ctx, opts, (o, d, wfx), res, pl = _adj_setup(q, orc, net, dem, iters)
    try:
        d2, cap2 = _perturbed(net, wfx, 4)
        fo = torch.empty(net.m, dtype=torch.float64, device="cuda")
        fid = ctx.model_forward(opts, dev(torch, d2), dev(torch, cap2), fo)
        f2, st2 = adj.forward_contract(pl, net.m, d2, net.fftt, cap2, 0.15, 4, dem.dt_s)
        assert sum(0.0 < s[2] < 1.0 for s in st2[1:]) >= 1
        rng = np.random.default_rng(8)
        fbar = np.where(rng.random(net.m) < 0.2, rng.standard_normal(net.m), 0.0)
        dbar = torch.empty(len(o), dtype=torch.float64, device="cuda")
        capbar = torch.empty(net.m, dtype=torch.float64, device="cuda")
        ctx.model_backward(fid, dev(torch, fbar), dbar, capbar)
        rd, rc = adj.backward(st2, fbar, pl, net.fftt, cap2, 0.15, 4, dem.dt_s)
        gd, gc = host(dbar), host(capbar)
        assert np.max(np.abs(gd - rd)) <= 1e-9 * np.max(np.abs(rd))
        assert np.max(np.abs(gc - rc)) <= 1e-9 * np.max(np.abs(rc))
        assert np.max(np.abs(rc)) > 0
    finally:
        ctx.close()


def test_model_autograd_function(torch_dev, q, orc):
    """torch.autograd through the frozen-path model: the squared count error
    on 10% of the links, gradients in the demand (float64) and the
    capacities (float32) against the oracle's reverse pass."""
    from oracle import adjoint as adj
    torch = torch_dev
    net, dem, iters = _adj_case("grid_trunc")
    ctx, opts, (o, d, wfx), res, pl = _adj_setup(q, orc, net, dem, iters)
    try:
        d2, cap2 = _perturbed(net, wfx, 6)
        rng = np.random.default_rng(9)
        obs = rng.random(net.m) < 0.1
        target = res.f / FX * (1.0 + 0.1 * rng.standard_normal(net.m))
        dt = dev(torch, d2).requires_grad_(True)
        ct = dev(torch, cap2).requires_grad_(True)
        f = q.frozen_path_flows(ctx, opts, dt, ct)
        m_obs = dev(torch, obs)
        loss = (((f - dev(torch, target)) ** 2) * m_obs).sum()
        loss.backward()
        f2, st2 = adj.forward_contract(pl, net.m, d2, net.fftt, cap2, 0.15, 4, dem.dt_s)
        fbar = np.where(obs, 2.0 * (f2 / FX - target), 0.0)
        rd, rc = adj.backward(st2, fbar, pl, net.fftt, cap2, 0.15, 4, dem.dt_s)
        assert np.max(np.abs(host(dt.grad) - rd)) <= 1e-9 * np.max(np.abs(rd))
        assert ct.grad.dtype == torch.float32
        assert np.allclose(host(ct.grad), rc.astype(np.float32), rtol=1e-6, atol=1e-6 * np.max(np.abs(rc)))
    finally:
        ctx.close()


def test_model_backward_refuses_a_stale_forward(torch_dev, q, orc):
    """Two forward passes before one backward: the context holds the second
    pass's iterates only, so the first pass's backward is refused (through
    the ABI and through torch.autograd) and the second one's still matches
    a fresh forward + backward at its own inputs."""
    torch = torch_dev
    net, dem, iters = _adj_case("grid_trunc")
    ctx, opts, (o, d, wfx), res, pl = _adj_setup(q, orc, net, dem, iters)
    try:
        d1, cap1 = _perturbed(net, wfx, 11)
        d2, cap2 = _perturbed(net, wfx, 12)
        fo = torch.empty(net.m, dtype=torch.float64, device="cuda")
        id1 = ctx.model_forward(opts, dev(torch, d1), dev(torch, cap1), fo)
        id2 = ctx.model_forward(opts, dev(torch, d2), dev(torch, cap2), fo)
        assert id2 != id1
        fbar = dev(torch, np.linspace(-1.0, 1.0, net.m))
        dbar = torch.empty(len(o), dtype=torch.float64, device="cuda")
        capbar = torch.empty(net.m, dtype=torch.float64, device="cuda")
        with pytest.raises(q.QdtaError) as e:
            ctx.model_backward(id1, fbar, dbar, capbar)
        assert e.value.code == q.ESTATE
        ctx.model_backward(id2, fbar, dbar, capbar)
        g2 = host(dbar).copy()
        id3 = ctx.model_forward(opts, dev(torch, d2), dev(torch, cap2), fo)
        ctx.model_backward(id3, fbar, dbar, capbar)
        assert np.array_equal(host(dbar), g2)
        # autograd: two losses built before one backward
        da = dev(torch, d1).requires_grad_(True)
        fa = q.frozen_path_flows(ctx, opts, da, None)
        fb = q.frozen_path_flows(ctx, opts, dev(torch, d2).requires_grad_(True), None)
        with pytest.raises(q.QdtaError):
            fa.sum().backward()
        del fb
    finally:
        ctx.close()


def test_model_needs_record_for_the_current_solve(torch_dev, q):
    torch = torch_dev
    w = synth.config1()
    with q.Context() as ctx:
        ctx.add(w.net)
        ctx.set_demand(0, w.demand.orig, w.demand.dest, w.demand.trips, w.demand.dt_s)
        opts = q.default_opts(fixed_iters=2, keep_history=1)
        P = ctx.layout().total_legs
        d = torch.ones(P, dtype=torch.float64, device="cuda")
        f = torch.empty(w.net.m, dtype=torch.float64, device="cuda")
        ctx.solve(opts)
        with pytest.raises(q.QdtaError) as e:
            ctx.model_forward(opts, d, None, f)
        assert e.value.code == q.ESTATE
        with pytest.raises(q.QdtaError) as e:
            ctx.adjoint_record(q.default_opts(fixed_iters=2))
        assert e.value.code == q.ESTATE
        ctx.adjoint_record(opts)
        ctx.model_forward(opts, d, None, f)
        ctx.solve(opts)                             # a new solve invalidates the record
        with pytest.raises(q.QdtaError) as e:
            ctx.model_forward(opts, d, None, f)
        assert e.value.code == q.ESTATE
    with q.Context() as ctx:
        ctx.add(w.net)
        ctx.add(w.net)
        for i in range(2):
            ctx.set_demand(i, w.demand.orig, w.demand.dest, w.demand.trips, w.demand.dt_s)
        opts = q.default_opts(fixed_iters=1, keep_history=1)
        ctx.solve(opts)
        with pytest.raises(q.QdtaError) as e:
            ctx.adjoint_record(opts)
        assert e.value.code == q.ESTATE


# ---------------------------------------------------------------------------
# The system optimum (marginal-cost routing, total travel time)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dt", [float("inf"), 900.0])
def test_bpr_marginal_bit_exact(torch_dev, q, orc, dt):
    torch = torch_dev
    w = synth.config2()
    rng = np.random.default_rng(21)
    f = rng.integers(0, 5000 * FX, w.net.m).astype(np.int64)
    ref, _ = orc.bpr(f, w.net.fftt, w.net.cap, 0.15, 4, dt, marginal=True)
    with q.Context() as ctx:
        ctx.add(w.net)
        ctx.set_demand(0, [], [], [], dt)
        c = torch.empty(w.net.m, dtype=torch.float32, device="cuda")
        ctx.bpr(q.default_opts(objective=q.OBJ_SO), dev(torch, f), c)
        assert np.array_equal(host(c).view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_fw_system_optimum_config1(torch_dev, q, orc, mode):
    w = synth.config1()
    st, f, off, (o, d, wfx), rc = _solve(torch_dev, q, [(w.net, w.demand)],
                                         q.default_opts(fixed_iters=50, ls_mode=mode, objective=q.OBJ_SO))
    ref = orc.fw_solve(w.net, o, d, wfx, fixed_iters=50, ls_mode=mode, objective=orc.OBJ_SO)
    _cmp_fw(st[0], None, f, ref)
    ue = orc.fw_solve(w.net, o, d, wfx, fixed_iters=50, ls_mode=mode)
    assert not np.array_equal(ue.f, ref.f)


def test_fw_system_optimum_truncated(torch_dev, q, orc):
    """Config 2 with its 900 s horizon: trees by marginal costs, the
    truncation clocked by the travel times, the objective stop rule."""
    w = synth.config2()
    opts = q.default_opts(objective=q.OBJ_SO, stop_rule=q.STOP_OBJ, tol=1e-4, max_iter=6)
    st, f, off, (o, d, wfx), rc = _solve(torch_dev, q, [(w.net, w.demand)], opts)
    ref = orc.fw_solve(w.net, o, d, wfx, dt_s=900.0, objective=orc.OBJ_SO, stop_rule=orc.STOP_OBJ, tol=1e-4,
                       max_iter=6, keep_history=False)
    _cmp_fw(st[0], None, f, ref)


def test_day_system_optimum_chain(torch_dev, q, orc):
    w = synth.config1()
    rng = np.random.default_rng(41)
    days = []
    for frac in (0.6, 0.4, 0.5):
        sel = rng.random(w.demand.P) < frac
        days.append(synth.demand.Demand(w.demand.orig[sel], w.demand.dest[sel], w.demand.trips[sel] / 2, 600.0))
    opts = q.default_opts(keep_history=1, tol=1e-3, max_iter=20, objective=q.OBJ_SO)
    g = _day_gpu(torch_dev, q, w.net, days, opts)
    ref, _ = orc.qdta_day(w.net, days, tol=1e-3, max_iter=20, objective=orc.OBJ_SO)
    for a, b in zip(g, ref):
        assert a["iters"] == b["iters"]
        assert np.array_equal(a["f"], b["f"])
        for x, y in zip(a["res"], b["res"]):
            assert np.array_equal(x, y)
    with q.Context() as ctx:
        ctx.add(w.net)
        ctx.set_demand(0, w.demand.orig, w.demand.dest, w.demand.trips, w.demand.dt_s)
        ctx.solve(opts)
        with pytest.raises(q.QdtaError) as e:
            ctx.adjoint_record(opts)
        assert e.value.code == q.ESTATE
        with pytest.raises(q.QdtaError) as e:
            ctx.solve(q.default_opts(objective=2))
        assert e.value.code == q.EARG
