"""Pins of the oracle's link-progress truncation (RULE_PROGRESS).

Section 3 notes that Eq. 2 keeps a trip at its origin whenever the interval
is shorter than the free-flow time of its first link, and suggests tracking
how far a trip got along its link instead.  The PROGRESS rule loads links as
CEIL does (a link entered before dt is loaded) but stops a trip still on a
link at dt at that link's head with the time it still needs to get there;
the next interval starts it with that delay on its clock.
"""
from __future__ import annotations

import numpy as np
import pytest

import synth
from synth.demand import Demand
from synth.networks import Network

FX = 1 << 20


def _long_link_net():
    # 0 -> 1 (720 s) -> 2 (60 s); capacities large and alpha_b = 0 keep the
    # costs at their free-flow values
    return Network(3, np.array([0, 1, 2, 2], np.int32), np.array([1, 2], np.int32),
                   np.array([720.0, 60.0], np.float32), np.array([1e6, 1e6], np.float32))


def _days(n_empty):
    one = Demand(np.array([0], np.int32), np.array([2], np.int32), np.array([1.0]), 300.0)
    empty = Demand(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0), 300.0)
    return [one] + [empty] * n_empty


def test_long_link_crosses_intervals_by_hand(orc):
    """5-minute intervals, a 12-minute first link.  PROGRESS: interval 0
    loads 0->1 and leaves the trip 420 s short of node 1; interval 1 loads
    nothing and leaves it 120 s short; interval 2 reaches node 1 at 120 s,
    loads 1->2 and completes.  CEIL puts the trip at node 1 after interval 0
    (12 minutes of travel in 5) and completes it in interval 1.  FLOOR never
    moves it off node 0: the limitation the paper points out."""
    net = _long_link_net()
    out, left = orc.qdta_day(net, _days(3), alpha_b=0.0, rule=orc.RULE_PROGRESS)
    assert [r["f"].tolist() for r in out] == [[FX, 0], [0, 0], [0, FX], [0, 0]]
    ro, rd, rw, rt = out[0]["res"]
    assert ro.tolist() == [1] and rd.tolist() == [2] and rw.tolist() == [FX] and rt.tolist() == [420.0]
    ro, rd, rw, rt = out[1]["res"]
    assert ro.tolist() == [1] and rt.tolist() == [120.0]
    assert out[2]["res"][0].size == 0 and out[2]["done_fx"] == FX
    out_c, _ = orc.qdta_day(net, _days(3), alpha_b=0.0, rule=orc.RULE_CEIL)
    assert [r["f"].tolist() for r in out_c] == [[FX, 0], [0, FX], [0, 0], [0, 0]]
    out_f, left_f = orc.qdta_day(net, _days(3), alpha_b=0.0, rule=orc.RULE_FLOOR)
    assert all(r["f"].tolist() == [0, 0] for r in out_f)
    assert left_f[0].tolist() == [0] and left_f[2].tolist() == [FX]


def test_progress_equals_ceil_loading_from_nodes(orc):
    """Legs that start at their origin node load exactly the links CEIL loads
    and stop at the same nodes; the delay is the overshoot past dt of the
    arrival at the stop node (0 when a node is reached exactly at dt or the
    leg completes)."""
    w = synth.config1()
    o, d, wfx = orc.demand_legs(w.demand.orig, w.demand.dest, w.demand.trips)
    rng = np.random.default_rng(3)
    cost = (w.net.fftt * rng.uniform(1, 3, w.net.m)).astype(np.float32)
    for dt in (120.0, 300.0, 777.0):
        yc, sc, _ = orc.aon(w.net, cost, o, d, wfx, dt, orc.RULE_CEIL)
        yp, sp, dl, _ = orc.aon(w.net, cost, o, d, wfx, dt, orc.RULE_PROGRESS, want_delay=True)
        assert np.array_equal(yc, yp) and np.array_equal(sc, sp)
        assert (dl >= 0).all() and (dl[sp == d] == 0).all()
        assert (dl > 0).mean() > 0.3


def test_progress_delay_equals_path_time_overshoot(orc):
    """On tiny graphs: walking each leg's tree path by hand in FP32 from its
    carried delay, the stop node and delay are the first node whose arrival
    time exceeds dt and the excess."""
    for seed in range(6):
        rng = np.random.default_rng(40 + seed)
        net = synth.tiny_network(9, 12, rng, costs="float")
        P = 30
        orig = rng.integers(0, 9, P).astype(np.int32)
        dest = rng.integers(0, 9, P).astype(np.int32)
        keep = orig != dest
        orig, dest = orig[keep], dest[keep]
        dfx = np.full(orig.size, FX, np.int64)
        tau0 = rng.uniform(0, 80, orig.size).astype(np.float32)
        tau0[::3] = 0.0
        dt = np.float32(60.0)
        _, stop, dl, _ = orc.aon(net, net.fftt, orig, dest, dfx, float(dt), orc.RULE_PROGRESS, delay=tau0,
                                 want_delay=True)
        for k in range(orig.size):
            D, succ, _ = orc.tree(net, net.fftt, int(dest[k]))
            u, t = int(orig[k]), np.float32(tau0[k])
            exp_s, exp_d = None, np.float32(0)
            if t >= dt:
                exp_s, exp_d = u, np.float32(t - dt)
            while exp_s is None:
                if u == dest[k] or t >= dt:
                    exp_s = u
                    break
                e = int(succ[u])
                t = np.float32(t + net.fftt[e])
                u = int(net.col[e])
                if t > dt:
                    exp_s = u
                    exp_d = np.float32(0) if u == dest[k] else np.float32(t - dt)
            assert stop[k] == exp_s and dl[k] == exp_d, (seed, k)


def test_progress_plain_interval_is_no_truncation(orc):
    w = synth.config1()
    o, d, wfx = orc.demand_legs(w.demand.orig, w.demand.dest, w.demand.trips)
    yn, sn, _ = orc.aon(w.net, w.net.fftt, o, d, wfx, float("inf"), orc.RULE_NONE)
    yp, sp, _ = orc.aon(w.net, w.net.fftt, o, d, wfx, float("inf"), orc.RULE_PROGRESS)
    assert np.array_equal(yn, yp) and np.array_equal(sn, sp) and (sp == d).all()


def test_progress_day_trip_conservation(orc):
    """Demand entering an interval = demand completing in it + residual
    carried out (with its delays), to within one fixed-point unit per
    (iterate, leg); trips in transit on a link longer than the interval are
    carried, not lost."""
    w = synth.config1()
    rng = np.random.default_rng(9)
    days = []
    for i in range(4):
        sel = rng.random(w.demand.P) < 0.3
        days.append(Demand(w.demand.orig[sel], w.demand.dest[sel], w.demand.trips[sel] / 4, 90.0))
    out, left = orc.qdta_day(w.net, days, tol=1e-3, max_iter=30, rule=orc.RULE_PROGRESS)
    in_transit = 0
    for r in out:
        res = int(r["res"][2].sum())
        slack = (r["iters"] + 1) * r["legs"]
        assert abs(r["in_fx"] - (r["done_fx"] + res)) <= slack
        in_transit += int((r["res"][3] > 0).sum())
    assert in_transit > 0


def _quantum(x, pq):
    """pq * ceil(x / pq) in FP64, rounded to FP32 (the delay rounding)."""
    return np.float32(pq * np.ceil(np.float64(x) / pq))


def test_progress_quantum_long_link_by_hand(orc):
    """A 700 s link then a 60 s link, 300 s intervals.  Exact delays: 400 s,
    then 100 s, completion in interval 2.  With delays rounded up to 250 s:
    400 -> 500; interval 1 keeps the trip (500 >= 300) with 200 -> 250;
    interval 2 reaches node 1 at 250 s and completes on the last link.  The
    loads are the same; only the carried delays differ."""
    net = Network(3, np.array([0, 1, 2, 2], np.int32), np.array([1, 2], np.int32),
                  np.array([700.0, 60.0], np.float32), np.array([1e6, 1e6], np.float32))
    for pq, delays in ((0.0, [400.0, 100.0]), (250.0, [500.0, 250.0]), (60.0, [420.0, 120.0])):
        out, _ = orc.qdta_day(net, _days(3), alpha_b=0.0, rule=orc.RULE_PROGRESS, pq=pq)
        assert [r["f"].tolist() for r in out] == [[FX, 0], [0, 0], [0, FX], [0, 0]], pq
        assert [r["res"][3].tolist() for r in out[:2]] == [[delays[0]], [delays[1]]], pq
        assert out[2]["res"][0].size == 0 and out[2]["done_fx"] == FX


def test_progress_quantum_rounds_stop_delays_up(orc):
    """Same trees, same walks: loads and stop nodes do not depend on the
    rounding, and every delay equals the exact one rounded up to a multiple
    of the quantum (at most one quantum above it)."""
    w = synth.config1()
    o, d, wfx = orc.demand_legs(w.demand.orig, w.demand.dest, w.demand.trips)
    rng = np.random.default_rng(5)
    cost = (w.net.fftt * rng.uniform(1, 3, w.net.m)).astype(np.float32)
    tau0 = rng.uniform(0, 500, o.size).astype(np.float32)
    for dt, pq in ((120.0, 30.0), (300.0, 60.0), (777.0, 7.5)):
        y0, s0, d0, _ = orc.aon(w.net, cost, o, d, wfx, dt, orc.RULE_PROGRESS, delay=tau0, want_delay=True)
        y1, s1, d1, _ = orc.aon(w.net, cost, o, d, wfx, dt, orc.RULE_PROGRESS, delay=tau0, want_delay=True, pq=pq)
        assert np.array_equal(y0, y1) and np.array_equal(s0, s1)
        exp = np.array([_quantum(x, pq) if x > 0 else np.float32(0) for x in d0], np.float32)
        assert np.array_equal(d1, exp), (dt, pq)
        assert (d1 >= d0).all() and (d1 - d0 < pq).all() and (d1 % np.float32(pq) == 0).all()


def test_progress_quantum_day_merges_pending_legs(orc):
    """Over a chain of short intervals, rounding the delays lets legs that
    stopped on the same link for the same destination merge: no more pending
    legs than with exact delays, every delay a multiple of the quantum, and
    trips conserved as with exact delays."""
    w = synth.config1()
    rng = np.random.default_rng(9)
    days = []
    for i in range(4):
        sel = rng.random(w.demand.P) < 0.3
        days.append(Demand(w.demand.orig[sel], w.demand.dest[sel], w.demand.trips[sel] / 4, 90.0))
    ex, _ = orc.qdta_day(w.net, days, tol=1e-3, max_iter=30, rule=orc.RULE_PROGRESS)
    qu, _ = orc.qdta_day(w.net, days, tol=1e-3, max_iter=30, rule=orc.RULE_PROGRESS, pq=30.0)
    for a, b in zip(ex, qu):
        assert b["res"][0].size <= a["res"][0].size
        assert (b["res"][3] % np.float32(30.0) == 0).all()
        slack = (b["iters"] + 1) * b["legs"]
        assert abs(b["in_fx"] - (b["done_fx"] + int(b["res"][2].sum()))) <= slack
    assert sum(r["res"][0].size for r in qu) < sum(r["res"][0].size for r in ex)
