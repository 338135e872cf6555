"""Pins of the oracle's reverse-mode derivative of the frozen-path
Frank-Wolfe flows (OD calibration): a two-route network whose step size and
derivatives have a closed form (beta = 1), central finite differences of the
FP64 model on a grid with and without truncation, and the contract replay
against the solver it freezes."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from synth.networks import Network

FX = 1 << 20


def _two_route_net(c0a=60.0, c0b=90.0, capa=900.0, capb=1800.0):
    # 0 -> 1 by link a (uid 0) and link b (uid 1)
    return Network(2, np.array([0, 2, 2], np.int32), np.array([1, 1], np.int32),
                   np.array([c0a, c0b], np.float32), np.array([capa, capb], np.float32))


def _frozen(orc, net, orig, dest, trips, dt_s, iters, **kw):
    from oracle import adjoint as adj
    d_fx = orc.trips_to_fx(trips)
    res = orc.fw_solve(net, orig, dest, d_fx, dt_s=dt_s, fixed_iters=iters, keep_history=True, **kw)
    return res, adj.frozen_paths(net, orig, dest, d_fx, res.hist_cost, dt_s)


def test_two_route_closed_form(orc):
    """Free flow loads link a; the next tree takes b; one update.  With
    beta = 1 the step size solves c_a((1 - x) D) = c_b(x D) in closed form:
    f_b = (c0a - c0b + c0a ka D) / (c0a ka + c0b kb), k = alpha_b kappa / C,
    whose derivatives in D, C_a and C_b are written out by hand here."""
    from oracle import adjoint as adj
    net = _two_route_net()
    D, ab = 6000.0, 0.15
    orig, dest = np.array([0], np.int32), np.array([1], np.int32)
    res, pl = _frozen(orc, net, orig, dest, [D], float("inf"), 1, alpha_b=ab, beta=1)
    assert [list(l) for _, l in pl] == [[0], [1]]
    c0a, c0b = float(net.fftt[0]), float(net.fftt[1])
    ca, cb = float(net.cap[0]), float(net.cap[1])
    ka, kb = ab / ca, ab / cb
    M = c0a * ka + c0b * kb
    N = c0a - c0b + c0a * ka * D
    fb = N / M
    f, st = adj.forward_exact(pl, 2, [D], net.fftt, net.cap, ab, 1, float("inf"))
    assert 0.0 < st[1][2] < 1.0
    assert abs(f[1] - fb) < 1e-9 * D and abs(f[0] - (D - fb)) < 1e-9 * D
    dbar, capbar = adj.backward(st, [0.0, 1.0], pl, net.fftt, net.cap, ab, 1, float("inf"), fixed_point=False)
    dfb_dD = c0a * ka / M
    dfb_dca = (c0a * D * M - N * c0a) / M ** 2 * (-ka / ca)
    dfb_dcb = (-N * c0b / M ** 2) * (-kb / cb)
    assert dbar[0] == pytest.approx(dfb_dD, rel=1e-12)
    assert capbar[0] == pytest.approx(dfb_dca, rel=1e-9)
    assert capbar[1] == pytest.approx(dfb_dcb, rel=1e-9)
    # the library's arithmetic reaches the same point to within its rounding
    ffx, stc = adj.forward_contract(pl, 2, [D], net.fftt, net.cap, ab, 1, float("inf"))
    assert np.array_equal(ffx, res.f)
    assert abs(ffx[1] / FX - fb) < 1e-3
    dbc, cbc = adj.backward(stc, [0.0, 1.0], pl, net.fftt, net.cap, ab, 1, float("inf"))
    assert dbc[0] == pytest.approx(dfb_dD, rel=1e-4)
    assert cbc[0] == pytest.approx(dfb_dca, rel=1e-3)


def _grid_case(dt_s, scale, seed):
    w = synth.config1()
    rng = np.random.default_rng(seed)
    sel = rng.random(w.demand.P) < 0.35
    return w.net, w.demand.orig[sel], w.demand.dest[sel], w.demand.trips[sel] * scale


@pytest.mark.parametrize("dt_s,scale", [(float("inf"), 1.0), (1800.0, 0.5)])
def test_backward_matches_finite_differences(orc, dt_s, scale):
    """Squared count error on 20% of the links; FP64 model with exact step
    sizes; central differences with h = 1e-3 veh on 8 legs and h = 1e-3 C on
    8 capacities against the reverse pass."""
    from oracle import adjoint as adj
    net, o, d, trips = _grid_case(dt_s, scale, 5)
    ab, beta = 0.15, 4
    res, pl = _frozen(orc, net, o, d, trips, dt_s, 4, alpha_b=ab, beta=beta)
    m = net.m
    rng = np.random.default_rng(11)
    obs = rng.random(m) < 0.2
    f0, st = adj.forward_exact(pl, m, trips, net.fftt, net.cap, ab, beta, dt_s)
    assert sum(0.0 < s[2] < 1.0 for s in st[1:]) >= 3
    target = f0 * (1.0 + 0.1 * rng.standard_normal(m))

    def loss(dv, capv):
        f, _ = adj.forward_exact(pl, m, dv, net.fftt, capv, ab, beta, dt_s)
        return float(np.sum((f - target)[obs] ** 2))

    fbar = np.where(obs, 2.0 * (f0 - target), 0.0)
    dbar, capbar = adj.backward(st, fbar, pl, net.fftt, net.cap, ab, beta, dt_s, fixed_point=False)
    cap64 = net.cap.astype(np.float64)
    gscale_d = np.max(np.abs(dbar))
    for p in rng.choice(len(trips), 8, replace=False):
        h = 1e-3
        dp, dm = trips.astype(np.float64).copy(), trips.astype(np.float64).copy()
        dp[p] += h
        dm[p] -= h
        fd = (loss(dp, cap64) - loss(dm, cap64)) / (2 * h)
        assert abs(fd - dbar[p]) < 1e-6 * gscale_d + 1e-6 * abs(fd), (p, fd, dbar[p])
    gscale_c = np.max(np.abs(capbar))
    assert gscale_c > 0
    for a in rng.choice(np.flatnonzero(np.abs(capbar) > 1e-3 * gscale_c), 8, replace=False):
        h = 1e-3 * cap64[a]
        cp, cm = cap64.copy(), cap64.copy()
        cp[a] += h
        cm[a] -= h
        fd = (loss(trips, cp) - loss(trips, cm)) / (2 * h)
        assert abs(fd - capbar[a]) < 1e-5 * gscale_c + 1e-5 * abs(fd), (a, fd, capbar[a])


@pytest.mark.parametrize("dt_s,scale", [(float("inf"), 1.0), (1800.0, 0.5)])
def test_contract_replay_reproduces_solver(orc, dt_s, scale):
    """Replaying the solve with its own demand on the frozen paths gives its
    flows bit for bit; every iterate's incidence loads exactly the AON of
    that iterate's costs, and every path is a chain of links from the
    origin."""
    from oracle import adjoint as adj
    net, o, d, trips = _grid_case(dt_s, scale, 7)
    res, pl = _frozen(orc, net, o, d, trips, dt_s, 5)
    d_fx = orc.trips_to_fx(trips)
    f, st = adj.forward_contract(pl, net.m, trips, net.fftt, net.cap, 0.15, 4, dt_s)
    assert np.array_equal(f, res.f)
    assert [s[2] for s in st[1:]] == list(res.hist_alpha[1:])
    tails = net.tails()
    for j, (ptr, links) in enumerate(pl):
        y, stop, _ = orc.aon(net, res.hist_cost[j], o, d, d_fx, dt_s)
        assert np.array_equal(st[j][1], y)
        for p in range(len(o)):
            seg = links[ptr[p]:ptr[p + 1]]
            u = o[p]
            for e in seg:
                assert tails[e] == u
                u = net.col[e]
            assert u == stop[p]


def test_fixed_steps_backward_is_lambda_weighted_gather(orc):
    """With MSA the step sizes are fixed, the flows are linear in the demand,
    f = sum_j lambda_j L_j d with lambda_j = alpha_j prod_{k>j} (1 - alpha_k)
    and alpha_0 = 1 (the path weights of Alg. 4), and the capacities do not
    enter: the reverse pass must give sum_j lambda_j L_j^T g and zero."""
    from oracle import adjoint as adj
    net, o, d, trips = _grid_case(float("inf"), 1.0, 13)
    res, pl = _frozen(orc, net, o, d, trips, float("inf"), 5, ls_mode=orc.LS_MSA)
    f, st = adj.forward_contract(pl, net.m, trips, net.fftt, net.cap, 0.15, 4, float("inf"), ls_mode=orc.LS_MSA)
    assert np.array_equal(f, res.f)
    alphas = [1.0] + [s[2] for s in st[1:]]
    assert alphas[1:] == [1.0 / (j + 1) for j in range(1, len(alphas))]
    g = np.random.default_rng(2).standard_normal(net.m)
    dbar, capbar = adj.backward(st, g, pl, net.fftt, net.cap, 0.15, 4, float("inf"), fixed_steps=True)
    want = np.zeros(len(trips))
    J = len(alphas) - 1
    for j in range(J + 1):
        lam = alphas[j]
        for k in range(j + 1, J + 1):
            lam *= 1.0 - alphas[k]
        ptr, links = pl[j]
        for p in range(len(trips)):
            want[p] += lam * g[links[ptr[p]:ptr[p + 1]]].sum()
    assert np.allclose(dbar, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())
    assert not np.any(capbar)

