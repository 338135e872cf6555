"""The allocation-free line-search entry point (qdta_ls_eval_noalloc), called
through the C ABI, against qdta_ls_eval on the same inputs: bit-identical
exact sums on two calls in a row, the second with a smaller input (fewer
links, fewer instances, fewer step sizes), with no hipMalloc made by the
call; sizes beyond its static scratch are refused."""
from __future__ import annotations

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

FX = 1 << 20


def _pair(m, seed):
    rng = np.random.default_rng(seed)
    f = rng.integers(0, 800 * FX, m).astype(np.int64)
    y = rng.integers(0, 1600 * FX, m).astype(np.int64)
    y[rng.random(m) < 0.3] = 0
    return f, y


def _both(torch, q, ctx, opts, f, y, alphas):
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    K = alphas.shape[-1]
    ni = ctx.layout().n_instances
    ref = torch.full((ni * K * 4,), -7, dtype=torch.int64, device="cuda")
    got = torch.full((ni * K * 4,), -9, dtype=torch.int64, device="cuda")
    ft, yt, at = d(f), d(y), d(alphas)
    ctx.ls_eval(opts, ft, yt, at, ref)
    before = ctx.alloc_count()[0]
    ctx.ls_eval_noalloc(opts, ft, yt, at, got)
    assert ctx.alloc_count()[0] == before
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_line_search_matches_allocating_entry_point():
    import torch
    from paper_2104_12911_amd import qdta as q
    opts = q.default_opts()
    # first call: three uneven instances (two config-2 networks and a grid), K = 32, 900 s interval
    w2 = synth.config2()
    w1 = synth.config1()
    with q.Context() as ctx:
        for net in (w2.net, w1.net, w2.net):
            i = ctx.add(net)
            ctx.set_demand(i, [], [], [], 900.0)
        li = ctx.layout()
        f, y = _pair(int(li.total_links), 1)
        alphas = np.tile(np.linspace(0.0, 1.0, 32), (3, 1))
        alphas[1, 7] = 0.123456789
        ref, got = _both(torch, q, ctx, opts, f, y, alphas)
        assert np.array_equal(ref, got)
        assert (ref != -7).all()
    # second call, smaller: the grid alone, K = 5, static assignment; the
    # scratch still holds the first call's larger sums
    with q.Context() as ctx:
        ctx.add(w1.net)
        ctx.set_demand(0, [], [], [], float("inf"))
        ctx.layout()
        f, y = _pair(w1.net.m, 2)
        alphas = np.array([0.0, 0.25, 0.5, 0.75, 1.0])
        ref, got = _both(torch, q, ctx, opts, f, y, alphas)
        assert np.array_equal(ref, got)
        # the oracle agrees with both
        import oracle
        Co, Do, _ = oracle.ls_eval(f, y, w1.net.fftt, w1.net.cap, 0.15, 4, float("inf"), alphas)
        s = got.reshape(5, 2, 2)
        for k in range(5):
            assert oracle.i128(s[k, 0]) == Co[k] and oracle.i128(s[k, 1]) == Do[k]


def test_noalloc_line_search_refusals():
    import torch
    from paper_2104_12911_amd import qdta as q
    w1 = synth.config1()
    opts = q.default_opts()
    with q.Context() as ctx:
        ctx.add(w1.net)
        ctx.set_demand(0, [], [], [], float("inf"))
        f = torch.zeros(w1.net.m, dtype=torch.int64, device="cuda")
        a = torch.zeros(4, dtype=torch.float64, device="cuda")
        s = torch.zeros(16, dtype=torch.int64, device="cuda")
        with pytest.raises(q.QdtaError) as e:              # not laid out yet
            ctx.ls_eval_noalloc(opts, f, f, a, s)
        assert e.value.code == q.ESTATE
    with q.Context() as ctx:
        for _ in range(65):
            ctx.add(w1.net)
        for i in range(65):
            ctx.set_demand(i, [], [], [], float("inf"))
        ctx.layout()
        f = torch.zeros(65 * w1.net.m, dtype=torch.int64, device="cuda")
        a = torch.zeros(65 * 64, dtype=torch.float64, device="cuda").reshape(65, 64)
        s = torch.zeros(65 * 64 * 4, dtype=torch.int64, device="cuda")
        with pytest.raises(q.QdtaError) as e:              # 65 x 64 sums exceed the scratch
            ctx.ls_eval_noalloc(opts, f, f, a, s)
        assert e.value.code == q.EARG
