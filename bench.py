#!/usr/bin/env python3
"""Throughput of the QDTA hot path on one MI355X.

One step = one Frank-Wolfe iteration of the link-flow form (Alg. 6): BPR link
costs, the all-or-nothing assignment (destination-rooted shortest-path trees,
truncation, loading), the relative-gap test, the K-section line search on the
Beckmann objective and the flow update -- i.e. one AON plus everything around
it.  No stop test ends the run early, so every timed step does the whole
iteration (a fixed iteration count disables every stop test).

Default workload: the 08:00 peak interval of the Bay-Area-shaped synthetic
day (550k nodes, 1.0M links, 5,000 zones) together with the residual demand
the four intervals before it (07:00-08:00) carry into it (Alg. 1, Alg. 4),
as in the full-day run: those intervals are solved first, untimed.

Prints one JSON line (rank 0, N = 1).  The SSSP kernel's duration comes from
HIP events the library records on its own stream.  Its roofline uses the
algorithmic bytes per tree 8n + 8m plus the shared topology once per launch
(every tree counted whole), and, next to it, the bytes of the work the
kernel counted (nodes taken and in-links relaxed: trees stop once their
origins are settled).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "AON assignments/s + GTEPS at 1M links; time to rel. gap 1e-4 vs plain form"
HBM_PEAK_GBS = 8000.0
FX = 1 << 20


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def workload(name):
    import synth
    if name == "config3":
        return synth.config3()
    if name == "config2":
        return synth.config2()
    if name == "config1":
        return synth.config1()
    raise SystemExit(f"unknown workload {name}")


def sssp_bytes_per_tree(n, m):
    """Algorithmic HBM bytes of one destination tree: label init (4n) and
    one label read per settled node (4n), one 4-byte label read and write per
    relaxed in-link (8m).  The reverse topology (source and cost per link,
    offsets per node: 8m + 4n bytes) is shared by every tree of the pass and
    is counted once per launch."""
    return 8.0 * n + 8.0 * m


# kernel instantiation per (sssp_shape, tree_waves): nodes per thread and
# in-links per thread of each relaxation chunk
WG_SHAPES = {1: (1, 2), 2: (1, 4), 3: (2, 4), 4: (4, 4), 5: (2, 2), 6: (4, 2)}
DS_SHAPES = {1: (1, 4), 2: (2, 4), 3: (4, 4), 4: (4, 8), 5: (8, 8), 6: (1, 1)}


BLK_SHAPES = {1: (128, 1), 2: (128, 2), 3: (64, 2), 4: (256, 1)}


WN_SHAPES = {1: (1, 4), 2: (2, 4), 3: (2, 2), 4: (1, 2)}


def sssp_kernel_name(shape, tree_waves, kernel=1):
    if kernel == 2:
        return "k_sssp_blk<%d, %d>" % BLK_SHAPES.get(shape, (128, 2))
    if kernel == 3:
        return "k_sssp_wn<%d, %d>" % WN_SHAPES.get(shape, (2, 4))
    shape = shape if shape in WG_SHAPES else 3
    if kernel == 4:
        # the <2, 4> form is instantiated with registers for 7 wavefronts per
        # SIMD; the trees are complete after the chain fill that follows
        return "k_sssp_wg<%d, %d, true%s> + k_chain_fill" % (WG_SHAPES[shape] + (", 7" if shape == 3 else "",))
    if (tree_waves or 4) == 1:
        return "k_sssp_ds<%d, %d>" % DS_SHAPES[shape]
    return "k_sssp_wg<%d, %d, false>" % WG_SHAPES[shape]


def reduce_traffic(fetch_db, write_db, kernel, calib_mib, out_path, commands, last=0):
    """HBM bytes per launch of `kernel` from two rocprofv3 PMC databases (one
    pass with FETCH_SIZE, one with WRITE_SIZE, both in KiB per dispatch),
    each scaled by what the counter reads for the calibration add kernel
    (reads and writes calib_mib MiB once, run by --copy-calib-mib).  last > 0:
    only the kernel's last `last` dispatches (the timed steps of the peak
    interval; earlier ones belong to the carried-in intervals).  A kernel
    named "A + B" is the sum of one launch of each."""
    import sqlite3

    def per_dispatch(db, counter):
        con = sqlite3.connect(db)
        rows = con.execute("select dispatch_id, name, counter_name, counter_value from pmc_events").fetchall()
        con.close()
        acc, names = {}, {}
        for did, name, cn, cv in rows:
            if cn == counter:
                acc[did] = acc.get(did, 0.0) + float(cv)
                names[did] = name
        return acc, names

    out = {"kernel": kernel, "calibration": {"kernel": f"torch.add of a {calib_mib} MiB float32 tensor (reads and "
                                                        f"writes {calib_mib} MiB once)"}}
    parts = [k.strip() for k in kernel.split(" + ")]
    for key, db, counter in (("fetch", fetch_db, "FETCH_SIZE"), ("write", write_db, "WRITE_SIZE")):
        acc, names = per_dispatch(db, counter)
        adds = [acc[d] for d in acc if "add" in names[d].lower() and "elementwise" in names[d].lower()]
        per_launch, launches = 0.0, []
        for part in parts:
            ks = [acc[d] for d in sorted(acc) if part in names[d]]
            if last > 0:
                ks = ks[-last:]
            if not ks:
                raise SystemExit(f"{db}: no dispatch of {part}")
            per_launch += sum(ks) / len(ks)
            launches.append(len(ks))
        if not adds:
            raise SystemExit(f"{db}: no dispatch of the calibration kernel")
        cal = max(adds)
        scale = (calib_mib * 1024.0) / cal
        out[f"{key}_kib_per_launch"] = per_launch
        out[f"{key}_launches"] = launches[0] if len(launches) == 1 else launches
        out["calibration"][f"{key}_kib"] = cal
        out["calibration"][f"{key}_scale"] = scale
    out["bytes_per_launch"] = 1024.0 * (out["fetch_kib_per_launch"] * out["calibration"]["fetch_scale"] +
                                        out["write_kib_per_launch"] * out["calibration"]["write_scale"])
    src = open(os.path.join(ROOT, "paper_2104_12911_amd", "csrc", "qdta_kernels.hip"), "rb").read()
    out["kernel_sha256"] = hashlib.sha256(src).hexdigest()
    out["commands"] = commands
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def trace_summary(db, kernel, last):
    """Markdown summary of a rocprofv3 --kernel-trace database: every kernel's
    calls, total and mean duration and share of GPU time, then the mean
    duration of `kernel`'s last `last` dispatches (the timed steps); for a
    kernel named "A + B", of each part and their sum."""
    import sqlite3
    con = sqlite3.connect(db)
    rows = con.execute("select name, dispatch_id, duration from kernels").fetchall()
    con.close()
    per = {}
    for name, did, dur in rows:
        short = name.split("(")[0].replace("void ", "")
        per.setdefault(short, []).append((did, dur))
    total = sum(d for _, _, d in rows)
    lines = ["| kernel | calls | total ms | mean ms | share of GPU time |", "|---|---|---|---|---|"]
    for short, v in sorted(per.items(), key=lambda kv: -sum(d for _, d in kv[1]))[:12]:
        t = sum(d for _, d in v)
        lines.append(f"| `{short}` | {len(v)} | {t / 1e6:.1f} | {t / len(v) / 1e6:.3f} | {100.0 * t / total:.1f}% |")
    lines.append("")
    mean_sum = 0.0
    parts = [k.strip() for k in kernel.split(" + ")]
    for part in parts:
        ks = sorted(v for short, vv in per.items() if part in short for v in vv)
        tail = [d for _, d in ks[-last:]] if last > 0 else [d for _, d in ks]
        mean_sum += sum(tail) / max(len(tail), 1)
        lines.append(f"`{part}`, last {len(tail)} dispatches (the timed steps): mean "
                     f"{sum(tail) / max(len(tail), 1) / 1e6:.2f} ms, min {min(tail) / 1e6:.2f}, "
                     f"max {max(tail) / 1e6:.2f}")
    if len(parts) > 1:
        lines.append(f"`{kernel}`: mean {mean_sum / 1e6:.2f} ms per launch of both")
    return "\n".join(lines)


def traffic_entry(kernel_src_hash, kernel):
    """HBM bytes per SSSP launch from the rocprofv3 PMC runs, if they were
    taken on the current kernel source and the same instantiation."""
    path = os.path.join(ROOT, "profiles", "sssp_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256") != kernel_src_hash or t.get("kernel") != kernel:
        return None
    return t.get("bytes_per_launch")


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(net, legs, f_fx, dt_s, alpha_b, beta, nthreads):
    """The oracle as it stands, timed on one whole Frank-Wolfe step of the
    same workload at the same iterate as the GPU's timed steps: BPR costs of
    f, the all-or-nothing assignment of every leg (all 5,000 trees, no
    sampling), the exact gap sums, the K-section line search (3 passes of
    32 step sizes over all links) and the update."""
    import oracle
    o, d, w = legs
    t0 = time.perf_counter()
    cost, _ = oracle.bpr(f_fx, net.fftt, net.cap, alpha_b, beta, dt_s)
    t1 = time.perf_counter()
    y, _, _ = oracle.aon(net, cost, o, d, w, dt_s, oracle.RULE_CEIL, nthreads=nthreads)
    t2 = time.perf_counter()
    oracle.sum_cx(cost, f_fx)
    oracle.sum_cx(cost, y)
    alpha, _, _ = oracle.line_search(f_fx, y, net.fftt, net.cap, alpha_b, beta, dt_s, 1)
    oracle.fw_update(f_fx, y, alpha)
    t3 = time.perf_counter()
    step = t3 - t0
    return {"value": 1.0 / step, "unit": "AON/s", "cores": nthreads, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"one whole FW step at the GPU's last timed iterate: BPR over {net.m} links ({t1 - t0:.2f} s), "
                      f"AON of all {len(o)} legs over all trees ({t2 - t1:.1f} s, {nthreads} threads), exact gap "
                      f"sums, K-section line search 3 x 32 and update ({t3 - t2:.2f} s); not extrapolated"}


def _ctx_for(qdta, stream, pairs):
    ctx = qdta.Context(0, stream)
    for net, dem in pairs:
        i = ctx.add(net)
        ctx.set_demand(i, dem.orig, dem.dest, dem.trips, dem.dt_s)
    return ctx


def _solve_timed(torch, ctx, opts):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, rc = ctx.solve(opts)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, st


def batched_vs_plain(torch, qdta, warm_iters=3):
    """Config 2 (255,754 links, 1,000 destinations, one congested 900 s
    interval): one FW iteration in the batched form (every tree in one
    launch, all step sizes in one pass, the iteration replayed as a HIP
    graph) against the plain form (one launch per destination tree and per
    step size), both timed at the same iterate after `warm_iters` updates.
    The two forms give bit-identical iterates."""
    w = workload("config2")
    stream = torch.cuda.current_stream()
    ctx = _ctx_for(qdta, stream, [(w.net, w.demand)])
    per = {}
    for form in (0, 2):
        o = qdta.default_opts(fixed_iters=1 << 30, launch_form=form)
        ctx.fw_begin(o)
        for _ in range(warm_iters):
            ctx.fw_step(qdta.default_opts(fixed_iters=1 << 30))
        n = 3
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            ctx.fw_step(o)
        torch.cuda.synchronize()
        per[form] = (time.perf_counter() - t0) / n
        log(f"config2 form {form}: {per[form] * 1e3:.1f} ms per FW iteration")
    ctx.close()
    return {"workload": f"config2: {w.net.n} nodes, {w.net.m} links, 1000 destinations, {w.demand.P} legs, dt 900 s",
            "batched_iter_ms": per[0] * 1e3, "plain_iter_ms": per[2] * 1e3, "speedup": per[2] / per[0],
            "iterate": f"FW iteration {warm_iters + 1} (congested)"}


def mode_plain(args, torch, qdta):
    """M3 on config 2: per-iteration time of the batched form (every tree in
    one launch, all step sizes in one pass, iteration replayed as a HIP graph)
    against the plain form (one launch per destination tree and per step
    size).  Both give bit-identical iterates, so they take the same number of
    iterations to any gap; time to gap = iterations x per-iteration time."""
    w = workload("config2")
    stream = torch.cuda.current_stream()
    ctx = _ctx_for(qdta, stream, [(w.net, w.demand)])
    out = {"mode": "plain", "workload": "config2"}
    opts_b = qdta.default_opts(tol=args.tol, max_iter=args.steps)
    if not args.no_autotune:
        # tuned under congested costs: a few iterations first (untimed)
        ctx.fw_begin(opts_b)
        for _ in range(3):
            ctx.fw_step(opts_b)
        opts_b, best = ctx.autotune(opts_b, 2000.0)
        log(f"autotune: sssp_shape={opts_b.sssp_shape} delta_scale={opts_b.delta_scale} "
            f"tree_waves={opts_b.tree_waves} ({best:.1f} ms)")
        out["autotuned"] = {"sssp_shape": opts_b.sssp_shape, "delta_scale": opts_b.delta_scale,
                            "tree_waves": opts_b.tree_waves}
    # the batched solve, step by step so that long runs report progress
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.fw_begin(opts_b)
    live, k = True, 0
    while live:
        st, live = ctx.fw_step(opts_b)
        k += 1
        if k % 1000 == 0:
            log(f"batched solve: {k} steps, gap {st[0]['gap']:.3e}, {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    out.update(tol=args.tol, batched_solve_s=t_solve, iterations=st[0]["iters"], gap=st[0]["gap"],
               stopped_by=st[0]["stopped_by"])
    log(f"batched solve: {t_solve:.2f} s, {st[0]['iters']} iterations, gap {st[0]['gap']:.3e}, "
        f"stopped_by {st[0]['stopped_by']}")
    per = {}
    for form in (0, 2):
        o = qdta.default_opts(fixed_iters=1 << 30, launch_form=form, sssp_shape=opts_b.sssp_shape,
                              delta_scale=opts_b.delta_scale, tree_waves=opts_b.tree_waves)
        ctx.fw_begin(o)
        ctx.fw_step(o)
        torch.cuda.synchronize()
        n = 3
        t0 = time.perf_counter()
        for _ in range(n):
            ctx.fw_step(o)
        torch.cuda.synchronize()
        per[form] = (time.perf_counter() - t0) / n
        log(f"form {form}: {per[form] * 1e3:.1f} ms per FW iteration")
    out.update(batched_iter_ms=per[0] * 1e3, plain_iter_ms=per[2] * 1e3, speedup=per[2] / per[0],
               plain_time_to_gap_s_extrapolated=per[2] * max(st[0]["iters"] + 1, 1))
    ctx.close()
    print(json.dumps(out), flush=True)


def mode_batch(args, torch, qdta):
    """Config 4: 64 uneven grids advanced together (one launch sequence and
    one HIP graph per FW iteration for all of them) against the same grids
    solved one after another.  Both run the same fixed number of iterations
    (the iterates are bit-identical, so the work is the same)."""
    import synth
    insts = synth.config4()
    stream = torch.cuda.current_stream()
    iters = args.steps
    opts = qdta.default_opts(fixed_iters=iters)
    ctx = _ctx_for(qdta, stream, [(x.net, x.demand) for x in insts])
    li = ctx.layout()
    log(f"config4: {len(insts)} instances, {li.total_links} links, {li.total_dests} destinations, {li.total_legs} legs")
    _solve_timed(torch, ctx, qdta.default_opts(fixed_iters=1))
    if not args.no_autotune:
        # kernel shape, bucket width, and walks or merged paths for the loading
        # (every grid is a plain static assignment), under the costs of the
        # iterate just solved; both forms use the result
        opts, best = ctx.autotune(opts, 2000.0)
        log(f"autotune: sssp_shape={opts.sssp_shape} delta_scale={opts.delta_scale} tree_waves={opts.tree_waves} "
            f"load_form={opts.load_form} ({best:.1f} ms)")
    ctx.profile(True)
    t_b, st_b = _solve_timed(torch, ctx, opts)
    prof = ctx.profile_read()
    # per-phase times of an iteration: three more with direct launches, timed per phase
    od = qdta.default_opts(fixed_iters=3, launch_form=1, sssp_shape=opts.sssp_shape, delta_scale=opts.delta_scale,
                           tree_waves=opts.tree_waves, load_form=opts.load_form)
    ctx.profile(True)
    _solve_timed(torch, ctx, od)
    pd = ctx.profile_read()
    ctx.profile(False)
    phase_iter = {k: round(v[0] / v[1], 2) for k, v in pd.items() if k != "sssp_work" and v[1]}
    log(f"phases per launch (ms), direct launches: {json.dumps(phase_iter)}")
    ctx.close()
    log(f"batched: {t_b:.2f} s for {iters} iterations; phases {json.dumps({k: round(v[0], 1) for k, v in prof.items()})}")
    t_s = 0.0
    for i, x in enumerate(insts):
        c1 = _ctx_for(qdta, stream, [(x.net, x.demand)])
        _solve_timed(torch, c1, qdta.default_opts(fixed_iters=1))
        t, st = _solve_timed(torch, c1, opts)
        t_s += t
        c1.close()
        log(f"sequential instance {i}: {t:.3f} s (total {t_s:.2f} s)")
    print(json.dumps({"mode": "batch", "workload": "config4", "instances": len(insts),
                      "load_form": {0: "walk", 1: "walk", 2: "merged paths"}[opts.load_form],
                      "links": int(li.total_links), "destinations": int(li.total_dests), "legs": int(li.total_legs),
                      "iterations": iters, "batched_s": t_b, "sequential_s": t_s, "speedup": t_s / t_b,
                      "gap_max_batched": max(s["gap"] for s in st_b),
                      "gap_median_batched": float(np.median([s["gap"] for s in st_b])),
                      "phase_ms_per_launch": phase_iter}), flush=True)


def mode_day(args, torch, qdta):
    """Full-day QDTA (Alg. 1): for each 15-min interval, d(i) = d^o(i) +
    d^r(i), Frank-Wolfe to relative gap 1e-4 (or stall / cap), then the
    residual demand of Alg. 4 carried into the next interval."""
    import synth
    w = synth.config3_day(args.scale)
    net = w.net
    days = w.demand[:args.intervals]
    stream = torch.cuda.current_stream()
    ctx = qdta.Context(0, stream)
    ctx.add(net)
    stop = qdta.STOP_OBJ if args.stop == "obj" else qdta.STOP_GAP
    ls_mode = {"ksection": qdta.LS_KSECTION, "qn": qdta.LS_QN, "msa": qdta.LS_MSA}[args.ls]
    trunc = {"ceil": qdta.RULE_CEIL, "floor": qdta.RULE_FLOOR, "progress": qdta.RULE_PROGRESS}[args.trunc]
    opts = qdta.default_opts(stop_rule=stop, tol=args.tol, max_iter=args.steps, keep_history=1, trunc_rule=trunc,
                             progress_quantum_s=args.progress_quantum,
                             launch_form=1 if args.profile_day else 0, tree_waves=args.tree_waves,
                             waves_per_cu=args.waves_per_cu, delta_scale=args.delta_scale, ls_mode=ls_mode,
                             objective=qdta.OBJ_SO if args.objective == "so" else qdta.OBJ_UE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, seg_s, gaps, stops, tot_trips, carried = [], [], [], [], 0.0, 0
    split = {"set_demand": 0.0, "solve": 0.0, "advance": 0.0, "residual_out": 0.0}
    if args.profile_day:
        ctx.profile(True)
    for i, dem in enumerate(days):
        ta = time.perf_counter()
        ctx.set_demand(0, dem.orig, dem.dest, dem.trips, dem.dt_s)
        tot_trips += dem.total()
        legs = ctx.layout().total_legs
        tb = time.perf_counter()
        if legs == 0:
            iters.append(0)
            seg_s.append(0.0)
            gaps.append(0.0)
            stops.append(-1)
            continue
        st, rc = ctx.solve(opts)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        ctx.advance_interval(opts)
        torch.cuda.synchronize()
        td = time.perf_counter()
        ro, rd, rw, done = ctx.residual(0)
        te = time.perf_counter()
        for k, v in zip(split, (tb - ta, tc - tb, td - tc, te - td)):
            split[k] += v
        iters.append(st[0]["iters"])
        seg_s.append(te - ta)
        gaps.append(st[0]["gap"])
        stops.append(st[0]["stopped_by"])
        carried = int(rw.sum())
        log(f"interval {i}: legs {legs} iters {st[0]['iters']} gap {st[0]['gap']:.2e} "
            f"stop {st[0]['stopped_by']} residual legs {ro.size} ({carried / FX:.0f} trips); "
            f"set {tb - ta:.2f} s solve {tc - tb:.2f} s advance {td - tc:.2f} s")
    if args.profile_day:
        prof = ctx.profile_read()
        log("phases (ms, count): " + json.dumps({k: [round(v[0], 1), v[1]] for k, v in prof.items()}))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.close()
    print(json.dumps({"mode": "day", "workload": f"config3 day, scale {args.scale}", "nodes": net.n, "links": net.m,
                      "intervals": len(days), "trips": tot_trips, "wall_s": wall, "fw_iterations": sum(iters),
                      "stop_rule": args.stop, "tol": args.tol, "line_search": args.ls, "objective": args.objective,
                      "truncation": args.trunc,
                      "progress_quantum_s": args.progress_quantum if args.trunc == "progress" else None,
                      "intervals_stopped_by": {k: stops.count(v) for k, v in
                                               (("gap", 1), ("objective_change", 2), ("stall", 3), ("cap", 0))},
                      "max_abs_gap": max((abs(g) for g in gaps), default=0.0),
                      "tree_waves": opts.tree_waves or 4,
                      "delta_scale": opts.delta_scale or 10.0, "left_after_last_trips": carried / FX,
                      "split_s": {k: round(v, 3) for k, v in split.items()},
                      "iters_per_interval": iters, "seconds_per_interval": [round(x, 3) for x in seg_s],
                      "gap_per_interval": [float("%.3g" % g) for g in gaps],
                      "stopped_by_per_interval": stops}), flush=True)


def mode_calib(args, torch, qdta):
    """OD calibration against link counts at the config-3 peak interval (the
    derivative pattern; not in the paper).  The interval is solved (FW to
    relative gap 1e-4, at most --calib-iters updates) and its iterations are
    frozen (qdta_adjoint_record).  Synthetic counts: the solved flows on 2% of
    the links with 10% Gaussian noise.  The demand starts from a lognormal
    perturbation of the truth; Adam runs --calib-steps steps on the squared
    count error, each one frozen-path forward replay and one reverse pass
    (the adjoint kernels) through torch.autograd.  Central differences
    (h = 2^-10 veh, about 1e-3 and a whole number of fixed-point units) on a
    few legs check the gradient at full size.  --calib-dt replaces the
    interval's 900 s horizon (0 keeps it; inf gives the static assignment of
    the same demand, whose step sizes stay inside (0, 1))."""
    import synth
    w = synth.config3()
    net, dem = w.net, w.demand
    stream = torch.cuda.current_stream()
    ctx = qdta.Context(0, stream)
    ctx.add(net)
    dt_s = args.calib_dt if args.calib_dt else dem.dt_s
    ctx.set_demand(0, dem.orig, dem.dest, dem.trips, dt_s)
    opts = qdta.default_opts(alpha=w.alpha, beta=w.beta, tol=1e-4, max_iter=args.calib_iters, keep_history=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, rc = ctx.solve(opts)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    log(f"solve (dt {dt_s:g} s): {st[0]['iters']} updates, gap {st[0]['gap']:.3e}, stopped_by "
        f"{st[0]['stopped_by']}, {t_solve:.2f} s")
    t0 = time.perf_counter()
    ctx.adjoint_record(opts)
    t_rec = time.perf_counter() - t0
    log(f"paths recorded for {st[0]['iters'] + 1} iterates in {t_rec:.2f} s")
    o, d, wfx = ctx.legs()
    m, P = net.m, len(o)
    d_true = torch.tensor(wfx / FX, dtype=torch.float64, device="cuda")
    f_true = torch.empty(m, dtype=torch.float64, device="cuda")
    ctx.model_forward(opts, d_true, None, f_true)
    rng = np.random.default_rng(2104129115)
    obs = torch.tensor(np.sort(rng.choice(m, int(0.02 * m), replace=False)), device="cuda")
    counts = f_true[obs] * torch.tensor(1.0 + 0.1 * rng.standard_normal(obs.numel()), device="cuda")
    d_start = d_true * torch.tensor(np.exp(0.5 * rng.standard_normal(P)), device="cuda")
    dp = d_start.clone().requires_grad_(True)
    cap = torch.tensor(net.cap, device="cuda").requires_grad_(True)
    optim = torch.optim.Adam([dp], lr=args.calib_lr)

    def loss_of(f):
        return ((f[obs] - counts) ** 2).sum()

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    losses, fwd_ms, bwd_ms = [], 0.0, 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.calib_steps):
        optim.zero_grad()
        ev[0].record()
        f = qdta.frozen_path_flows(ctx, opts, dp, cap)
        loss = loss_of(f)
        ev[1].record()
        loss.backward()
        ev[2].record()
        optim.step()
        with torch.no_grad():
            dp.clamp_(min=0.0)
        ev[2].synchronize()
        fwd_ms += ev[0].elapsed_time(ev[1])
        bwd_ms += ev[1].elapsed_time(ev[2])
        losses.append(float(loss))
        if k % 20 == 0 or k == args.calib_steps - 1:
            log(f"adam step {k}: loss {losses[-1]:.6e}")
    torch.cuda.synchronize()
    t_adam = time.perf_counter() - t0
    n = max(args.calib_steps, 1)
    gcap = float(cap.grad.abs().max()) if cap.grad is not None else 0.0
    # central differences of the full-size model at the final demand
    dfin = dp.detach().clone()
    fo = torch.empty(m, dtype=torch.float64, device="cuda")

    def loss_at(dv):
        ctx.model_forward(opts, dv, None, fo)
        return float(loss_of(fo))

    g = torch.empty(P, dtype=torch.float64, device="cuda")
    capbar = torch.empty(m, dtype=torch.float64, device="cuda")
    fid = ctx.model_forward(opts, dfin, None, fo)
    fbar = torch.zeros(m, dtype=torch.float64, device="cuda")
    fbar[obs] = 2.0 * (fo[obs] - counts)
    ctx.model_backward(fid, fbar, g, capbar)
    gh = g.cpu().numpy()
    fd_err = []
    for l in np.argsort(-np.abs(gh))[:4]:
        h = 2.0 ** -10
        e = torch.zeros(P, dtype=torch.float64, device="cuda")
        e[int(l)] = h
        fd = (loss_at(dfin + e) - loss_at(dfin - e)) / (2 * h)
        fd_err.append(abs(fd - gh[l]) / max(abs(gh[l]), 1e-300))
        log(f"leg {int(l)}: adjoint {gh[l]:.6e}, central difference {fd:.6e}")
    dt_h = d_true.cpu().numpy()
    out = {"mode": "calib", "workload": f"config3 peak interval: {net.n} nodes, {m} links, {P} legs, dt {dt_s:g} s",
           "observed_links": int(obs.numel()), "fw_updates": st[0]["iters"], "solve_s": t_solve, "record_s": t_rec,
           "adam_steps": args.calib_steps, "lr": args.calib_lr, "step_ms": t_adam / n * 1e3,
           "forward_ms": fwd_ms / n, "backward_ms": bwd_ms / n, "loss_first": losses[0] if losses else None,
           "loss_last": losses[-1] if losses else None,
           "demand_rmse_start": float(np.sqrt(np.mean((d_start.cpu().numpy() - dt_h) ** 2))),
           "demand_rmse_end": float(np.sqrt(np.mean((dfin.cpu().numpy() - dt_h) ** 2))),
           "cap_grad_max_abs": gcap, "fd_rel_err_max": max(fd_err) if fd_err else None}
    ctx.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10,
                    help="aon: timed FW iterations; day: FW iteration cap per interval (use 200); "
                         "plain: cap of the batched solve; batch: fixed iterations")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--delta-scale", type=float, default=0.0, help="bucket width / mean link cost (0: library default)")
    ap.add_argument("--waves-per-cu", type=int, default=0, help="wavefronts in flight per CU (0: library default)")
    ap.add_argument("--tree-waves", type=int, default=0, help="wavefronts per tree, 1 or 4 (0: library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the batched-vs-plain record on config 2")
    ap.add_argument("--carry", type=int, default=4,
                    help="aon: earlier intervals solved first to carry their residual into the peak interval")
    ap.add_argument("--sssp-kernel", type=int, default=0, help="shortest-path kernel (0 library default, 1 node "
                                                               "queue, 2 block-local, 3 node per thread, 4 node "
                                                               "queue over the chain-contracted search)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="also run a plain device copy of this size (MiB) once, for counter calibration")
    ap.add_argument("--no-autotune", action="store_true", help="skip the kernel-shape / bucket-width autotuner")
    ap.add_argument("--reduce-traffic", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="write profiles/sssp_traffic.json from two rocprofv3 --pmc databases (FETCH_SIZE, "
                         "WRITE_SIZE) of runs made with --copy-calib-mib, and exit")
    ap.add_argument("--traffic-kernel", default="k_sssp_wg<2, 4, true, 7> + k_chain_fill",
                    help="kernel instantiation the traffic reduction averages")
    ap.add_argument("--traffic-commands", default="", help="the rocprofv3 commands, ' ;; '-separated, recorded")
    ap.add_argument("--traffic-out", default=os.path.join(ROOT, "profiles", "sssp_traffic.json"))
    ap.add_argument("--traffic-last", type=int, default=0,
                    help="only the kernel's last N dispatches (the timed steps: 2 x --steps of the profiled run)")
    ap.add_argument("--summarize-trace", metavar="DB",
                    help="print a markdown summary of a rocprofv3 --kernel-trace database and exit")
    ap.add_argument("--mode", default="aon", choices=["aon", "plain", "batch", "day", "calib"],
                    help="aon: the headline AON/s line; plain: batched vs per-destination launches (config 2); "
                         "batch: 64 uneven instances together vs one after another (config 4); day: full-day QDTA; "
                         "calib: OD calibration against link counts (Adam through the adjoint)")
    ap.add_argument("--calib-steps", type=int, default=200, help="calib mode: Adam steps")
    ap.add_argument("--calib-iters", type=int, default=40, help="calib mode: cap on the solve's FW updates")
    ap.add_argument("--calib-lr", type=float, default=0.02, help="calib mode: Adam learning rate (veh per leg)")
    ap.add_argument("--calib-dt", type=float, default=0.0,
                    help="calib mode: horizon in s (0: the interval's 900 s; inf: static assignment)")
    ap.add_argument("--scale", type=float, default=1.0, help="day mode: network/demand scale (1 = 1.0M links)")
    ap.add_argument("--intervals", type=int, default=96, help="day mode: number of 15-min intervals")
    ap.add_argument("--profile-day", action="store_true", help="day mode: per-phase event timing (direct launches)")
    ap.add_argument("--stop", default="obj", choices=["obj", "gap"],
                    help="day mode: stop rule, objective change (Eq. 7) or relative gap, both at 1e-4")
    ap.add_argument("--objective", default="ue", choices=["ue", "so"],
                    help="day mode: user equilibrium (the paper's) or system optimum (marginal-cost routing)")
    ap.add_argument("--ls", default="ksection", choices=["ksection", "qn", "msa"],
                    help="day mode: step rule (K-section line search, quasi-Newton of Alg. 8, or MSA)")
    ap.add_argument("--tol", type=float, default=1e-4, help="day and plain modes: stop tolerance")
    ap.add_argument("--trunc", default="ceil", choices=["ceil", "floor", "progress"],
                    help="day mode: truncation rule (Eq. 2 read as CEIL or FLOOR, or link progress)")
    ap.add_argument("--progress-quantum", type=float, default=60.0,
                    help="day mode, link progress: delays rounded up to multiples of this many seconds (0 exact)")
    args = ap.parse_args()
    if args.reduce_traffic:
        out = reduce_traffic(args.reduce_traffic[0], args.reduce_traffic[1], args.traffic_kernel,
                             args.copy_calib_mib or 1024, args.traffic_out,
                             [c.strip() for c in args.traffic_commands.split(";;") if c.strip()], args.traffic_last)
        print(json.dumps(out))
        return
    if args.summarize_trace:
        print(trace_summary(args.summarize_trace, args.traffic_kernel, args.traffic_last))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2104_12911_amd import qdta

    if args.mode != "aon":
        {"plain": mode_plain, "batch": mode_batch, "day": mode_day, "calib": mode_calib}[args.mode](args, torch, qdta)
        return

    import synth
    first = synth.configs.PEAK_INTERVAL - args.carry
    log(f"generating config3 intervals {first}..{synth.configs.PEAK_INTERVAL}")
    w = synth.config3_window(first)
    net, days = w.net, w.demand
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    ctx = qdta.Context(0, stream)
    ctx.add(net)
    kern = dict(sssp_kernel=args.sssp_kernel)
    # the intervals before the peak, solved as in the full day, carry their
    # residual demand into it (untimed)
    day_opts = qdta.default_opts(alpha=w.alpha, beta=w.beta, stop_rule=qdta.STOP_OBJ, tol=1e-4, max_iter=200,
                                 keep_history=1, **kern)
    for dem in days[:-1]:
        ctx.set_demand(0, dem.orig, dem.dest, dem.trips, dem.dt_s)
        st, _ = ctx.solve(day_opts)
        ctx.advance_interval(day_opts)
        log(f"carry-in interval: {dem.P} legs, {st[0]['iters']} FW updates, stop {st[0]['stopped_by']}")
    ro, rd, rw, _ = ctx.residual(0)
    dem = days[-1]
    ctx.set_demand(0, dem.orig, dem.dest, dem.trips, dem.dt_s)
    li = ctx.layout()
    Q, P = int(li.total_dests), int(li.total_legs)
    log(f"peak interval: {dem.P} original legs + {ro.size} residual legs ({rw.sum() / FX:.0f} trips) -> {P} legs")
    opts = qdta.default_opts(alpha=w.alpha, beta=w.beta, fixed_iters=1 << 30, delta_scale=args.delta_scale,
                             waves_per_cu=args.waves_per_cu, tree_waves=args.tree_waves, **kern)
    t0 = time.perf_counter()
    ctx.fw_begin(opts)
    log(f"initial AON {time.perf_counter() - t0:.3f} s")
    for i in range(args.warmup):
        st, live = ctx.fw_step(opts)
        log(f"warmup {i + 1}/{args.warmup}: gap={st[0]['gap']:.4e} alpha={st[0]['last_alpha']:.4f}")
    if not args.no_autotune and not args.delta_scale:
        # trials under the costs of the current (congested) iterate, then one
        # more untimed step so that the timed ones replay the tuned graph
        opts, best = ctx.autotune(opts, 2000.0)
        log(f"autotune: kernel={opts.sssp_kernel} sssp_shape={opts.sssp_shape} delta_scale={opts.delta_scale} "
            f"tree_waves={opts.tree_waves} ({best:.1f} ms)")
        st, live = ctx.fw_step(opts)
        log(f"warmup after autotune: gap={st[0]['gap']:.4e} alpha={st[0]['last_alpha']:.4f}")
    if args.copy_calib_mib:
        # a streaming kernel of known size (reads and writes N bytes once) to
        # scale the HBM counters
        a = torch.ones(args.copy_calib_mib << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.add(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gaps, alphas = [], []
    for i in range(args.steps):
        st, live = ctx.fw_step(opts)
        gaps.append(st[0]["gap"])
        alphas.append(st[0]["last_alpha"])
        log(f"step {i + 1}/{args.steps}: gap={st[0]['gap']:.4e} alpha={st[0]['last_alpha']:.4f}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile(False)
    f_now = torch.empty(net.m, dtype=torch.int64, device="cuda")
    ctx.get_flows(f_now)
    f_host = f_now.cpu().numpy()

    ms_step = elapsed / args.steps * 1e3
    kernel_timing = "HIP events around the kernel, timed steps"
    work_nodes, work_links = prof["sssp_work"]
    if prof["sssp"][1] == 0:
        # the timed steps replayed a HIP graph, whose kernels carry no events:
        # time the same number of steps once more launched directly (same
        # kernels and inputs; only the launch path differs)
        kernel_timing = "HIP events around direct launches of the same number of steps, after the timed graph replays"
        od = qdta.default_opts(alpha=w.alpha, beta=w.beta, fixed_iters=1 << 30, delta_scale=opts.delta_scale,
                               sssp_shape=opts.sssp_shape, waves_per_cu=opts.waves_per_cu,
                               tree_waves=opts.tree_waves, sssp_kernel=opts.sssp_kernel, launch_form=1)
        ctx.profile(True)
        for _ in range(args.steps):
            ctx.fw_step(od)
        prof_d = ctx.profile_read()
        ctx.profile(False)
        prof["sssp"] = prof_d["sssp"]
        prof["walk"] = prof_d["walk"]
        prof["fill"] = prof_d["fill"]
    sssp_ms, sssp_n = prof["sssp"]
    sssp_avg_s = sssp_ms / max(sssp_n, 1) / 1e3
    # the contracted search's trees are complete after the chain fill
    fill_ms, fill_n = prof["fill"]
    if fill_n > 0:
        sssp_avg_s += fill_ms / fill_n / 1e3
    bytes_launch = Q * sssp_bytes_per_tree(net.n, net.m) + 8.0 * net.m + 4.0 * net.n
    achieved = bytes_launch / sssp_avg_s / 1e9
    # the work the kernel counted over the timed steps: per launch, 8 bytes
    # per node taken (label written and read) and per in-link relaxed
    # (label read and written), plus the shared topology once
    n_launch = max(args.steps, 1)
    touched = (8.0 * work_nodes + 8.0 * work_links) / n_launch + 8.0 * net.m + 4.0 * net.n
    src = open(os.path.join(ROOT, "paper_2104_12911_amd", "csrc", "qdta_kernels.hip"), "rb").read()
    kname = sssp_kernel_name(opts.sssp_shape, opts.tree_waves,
                             opts.sssp_kernel or (1 if opts.tree_waves == 1 else 4))
    traffic = traffic_entry(hashlib.sha256(src).hexdigest(), kname)
    result = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "AON/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"config3 08:00 peak interval with the residual carried from {args.carry} earlier "
                               f"intervals: {net.n} nodes, {net.m} links, {Q} destinations, {P} legs "
                               f"({dem.P} original + {ro.size} residual), dt {dem.dt_s:g} s",
                   "sssp_kernel": kname, "delta_scale": opts.delta_scale or 10.0,
                   "waves_per_cu": opts.waves_per_cu or (32 if opts.tree_waves == 1 else 28),
                   "line_search": "K-section K=32 x3", "launch": "HIP graph per FW iteration"},
        "gteps": Q * net.m / sssp_avg_s / 1e9,
        "gteps_counted": work_links / n_launch / sssp_avg_s / 1e9,
        "sssp_work_per_launch": {"nodes_taken": work_nodes / n_launch, "links_relaxed": work_links / n_launch,
                                 "of_full_trees": (work_links / n_launch) / (Q * net.m)},
        "phase_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in prof.items() if k != "sssp_work"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kname, "kernel_ms": sssp_avg_s * 1e3, "algorithmic_bytes_per_launch": bytes_launch,
                     "algorithmic_bytes": "8n + 8m per tree (every tree counted whole) + 8m + 4n topology",
                     "achieved_counted": touched / sssp_avg_s / 1e9,
                     "frac_counted": touched / sssp_avg_s / 1e9 / HBM_PEAK_GBS,
                     "counted_bytes": "8 per node taken + 8 per in-link relaxed, as counted by the kernel, "
                                      "+ topology once",
                     "kernel_timing": kernel_timing},
        "gaps": gaps, "alphas": alphas,
    }
    if not args.no_cpu_baseline:
        nthreads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
        log(f"cpu baseline: oracle with {nthreads} threads")
        import oracle
        legs = oracle.demand_legs(np.concatenate([dem.orig, ro]), np.concatenate([dem.dest, rd]),
                                  np.concatenate([dem.trips, rw / FX]))
        result["cpu_baseline"] = cpu_baseline(net, legs, f_host, dem.dt_s, w.alpha, w.beta, nthreads)
    ctx.close()
    if not args.no_plain:
        result["batched_vs_plain"] = batched_vs_plain(torch, qdta)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
