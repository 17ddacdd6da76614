#!/usr/bin/env python3
"""Benchmark of the Anderson-acceleration hot path on one MI355X.

Headline (the metric: QRAdd GB/s as a fraction of HBM peak): one QRAdd of a
Gaussian column v into a basis of k = 19 orthonormal columns (the add into a
20-column window) at n = 2^26, FP64, by the chosen variant (default ICWY,
Alg. 4).  A "step" is one such add: W untimed and K timed adds, each followed
by an untimed QRDelete that restores k.  Every add is bracketed by its own
pair of HIP events on the context's stream with the library's per-launch
profiling off, so its time is its span on the GPU (kernels and the gaps
between them).  value = algorithmic bytes of the add / median add time, where
every n-vector a kernel must read or write counts 8 n bytes once (ICWY:
(2k + 5) vectors; the library accounts this per launch).  The roofline object
names the add's dominant kernel, timed per launch by events in a separate
profiled pass.

Also measured: the QRAdd / QRDelete table for every variant (n = 2^24 with
k = m - 1, n = 2^26 with k = 1 .. 64; 10 reps, median and best), the
bandwidth ceilings of plain access patterns with the passes' tiles and loads
(aa_bandwidth_probe), the 3D nonlinear AA recycle iteration (G(u) = u -
omega (A u + u^3 - f) on 256^3, window m = 20) per variant with its loss of
orthogonality, the pass fusions, the window sweep, graph replay at mid
sizes, the 1D Poisson solves, and the batched / learned-guarded /
one-at-a-time comparison on the 4096-instance 2D table.

The CPU baseline is the oracle (its OpenMP build, bitwise the serial results)
on a bounded sample of the headline: the same add at n = 2^22, on one and on
every host core.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("QRAdd GB/s (% HBM peak) per variant; time-to-1e-8, learned/batched vs plain AA")
HBM_PEAK_GBS = 8000.0
VARIANTS = ["mgs", "cgs2", "dcgs2", "icwy"]
PROFILE_JSON = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def run_variant(prob, m, variant, steps, warmup, grid=None, profile=True, flags=0,
                keep_ctx=False):
    import torch
    from paper_2110_09667_amd import aa

    n = prob.n
    dev = torch.device("cuda:0")
    f_d = device_rhs(prob)
    ctx = aa.AAContext(n, m, variant, flags)
    if grid:
        ctx.set_grid(*grid)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    g = torch.empty_like(x)

    def step():
        aa.aa_problem_apply(prob.d, prob.s, prob.h, prob.omega, prob.c, f_d, x, g)
        ctx.step(x, g, x)

    for _ in range(m + 1 + warmup):
        step()
    torch.cuda.synchronize(dev)
    # timed steps, unprofiled (the step time reported)
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    # the same number of steps again with per-launch events (kernel breakdown)
    prof = {}
    if profile:
        ctx.profile(True)
        for _ in range(steps):
            step()
        torch.cuda.synchronize(dev)
        prof = ctx.profile_read()
        ctx.profile(False)
    info = ctx.info()
    if info.status != 0:
        raise RuntimeError(f"{variant}: device status {info.status}")
    u_bytes = 8.0 * n
    bytes_per_step = (sum(b for (_, _, b) in prof.values()) / steps + 3 * u_bytes) if prof else None
    out = {
        "variant": variant,
        "steps": steps,
        "ms_per_step": ms_total / steps,
        "wall_ms_per_step": 1e3 * wall / steps,
        "bytes_per_step": bytes_per_step,
        "gbs": (bytes_per_step / (ms_total / steps) / 1e6) if bytes_per_step else None,
        "res_norm": info.res_norm,
        "res0_norm": info.res0_norm,
        "kernels": {k: {"ms": v[0], "launches": v[1], "bytes": v[2],
                        "gbs": (v[2] / v[0] / 1e6) if v[0] > 0 else None}
                    for k, v in prof.items() if v[1] > 0},
    }
    if keep_ctx:
        out["ctx"] = ctx  # the caller closes it
    else:
        ctx.close()
    del x, g, f_d
    torch.cuda.empty_cache()
    return out


def graph_replay(sizes=(32, 48, 64, 96, 128), m=20, variant="icwy", steps=40):
    """Mid-size 3D workloads, where an iteration is launch-bound: ms per AA
    step (G included) enqueuing every pass vs. replaying captured graphs of
    the steady-state iteration (aa_set_graph)."""
    import torch
    from paper_2110_09667_amd import aa
    out = {}
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for s_ in sizes:
            prob = Problem3D(s_)
            f_d = device_rhs(prob)
            row = {}
            for graph in (False, True):
                ctx = aa.AAContext(prob.n, m, variant, stream=stream)
                ctx.set_fused_threshold(0)
                ctx.set_graph(graph)
                x = torch.zeros(prob.n, dtype=torch.float64, device="cuda:0")
                g = torch.empty_like(x)

                def step():
                    aa.aa_problem_apply(3, s_, prob.h, prob.omega, prob.c, f_d, x, g,
                                        stream=stream)
                    ctx.step(x, g, x)

                for _ in range(2 * m + 2):  # fill the window; capture every phase
                    step()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    step()
                torch.cuda.synchronize()
                row["graph_ms" if graph else "direct_ms"] = round(
                    1e3 * (time.perf_counter() - t0) / steps, 4)
                ctx.close()
            row["n"] = prob.n
            row["speedup"] = round(row["direct_ms"] / row["graph_ms"], 3)
            out[f"s={s_}"] = row
            print(f"# graph replay s={s_} (n={prob.n}): direct {row['direct_ms']:.3f} ms, "
                  f"graph {row['graph_ms']:.3f} ms", file=sys.stderr, flush=True)
    return out


def qr_micro(n, ks, variant, flags=0, reps=10, busy_reps=3, warmup=1):
    """QRAdd / QRDelete on their own (the standalone microbenchmark): a basis
    of k orthonormal columns (seeded Gaussian columns added one by one), then
    ``warmup`` untimed and ``reps`` timed cycles of [QRAdd of a Gaussian v;
    QRDelete], which keeps k fixed; every cycle adds a fresh v (generated
    before the add's events: re-adding the same v after a delete that kept it
    would add a vector already in the span).  Timing runs with the library's
    per-launch profiling off: a pair of events on the context's stream
    brackets each add (and, separately, each delete), so a time is the add's
    span on the GPU (its kernels and the gaps between them).  Then
    ``busy_reps`` more cycles with per-launch profiling give the add's
    algorithmic bytes (the library's accounting), its busy time (sum of its
    kernels' event-timed durations) and its dominant kernel.  Returns
    {k: {...}} with minima and medians."""
    import numpy as np
    import torch
    from paper_2110_09667_amd import aa
    import aa_workloads as W

    dev = torch.device("cuda:0")
    kmax = max(ks)
    ctx = aa.AAContext(n, kmax + 1, variant, flags=flags | aa.QR_ONLY)
    col = torch.empty(n, dtype=torch.float64, device=dev)
    v = torch.empty(n, dtype=torch.float64, device=dev)
    aa.aa_fill_normal(v, W.SEED_QR_V, 0)
    stream = torch.cuda.current_stream(dev)
    out = {}
    j = 0
    for k in sorted(ks):
        while ctx.info().k < k:
            aa.aa_fill_normal(col, W.SEED_QR_Q, j)
            ctx.qr_add(col)
            j += 1
        cyc = 0

        def fresh_v():
            nonlocal cyc
            aa.aa_fill_normal(v, W.SEED_QR_V, 1000 * k + cyc)
            cyc += 1

        for _ in range(warmup):
            fresh_v()
            ctx.qr_add(v)
            ctx.qr_delete()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(reps)]
        torch.cuda.synchronize(dev)
        for r in range(reps):
            fresh_v()
            ev[r][0].record(stream)
            ctx.qr_add(v)
            ev[r][1].record(stream)
            ev[r][2].record(stream)
            ctx.qr_delete()
            ev[r][3].record(stream)
        torch.cuda.synchronize(dev)
        t_add = np.array([e[0].elapsed_time(e[1]) for e in ev])
        t_del = np.array([e[2].elapsed_time(e[3]) for e in ev])
        # per-launch profiling: bytes, busy time, per-kernel breakdown
        ctx.profile(True)
        busy, kerns, b_add, b_del = [], {}, 0.0, 0.0
        for _ in range(busy_reps):
            fresh_v()
            aa.aa_profile_reset(ctx.ctx)
            ctx.qr_add(v)
            prof = ctx.profile_read()
            busy.append(sum(ms for (ms, _, _) in prof.values()))
            b_add = sum(b for (_, _, b) in prof.values())
            for kind, (ms, la, by) in prof.items():
                if la:
                    kk = kerns.setdefault(kind, [0.0, 0, 0.0])
                    kk[0] += ms
                    kk[1] += la
                    kk[2] += by
            aa.aa_profile_reset(ctx.ctx)
            ctx.qr_delete()
            b_del = sum(b for (_, _, b) in ctx.profile_read().values())
        ctx.profile(False)
        if ctx.info().status != 0:
            raise RuntimeError(f"qr_micro {variant} k={k}: status {ctx.info().status}")
        stream_kinds = {kd: d for kd, d in kerns.items() if d[2] > 0}
        dom = max(stream_kinds, key=lambda kd: stream_kinds[kd][0]) if stream_kinds else None
        med_a, min_a = float(np.median(t_add)), float(t_add.min())
        med_d = float(np.median(t_del))
        out[k] = {"add_bytes": b_add,
                  "add_us_median": 1e3 * med_a, "add_us_min": 1e3 * min_a,
                  "add_gbs": b_add / med_a / 1e6, "add_gbs_best": b_add / min_a / 1e6,
                  "add_busy_us": 1e3 * float(np.median(busy)),
                  "add_busy_gbs": b_add / float(np.median(busy)) / 1e6,
                  "delete_us_median": 1e3 * med_d,
                  "delete_gbs": (b_del / med_d / 1e6) if med_d > 0 else None,
                  "reps": reps,
                  "dominant_kernel": dom,
                  "kernels": {kd: {"us_per_launch": 1e3 * d[0] / d[1],
                                   "bytes_per_launch": d[2] / d[1],
                                   "gbs": (d[2] / d[0] / 1e6) if d[0] > 0 and d[2] > 0 else None}
                              for kd, d in kerns.items()}}
    ctx.close()
    del col, v
    torch.cuda.empty_cache()
    return out


def ceilings(n=1 << 26, reps=10):
    """Sustained bandwidth of plain access patterns with the passes' tiles,
    loads and launch shape (aa_bandwidth_probe): read streams (1, 4, 8
    vectors), copy (1 read, 1 write), the MGS update's 3 reads + 1 write and
    8 reads + 1 write; GB/s of the bytes read and written, best and median
    of ``reps`` launches."""
    import numpy as np
    import torch
    from paper_2110_09667_amd import aa
    # the library's column stride for long columns: 1024 (mod 2048) doubles
    ld = (n + 63) // 64 * 64
    ld = (ld + 2047) // 2048 * 2048 + 1024
    src = torch.ones(8 * ld, dtype=torch.float64, device="cuda:0")
    dst = torch.empty(2 * ld, dtype=torch.float64, device="cuda:0")
    sink = torch.empty(4096, dtype=torch.float64, device="cuda:0")
    stream = torch.cuda.current_stream()
    out = {}
    for (rd, wr) in ((1, 0), (4, 0), (8, 0), (1, 1), (3, 1), (8, 1)):
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(reps + 1)]
        for r in range(reps + 1):
            ev[r][0].record(stream)
            aa.aa_bandwidth_probe(rd, wr, src, ld, dst, n, sink)
            ev[r][1].record(stream)
        torch.cuda.synchronize()
        t = np.array([e[0].elapsed_time(e[1]) for e in ev[1:]])
        byt = 8.0 * n * (rd + wr)
        out[f"{rd}r{wr}w"] = {"gbs_best": round(byt / t.min() / 1e6, 1),
                              "gbs_median": round(byt / float(np.median(t)) / 1e6, 1)}
    del src, dst, sink
    torch.cuda.empty_cache()
    return out


class BatchProblem2D:
    """One instance of the batched 2D workload, f generated on the GPU by the
    library's generator (bit-identical to aa_workloads.batch_problem)."""

    def __init__(self, inst):
        import torch
        import aa_workloads as W
        from paper_2110_09667_amd import aa
        self.d, self.s, self.c = 2, inst.s, inst.c
        self.n = inst.n
        self.h = 1.0 / (inst.s + 1)
        self.omega = 0.9 / W.laplacian_lambda_max(2, inst.s)
        self.f = torch.empty(self.n, dtype=torch.float64, device="cuda:0")
        aa.aa_fill_uniform(self.f, inst.seed, 1)


def batch_iter_vectors(variant, m, m_i, k_before, fuse=0):
    """Algorithmic n-vectors of one batched iteration of one instance with a
    full window (the same byte model as the library's accounting, G
    included)."""
    from paper_2110_09667_amd import aa
    k = k_before
    add = {"mgs": 4 * k + 3 if k else 3, "cgs2": 3 * k + 6, "dcgs2": 2 * k + (6 if k >= 3 else 5),
           "icwy": 2 * k + 5}[variant]
    delete = (2 * m - 1) if m_i == m else 0
    rhs = m_i + 1
    fold = bool(fuse & aa.FUSE_RHS) and variant != "mgs" and k >= 1
    fused_del = bool(fuse & aa.FUSE_DELETE) and variant != "mgs" and m_i == m and k >= 1
    if fused_del:
        add -= k + 1
        delete += 2 if fold else 1
    if fold:
        rhs = 0
        add += 1 if fused_del else 2
    return 3 + 8 + delete + add + rhs + (m_i + 3)


def batched_run(probs, ms, variant, tol, cap, chunk, stream, net=None, steady=20, tune=True,
                fuse=0):
    """Drive a batch to tolerance (or the iteration cap): returns the time of
    the first 21 iterations (every window full after them), the schedule the
    autotuner picked (plain batches), the steady per-iteration time, the wall
    time until no instance is active and the final states."""
    import torch
    from paper_2110_09667_amd import aa
    flags = (aa.BATCH_LEARNED if net is not None else 0) | fuse
    b = aa.AABatch(probs, ms, variant, flags=flags, tol=tol, max_iter=cap, stream=stream)

    def run(k):
        if net is None:
            b.run(k)
        else:
            b.run_learned(net, k)

    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e[0].record(stream)
    run(21)
    e[1].record(stream)
    it = 21
    sched = None
    if tune and net is None:
        # the schedule autotuner times real iterations under each candidate
        sched = b.autotune(3)
        it += 3 * sched.trials
    e[2].record(stream)
    run(steady)
    e[3].record(stream)
    it += steady
    while True:
        st, active = b.read()
        if active == 0 or it >= cap:
            break
        run(chunk)
        it += chunk
    wall = time.perf_counter() - t0
    out = {"fill_ms": e[0].elapsed_time(e[1]), "steady_ms_per_iter": e[2].elapsed_time(e[3]) / steady,
           "wall_s": wall, "states": st, "iters_run": it,
           "schedule": ({"grid": sched.grid, "order": ["largest n*m first", "as given"][sched.order],
                         "ms_per_iter": round(sched.ms_per_iter, 3), "trials": sched.trials}
                        if sched else None)}
    b.close()
    del b
    return out


def batched_tail(variant, takes=(8, 32, 128), fuse=0, steady=20):
    """The tail of a batch: only the `take` largest instances of the batched
    table still active.  Steady time per iteration with every instance in the
    persistent kernel (one workgroup each) against the split path (each
    instance on the grid-wide passes, one after another)."""
    import torch
    import aa_workloads as W
    from paper_2110_09667_amd import aa
    table = W.batch_table(4096)
    order = sorted(range(len(table)), key=lambda j: (table[j].s * table[j].s * table[j].m, -j),
                   reverse=True)
    stream = torch.cuda.Stream()
    out = {}
    for take in takes:
        insts = [table[j] for j in order[:take]]
        probs = [BatchProblem2D(i) for i in insts]
        ms = [i.m for i in insts]
        vec = sum(batch_iter_vectors(variant, i.m, i.m, i.m - 1, fuse) * p.n
                  for i, p in zip(insts, probs))
        row = {"instances": take, "n_min": min(p.n for p in probs),
               "n_max": max(p.n for p in probs)}
        with torch.cuda.stream(stream):
            for mode in ("persistent", "split"):
                b = aa.AABatch(probs, ms, variant, flags=fuse, tol=0.0, max_iter=10**9,
                               stream=stream)
                b.set_split(1 if mode == "split" else 0, take)
                b.run(21)   # every window full
                b.run(1)    # the split policy applies at the start of a run
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                e0.record(stream)
                b.run(steady)
                e1.record(stream)
                torch.cuda.synchronize()
                wall = (time.perf_counter() - t0) / steady
                ms_it = e0.elapsed_time(e1) / steady
                row[mode] = {"ms_per_iter": round(ms_it, 3),
                             "host_ms_per_iter": round(1e3 * wall, 3),
                             "algorithmic_gbs": round(8.0 * vec / (ms_it * 1e-3) / 1e9, 1),
                             "split_instances": b.split_count()}
                b.close()
                del b
        row["split_speedup"] = round(row["persistent"]["ms_per_iter"] /
                                     row["split"]["ms_per_iter"], 2)
        out[str(take)] = row
        print(f"# batched tail, {take} largest instances: persistent "
              f"{row['persistent']['ms_per_iter']:.2f} ms/iter, split "
              f"{row['split']['ms_per_iter']:.2f} ms/iter", file=sys.stderr, flush=True)
        del probs
        torch.cuda.empty_cache()
    return out


def poisson1d_to_tolerance(variant, tol=1e-8, cap=300, check_every=1):
    """The 1D Poisson workload (n = 4096, m = 5) solved to ||f|| <= tol ||f_0||
    with the single-instance entry points (the one-workgroup step at this n),
    host stop test every step, and with the batched entry points for one
    instance (stop test on the device).  The oracle's time for the same solve
    is part of the CPU baseline."""
    import torch
    import aa_workloads as W
    from paper_2110_09667_amd import aa
    prob = W.poisson1d()
    m = 5
    f_d = torch.from_numpy(prob.f).cuda()
    ctx = aa.AAContext(prob.n, m, variant)
    x = torch.zeros(prob.n, dtype=torch.float64, device="cuda:0")
    g = torch.empty_like(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = 0
    while it < cap:
        aa.aa_problem_apply(prob.d, prob.s, prob.h, prob.omega, prob.c, f_d, x, g)
        ctx.step(x, g, x)
        it += 1
        if it % check_every == 0:
            info = ctx.info()
            if info.iter > 1 and info.res_norm <= tol * info.res0_norm:
                break
    torch.cuda.synchronize()
    gpu_s = time.perf_counter() - t0
    info = ctx.info()
    ctx.close()
    # the same solve through the batched entry points with one instance: the
    # stop test runs on the device, one launch per iteration, one wait at the end
    stream = torch.cuda.Stream()
    batch_s = {}
    with torch.cuda.stream(stream):
        for label, flags in (("separate", 0), ("fused", aa.FUSE_RHS | aa.FUSE_DELETE)):
            b = aa.AABatch([prob], [m], variant, flags=flags, tol=tol, max_iter=cap, stream=stream)
            b.set_schedule(use_graph=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.run(cap + 1)
            bst, _ = b.read()
            batch_s[label] = time.perf_counter() - t0
            b.close()
    return {"iterations": it, "converged": bool(info.res_norm <= tol * info.res0_norm),
            "final_rel_residual": info.res_norm / info.res0_norm,
            "gpu_ms": round(1e3 * gpu_s, 3), "us_per_iter": round(1e6 * gpu_s / max(it, 1), 1),
            "batch_api_iterations": int(bst[0].stop_iter if not bst[0].active else bst[0].iter),
            "batch_api_ms": round(1e3 * batch_s["separate"], 3),
            "batch_api_fused_passes_ms": round(1e3 * batch_s["fused"], 3)}


def nonlinear3d_to_tolerance(prob, m, variant, tol=1e-8, cap=20000, check_every=10, flags=0):
    """The 3D nonlinear workload solved from u_0 = 0 to ||f_i|| <= tol ||f_0||
    (or the cap) with the single-instance entry points and the device-side
    stop test (aa_set_stop), the host reading the state every
    ``check_every`` steps (steps after the end return at once).  Returns
    iterations, wall seconds (G evaluations included), the final relative
    residual and whether it converged."""
    import torch
    from paper_2110_09667_amd import aa
    dev = torch.device("cuda:0")
    f_d = device_rhs(prob)
    ctx = aa.AAContext(prob.n, m, variant, flags)
    ctx.set_stop(tol, cap)  # the stopping test runs on the device
    x = torch.zeros(prob.n, dtype=torch.float64, device=dev)
    g = torch.empty_like(x)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    calls = 0
    while True:
        for _ in range(check_every):
            aa.aa_problem_apply(prob.d, prob.s, prob.h, prob.omega, prob.c, f_d, x, g)
            ctx.step(x, g, x)
            calls += 1
        info = ctx.info()
        if info.stopped:
            break
    wall = time.perf_counter() - t0
    ctx.close()
    del f_d, x, g
    torch.cuda.empty_cache()
    it = int(info.stop_iter)
    rel = info.res_norm / info.res0_norm
    return {"iterations": it, "converged": info.stopped == aa.STOPPED_TEST,
            "final_rel_residual": rel, "wall_s": round(wall, 3),
            "ms_per_iter": round(1e3 * wall / max(it, 1), 4), "status": int(info.status),
            "stopped": int(info.stopped)}


def em_to_tolerance(variant, flags=0, replicas=500_000, nsamples=100_000, m=3, tol=1e-8,
                    cap=100, reps=5):
    """The EM workload (Sec. 5.3): n = 3 x replicas (1.5 million, the paper's
    vector per GPU), 100,000 samples, m = 3, from the samples' 1/6, 1/2, 5/6
    quantiles to ||f_i|| <= tol ||f_0|| with the library's device-side stop
    test (aa_set_stop), the host reading the state every 4 steps.  Returns
    the iterations and the best of ``reps`` wall times (G and AA, up to the
    host seeing the end), with the time in G and in aa_step up to the end
    split by events."""
    import numpy as np
    import torch
    import aa_workloads as W
    from paper_2110_09667_amd import aa
    prob = W.em_problem(nsamples=nsamples, replicas=replicas)
    xd = torch.from_numpy(prob.samples).cuda()
    work = torch.empty(aa.EM_WORK_DOUBLES, dtype=torch.float64, device="cuda")
    u0 = torch.from_numpy(prob.u0()).cuda()
    stream = torch.cuda.current_stream()
    best = None
    for _ in range(reps):
        ctx = aa.AAContext(prob.n, m, variant, flags)
        ctx.set_stop(tol, cap)  # tested on the device: no per-step wait
        x = u0.clone()
        g = torch.empty_like(x)
        evs = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        calls = 0
        while True:
            for _ in range(4):  # steps after the end return at once
                e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
                e[0].record(stream)
                aa.aa_em_apply(prob.alpha, prob.sigma, xd, x, g, work)
                e[1].record(stream)
                ctx.step(x, g, x)
                e[2].record(stream)
                evs.append(tuple(e))
                calls += 1
            info = ctx.info()
            if info.stopped:
                break
        wall = time.perf_counter() - t0
        its = info.stop_iter  # x_its is the answer: its steps were taken
        g_ms = sum(a.elapsed_time(b) for a, b, _ in evs[:its + 1])
        aa_ms = sum(b.elapsed_time(c) for a, b, c in evs[:its])
        ctx.close()
        r = {"iterations": its, "converged": info.stopped == aa.STOPPED_TEST,
             "wall_ms": round(1e3 * wall, 3), "g_ms": round(g_ms, 3), "aa_ms": round(aa_ms, 3),
             "calls_enqueued": calls}
        if best is None or r["wall_ms"] < best["wall_ms"]:
            best = r
    best["n"] = prob.n
    best["nsamples"] = nsamples
    return best


PDE_PROBLEMS = (("heat_nl1", 1), ("heat_nl2", 2), ("bratu", 3))


def pde_to_tolerance(problem, variant, flags=0, N=1024, cap=150, reps=3):
    """The 2D test problems of Sec. 5.1 (heat equation with nonlinear term 1,
    m = 5; term 2, m = 10) and Sec. 5.2 (Bratu, lambda = 6.7, m = 30) on the
    paper's 1024 x 1024 grid from u_0 = 0 to ||f_i|| <= 1e-10 ||f_0|| (the
    paper's nonlinear tolerance; the stop test on the device), each G a PCG
    solve to 1e-10 preconditioned by the library's multigrid cycle.  The map
    returns after its solve has ended on the GPU (it reads the PCG state), so
    the host reads the AA state after every step.  Returns the iterations,
    the best of ``reps`` wall times up to the host seeing the end, and the GPU
    time in G and in aa_step (events)."""
    import torch
    import aa_workloads as W
    from paper_2110_09667_amd import aa
    prob = W.bratu2d(N) if problem == W.PDE_BRATU else W.heat2d(N, problem)
    b = torch.from_numpy(prob.b).cuda() if prob.b is not None else None
    stream = torch.cuda.current_stream()
    pde = aa.PDE2D(N, problem, lam=prob.lam, tol=prob.tol, max_iter=200)
    best = None
    for _ in range(reps):
        ctx = aa.AAContext(prob.n, prob.m, variant, flags)
        ctx.set_stop(prob.tol, cap)
        x = torch.zeros(prob.n, dtype=torch.float64, device="cuda")
        g = torch.empty_like(x)
        evs, pcg = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while True:
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record(stream)
            pde.apply(b, x, g)
            e[1].record(stream)
            ctx.step(x, g, x)
            e[2].record(stream)
            evs.append(tuple(e))
            pcg.append(pde.last()[0])
            info = ctx.info()
            if info.stopped:
                break
        wall = time.perf_counter() - t0
        its = info.stop_iter
        g_ms = sum(a.elapsed_time(bb) for a, bb, _ in evs)
        aa_ms = sum(bb.elapsed_time(c) for a, bb, c in evs[:its])
        ctx.close()
        r = {"iterations": its, "converged": info.stopped == aa.STOPPED_TEST,
             "stopped": int(info.stopped), "wall_ms": round(1e3 * wall, 2),
             "g_ms": round(g_ms, 2), "aa_ms": round(aa_ms, 3),
             "g_evaluations": len(evs), "pcg_iterations_per_g": sorted(set(pcg))}
        if best is None or r["wall_ms"] < best["wall_ms"]:
            best = r
    best["n"] = prob.n
    best["m"] = prob.m
    return best


def one_at_a_time(probs, ms, variant, tol, cap, check_every=10, flags=0):
    """The same instances solved one after another through the single-instance
    entry points (aa_problem_apply + aa_step on one context per instance),
    each until ||f_i|| <= tol ||f_0|| (tested every ``check_every`` steps) or
    ``cap`` iterations.  Returns (seconds, iterations, converged) per instance."""
    import torch
    from paper_2110_09667_amd import aa
    out = []
    for p, m in zip(probs, ms):
        ctx = aa.AAContext(p.n, m, variant, flags)
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda:0")
        g = torch.empty_like(x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, conv = 0, False
        while it < cap:
            for _ in range(check_every):
                aa.aa_problem_apply(p.d, p.s, p.h, p.omega, p.c, p.f, x, g)
                ctx.step(x, g, x)
                it += 1
            info = ctx.info()
            if info.iter > 1 and info.res_norm <= tol * info.res0_norm:
                conv = True
                break
        torch.cuda.synchronize()
        out.append((time.perf_counter() - t0, it, conv))
        ctx.close()
        del x, g
    return out


def batched_suite(variant, count, cap, train_count, train_iters, sample, lr=1e-3, fuse=0,
                  ablation_cap=600):
    """Batched AA on the 2D workload table (instance seeds 0..count-1):
    plain batched to tol 1e-8 (or the cap), the learned-guarded batch with a
    network trained on instances of disjoint seeds, and a seeded sample of
    the same instances run one at a time through the single-instance path;
    the guard with the untrained network (what the training adds) to
    ``ablation_cap`` iterations, beside the other two at that cap read from
    their iteration counts."""
    import numpy as np
    import torch
    import aa_workloads as W
    from paper_2110_09667_amd import aa

    tol = 1e-8
    insts = W.batch_table(count)
    probs = [BatchProblem2D(i) for i in insts]
    ms = [i.m for i in insts]
    sum_n = sum(p.n for p in probs)
    stream = torch.cuda.Stream()
    res = {"instances": count, "sum_n": sum_n, "variant": variant, "tol": tol,
           "max_iter": cap, "ablation_max_iter": min(cap, ablation_cap),
           "passes": ("RHS folded into QRAdd, QRDelete fused with its first pass"
                      if fuse == (aa.FUSE_RHS | aa.FUSE_DELETE) else
                      "separate" if fuse == 0 else f"flags {fuse}")}
    with torch.cuda.stream(stream):
        # algorithmic bytes of one full-window iteration of every instance
        vec = sum(batch_iter_vectors(variant, i.m, i.m, i.m - 1, fuse) * p.n
                  for i, p in zip(insts, probs))
        plain = batched_run(probs, ms, variant, tol, cap, 50, stream, fuse=fuse)
        print(f"# batched plain: {plain['steady_ms_per_iter']:.2f} ms/iter, "
              f"{plain['wall_s']:.1f} s", file=sys.stderr, flush=True)
        # training on disjoint seeds: plain-AA trajectories, one Adam step per
        # iteration over the whole training batch
        tinsts = W.batch_table(train_count, first_seed=W.SEED_TRAIN_BASE)
        tprobs = [BatchProblem2D(i) for i in tinsts]
        net = aa.AAMlp(max(count, train_count), seed=1, stream=stream)
        tb = aa.AABatch(tprobs, [i.m for i in tinsts], variant, flags=aa.BATCH_LEARNED | fuse,
                        tol=0.0, max_iter=10**9, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tb.train(net, train_iters, lr)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t0
        tstates, _ = tb.read()
        tb.close()
        del tb, tprobs
        torch.cuda.empty_cache()
        learned = batched_run(probs, ms, variant, tol, cap, 50, stream, net=net, fuse=fuse)
        print(f"# batched learned: {learned['steady_ms_per_iter']:.2f} ms/iter, "
              f"{learned['wall_s']:.1f} s", file=sys.stderr, flush=True)
        # ablation: the same guard with the untrained network (delta gamma = 0,
        # beta = sigmoid(4)): what the training itself adds
        net0 = aa.AAMlp(count, seed=1, stream=stream)
        untrained = batched_run(probs, ms, variant, tol, min(cap, ablation_cap), 50, stream,
                                net=net0, fuse=fuse)
        print(f"# batched guarded, untrained network: {untrained['wall_s']:.1f} s",
              file=sys.stderr, flush=True)
    rng = np.random.default_rng(12345)
    pick = sorted(rng.choice(count, size=min(sample, count), replace=False).tolist())
    single = one_at_a_time([probs[j] for j in pick], [ms[j] for j in pick], variant, tol, cap,
                           flags=fuse)
    print(f"# one at a time ({len(pick)} sampled): {sum(t for t, _, _ in single):.1f} s",
          file=sys.stderr, flush=True)

    def summary(run):
        st = run["states"]
        conv = [s for s in st if s.res_norm <= tol * s.res0_norm]
        its = np.array([s.stop_iter for s in conv]) if conv else np.array([0])
        return {"wall_s": round(run["wall_s"], 3),
                "steady_ms_per_iter": round(run["steady_ms_per_iter"], 3),
                "converged": len(conv),
                "converged_within_ablation_cap": int(sum(1 for s in conv
                                                         if s.stop_iter <= ablation_cap)),
                "median_iters_converged": float(np.median(its)),
                "p90_iters_converged": float(np.percentile(its, 90)),
                "g_evals_total": int(sum(s.g_evals for s in st)),
                "accepted_total": int(sum(s.accepted for s in st))}

    sp, sl, su = summary(plain), summary(learned), summary(untrained)
    both = [j for j in range(count)
            if plain["states"][j].res_norm <= tol * plain["states"][j].res0_norm
            and learned["states"][j].res_norm <= tol * learned["states"][j].res0_norm]
    gi = np.array([learned["states"][j].stop_iter / plain["states"][j].stop_iter for j in both]) \
        if both else np.array([np.nan])
    t_single = sum(t for t, _, _ in single)
    res.update({
        "plain": {**sp, "schedule": plain["schedule"],
                  "inst_iters_per_s": round(count / (plain["steady_ms_per_iter"] * 1e-3)),
                  "algorithmic_gbs": round(8.0 * vec / (plain["steady_ms_per_iter"] * 1e-3) / 1e9, 1)},
        "learned": {**sl, "train_instances": train_count, "train_iters": train_iters,
                    "train_samples": train_count * max(0, train_iters - 1), "train_s": round(train_s, 2),
                    "train_final_mean_loss": float(np.mean([s.loss for s in tstates])),
                    "both_converged": len(both),
                    "median_iter_ratio_learned_over_plain": float(np.median(gi))},
        "guarded_untrained_network": su,
        "one_at_a_time_sample": {
            "instances": len(pick), "seconds": round(t_single, 3),
            "converged": sum(1 for _, _, c in single if c),
            "iterations": int(sum(i for _, i, _ in single)),
            "estimated_seconds_all": round(t_single * count / len(pick), 1),
            "stop_test_every": 10},
    })
    return res


def device_rhs(prob):
    """f ~ U[0, 1] of the 3D workload (seed 2, stream 0), generated on the GPU
    by the library's generator (bit-identical to aa_workloads.uniform)."""
    import torch
    from paper_2110_09667_amd import aa
    import aa_workloads as W
    f = torch.empty(prob.n, dtype=torch.float64, device="cuda:0")
    aa.aa_fill_uniform(f, W.SEED_POISSON3D_F, 0)
    return f


class Problem3D:
    """Parameters of G(u) = u - omega (A u + u^3 - f) on an s^3 grid (f on device)."""

    def __init__(self, s):
        import aa_workloads as W
        self.d, self.s, self.c = 3, s, 1.0
        self.n = s ** 3
        self.h = 1.0 / (s + 1)
        self.omega = 0.9 / W.laplacian_lambda_max(3, s)


def cpu_baseline(n=1 << 22, k=19, variant="icwy", reps=5, c2_s=256, c2_m=20, c2_iters=3):
    """The oracle (its OpenMP build: fixed row blocks, bitwise the serial
    results) on a bounded sample of the headline measurement: QRAdds of a
    Gaussian column into a k-column basis at n = 2^22 (the GPU measures
    n = 2^26), each followed by an untimed QRDelete, median of ``reps`` at 1
    thread and at every host core; GB/s with the same byte model.  Also the
    1D Poisson solves (1 thread), and the 3D workload's AA iteration at the
    GPU's size (s^3 grid, window c2_m) on every core: the window filled
    (c2_m + 1 iterations, untimed), then ``c2_iters`` recycled iterations
    timed (one core would take minutes)."""
    import numpy as np

    import aa_workloads as W
    import oracle as O
    allc = len(os.sched_getaffinity(0))
    O.use_openmp(allc)
    q = O.QR(n, k + 1, variant)
    for j in range(k):
        q.add(W.normal(W.SEED_QR_Q, j, n))
    u = 8.0 * n
    vecs = {"mgs": 4 * k + 3, "cgs2": 3 * k + 6, "dcgs2": 2 * k + 6, "icwy": 2 * k + 5,
            "dcgs2_lag": 2 * k + 4}[variant]
    res = {}
    cycle = 0
    for threads in (1, allc):
        used = O.use_openmp(threads)
        ts = []
        for _ in range(reps):
            # a fresh column every cycle: the delete drops the oldest column,
            # so the last v stays in the basis
            v = W.normal(W.SEED_QR_V, cycle, n)
            cycle += 1
            t0 = time.perf_counter()
            assert q.add(v) == O.OK
            ts.append(time.perf_counter() - t0)
            assert q.delete() == O.OK
        dt = float(np.median(ts))
        res[threads] = (vecs * u / dt / 1e9, dt, used)
    O.use_openmp(1)
    p1 = W.poisson1d()
    poisson = {}
    for vv in VARIANTS:
        t1 = time.perf_counter()
        _, _, r = O.run_aa(lambda z: O.G_stencil(p1, z), np.zeros(p1.n), 5, vv, 300, tol=1e-8,
                           record=False)
        poisson[vv] = {"iterations": len(r), "ms": round(1e3 * (time.perf_counter() - t1), 3)}
    c2_threads = O.use_openmp(allc)
    p3 = W.nonlinear3d(c2_s)
    st = O.AA(p3.n, c2_m, variant)
    x = np.zeros(p3.n)
    for _ in range(c2_m + 1):
        x = st.step(x, O.G_stencil(p3, x))
    t0 = time.perf_counter()
    for _ in range(c2_iters):
        x = st.step(x, O.G_stencil(p3, x))
    c2_ms = 1e3 * (time.perf_counter() - t0) / c2_iters
    c2 = {"workload": f"3D nonlinear {c2_s}^3, {variant}, m = {c2_m}, window full",
          "ms_per_iteration": round(c2_ms, 1), "threads": c2_threads,
          "timed_iterations": c2_iters, "untimed_fill_iterations": c2_m + 1}
    del st, x, p3
    O.use_openmp(1)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    gb_all, dt_all, used_all = res[allc]
    gb_1, dt_1, _ = res[1]
    return {"value": round(gb_all, 3), "unit": "GB/s", "cores": used_all, "kind": "oracle",
            "one_core_value": round(gb_1, 3), "nproc": os.cpu_count(), "cpu_model": model,
            "poisson1d_to_1e-8_one_core": poisson,
            "c2_iteration_all_cores": c2,
            "sample": (f"FP64 C oracle (OpenMP build, fixed row blocks): one {variant} QRAdd "
                       f"into a {k}-column basis at n = {n} (the GPU line is n = 2^26), "
                       f"median of {reps}: {dt_all:.2f} s on {used_all} threads, {dt_1:.2f} s "
                       f"on 1; and {c2_iters} recycled iterations of the 3D AA workload at "
                       f"{c2_s}^3, m = {c2_m}, {c2_ms / 1e3:.2f} s each on {c2_threads} "
                       f"threads")}


def load_traffic(workload, kind):
    """HBM bytes per launch measured with rocprofv3 counters, if a summary for
    this kernel and workload is committed and its kernel sources have not
    changed since."""
    try:
        with open(PROFILE_JSON) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    key = f"{workload}/{kind}"
    ent = d.get(key)
    if not ent or ent.get("source_hash") != source_hash():
        return None
    return ent.get("bytes_per_launch")


def source_hash():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2110_09667_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


QR_VARIANTS = [("mgs", 0), ("cgs2", 0), ("dcgs2", 0), ("icwy", 0), ("dcgs2_lag", 0),
               ("icwy_T_transform", 1 << 2)]


def variant_name(label):
    return "icwy" if label == "icwy_T_transform" else label


def orthogonality(ctx, m):
    """||I - Q^T Q||_F of the context's basis (torch FP64 products, column by
    column block) and kappa_2(R), for the bounds of Sec. 2.2."""
    import numpy as np
    import torch
    Q = ctx.basis(m).contiguous()
    G = torch.empty((m, m), dtype=torch.float64, device=Q.device)
    for a in range(m):
        G[a] = Q[:, a] @ Q
    orth = torch.linalg.norm(torch.eye(m, dtype=torch.float64, device=Q.device) - G).item()
    R = ctx.get_qr()[0]
    return orth, float(np.linalg.cond(R))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="timed QRAdds of the headline measurement (and AA steps of the "
                         "3D workload)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variant", default="icwy", choices=VARIANTS)
    ap.add_argument("--k", type=int, default=19, help="columns before the headline QRAdd")
    ap.add_argument("--m", type=int, default=20, help="window of the 3D AA step")
    ap.add_argument("--s", type=int, default=256, help="grid points per side (3D AA step)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other-variants", action="store_true")
    ap.add_argument("--grid", type=int, nargs=2, default=None,
                    help="max workgroups: streaming passes, Gram pass")
    ap.add_argument("--no-qr-micro", action="store_true",
                    help="skip the QRAdd/QRDelete table (the headline add still runs)")
    ap.add_argument("--rhs", choices=["separate", "fused"], default="separate",
                    help="R gamma = Q^T f_i as its own pass (as Alg. 2 writes it) or folded "
                         "into the QRAdd passes (AA_FUSE_RHS) in the 3D AA steps")
    ap.add_argument("--batch-passes", choices=["separate", "fused"], default="fused",
                    help="batched runs with the paper's separate passes or with the RHS folded "
                         "into QRAdd and QRDelete fused with its first pass")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched / learned-guarded / one-at-a-time comparison")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--batch-cap", type=int, default=5000,
                    help="iteration cap of the batched time-to-tolerance runs")
    ap.add_argument("--ablation-cap", type=int, default=600,
                    help="iteration cap of the untrained-network ablation")
    ap.add_argument("--train-count", type=int, default=4096)
    ap.add_argument("--train-iters", type=int, default=50)
    ap.add_argument("--single-sample", type=int, default=64,
                    help="instances run one at a time for the comparison")
    ap.add_argument("--qr-micro-only", action="store_true",
                    help="only the QRAdd / QRDelete table at n = 2^26 (one JSON line per "
                         "variant; for kernel traces)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline QRAdd (for kernel traces and counters)")
    ap.add_argument("--em-only", action="store_true",
                    help="only the EM workload (Sec. 5.3) solved to 1e-8 per variant")
    ap.add_argument("--pde-only", action="store_true",
                    help="only the 2D heat (both nonlinear terms) and Bratu problems of Sec. "
                         "5.1-5.2 on the 1024 x 1024 grid solved to 1e-10 per variant")
    ap.add_argument("--ceilings-only", action="store_true",
                    help="only the bandwidth probes (read streams, copy, 3 reads + 1 write)")
    ap.add_argument("--c2-to-tol", action="store_true",
                    help="only the 3D nonlinear workload (256^3) solved to 1e-8 per variant and "
                         "m in {5, 10, 20, 50} (long: several minutes; one JSON line each)")
    ap.add_argument("--c2-cap", type=int, default=20000,
                    help="iteration cap of --c2-to-tol")
    ap.add_argument("--c2-only", action="store_true",
                    help="only the 3D AA step of --variant and --m (for kernel traces)")
    ap.add_argument("--poisson-only", action="store_true",
                    help="only the 1D Poisson time-to-tolerance measurement (for profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (5 times), to "
                         "calibrate the HBM byte counters of a profiler")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        nbytes = 1 << 30
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes,
                          "repeats": 5}), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_2110_09667_amd import aa
    if not os.path.exists(aa.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    aa.lib()

    if args.poisson_only:
        for v in VARIANTS:
            print(json.dumps({v: poisson1d_to_tolerance(v)}), flush=True)
        return
    if args.em_only:
        for label, fl in QR_VARIANTS:
            print(json.dumps({label: em_to_tolerance(variant_name(label), fl)}), flush=True)
        return
    if args.ceilings_only:
        print(json.dumps({"ceilings_n2e26": ceilings()}), flush=True)
        return
    if args.pde_only:
        for pname, pid in PDE_PROBLEMS:
            for label, fl in QR_VARIANTS:
                print(json.dumps({"problem": pname, "variant": label,
                                  **pde_to_tolerance(pid, variant_name(label), fl)}), flush=True)
        return
    if args.qr_micro_only:
        for label, fl in QR_VARIANTS:
            v = variant_name(label)
            ks = [min(k, 63) if v == "icwy" else k for k in (1, 2, 4, 8, 16, 32, 64)]
            r = qr_micro(1 << 26, ks, v, fl)
            print(json.dumps({"variant": label, "n": 1 << 26,
                              **{f"k={k}": {kk: d[kk] for kk in ("add_us_median", "add_gbs",
                                                                  "add_busy_gbs", "delete_gbs")}
                                 for k, d in r.items()}}), flush=True)
        return
    if args.c2_to_tol:
        prob = Problem3D(args.s)
        for mm in (5, 10, 20, 50):
            for v in VARIANTS:
                r = nonlinear3d_to_tolerance(prob, mm, v, cap=args.c2_cap)
                print(json.dumps({"workload": f"3D nonlinear {args.s}^3 to 1e-8", "m": mm,
                                  "variant": v, **r}), flush=True)
        return
    if args.c2_only:
        prob = Problem3D(args.s)
        r = run_variant(prob, args.m, args.variant, args.steps, args.warmup, args.grid,
                        flags=aa.FUSE_RHS if args.rhs == "fused" else 0)
        print(json.dumps({"variant": args.variant, "m": args.m, "ms_per_step": r["ms_per_step"],
                          "gbs": r["gbs"]}), flush=True)
        return

    # ---- the headline: one QRAdd into a k-column basis at n = 2^26 ------------
    n_head = 1 << 26
    head = qr_micro(n_head, [args.k], args.variant, reps=args.steps, warmup=args.warmup)[args.k]
    print(f"# headline QRAdd {args.variant} n=2^26 k={args.k}: {head['add_us_median']:.1f} us "
          f"(min {head['add_us_min']:.1f}), {head['add_gbs']:.0f} GB/s "
          f"({100 * head['add_gbs'] / HBM_PEAK_GBS:.1f} % of HBM peak); busy "
          f"{head['add_busy_gbs']:.0f} GB/s", file=sys.stderr, flush=True)
    if args.headline_only:
        print(json.dumps({"headline": head}), flush=True)
        return

    ceil = ceilings()
    print("# ceilings: " + ", ".join(f"{k} {d['gbs_best']:.0f}" for k, d in ceil.items()),
          file=sys.stderr, flush=True)

    qradd = {}
    if not args.no_qr_micro:
        # QRAdd / QRDelete alone: at the 3D workload's n with k = m - 1 (the
        # add that follows a delete in a full window, m = 5, 10, 20, 50), and
        # at n = 2^26 for k = 1..64
        for label_n, n_q, ks in (("n=%d" % (1 << 24), 1 << 24, [4, 9, 19, 49]),
                                 ("n=%d" % n_head, n_head, [1, 2, 4, 8, 9, 16, 19, 32, 64])):
            qradd[label_n] = {}
            for label, fl in QR_VARIANTS:
                v = variant_name(label)
                # the ICWY window holds at most 64 columns: its largest add is k = 63
                r = qr_micro(n_q, [min(k, 63) if v == "icwy" else k for k in ks], v, fl)
                qradd[label_n][label] = {
                    f"k={k}": {"add_us_median": round(d["add_us_median"], 1),
                               "add_us_min": round(d["add_us_min"], 1),
                               "add_gbs": round(d["add_gbs"], 1),
                               "add_gbs_best": round(d["add_gbs_best"], 1),
                               "add_pct_hbm": round(100 * d["add_gbs"] / HBM_PEAK_GBS, 1),
                               "add_busy_gbs": round(d["add_busy_gbs"], 1),
                               "delete_us_median": round(d["delete_us_median"], 1),
                               "delete_gbs": (round(d["delete_gbs"], 1)
                                              if d["delete_gbs"] else None),
                               "dominant_kernel": d["dominant_kernel"]}
                    for k, d in r.items()}
                print(f"# qradd {label_n} {label}: " + ", ".join(
                    f"k={k} {d['add_gbs']:.0f}" for k, d in r.items()), file=sys.stderr,
                    flush=True)

    # ---- the 3D AA recycle iteration (C2) per variant --------------------------
    prob = Problem3D(args.s)
    c2_flags = aa.FUSE_RHS if args.rhs == "fused" else 0
    c2 = {}
    if not args.no_other_variants:
        for label, fl in QR_VARIANTS:
            v = variant_name(label)
            r = run_variant(prob, args.m, v, max(5, args.steps // 2), 2, args.grid,
                            flags=fl | c2_flags, keep_ctx=True)
            orth, kap = orthogonality(r["ctx"], args.m)
            r["ctx"].close()
            c2[label] = {"ms_per_step": round(r["ms_per_step"], 4), "gbs": round(r["gbs"], 1),
                         "pct_hbm_peak": round(100 * r["gbs"] / HBM_PEAK_GBS, 1),
                         "orthogonality_loss": orth, "kappa_R": kap,
                         "kernels": {kk: {"gbs": round(d["gbs"], 1) if d["gbs"] else None,
                                          "us_per_step": round(1e3 * d["ms"] / r["steps"], 1)}
                                     for kk, d in r["kernels"].items()}}
            print(f"# c2 {label} m={args.m}: {r['ms_per_step']:.3f} ms/step, "
                  f"{r['gbs']:.0f} GB/s, ||I-Q^TQ|| {orth:.1e} (kappa(R) {kap:.1e})",
                  file=sys.stderr, flush=True)

    fused = {}
    if not args.no_other_variants:
        # the same steps with R gamma = Q^T f_i folded into the QRAdd passes and
        # QRDelete fused with the QRAdd's first pass (same method, fewer passes)
        for v in ("cgs2", "dcgs2", "icwy"):
            r2 = run_variant(prob, args.m, v, max(5, args.steps // 2), 2, args.grid,
                             profile=False, flags=aa.FUSE_RHS | aa.FUSE_DELETE)
            fused[v] = {"ms_per_step": round(r2["ms_per_step"], 4),
                        "speedup_vs_separate": round(c2[v]["ms_per_step"] / r2["ms_per_step"], 3)}
            print(f"# {v} with the RHS folded and QRDelete fused with QRAdd: "
                  f"{r2['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)

    m_sweep = {}
    if not args.no_other_variants:
        # the other windows of the 3D workload (m = 5, 10, 50), paper passes
        for label, fl in QR_VARIANTS:
            v = variant_name(label)
            m_sweep[label] = {}
            for mm in (5, 10, 50):
                if mm == args.m:
                    continue
                r = run_variant(prob, mm, v, 5, 2, args.grid, flags=fl)
                m_sweep[label][f"m={mm}"] = {"ms_per_step": round(r["ms_per_step"], 4),
                                             "gbs": round(r["gbs"], 1),
                                             "pct_hbm_peak": round(100 * r["gbs"] / HBM_PEAK_GBS, 1)}
            print(f"# {label} m sweep: " + ", ".join(f"{k} {d['ms_per_step']:.2f} ms "
                                                      f"{d['gbs']:.0f} GB/s"
                                                      for k, d in m_sweep[label].items()),
                  file=sys.stderr, flush=True)

    graphs = graph_replay() if not args.no_other_variants else {}

    poisson = {}
    if not args.no_other_variants:
        for v in VARIANTS:
            poisson[v] = poisson1d_to_tolerance(v)
            print(f"# 1D Poisson n=4096 m=5 {v}: {poisson[v]['iterations']} iterations, "
                  f"{poisson[v]['gpu_ms']:.1f} ms (one-instance batch: "
                  f"{poisson[v]['batch_api_ms']:.1f} ms)", file=sys.stderr, flush=True)

    em = {}
    if not args.no_other_variants:
        for label, fl in QR_VARIANTS:
            em[label] = em_to_tolerance(variant_name(label), fl)
            print(f"# EM (n = 1.5e6, m = 3) {label}: {em[label]['iterations']} iterations to 1e-8, "
                  f"{em[label]['wall_ms']:.2f} ms (G {em[label]['g_ms']:.2f}, AA "
                  f"{em[label]['aa_ms']:.2f})", file=sys.stderr, flush=True)

    pde = {}
    if not args.no_other_variants:
        for pname, pid in PDE_PROBLEMS:
            pde[pname] = {}
            for label, fl in QR_VARIANTS:
                r = pde_to_tolerance(pid, variant_name(label), fl)
                pde[pname][label] = r
                print(f"# 2D {pname} (N = 1024, m = {r['m']}) {label}: {r['iterations']} "
                      f"iterations to 1e-10{'' if r['converged'] else ' (not converged)'}, "
                      f"{r['wall_ms']:.1f} ms (G {r['g_ms']:.1f}, AA {r['aa_ms']:.2f}; PCG "
                      f"{r['pcg_iterations_per_g']} per G)", file=sys.stderr, flush=True)

    batched = None
    if not args.no_batch:
        batched = batched_suite(args.variant, args.batch_count, args.batch_cap, args.train_count,
                                args.train_iters, args.single_sample,
                                ablation_cap=args.ablation_cap,
                                fuse=(aa.FUSE_RHS | aa.FUSE_DELETE)
                                if args.batch_passes == "fused" else 0)
        batched["tail_largest_instances"] = batched_tail(
            args.variant, fuse=(aa.FUSE_RHS | aa.FUSE_DELETE)
            if args.batch_passes == "fused" else 0)

    # the roofline of the headline add's dominant kernel: algorithmic bytes per
    # launch / its average launch duration (per-launch events on the
    # context's stream)
    dom = head["dominant_kernel"]
    kd = head["kernels"][dom]
    achieved = kd["gbs"]
    traffic = load_traffic(f"qradd_{args.variant}_k{args.k}_n2e26", dom)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "algorithmic_bytes_per_launch": kd["bytes_per_launch"],
                "us_per_launch": round(kd["us_per_launch"], 2),
                "frac_of_measured_ceiling": round(
                    achieved / max(ceil["8r0w"]["gbs_best"], ceil["8r1w"]["gbs_best"]), 4)}

    cpu = None
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(k=args.k, variant=args.variant, c2_s=args.s, c2_m=args.m)
        gpu_c2 = c2.get(args.variant)
        if gpu_c2:
            # the oracle's per-iteration time over the GPU's on the same
            # iteration: the ratio of the two solves' times to tolerance, whose
            # iteration counts agree (the host run itself would take hours)
            cpu["c2_iteration_all_cores"]["gpu_ms_per_iteration"] = gpu_c2["ms_per_step"]
            cpu["c2_iteration_all_cores"]["cpu_over_gpu"] = round(
                cpu["c2_iteration_all_cores"]["ms_per_iteration"] / gpu_c2["ms_per_step"], 1)

    line = {
        "metric": METRIC,
        "value": round(head["add_gbs"], 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["add_us_median"] / 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"QRAdd microbenchmark: {args.variant}, n = 2^26, k = {args.k} "
                               f"(the add into a {args.k + 1}-column window), seeded Gaussian "
                               f"columns orthonormalized by the library, v ~ N(0, 1)",
                   "variant": args.variant, "n": n_head, "k": args.k,
                   "parallelism": "single GPU"},
        "pct_hbm_peak": round(100.0 * head["add_gbs"] / HBM_PEAK_GBS, 2),
        "headline_add": {"us_median": round(head["add_us_median"], 1),
                         "us_min": round(head["add_us_min"], 1),
                         "gbs_median": round(head["add_gbs"], 1),
                         "gbs_best": round(head["add_gbs_best"], 1),
                         "busy_gbs": round(head["add_busy_gbs"], 1),
                         "algorithmic_bytes": head["add_bytes"],
                         "pct_of_measured_read_ceiling": round(
                             100 * head["add_gbs"] / ceil["8r0w"]["gbs_best"], 1),
                         "kernels": {kk: {a: round(b, 2) if isinstance(b, float) else b
                                          for a, b in d.items()}
                                     for kk, d in head["kernels"].items()}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "ceilings_n2e26": ceil,
        "qradd": qradd,
        "c2_step_256cubed": {"m": args.m, "rhs": args.rhs, "variants": c2,
                             "with_fused_rhs_and_delete": fused, "m_sweep": m_sweep},
        "poisson1d_to_1e-8": poisson,
        "em_to_1e-8": em,
        "pde2d_1024_to_1e-10": pde,
        "graph_replay_icwy_m20": graphs,
        "batched": batched,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
