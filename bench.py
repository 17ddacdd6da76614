#!/usr/bin/env python3
"""Benchmark of the Anderson-acceleration hot path on one MI355X.

Workload (the 3D nonlinear fixed-point problem): G(u) = u - omega (A u + u^3 - f)
on a 256^3 Dirichlet grid (n = 16,777,216), f ~ U[0, 1] (seed 2), u_0 = 0,
window m = 20, FP64.  A step is one full recycle iteration of Alg. 1: one
evaluation of G (HIP stencil kernel) and one ``aa_step`` -- history
formation, QRDelete by Givens rotations, QRAdd of Delta f_{i-1} by the chosen
variant, R gamma = Q^T f_i and the x update.  The window is filled (m + 1
untimed start-up iterations) before the warmup, so every timed step deletes
and adds a column.

value = algorithmic HBM bytes of one step / time of one step, in GB/s, where
every n-vector a kernel must read or write counts 8 n bytes once (the library
accounts this per launch from its column counts; the stencil counts 3
vectors).  The roofline object reports the kernel kind with the largest
share of the step time, timed by HIP events that the library records around
each launch on its stream during the timed steps.

The CPU baseline is the FP64 oracle (single thread) on a bounded sample of the
same configuration: a 128^3 grid, same m and variant, 3 recycle iterations
timed after filling the window; same byte model.
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


def run_variant(prob, m, variant, steps, warmup, grid=None, profile=True):
    import torch
    from paper_2110_09667_amd import aa

    n = prob.n
    dev = torch.device("cuda:0")
    f_d = device_rhs(prob)
    ctx = aa.AAContext(n, m, variant)
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
    if profile:
        ctx.profile(True)
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    prof = ctx.profile_read() if profile else {}
    info = ctx.info()
    if info.status != 0:
        raise RuntimeError(f"{variant}: device status {info.status}")
    u_bytes = 8.0 * n
    bytes_per_step = (sum(b for (_, _, b) in prof.values()) / steps + 3 * u_bytes) if prof else None
    out = {
        "variant": variant,
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
    ctx.close()
    del x, g, f_d
    torch.cuda.empty_cache()
    return out


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


def cpu_baseline(m, variant, s=128, timed_steps=3):
    import numpy as np

    import aa_workloads as W
    import oracle as O
    if not os.path.exists(O.LIB_PATH):
        O.build()
    prob = W.nonlinear3d(s=s)
    n = prob.n
    st = O.AA(n, m, variant)
    x = np.zeros(n)
    for _ in range(m + 1):
        x = st.step(x, O.G_stencil(prob, x))
    t0 = time.perf_counter()
    for _ in range(timed_steps):
        x = st.step(x, O.G_stencil(prob, x))
    dt = time.perf_counter() - t0
    u = 8.0 * n
    k = m - 1
    add = {"mgs": 4 * k + 3, "cgs2": 3 * k + 6, "dcgs2": 2 * k + (6 if k >= 3 else 5),
           "icwy": 2 * k + 5}[variant]
    vecs = 3 + 8 + (2 * m - 1) + add + 2 + (m + 1) + (m + 3)
    return {"value": vecs * u * timed_steps / dt / 1e9, "unit": "GB/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"FP64 C oracle, 1 thread: {timed_steps} recycle iterations of the same "
                       f"configuration (m={m}, {variant}) on a {s}^3 grid (n={n}) after "
                       f"filling the window; {dt:.2f} s timed")}


def load_traffic(kind, variant, m):
    """HBM bytes per launch measured with rocprofv3 counters, if a summary for
    this kernel and configuration is committed and still current."""
    try:
        with open(PROFILE_JSON) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    key = f"{kind}/{variant}/m{m}"
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


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variant", default="icwy", choices=VARIANTS)
    ap.add_argument("--m", type=int, default=20)
    ap.add_argument("--s", type=int, default=256, help="grid points per side")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other-variants", action="store_true")
    ap.add_argument("--grid", type=int, nargs=2, default=None,
                    help="max workgroups: streaming passes, Gram pass")
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
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import aa_workloads as W
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_2110_09667_amd import aa
    if not os.path.exists(aa.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    aa.lib()

    prob = Problem3D(args.s)
    print(f"# workload: 3D nonlinear, s={args.s}, n={prob.n}, m={args.m}", file=sys.stderr,
          flush=True)
    main_res = run_variant(prob, args.m, args.variant, args.steps, args.warmup, args.grid)
    print(f"# {args.variant}: {main_res['ms_per_step']:.3f} ms/step, "
          f"{main_res['gbs']:.0f} GB/s", file=sys.stderr, flush=True)
    others = {}
    if not args.no_other_variants:
        for v in VARIANTS:
            if v == args.variant:
                continue
            r = run_variant(prob, args.m, v, max(5, args.steps // 2), 2, args.grid)
            others[v] = r
            print(f"# {v}: {r['ms_per_step']:.3f} ms/step, {r['gbs']:.0f} GB/s",
                  file=sys.stderr, flush=True)

    kern = main_res["kernels"]
    dom = max(kern, key=lambda k: kern[k]["ms"])
    achieved = kern[dom]["gbs"]
    traffic = load_traffic(dom, args.variant, args.m)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": traffic,
                "launches": kern[dom]["launches"],
                "algorithmic_bytes_per_launch": kern[dom]["bytes"] / kern[dom]["launches"]}

    cpu = None
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.m, args.variant)

    per_variant = {args.variant: main_res, **others}
    line = {
        "metric": METRIC,
        "value": main_res["gbs"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"AA recycle iteration, 3D nonlinear {args.s}^3 "
                               f"(n={prob.n}), m={args.m}",
                   "variant": args.variant, "n": prob.n, "m": args.m,
                   "parallelism": "single GPU"},
        "pct_hbm_peak": 100.0 * main_res["gbs"] / HBM_PEAK_GBS,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "per_variant": {v: {"ms_per_step": r["ms_per_step"], "gbs": r["gbs"],
                            "pct_hbm_peak": 100.0 * r["gbs"] / HBM_PEAK_GBS,
                            "kernels": {k: round(d["gbs"], 1) if d["gbs"] else None
                                        for k, d in r["kernels"].items()}}
                        for v, r in per_variant.items()},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
