#!/usr/bin/env python3
"""Throughput of the LEE + ghost-point IBM + ADE stage on one MI355X.

Metric: fluid grid-point Runge-Kutta stage updates per second, FP32 (the
reported value) and FP64, with the FP32 result's relative L2 error against
the FP64 oracle on the same workload.  Workload: the cylinder reflecting a
pulse on a 1024^2 grid (16/1024 spacing, r_c = 0.5, impedance (0.5, 0.02,
10), 11-point DRP + 11-point filter).  A "step" is one full RK4 time step:
four stages, each a ghost fill + ADE launch and a stage-sweep launch, plus
the step-end probe kernel, replayed from a captured hipGraph.

Roofline: the stage sweep dominates (>99% of bytes).  Its algorithmic traffic
per launch is the average over the four stages of (stage 1: read q^n,
write q^(1): 24 B; stages 2-4: read q^n and q^(l-1), write q^(l): 36 B) per
fluid node = 33 B (FP32), divided by the launch duration measured with HIP
events on the library's stream.

Also reported: FP64 throughput, the batched workload (uneven instances in
one launch per phase) when --batch is given, and the oracle on the host
cores over a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "grid-pt RK-stage updates/s FP32 vs FP64 at 1e-4 rel L2; p50/p99 solve latency"
UNIT = "grid-pt RK-stage updates/s"
HBM_PEAK_GBS = 8000.0


def _kernel_hash() -> str:
    with open(os.path.join(HERE, "paper_2609_24785_amd", "csrc", "lee_kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(bytes_alg_per_launch: float):
    """HBM bytes per sweep launch from the committed counter summary, if it was
    taken on the current kernel source."""
    path = os.path.join(HERE, "profiles", "sweep_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_sha") != _kernel_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def run(args):
    import numpy as np
    import torch

    import lee_cases as lc
    from paper_2609_24785_amd.lee import Instance

    if not torch.cuda.is_available():
        print(json.dumps({"metric": METRIC, "error": "no GPU visible"}))
        return 1
    torch.cuda.set_device(0)
    case = lc.cylinder_pulse_1024(steps=args.steps)
    total = args.warmup + args.steps + args.kernel_steps
    res = {}
    insts = {}
    for prec in ("f32", "f64"):
        inst = Instance(case, prec, trace_capacity=max(total, 1))
        insts[prec] = inst
        fluid = inst.summary.fluid_nodes
        inst.step_n(args.warmup)
        inst.synchronize()
        steps = args.steps if prec == "f32" else args.steps
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(inst.stream):
            ev0.record()
        t0 = time.perf_counter()
        inst.step_n(steps)
        with torch.cuda.stream(inst.stream):
            ev1.record()
        inst.synchronize()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        wall = t1 - t0
        gpu_ms = ev0.elapsed_time(ev1)
        # per-launch durations of the sweep and ghost kernels (HIP events on the
        # library's stream around every launch)
        sweep_us, ghost_us, eager_step_us = inst.time_kernels(args.kernel_steps)
        res[prec] = dict(wall=wall, gpu_ms=gpu_ms, steps=steps, fluid=fluid, sweep_us=sweep_us,
                         ghost_us=ghost_us, eager_step_us=eager_step_us,
                         value=fluid * 4.0 * steps / wall)
    p32 = insts["f32"].fields()
    p64 = insts["f64"].fields()
    import oracle.solver as osv   # CPU baseline and error reference (test infrastructure)
    from oracle.geometry import fluid_mask
    mask = fluid_mask(case)
    rel_32_64 = max(osv.relative_l2(a, b, mask) for a, b in zip(p32, p64))

    r = res["f32"]
    esz = 4
    bytes_per_node = (24.0 + 3 * 36.0) / 4.0          # average over the four stages (FP32)
    alg_bytes = bytes_per_node * r["fluid"]
    achieved = alg_bytes / (r["sweep_us"] * 1e-6) / 1e9
    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * r["wall"] / r["steps"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "cylinder-pulse 1024x1024, dx=1/64 on [-8,8)^2, r_c=0.5 shifted (0.3h,0.3h), "
                        "Gaussian pulse (4,0) a=1e-3 w=0.2, MSD R=0.5 m=0.02 k=10, 11-pt DRP + 11-pt filter "
                        "sigma=0.2, LSRK4 CFL 0.5, 8 probes on r=5",
            "grid": [case.nx, case.ny],
            "fluid_nodes": r["fluid"],
            "ghosts": int(insts["f32"].summary.G),
            "stages_per_step": 4,
            "launch": "hipGraph per step: 4 x (ghost fill+ADE, stage sweep) + step end",
        },
        "fp64_value": res["f64"]["value"],
        "fp32_vs_fp64_rel_l2": rel_32_64,
        "gpu_event_ms_per_step": r["gpu_ms"] / r["steps"],
        "kernels_us": {"sweep_f32": r["sweep_us"], "ghost_f32": r["ghost_us"],
                       "sweep_f64": res["f64"]["sweep_us"], "ghost_f64": res["f64"]["ghost_us"],
                       "eager_step_f32": r["eager_step_us"]},
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": _traffic(alg_bytes),
            "kernel": "k_sweep<float,4,filter,1>",
            "alg_bytes_per_launch": alg_bytes,
        },
    }
    # FP64 roofline of the same kernel (66 B per node-stage)
    out["roofline_f64_frac"] = (2 * alg_bytes / (res["f64"]["sweep_us"] * 1e-6) / 1e9) / HBM_PEAK_GBS

    if not args.no_cpu_baseline:
        nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        s = osv.OracleSolver(case)
        t0 = time.perf_counter()
        s.run(args.cpu_steps)
        t1 = time.perf_counter()
        cpu_rate = r["fluid"] * 4.0 * args.cpu_steps / (t1 - t0)
        # the FP32 GPU path on the same sample, against the oracle
        g = Instance(case, "f32")
        g.step_n(args.cpu_steps)
        g.synchronize()
        gf = g.fields()
        of = s.fields()
        rel = max(osv.relative_l2(a, b, mask) for a, b in zip(gf, of))
        out["cpu_baseline"] = {
            "value": cpu_rate, "unit": UNIT, "cores": nthreads, "kind": "oracle",
            "sample": f"same workload, first {args.cpu_steps} steps, FP64 C core with OpenMP over rows, "
                      f"stepping loop only ({t1 - t0:.1f} s)",
        }
        out["fp32_vs_oracle_rel_l2"] = rel
        out["fp32_vs_oracle_steps"] = args.cpu_steps
    print(json.dumps(out), flush=True)
    return 0


def profile_run(args):
    """A short fixed sequence for hardware profilers: the benchmark workload for
    a few steps (graph replay, FP32), then a copy of known size."""
    import torch

    import lee_cases as lc
    from paper_2609_24785_amd import _lib
    from paper_2609_24785_amd.lee import Instance

    torch.cuda.set_device(0)
    case = lc.cylinder_pulse_1024(steps=args.steps)
    inst = Instance(case, "f32", trace_capacity=args.steps + args.warmup)
    inst.step_n(args.warmup + args.steps)
    inst.synchronize()
    nbytes = 1 << 30
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream()
    for _ in range(3):
        _lib.check(_lib.load().lee_stream_copy(a.data_ptr(), b.data_ptr(), nbytes, s.cuda_stream), "copy")
    torch.cuda.synchronize()
    print(json.dumps({"profile_run": True, "steps": args.steps + args.warmup, "copy_bytes": nbytes,
                      "fluid_nodes": inst.summary.fluid_nodes}), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--kernel-steps", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-run", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the path is a single-GPU kernel and this build has no "
              "multi-GPU mode (instances shard by bytes with no communication; see the design notes).",
              file=sys.stderr)
        return 2
    if args.profile_run:
        return profile_run(args)
    return run(args)


if __name__ == "__main__":
    sys.exit(main())
