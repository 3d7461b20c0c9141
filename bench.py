#!/usr/bin/env python3
"""Throughput of the LEE + ghost-point IBM + ADE stage on one MI355X.

Metric: fluid grid-point Runge-Kutta stage updates per second.  The reported
value is FP32; FP64 is reported beside it, with the FP32 result's relative L2
error against the FP64 run at the workload's stated step count, against the
FP64 oracle over a bounded sample, and the served stream's p50/p99 latency.

Workload: the cylinder scattering a harmonic monopole on a 4096^2 grid
(h = 1/128 on [-16, 16)^2, r_c = 1, impedance (R, m, k) = (1, 0.01, 5) with
two real poles, monopole at (4, 0) with omega = 4 pi and half-width 3 h,
64-cell sponge, 11-point DRP and 11-point filter, LSRK4 at CFL 0.5, 20000
steps, amplitudes by a running DFT over the last 10 periods on two rings of
180 points).  Its working set (about 600 MB in FP32) exceeds the on-chip
cache, so its fraction of the HBM roofline is meaningful.  A step is one full
RK4 time step (four stages of ghost fill + ADE update and stage sweep),
replayed from captured hipGraphs.  Inputs are resident in HBM when the timed
region starts, and the graphs for the timed run length are captured before
it.

Roofline: the stage sweep moves more than 99% of the bytes.  Its algorithmic
traffic per launch is the mean over the four stages of 24 B (stage 1: read
q^n, write q^(1)) and 36 B (stages 2-4: read q^n and q^(l-1), write q^(l))
per fluid node, 33 B in FP32, plus the fused launch's ghost fill, divided by
the mean launch time measured with HIP events on the library's stream over
back-to-back launches.

The launch configuration (tile shape, fused or two-launch stage, steps per
graph) is chosen by the library's autotuner (shipped table, else trials).
Also reported: the oracle on the host cores over a bounded sample of the
workload (all threads and one thread).

Other modes: --extras (a second JSON line: the 1024^2 cylinder pulse, whose
working set sits in the on-chip cache and is reported as effective
bandwidth; the flat-wall case against the oracle; the 1024^2 case with the
paper's 7-point stencils and no filter, with a multi-pole wall and with the
radiation band; the paper's own configuration; the spectral analysis; the
batch of 256 uneven instances),
--serve (the served request stream: Poisson arrivals, continuous batching,
admission by HBM budget; throughput and p50/p99 latency),
--profile-run (a short fixed sequence for rocprofv3), and
--counters FETCH_CSV WRITE_CSV KERNEL (turns two rocprofv3 --pmc counter
files of the profile run into KERNEL's HBM traffic per launch, calibrated by
the copy kernel of known size the profile run ends with).
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
BYTES_PER_NODE_STAGE = {"f32": (24.0 + 3 * 36.0) / 4.0, "f64": (48.0 + 3 * 72.0) / 4.0}


def ghost_bytes(prec: str, G: int, nnz: int) -> float:
    """Algorithmic bytes of one stage's ghost fill: per cloud entry 4 weights
    and an offset; per ghost its geometry, two ADE state reads and one write,
    its offset and the three ghost values written (the gathered fluid values
    are the sweep's)."""
    e = 4 if prec == "f32" else 8
    return nnz * (4 * e + 4) + G * (4 * e + 3 * 2 * e + 4 + 3 * e)
COUNTERS_JSON = os.path.join(HERE, "profiles", "sweep_counters.json")
COPY_BYTES = 1 << 28                     # the profile run's calibration copy (256 MiB)


def _kernel_hash() -> str:
    """Hash of the kernels and of the code that orders their work (the tile
    order sets which halos the L2s still hold, hence the HBM traffic)."""
    h = hashlib.sha256()
    for name in ("lee_kernels.hip", "lee_device.h", "lee_api.hip"):
        with open(os.path.join(HERE, "paper_2609_24785_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _traffic(kernel: str):
    """HBM bytes per sweep launch from the committed counter summary, when it
    was taken on the current kernel source and the same kernel instance."""
    if not os.path.exists(COUNTERS_JSON):
        return None
    with open(COUNTERS_JSON) as f:
        d = json.load(f)
    if d.get("kernel_sha") != _kernel_hash() or d.get("kernel") != kernel:
        return None
    return d.get("hbm_bytes_per_launch")


def _kernel_name(tiling: dict, prec: str) -> str:
    t = "float, 4" if prec == "f32" else "double, 2"
    if tiling["kind"] == "tile":
        k = "k_stage" if tiling.get("fused") else "k_tile"
        extra = ", 32, 1" if tiling.get("fused") else ""        # lanes per ghost (fused), one-instance variant
        return f"lee::{k}<{t}, true, {tiling['cols']}, {tiling['rows']}{extra}>"
    return f"lee::k_sweep<{t.split(',')[0]}, {tiling['vec']}, true, {tiling['waves']}>"


def _apply(inst, choice):
    if choice:
        inst.set_tiling(**choice["tiling"])
        inst.set_graph_steps(choice["graph_steps"])


def _timed(case, prec: str, steps: int, warmup: int, choice=None, dft=None, trace_capacity=None, fresh=False):
    """Graph-replayed steps of one instance; returns the rate and the instance.
    The run of `steps` steps is issued once untimed first, so that its graphs
    are captured before the timed run; with fresh, the instance then goes
    back to its initial state (the graphs stay), so that the timed run is
    the case's own time span."""
    import torch
    from paper_2609_24785_amd.lee import Instance

    cap = trace_capacity if trace_capacity is not None else max(2 * steps + warmup, 1)
    inst = Instance(case, prec, trace_capacity=cap, dft=dft)
    _apply(inst, choice)
    inst.step_n(warmup)
    inst.step_n(steps)
    inst.synchronize()
    if fresh:
        inst.init_fields()
        inst.synchronize()
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
    wall = time.perf_counter() - t0
    fluid = inst.summary.fluid_nodes
    return dict(inst=inst, wall=wall, gpu_ms=ev0.elapsed_time(ev1), steps=steps, fluid=fluid,
                value=fluid * 4.0 * steps / wall)


def _kernel_times(case, prec: str, n: int, choice=None):
    """Mean per-launch times of the sweep and ghost kernels (back-to-back
    launches on the library's stream, one event pair per kernel kind)."""
    from paper_2609_24785_amd.lee import Instance

    inst = Instance(case, prec, trace_capacity=1)
    _apply(inst, choice)
    inst.time_kernels(2)                                  # warm the code objects
    sweep_us, ghost_us, step_us = inst.time_kernels(n)
    tiling = inst.get_tiling()
    fluid = inst.summary.fluid_nodes
    ghosts = inst.summary.G
    nnz = inst.summary.nnz
    inst.close()
    alg = BYTES_PER_NODE_STAGE[prec] * fluid + (ghost_bytes(prec, ghosts, nnz) if tiling.get("fused") else 0.0)
    return dict(sweep_us=sweep_us, ghost_us=ghost_us, eager_step_us=step_us, tiling=tiling, fluid=fluid,
                ghosts=ghosts, nnz=nnz, kernel=_kernel_name(tiling, prec), alg_bytes=alg)


def _copy_rate(nbytes: int = 1 << 30, reps: int = 10) -> float:
    """Achievable HBM rate: the library's plain copy kernel, GB/s (read + write)."""
    import torch
    from paper_2609_24785_amd import _lib

    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream()
    lib = _lib.load()
    for _ in range(2):
        _lib.check(lib.lee_stream_copy(b.data_ptr(), a.data_ptr(), nbytes, s.cuda_stream), "copy")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        _lib.check(lib.lee_stream_copy(b.data_ptr(), a.data_ptr(), nbytes, s.cuda_stream), "copy")
    e1.record()
    torch.cuda.synchronize()
    rate = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return rate


def _max_rel_l2(a, b, mask):
    from oracle.solver import relative_l2
    return max(relative_l2(x, y, mask) for x, y in zip(a, b))


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _ring_dft(inst, case):
    """Complex ring amplitudes P = (2i/N) sum_n p(t_n) exp(-i omega t_n) over
    the last N = dft_steps steps (p(t) = Im(P exp(i omega t))), as
    lee_probe_dft returns them."""
    return inst.dft()


def _serve_short(args):
    """A short window of the served request stream (its p50/p99 latency)."""
    import lee_cases as lc
    from paper_2609_24785_amd.serve import GpuBackend, Request, Server

    reqs = [Request(k, c, t) for k, (t, c) in
            enumerate(lc.request_stream(seed=26091, rate=args.serve_rate, duration=args.serve_duration))]
    be = GpuBackend("f32")
    try:
        srv = Server(be, budget_bytes=args.serve_budget_gb * 1e9, chunk=args.serve_chunk,
                     report=lambda st: print(f"[serve] {json.dumps(st)}", file=sys.stderr, flush=True))
        res = srv.run(reqs)
    finally:
        be.close()
    return srv, res


def run(args):
    import numpy as np
    import torch

    import lee_cases as lc

    if not torch.cuda.is_available():
        print(json.dumps({"metric": METRIC, "error": "no GPU visible"}))
        return 1
    torch.cuda.set_device(0)
    from paper_2609_24785_amd import tune
    case = lc.monopole_4096()
    dft = (case.source.omega, case.steps - case.dft_steps, case.dft_steps)
    print("[bench] autotuning the launch configuration", file=sys.stderr, flush=True)
    cache = tune.TuneCache(args.tune_cache, shipped=not args.retune)   # the shipped table, then live trials
    ch32 = tune.tune_case(case, "f32", cache)
    ch64 = tune.tune_case(case, "f64", cache)
    print(f"[bench] {case.name}: {args.steps} steps after {args.warmup} warm-up, FP32 then FP64",
          file=sys.stderr, flush=True)
    r32 = _timed(case, "f32", args.steps, args.warmup, ch32, dft=dft, trace_capacity=1)
    r64 = _timed(case, "f64", args.steps, args.warmup, ch64, dft=dft, trace_capacity=1)
    print("[bench] kernel timing", file=sys.stderr, flush=True)
    k32 = _kernel_times(case, "f32", args.kernel_steps, ch32)
    k64 = _kernel_times(case, "f64", args.kernel_steps, ch64)
    copy_gbs = _copy_rate()

    import oracle.solver as osv          # error reference and CPU baseline (test infrastructure)
    from oracle.geometry import fluid_mask
    mask = fluid_mask(case)
    rel_timed = _max_rel_l2(r32["inst"].fields(), r64["inst"].fields(), mask)

    # the stated step count: both timed instances continue to the workload's
    # 20000 steps (the DFT window is its last 10 periods)
    stated = {}
    if not args.no_stated:
        print(f"[bench] FP32 and FP64 to the stated {case.steps} steps", file=sys.stderr, flush=True)
        for r in (r32, r64):
            left = case.steps - r["inst"].step
            if left > 0:
                r["inst"].step_n(left)
            r["inst"].synchronize()
        f32, f64 = r32["inst"].fields(), r64["inst"].fields()
        a32, a64 = _ring_dft(r32["inst"], case), _ring_dft(r64["inst"], case)
        rel = _max_rel_l2(f32, f64, mask)
        ring = float(np.abs(a32 - a64).max() / np.abs(a64).max())
        stated = {"steps": case.steps, "fp32_vs_fp64_rel_l2": rel,
                  "ring_dft_fp32_vs_fp64_max_rel": ring,
                  "ring_amplitude_abs_mean": {"r=1.1": float(np.abs(a64[:180]).mean()),
                                              "r=5": float(np.abs(a64[180:]).mean())},
                  "within_tolerance": bool(rel <= 1e-4 and ring <= 1e-4)}

    alg_bytes = k32["alg_bytes"]
    achieved = alg_bytes / (k32["sweep_us"] * 1e-6) / 1e9
    ach64 = k64["alg_bytes"] / (k64["sweep_us"] * 1e-6) / 1e9
    traffic = _traffic(k32["kernel"])
    out = {
        "metric": METRIC,
        "value": r32["value"],
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * r32["wall"] / r32["steps"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "monopole-cylinder 4096x4096, h=1/128 on [-16,16)^2, r_c=1 at the origin, monopole (4,0) "
                        "a=1 omega=4pi half-width 3h, MSD R=1 m=0.01 k=5 (two real poles), 64-cell sponge, 11-pt "
                        "DRP + 11-pt filter sigma=0.2, LSRK4 CFL 0.5, 20000 steps, running DFT over the last 10 "
                        "periods on rings r=1.1 and r=5 (360 probes)",
            "grid": [case.nx, case.ny],
            "fluid_nodes": r32["fluid"],
            "ghosts": int(r32["inst"].summary.G),
            "tiling_f32": k32["tiling"],
            "tiling_f64": k64["tiling"],
            "graph_steps": ch32["graph_steps"],
            "tuning_from": "table" if ch32.get("cached") else "trials",
            "launch": "hipGraphs of captured runs of steps (one graph per run length, captured before the timed "
                      "run); a step is 4 x (ghost fill + ADE, stage sweep; one launch when fused), probes and DFT "
                      "riding in the next step's second stage",
        },
        "fp64_value": r64["value"],
        "fp64_ms_per_step": 1000.0 * r64["wall"] / r64["steps"],
        "fp32_vs_fp64_rel_l2_timed_run": rel_timed,
        "stated_steps": stated,
        "gpu_event_ms_per_step": r32["gpu_ms"] / r32["steps"],
        "kernels_us": {"sweep_f32": k32["sweep_us"], "ghost_f32": k32["ghost_us"],
                       "sweep_f64": k64["sweep_us"], "ghost_f64": k64["ghost_us"],
                       "eager_step_f32": k32["eager_step_us"], "eager_step_f64": k64["eager_step_us"]},
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": k32["kernel"],
            "alg_bytes_per_launch": alg_bytes,
            "launch_us": k32["sweep_us"],
            "copy_kernel_GBs": copy_gbs,
        },
        "roofline_f64": {"kernel": k64["kernel"], "achieved": ach64, "frac": ach64 / HBM_PEAK_GBS,
                         "launch_us": k64["sweep_us"]},
    }
    r32["inst"].close()
    r64["inst"].close()
    torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        print(f"[bench] oracle on the host: {args.cpu_steps} steps, then {args.cpu_steps_1t} on one thread",
              file=sys.stderr, flush=True)
        s = osv.OracleSolver(case)
        nthreads = osv.set_threads(0)
        t0 = time.perf_counter()
        s.run(args.cpu_steps)
        t1 = time.perf_counter()
        cpu_rate = r32["fluid"] * 4.0 * args.cpu_steps / (t1 - t0)
        from paper_2609_24785_amd.lee import Instance
        g = Instance(case, "f32", trace_capacity=1)
        _apply(g, ch32)                                 # the configuration timed above
        g.step_n(args.cpu_steps)
        g.synchronize()
        out["fp32_vs_oracle_rel_l2"] = _max_rel_l2(g.fields(), s.fields(), mask)
        out["fp32_vs_oracle_steps"] = args.cpu_steps
        g.close()
        del s
        s1 = osv.OracleSolver(case)
        osv.set_threads(1)
        t2 = time.perf_counter()
        s1.run(args.cpu_steps_1t)
        t3 = time.perf_counter()
        osv.set_threads(nthreads)
        del s1
        out["cpu_baseline"] = {
            "value": cpu_rate, "unit": UNIT, "cores": nthreads, "kind": "oracle",
            "sample": f"the workload's first {args.cpu_steps} steps (FP64 C core, OpenMP over rows, stepping loop "
                      f"only, {t1 - t0:.1f} s)",
            "cpu_model": _cpu_model(),
            "one_thread_value": r32["fluid"] * 4.0 * args.cpu_steps_1t / (t3 - t2),
            "one_thread_sample": f"the workload's first {args.cpu_steps_1t} steps on one thread ({t3 - t2:.1f} s)",
        }

    if not args.no_serve:
        print(f"[bench] served stream: {args.serve_duration} s of arrivals at {args.serve_rate}/s",
              file=sys.stderr, flush=True)
        srv, res = _serve_short(args)
        st = srv.stats
        out["serve"] = {"window_s": args.serve_duration, "arrival_rate": args.serve_rate,
                        "requests": len(res), "served": sum(1 for r in res if r.error is None),
                        "refused": sum(1 for r in res if r.error is not None),
                        "latency_p50_s": st.get("p50_latency_s"), "latency_p99_s": st.get("p99_latency_s"),
                        "throughput": st.get("throughput")}
    print(json.dumps(out), flush=True)
    return 0


def extras(args):
    """Second JSON line: the other configurations (not the benchmark line)."""
    import torch

    import lee_cases as lc
    import oracle.solver as osv
    from paper_2609_24785_amd import tune
    from paper_2609_24785_amd._lib import LeeError
    from paper_2609_24785_amd.lee import Batch, Instance

    torch.cuda.set_device(0)
    out = {"extras": True}
    cache = tune.TuneCache(args.tune_cache, shipped=not args.retune)

    # the cylinder pulse on 1024^2 at its stated 4000 steps: its working set
    # (about 38 MB in FP32) sits in the on-chip cache, so its rate is an
    # effective bandwidth, not an HBM fraction
    print("[extras] cylinder pulse 1024^2, 4000 steps", file=sys.stderr, flush=True)
    import numpy as np
    from oracle.geometry import fluid_mask
    cp = lc.cylinder_pulse_1024()
    cres, flds = {}, {}
    for prec in ("f32", "f64"):
        ch = tune.tune_case(cp, prec, cache)
        rc_ = _timed(cp, prec, cp.steps, 0, ch, fresh=True)
        k = _kernel_times(cp, prec, args.kernel_steps, ch)
        cres[prec] = {"value": rc_["value"], "ms_per_step": 1000.0 * rc_["wall"] / rc_["steps"],
                      "tiling": ch["tiling"], "graph_steps": ch["graph_steps"], "kernel": k["kernel"],
                      "launch_us": k["sweep_us"],
                      "effective_GBs": k["alg_bytes"] / (k["sweep_us"] * 1e-6) / 1e9}
        flds[prec] = rc_["inst"].fields()
        rc_["inst"].close()
    cres["fp32_vs_fp64_rel_l2_after_4000_steps"] = _max_rel_l2(flds["f32"], flds["f64"], fluid_mask(cp))
    out["cylinder_pulse_1024"] = dict(steps=cp.steps, unit=UNIT, working_set="cache-resident", **cres)

    print("[extras] flat wall 201^2 FP64 against the oracle", file=sys.stderr, flush=True)
    flat = lc.flat_wall_201(500)
    rf = _timed(flat, "f64", 500, 0, fresh=True)
    s = osv.OracleSolver(flat)
    s.run(500)
    out["flat_wall_201_f64"] = {"value": rf["value"], "unit": UNIT, "steps": 500,
                                "rel_l2_vs_oracle": _max_rel_l2(rf["inst"].fields(), s.fields(), s.fluid)}
    rf["inst"].close()
    print("[extras] monopole 4096^2", file=sys.stderr, flush=True)
    mono = lc.monopole_4096(args.mono_steps)
    mres = {}
    for prec in ("f32", "f64"):
        ch = tune.tune_case(mono, prec, cache)
        rm = _timed(mono, prec, args.mono_steps, 16, ch)
        mres[prec] = {"value": rm["value"], "ms_per_step": 1000.0 * rm["wall"] / rm["steps"],
                      "fluid_nodes": rm["fluid"], "tiling": ch["tiling"]}
        rm["inst"].close()
        torch.cuda.empty_cache()
    out["monopole_4096"] = dict(steps=args.mono_steps, unit=UNIT, **mres)

    # the benchmark workload in the paper's own scheme: 7-point DRP stencils
    # (H = 3) and no selective filter; FP64 is checked against the oracle
    print("[extras] cylinder pulse 1024^2, 7-point DRP without filter", file=sys.stderr, flush=True)
    pm_steps = 500
    pm = lc.cylinder_pulse_1024(pm_steps).replace(H=3, filter_sigma=0.0)
    pres = {}
    for prec in ("f32", "f64"):
        ch = tune.tune_case(pm, prec, cache)
        rp = _timed(pm, prec, pm_steps, 0, ch, fresh=True)
        pres[prec] = {"value": rp["value"], "ms_per_step": 1000.0 * rp["wall"] / rp["steps"],
                      "tiling": ch["tiling"]}
        if prec == "f64":
            s = osv.OracleSolver(pm)
            s.run(pm_steps)
            pres[prec]["rel_l2_vs_oracle"] = _max_rel_l2(rp["inst"].fields(), s.fields(), s.fluid)
        rp["inst"].close()
    out["cylinder_pulse_1024_7pt"] = dict(steps=pm_steps, unit=UNIT, **pres)

    # the benchmark workload with a broadband multi-pole wall (Sec. 2.3): two
    # relaxation terms and three resonances, eight auxiliary states per ghost
    print("[extras] cylinder pulse 1024^2, multi-pole wall", file=sys.stderr, flush=True)
    mp = lc.cylinder_pulse_1024(pm_steps).replace(impedance=lc.Impedance(
        "poles", real=((-5.0, 8.0), (-40.0, 4.0)),
        pairs=((-12.5, 18.5, 12.0, -8.0), (-3.0, 30.0, 2.0, 1.0), (-20.0, 60.0, 1.5, 0.5))))
    mres = {}
    for prec in ("f32", "f64"):
        ch = tune.tune_case(mp, prec, cache)
        rp = _timed(mp, prec, pm_steps, 0, ch, fresh=True)
        mres[prec] = {"value": rp["value"], "ms_per_step": 1000.0 * rp["wall"] / rp["steps"],
                      "tiling": ch["tiling"]}
        if prec == "f64":
            s = osv.OracleSolver(mp)
            s.run(pm_steps)
            mres[prec]["rel_l2_vs_oracle"] = _max_rel_l2(rp["inst"].fields(), s.fields(), s.fluid)
        rp["inst"].close()
    out["cylinder_pulse_1024_multipole"] = dict(steps=pm_steps, unit=UNIT, ade_states=8, **mres)

    # the benchmark workload truncated by the outer radiation condition
    # instead of the zero frame; FP64 is checked against the oracle
    print("[extras] cylinder pulse 1024^2, radiation condition", file=sys.stderr, flush=True)
    rc = lc.cylinder_pulse_1024(pm_steps).replace(radiation=True, rad_center=(0.0, 0.0))
    rres = {}
    for prec in ("f32", "f64"):
        ch = tune.tune_case(rc, prec, cache)
        rp = _timed(rc, prec, pm_steps, 0, ch, fresh=True)
        rres[prec] = {"value": rp["value"], "ms_per_step": 1000.0 * rp["wall"] / rp["steps"],
                      "tiling": ch["tiling"]}
        if prec == "f64":
            s = osv.OracleSolver(rc)
            s.run(pm_steps)
            rres[prec]["rel_l2_vs_oracle"] = _max_rel_l2(rp["inst"].fields(), s.fields(), s.fluid)
        rp["inst"].close()
    out["cylinder_pulse_1024_radiation"] = dict(steps=pm_steps, unit=UNIT, **rres)

    # the paper's own cylinder-pulse configuration (7-point scheme, no filter,
    # radiation on all four sides, 301^2); FP64 is checked against the oracle
    print("[extras] paper cylinder pulse 301^2", file=sys.stderr, flush=True)
    pc_steps = 400
    pc = lc.paper_cylinder_pulse(pc_steps)
    pres = {}
    for prec in ("f32", "f64"):
        ch = tune.tune_case(pc, prec, cache)
        rp = _timed(pc, prec, pc_steps, 0, ch, fresh=True)
        pres[prec] = {"value": rp["value"], "ms_per_step": 1000.0 * rp["wall"] / rp["steps"],
                      "tiling": ch["tiling"]}
        if prec == "f64":
            s = osv.OracleSolver(pc)
            s.run(pc_steps)
            pres[prec]["rel_l2_vs_oracle"] = _max_rel_l2(rp["inst"].fields(), s.fields(), s.fluid)
        rp["inst"].close()
    out["paper_cylinder_pulse_301"] = dict(steps=pc_steps, unit=UNIT, **pres)

    # the paper's own monopole configuration (Sec. 4.3), its whole time span,
    # ring amplitudes over its window against App. C: the total field, and
    # the scattered field (the run minus the same grid without the cylinder,
    # against the exact total minus the free field), the paper's measure
    print("[extras] paper monopole 601^2", file=sys.stderr, flush=True)
    from tests import refsol
    pmc = lc.paper_monopole()
    xy = np.array(pmc.probes)
    imp = pmc.impedance
    om = pmc.source.omega
    Z = imp.R + 1j * (imp.M * om - imp.K / om)
    P, Pfree = refsol.monopole_cylinder(xy[:, 0], xy[:, 1], om, 1.0, 0.2, 4.0, 0.0, 0.5, Z=Z)
    dft = (om, pmc.steps - pmc.dft_steps, pmc.dft_steps)
    rings = {"r=0.6": slice(0, 72), "r=5": slice(72, 144)}

    def ring_err(got, ref):
        return {k: float(np.linalg.norm(got[sl] - ref[sl]) / np.linalg.norm(ref[sl])) for k, sl in rings.items()}

    pres = {}
    for prec in ("f32", "f64"):
        ch = tune.tune_case(pmc, prec, cache)
        rp = _timed(pmc, prec, pmc.steps, 0, ch, dft=dft, fresh=True)
        got = rp["inst"].dft()
        rp["inst"].close()
        free = Instance(pmc.replace(wall=lc.Wall()), prec, dft=dft)
        free.step_n(pmc.steps)
        free.synchronize()
        got_free = free.dft()
        free.close()
        pres[prec] = {"value": rp["value"], "ms_per_step": 1000.0 * rp["wall"] / rp["steps"],
                      "tiling": ch["tiling"], "steps_timed": pmc.steps,
                      "ring_error_vs_app_c": ring_err(got, P),
                      "scattered_ring_error_vs_app_c": ring_err(got - got_free, P - Pfree),
                      "free_field_ring_error": ring_err(got_free, Pfree)}
    out["paper_monopole_601"] = dict(unit=UNIT, steps=pmc.steps, **pres)

    # spectral stability of the step map (abstract): assembled on the GPU for
    # coarse cylinders and checked against the oracle's assembly; the growth
    # per step of the worst mode of the benchmark grid by power iteration
    print("[extras] spectral analysis", file=sys.stderr, flush=True)
    import numpy as np
    from oracle import spectral as osp
    from paper_2609_24785_amd import stability
    scan = []
    for d in (0.0, 0.25, 0.49):
        sc = lc.coarse_cylinder(28, 4.0, d, 0.5 * d)
        inst = Instance(sc, "f64")
        t0 = time.perf_counter()
        G = stability.step_matrix(inst)
        t_gpu = time.perf_counter() - t0
        inst.close()
        t0 = time.perf_counter()
        R = osp.step_matrix(sc)
        t_cpu = time.perf_counter() - t0
        scan.append({"shift": [d, 0.5 * d], "states": int(G.shape[0]),
                     "spectral_radius": stability.spectral_radius(G),
                     "spectral_radius_oracle": osp.spectral_radius(R),
                     "max_abs_diff_vs_oracle": float(np.abs(G - R).max()),
                     "gpu_columns_per_s": G.shape[0] / t_gpu, "oracle_columns_per_s": R.shape[0] / t_cpu})
    # the semi-discrete operator L (growth rates per unit time, free of dt):
    # the paper's scheme and the filtered one on the same coarse cylinders,
    # through the library (lee_rhs) and the oracle
    semi = []
    for d in (0.0, 0.25, 0.49):
        for name, H, fs in (("paper-scheme", 3, 0.0), ("11pt-filter", 5, 0.2)):
            sc = lc.coarse_cylinder(28, 4.0, d, 0.5 * d, H=H, filter_sigma=fs)
            inst = Instance(sc, "f64")
            Lg = stability.operator_matrix(inst)
            inst.close()
            Lo = osp.operator_matrix(sc)
            semi.append({"shift": [d, 0.5 * d], "scheme": name, "states": int(Lg.shape[0]),
                         "abscissa_per_unit_time": stability.spectral_abscissa(Lg),
                         "abscissa_oracle": osp.spectral_abscissa(Lo),
                         "max_abs_diff_vs_oracle": float(np.abs(Lg - Lo).max())})
    # flat walls through a 24^2 grid swept in angle (oracle; the wall meets
    # the domain edges, whose cut clouds weigh on these small grids)
    sweep = []
    for ang in (0.0, 1.0, 2.0, 5.0, 10.0, 20.0, 30.0, 45.0):
        nxw, nyw = lc.line_normal(ang)
        for name, H, fs in (("paper-scheme", 3, 0.0), ("11pt-filter", 5, 0.2)):
            fc = lc.Case(nx=24, ny=24, x0=-11.5, y0=-11.5, h=1.0, H=H, cfl=0.5, filter_sigma=fs,
                         wall=lc.Wall("line", 0.13, 0.21, nxw, nyw), impedance=lc.Impedance())
            sweep.append({"angle_deg": ang, "scheme": name,
                          "abscissa_per_unit_time": osp.spectral_abscissa(osp.operator_matrix(fc))})
    bench_case = lc.cylinder_pulse_1024(10).replace(ic=None, probes=())
    power = {}
    for prec in ("f32", "f64"):
        inst = Instance(bench_case, prec)
        ch = tune.tune_case(bench_case, prec, cache)
        inst.set_tiling(**ch["tiling"])
        inst.set_graph_steps(ch["graph_steps"])
        n = stability.StatePacker(inst).n
        x0 = np.random.default_rng(2609).standard_normal(n)
        t0 = time.perf_counter()
        est, logs = stability.power_growth(inst, x0, args.power_steps, chunk=100)
        wall = time.perf_counter() - t0
        inst.close()
        power[prec] = {"growth_per_step": est, "over_4000_steps": est ** 4000,
                       "last_chunk_growth": float(np.exp((logs[-1] - logs[-2]) / 100)),
                       "steps": args.power_steps, "wall_s": wall}
    out["spectral"] = {"coarse_cylinder_28_rc4_f64": scan, "benchmark_grid_power_iteration": power,
                       "semi_discrete_operator_coarse_cylinder_28_rc4": semi,
                       "semi_discrete_flat_wall_angle_sweep_24_oracle": sweep}

    print(f"[extras] batch of {args.batch_size} uneven instances", file=sys.stderr, flush=True)
    gen = lc.batch_candidates(steps=args.batch_steps)
    members, rejected = [], 0
    t0 = time.perf_counter()
    while len(members) < args.batch_size:
        c = next(gen)
        try:
            members.append(Instance(c, "f32", trace_capacity=1))
        except LeeError:
            rejected += 1
    setup_s = time.perf_counter() - t0
    fluid = sum(m.summary.fluid_nodes for m in members)
    b = Batch(members)
    ch = tune.tune_batch(b, cache)
    b.step_n(4)
    b.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(members[0].stream):
        ev0.record()
    t0 = time.perf_counter()
    b.step_n(args.batch_steps)
    with torch.cuda.stream(members[0].stream):
        ev1.record()
    b.synchronize()
    wall = time.perf_counter() - t0
    sides = [m.case.nx for m in members]
    out["batch_256"] = {"value": fluid * 4.0 * args.batch_steps / wall, "unit": UNIT, "members": len(members),
                        "rejected_candidates": rejected, "fluid_nodes": fluid, "steps": args.batch_steps,
                        "ms_per_step": 1000.0 * wall / args.batch_steps,
                        "gpu_ms_per_step": ev0.elapsed_time(ev1) / args.batch_steps,
                        "sides": {str(k): sides.count(k) for k in sorted(set(sides))},
                        "host_setup_s": setup_s, "tiling": ch["tiling"], "graph_steps": ch["graph_steps"],
                        "roofline_frac": fluid * 4.0 * args.batch_steps * BYTES_PER_NODE_STAGE["f32"]
                        / wall / 1e9 / HBM_PEAK_GBS}
    print(json.dumps(out), flush=True)
    return 0


def serve(args):
    """Served request stream: a JSON line with throughput and p50/p99 latency."""
    import numpy as np
    import torch

    import lee_cases as lc
    from paper_2609_24785_amd.serve import GpuBackend, Request, Server

    torch.cuda.set_device(0)
    reqs = [Request(k, c, t) for k, (t, c) in
            enumerate(lc.request_stream(seed=26091, rate=args.serve_rate, duration=args.serve_duration))]
    print(f"[serve] {len(reqs)} requests over {args.serve_duration} s at {args.serve_rate}/s", file=sys.stderr,
          flush=True)
    be = GpuBackend("f32")
    try:
        srv = Server(be, budget_bytes=args.serve_budget_gb * 1e9, chunk=args.serve_chunk,
                     report=lambda st: print(f"[serve] {json.dumps(st)}", file=sys.stderr, flush=True))
        res = srv.run(reqs)
    finally:
        be.close()
    ok = [r for r in res if r.error is None]
    # the reflection estimate at resonance against the exact value
    dev = []
    for r in ok:
        if r.reflection and r.reflection.get("R_est") and r.reflection["R_est"][1] is not None:
            a, b = r.reflection["R_est"][1], r.reflection["R_exact"][1]
            dev.append(math.hypot(a[0] - b[0], a[1] - b[1]))
    out = {"serve": True, "metric": "served solves: throughput and p50/p99 latency", "unit": UNIT,
           "arrival_rate": args.serve_rate, "window_s": args.serve_duration, "chunk_steps": args.serve_chunk,
           "budget_gb": args.serve_budget_gb, "dtype": "f32",
           "value": srv.stats["throughput"], **srv.stats, "gpu_s": be.gpu_s,
           "mean_steps": float(np.mean([r.steps for r in ok])) if ok else 0.0,
           "mean_fluid_nodes": float(np.mean([r.nodes for r in ok])) if ok else 0.0,
           "rejected_reasons": sorted({(r.error or "")[:60] for r in res if r.error}),
           "reflection_at_resonance_abs_dev_median": float(np.median(dev)) if dev else None}
    print(json.dumps(out), flush=True)
    return 0


def _workload(name: str):
    import lee_cases as lc
    return {"monopole-4096": lc.monopole_4096, "cylinder-pulse-1024": lc.cylinder_pulse_1024}[name]()


def profile_run(args):
    """A short fixed sequence for hardware profilers: the workload named by
    --workload (FP32, graph replay), then three copies of COPY_BYTES bytes.
    It imports no torch: device memory and the stream come from hipmem, so
    the process holds the one HIP runtime the library links (a profiler that
    preloads the system runtime would otherwise leave torch's own runtime
    beside it).  The run checks its fields against the oracle over the same
    steps and prints the error."""
    import oracle.solver as osv
    from paper_2609_24785_amd import _lib, hipmem, tune
    from paper_2609_24785_amd.lee import Instance

    _lib.without_torch()
    hipmem.set_device(0)
    case = _workload(args.workload)
    n = args.warmup + args.steps
    inst = Instance(case, "f32", trace_capacity=n, bind=False)
    ch = tune.lookup(case, "f32", inst.summary.fluid_nodes, inst.summary.G)
    stream = hipmem.Stream()
    buf = hipmem.DeviceBuffer(inst.required_bytes())
    inst.bind_raw(buf, stream)
    _apply(inst, ch)
    inst.step_n(n)
    inst.synchronize()
    got = inst.fields()
    tiling = inst.get_tiling()
    inst.close()
    buf.close()
    a = hipmem.DeviceBuffer(COPY_BYTES)
    b = hipmem.DeviceBuffer(COPY_BYTES)
    for _ in range(3):
        _lib.check(_lib.load().lee_stream_copy(a.ptr, b.ptr, COPY_BYTES, stream.handle), "copy")
    stream.synchronize()
    a.close()
    b.close()
    stream.close()
    ora = osv.OracleSolver(case)
    ora.run(n)
    err = _max_rel_l2(got, ora.fields(), ora.fluid)
    print(json.dumps({"profile_run": True, "workload": args.workload, "steps": n, "copy_bytes": COPY_BYTES,
                      "fluid_nodes": int(ora.fluid.sum()), "tiling": tiling,
                      "kernel": _kernel_name(tiling, "f32"), "fp32_vs_oracle_rel_l2": err}), flush=True)
    return 0 if err <= 1e-4 else 3


def counters(args):
    """Sweep traffic per launch from two rocprofv3 --pmc runs of --profile-run
    (FETCH_SIZE, WRITE_SIZE in KiB per dispatch), each scaled so that the copy
    kernel of known size reads as COPY_BYTES fetched and COPY_BYTES written."""
    import csv

    import lee_cases as lc

    def per_kernel(path, counter):
        sums, counts = {}, {}
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                k = r["Kernel_Name"]
                sums[k] = sums.get(k, 0.0) + float(r["Counter_Value"])
                counts[k] = counts.get(k, 0) + 1
        return {k: (sums[k] / counts[k], counts[k]) for k in sums}

    fetch = per_kernel(args.counters[0], "FETCH_SIZE")
    write = per_kernel(args.counters[1], "WRITE_SIZE")
    copy_name = next(k for k in fetch if "k_copy" in k)
    sweep_name = next(k for k in fetch if k.replace("void ", "").startswith(args.counters[2] + "("))
    kib = 1024.0
    fetch_scale = COPY_BYTES / (fetch[copy_name][0] * kib)
    write_scale = COPY_BYTES / (write[copy_name][0] * kib)
    fb = fetch[sweep_name][0] * kib * fetch_scale
    wb = write[sweep_name][0] * kib * write_scale
    case = _workload(args.workload)
    from paper_2609_24785_amd.lee import Instance
    inst = Instance(case, "f32", bind=False)
    fluid = inst.summary.fluid_nodes
    alg = BYTES_PER_NODE_STAGE["f32"] * fluid
    if "k_stage" in sweep_name:                       # the fused launch also fills the ghosts
        alg += ghost_bytes("f32", inst.summary.G, inst.summary.nnz)
    short = sweep_name.split("(")[0].replace("void ", "")
    d = {"kernel": short, "workload": args.workload, "kernel_sha": _kernel_hash(), "dispatches": fetch[sweep_name][1],
         "fetch_kib_per_dispatch": fetch[sweep_name][0], "write_kib_per_dispatch": write[sweep_name][0],
         "copy_fetch_kib": fetch[copy_name][0], "copy_write_kib": write[copy_name][0],
         "fetch_scale": fetch_scale, "write_scale": write_scale,
         "hbm_bytes_per_launch": fb + wb, "alg_bytes_per_launch": alg, "traffic_over_alg": (fb + wb) / alg}
    os.makedirs(os.path.dirname(COUNTERS_JSON), exist_ok=True)
    with open(COUNTERS_JSON, "w") as f:
        json.dump(d, f, indent=1)
    print(json.dumps(d))
    return 0


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--kernel-steps", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=150, help="oracle sample on all host threads")
    ap.add_argument("--cpu-steps-1t", type=int, default=3, help="oracle sample on one thread")
    ap.add_argument("--no-stated", action="store_true", help="skip the run to the stated 20000 steps")
    ap.add_argument("--no-serve", action="store_true", help="skip the short served window")
    ap.add_argument("--mono-steps", type=int, default=200)
    ap.add_argument("--power-steps", type=int, default=4000, help="power-iteration steps on the benchmark grid (--extras)")
    ap.add_argument("--extras", action="store_true", help="the other configurations, as a second JSON line")
    ap.add_argument("--batch-size", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-run", action="store_true")
    ap.add_argument("--serve", action="store_true", help="the served request stream, as its own JSON line")
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--serve-duration", type=float, default=2.0)
    ap.add_argument("--serve-chunk", type=int, default=100)
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--counters", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "KERNEL"))
    ap.add_argument("--workload", default="monopole-4096", choices=["monopole-4096", "cylinder-pulse-1024"],
                    help="workload of --profile-run and --counters")
    ap.add_argument("--tune-cache", default=None, help="JSON file for autotuner choices (over the shipped table)")
    ap.add_argument("--retune", action="store_true", help="ignore the shipped tuning table (trials only)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (asked for {args.gpus}): the stage is a single-GPU kernel and this "
              "library has no multi-GPU mode.  Independent instances would shard across GPUs by bytes with no "
              "communication; see the design notes.", file=sys.stderr)
        return 2
    if args.counters:
        return counters(args)
    if args.profile_run:
        return profile_run(args)
    if args.extras:
        return extras(args)
    if args.serve:
        return serve(args)
    return run(args)


if __name__ == "__main__":
    sys.exit(main())
