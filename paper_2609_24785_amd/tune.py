"""Autotuner for the stage sweep of one instance or one batch.

It times candidate launch configurations on the device and keeps the
fastest.  Each candidate is a tile shape, the fused or two-launch form of a
stage, and a number of steps per captured graph.  The figure of merit is the
mean time of a graph-replayed RK4 step, which is what a run pays.  Choices
are cached in a JSON file, keyed by the device architecture, the precision,
the problem's size class (fluid nodes and ghosts, in powers of two) and its
kernel variant (stencil half-width, filter on or off, radiation band, wall
kind), so a later problem of the same class and variant skips the trials.  The package ships such a
table (tuned_gfx950.json, written by this module on an MI355X) as a read-only
base layer under every cache.

The trial steps advance the instance, so the tuned instance (or every member
of a tuned batch) is reset to its initial condition afterwards.  Tune before
stepping, or tune a twin made with tune_case.
"""
from __future__ import annotations

import json
import math
import os
from typing import Callable, Dict, Iterable, List, Optional, Sequence, Tuple

# Tile shapes the library supports that are worth timing (narrow tiles keep
# more workgroups in flight; wide ones read fewer halo columns), each in the
# fused and the two-launch form.
_SHAPES = {
    "f32": [(64, 16), (64, 8), (64, 32), (128, 8), (128, 16)],
    "f64": [(64, 8), (64, 16), (128, 4), (128, 8)],
}
GRAPH_STEPS = (16, 32)      # trial runs are whole graphs of either length


def candidates(precision: str) -> List[dict]:
    """Candidate configurations for a precision ("f32" or "f64")."""
    out = []
    for cols, rows in _SHAPES[precision]:
        for fused in (0, 1):
            for g in GRAPH_STEPS:
                out.append({"tiling": {"kind": "tile", "cols": cols, "rows": rows, "fused": fused},
                            "graph_steps": g})
    return out


def size_class(fluid_nodes: int, ghosts: int, members: int = 1) -> str:
    """Problems within a factor of about 1.4 in fluid nodes and ghosts share a class."""
    def b(x):
        return int(round(2.0 * math.log2(max(int(x), 1))))
    return f"m{members}-f{b(fluid_nodes)}-g{b(ghosts)}"


def variant_of(case) -> str:
    """The parts of a case that select different kernel code or cost: the
    stencil half-width, the filter (off, in the stages, once per step), the
    radiation band and the wall kind (rigid, mass-spring-damper,
    multi-pole)."""
    wall = case.impedance.kind if case.wall.kind != "none" else "none"
    form = 0 if case.filter_sigma <= 0.0 else (2 if getattr(case, "filter_explicit", False) else 1)
    return f"H{case.H}-s{form}-r{int(bool(case.radiation))}-{wall}"


def cache_key(arch: str, precision: str, cls: str, variant: str) -> str:
    return f"{arch.split(':')[0]}|{precision}|{cls}|{variant}"


def select(measure: Callable[[dict], float], cands: Iterable[dict], rounds: int = 3) -> Tuple[dict, List[dict]]:
    """Time every candidate with measure (microseconds per step; it may raise,
    which rejects the candidate) in `rounds` interleaved passes, keep each
    candidate's best time (candidates a few per cent apart are otherwise
    ordered by run-to-run noise), and return the fastest and the table."""
    cands = list(cands)
    table = [dict(c, step_us=None, trials=[]) for c in cands]
    for _ in range(max(int(rounds), 1)):
        for row, c in zip(table, cands):
            if "error" in row:
                continue
            try:
                us = float(measure(c))
            except Exception as e:        # a configuration the device rejects
                row.update(step_us=None, error=str(e))
                continue
            if not math.isfinite(us) or us <= 0.0:
                row.update(step_us=None, error="no time")
                continue
            row["trials"].append(us)
            row["step_us"] = min(row["trials"])
    best = None
    for row, c in zip(table, cands):
        if row["step_us"] is not None and "error" not in row and (best is None or row["step_us"] < best["step_us"]):
            best = dict(c, step_us=row["step_us"])
    if best is None:
        raise RuntimeError("no candidate configuration ran")
    return best, table


SHIPPED_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_gfx950.json")


class TuneCache:
    """Choices by key, in a JSON file (written on every update), over the
    shipped table unless shipped=False."""

    def __init__(self, path: Optional[str] = None, shipped: bool = True):
        self.path = path
        self.base: Dict[str, dict] = {}
        self.data: Dict[str, dict] = {}
        if shipped and os.path.exists(SHIPPED_TABLE):
            with open(SHIPPED_TABLE) as f:
                self.base = json.load(f)
        if path and os.path.exists(path):
            with open(path) as f:
                self.data = json.load(f)

    def get(self, key: str) -> Optional[dict]:
        hit = self.data.get(key)
        return hit if hit is not None else self.base.get(key)

    def put(self, key: str, value: dict) -> None:
        self.data[key] = value
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.data, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def _device_arch() -> str:
    import torch
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName


def _time_steps(target, stream, steps: int, warmup: int) -> float:
    import torch
    target.step_n(warmup)
    target.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        e0.record()
    target.step_n(steps)
    with torch.cuda.stream(stream):
        e1.record()
    target.synchronize()
    return e0.elapsed_time(e1) * 1e3 / steps


def _apply(target, choice: dict) -> None:
    target.set_tiling(**choice["tiling"])
    target.set_graph_steps(choice["graph_steps"])


def tune_instance(inst, cache: Optional[TuneCache] = None, steps: int = 64, warmup: int = 32,
                  cands: Optional[Sequence[dict]] = None) -> dict:
    """Pick and apply the fastest configuration for a bound instance, then
    reset it to its initial condition.  Returns the choice (with its time and,
    when measured here, the table of trials)."""
    s = inst.summary
    key = cache_key(_device_arch(), inst.precision, size_class(s.fluid_nodes, s.G), variant_of(inst.case))
    hit = cache.get(key) if cache else None
    if hit is not None:
        _apply(inst, hit)
        return dict(hit, cached=True, key=key)

    def measure(c):
        _apply(inst, c)
        return _time_steps(inst, inst.stream, steps, warmup)

    best, table = select(measure, cands if cands is not None else candidates(inst.precision))
    _apply(inst, best)
    inst.init_fields()
    if cache:
        cache.put(key, best)
    return dict(best, cached=False, key=key, table=table)


def tune_case(case, precision: str = "f32", cache: Optional[TuneCache] = None, **kw) -> dict:
    """Tune on a scratch instance of a case; apply the result to others with
    Instance.set_tiling(**choice["tiling"]) and set_graph_steps."""
    from .lee import Instance
    inst = Instance(case, precision, trace_capacity=1)
    try:
        return tune_instance(inst, cache, **kw)
    finally:
        inst.close()


def tune_batch(batch, cache: Optional[TuneCache] = None, steps: int = 32, warmup: int = 32,
               cands: Optional[Sequence[dict]] = None) -> dict:
    """Pick and apply the fastest configuration for a batch, then reset every
    member to its initial condition (budgets become unlimited)."""
    members = batch.members
    fluid = sum(m.summary.fluid_nodes for m in members)
    ghosts = sum(m.summary.G for m in members)
    prec = members[0].precision
    variants = sorted({variant_of(m.case) for m in members})
    key = cache_key(_device_arch(), prec, size_class(fluid, ghosts, len(members)),
                    variants[0] if len(variants) == 1 else "mixed")
    hit = cache.get(key) if cache else None
    if hit is not None:
        _apply(batch, hit)
        return dict(hit, cached=True, key=key)

    def measure(c):
        _apply(batch, c)
        return _time_steps(batch, members[0].stream, steps, warmup)

    best, table = select(measure, cands if cands is not None else candidates(prec))
    _apply(batch, best)
    batch.init_fields()
    if cache:
        cache.put(key, best)
    return dict(best, cached=False, key=key, table=table)


def lookup(case, precision: str, fluid_nodes: int, ghosts: int, arch: str = "gfx950",
           cache: Optional[TuneCache] = None) -> Optional[dict]:
    """The cached choice for a case without touching the device (None if
    there is none)."""
    cache = cache if cache is not None else TuneCache()
    return cache.get(cache_key(arch, precision, size_class(fluid_nodes, ghosts), variant_of(case)))


__all__ = ["candidates", "size_class", "variant_of", "cache_key", "lookup", "select", "TuneCache", "tune_instance", "tune_case",
           "tune_batch"]
