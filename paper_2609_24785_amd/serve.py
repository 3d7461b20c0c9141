"""Serving loop: continuous batching of solve requests on one GPU.

A request is a case (grid, wall, impedance, pulse, probes, step count) with
an arrival time.  The server:
- prepares each arriving request on the host (mask, ghosts, least-squares
  weights) in worker threads;
- admits prepared requests in arrival order while their device footprints
  (known before binding) fit the HBM budget and a slot is free;
- keeps every admitted request's fields and ADE states resident;
- advances all of them together as one batch, one chunk of steps at a time;
  per-member budgets on the device stop a request mid-chunk when its steps
  are done.

After every chunk the finished requests are retired (results copied out)
and waiting ones admitted; the batch takes the chunk's removals and
additions in one membership update before the next chunk, and the retired
requests' device memory is released then.  The budget counts a retired
request's bytes as free from its retirement, so the device can hold up to
one chunk's retirements beyond the budget until that update.  A request
that arrives while others are on the GPU therefore joins the running batch
at the next chunk boundary, and its work overlaps theirs in the same
launches.

Each result carries:
- the probe traces;
- the watched ghost's boundary pressure, the ADE's wall normal velocity and
  the normal velocity read out of the fluid at the same boundary point (the
  ghost whose boundary point is nearest the pulse centre);
- the reflection coefficient estimated from the pressure and the fluid's
  normal velocity;
- the latency (completion - arrival) and the wait (admission - arrival).

The reflection coefficient estimate: Z = P/U_f from the discrete Fourier
transforms of p_BP and of the fluid's normal velocity u_n at the boundary
point (the least-squares read-out, not the ADE's own u_n,BP, which equals
Y p_BP by construction), and R = (Z - 1)/(Z + 1), beside the exact
(Z - 1)/(Z + 1) of the mass-spring-damper impedance Z = R + i (M w - K / w)
(Single-resonance mass spring damper wall).  The ratio of the two normal
velocities' transforms is reported too: the fluid realises the wall's
velocity where it is close to 1 (Sec. 4.3).

The scheduler is written against a small backend interface.  GpuBackend
drives the library; tests drive the same scheduler with a simulated one.
"""
from __future__ import annotations

import math
import time
from concurrent.futures import ThreadPoolExecutor
from concurrent.futures import wait as wait_futures
from dataclasses import dataclass, field
from typing import Any, Callable, Dict, Iterable, List, Optional, Sequence

import numpy as np


@dataclass
class Request:
    rid: int
    case: Any
    arrival: float                     # seconds after the server starts


@dataclass
class Result:
    rid: int
    steps: int
    arrival: float
    admitted: float
    finished: float
    nodes: int
    traces: Optional[np.ndarray] = None
    watch: Optional[np.ndarray] = None
    reflection: Optional[Dict[str, Any]] = None
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival

    @property
    def wait(self) -> float:
        return self.admitted - self.arrival


def reflection(watch: np.ndarray, dt: float, impedance, omegas: Sequence[float]) -> Dict[str, Any]:
    """R = (Z - 1)/(Z + 1) with Z = P/U_f from the transforms of the watched
    ghost's p_BP trace and of the fluid's normal velocity at its boundary
    point (watch columns 0 and 2), at each angular frequency in omegas,
    beside the exact value of the wall's impedance and the ratio U_f/U of the
    fluid's and the ADE's normal velocity transforms."""
    if watch is None or len(watch) == 0:
        return {}
    t = dt * np.arange(len(watch))
    out = {"omega": [], "R_est": [], "R_exact": [], "un_fluid_over_ade": []}
    for w in omegas:
        e = np.exp(-1j * w * t) * dt
        P = np.sum(watch[:, 0] * e)
        Ua = np.sum(watch[:, 1] * e)
        Uf = np.sum(watch[:, 2] * e)
        out["omega"].append(float(w))
        if abs(Uf) > 0:
            Z = P / Uf
            r = (Z - 1.0) / (Z + 1.0)
            out["R_est"].append([float(r.real), float(r.imag)])
        else:
            out["R_est"].append(None)
        q = Uf / Ua if abs(Ua) > 0 else None
        out["un_fluid_over_ade"].append(None if q is None else [float(q.real), float(q.imag)])
        if impedance.kind == "msd":
            Ze = impedance.R + 1j * (impedance.M * w - impedance.K / w)
            re = (Ze - 1.0) / (Ze + 1.0)
            out["R_exact"].append([float(re.real), float(re.imag)])
        else:
            out["R_exact"].append([1.0, 0.0])
    return out


def _omegas(case) -> List[float]:
    imp = case.impedance
    if imp.kind == "msd":
        w0 = math.sqrt(imp.K / imp.M)
        return [0.5 * w0, w0, 2.0 * w0]
    return [1.0, 4.0, 16.0]


class GpuBackend:
    """The library: one batch whose members are the admitted requests, all on
    the server's stream."""

    def __init__(self, precision: str = "f32", device: str = "cuda:0", tiling: Optional[dict] = None,
                 graph_steps: int = 0, prepare_threads: int = 8):
        import torch
        self.torch = torch
        self.precision = precision
        self.device = device
        torch.cuda.set_device(torch.device(device))
        self.stream = torch.cuda.Stream(device=device)
        self.tiling = tiling
        self.graph_steps = graph_steps
        self.batch = None
        self.pool = ThreadPoolExecutor(max_workers=prepare_threads)
        self.gpu_s = 0.0                         # device time of the chunks (events on the stream)
        # membership changes since the last chunk, applied together before the
        # next one (one rebuild of the batch's lists instead of one per change)
        self._add: List[Any] = []
        self._remove: List[Any] = []

    # host side, in worker threads: the library releases the GIL in its calls
    def prepare(self, case):
        from .lee import Instance
        c = case.ic
        watch = (c.xs, c.ys, case.steps) if c is not None else None
        return Instance(case, self.precision, bind=False, trace_capacity=case.steps, watch=watch)

    def prepare_async(self, case):
        return self.pool.submit(self.prepare, case)

    def footprint(self, inst) -> int:
        return inst.required_bytes() + 256

    def nodes(self, inst) -> int:
        return int(inst.summary.fluid_nodes)

    def admit(self, inst) -> None:
        inst.bind(self.device, self.stream)
        self._add.append(inst)

    def _flush(self) -> None:
        """The pending removals and additions in one lee_batch_update; the
        removed instances are closed after it."""
        from .lee import Batch
        if not self._add and not self._remove:
            return
        if self.batch is None:
            self.batch = Batch(self._add, tiling=self.tiling, graph_steps=self.graph_steps)
        else:
            self.batch.update(add=self._add, remove=self._remove)
        for inst in self._remove:
            inst.close()
            inst.buf = None                  # the device memory returns to torch's cache
        self._add, self._remove = [], []

    def step(self, insts: Sequence, budgets: Sequence[int], n: int) -> None:
        self._flush()
        # budgets are per position: the batch must hold the scheduler's members in its order
        if [id(m) for m in self.batch.members] != [id(m) for m in insts]:
            raise RuntimeError("batch members and scheduler order differ")
        self.batch.set_budget(budgets)
        ev = [self.torch.cuda.Event(enable_timing=True) for _ in range(2)]
        with self.torch.cuda.stream(self.stream):
            ev[0].record()
        self.batch.step_n(n)
        with self.torch.cuda.stream(self.stream):
            ev[1].record()
        self.batch.synchronize()
        self.gpu_s += ev[0].elapsed_time(ev[1]) * 1e-3

    def retire(self, inst) -> Dict[str, Any]:
        out = {"traces": inst.traces(), "watch": inst.watch_traces() if inst.watch_g >= 0 else None}
        self._remove.append(inst)            # leaves the batch before the next chunk
        return out

    def close(self):
        if self.batch is not None:
            self.batch.close()
        for inst in self._remove + self._add:
            inst.close()
        self._add, self._remove = [], []
        self.pool.shutdown(wait=True)


class SimBackend:
    """A simulated device for testing the scheduler: memory is counted, and a
    chunk costs `cost_per_node_step` seconds per fluid node-step of the
    members that are still working, on a virtual clock."""

    def __init__(self, clock, cost_per_node_step: float = 1e-9):
        self.clock = clock
        self.cost = cost_per_node_step
        self.members: List[Any] = []
        self.launches = []

    class _Prepared:
        def __init__(self, case):
            self.case = case
            self.done = 0

    def prepare(self, case):
        return SimBackend._Prepared(case)

    def prepare_async(self, case):
        from concurrent.futures import Future
        f = Future()
        f.set_result(self.prepare(case))
        return f

    def footprint(self, p) -> int:
        return 36 * p.case.nx * p.case.ny

    def nodes(self, p) -> int:
        return p.case.nx * p.case.ny

    def admit(self, p) -> None:
        self.members.append(p)

    def step(self, insts, budgets, n) -> None:
        assert [id(x) for x in insts] == [id(x) for x in self.members]
        self.launches.append([(p.case.name, b) for p, b in zip(insts, budgets)])
        work = 0
        for p, b in zip(insts, budgets):
            k = min(b, n)
            p.done += k
            work += self.nodes(p) * k
        self.clock.advance(work * self.cost)

    def retire(self, p) -> Dict[str, Any]:
        self.members.remove(p)
        return {"traces": np.array([p.done]), "watch": None}

    def close(self):
        pass


class Server:
    """Continuous batching over a backend; run() serves a request list whose
    arrival times are seconds from the start."""

    def __init__(self, backend, budget_bytes: float = 200e9, chunk: int = 100, max_members: int = 512,
                 clock: Callable[[], float] = time.monotonic, sleep: Callable[[float], None] = time.sleep,
                 dt_of: Optional[Callable[[Any], float]] = None,
                 report: Optional[Callable[[Dict[str, Any]], None]] = None, report_every: float = 20.0):
        self.backend = backend
        self.budget = budget_bytes
        self.chunk = chunk
        self.max_members = max_members
        self.clock = clock
        self.sleep = sleep
        self.dt_of = dt_of or (lambda case: case.dt)
        self.report = report                     # called with a state summary after a chunk,
        self.report_every = report_every         # at most once per report_every seconds
        self.stats: Dict[str, Any] = {}

    def run(self, requests: Iterable[Request]) -> List[Result]:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        t0 = self.clock()
        now = lambda: self.clock() - t0             # noqa: E731
        nxt = 0                                      # next request not yet arrived
        preparing: List[tuple] = []                  # (request, future), arrival order
        active: List[dict] = []                      # admitted: request, handle, remaining, admitted
        results: List[Result] = []
        in_use = 0
        peak_mem = 0
        peak_members = 0
        node_steps = 0
        busy = 0.0
        spent = {"admit_s": 0.0, "retire_s": 0.0, "setup_wait_s": 0.0}   # host phases between chunks
        last_report = 0.0
        while nxt < len(reqs) or preparing or active:
            t = now()
            while nxt < len(reqs) and reqs[nxt].arrival <= t:
                preparing.append((reqs[nxt], self.backend.prepare_async(reqs[nxt].case)))
                nxt += 1
            # admission in arrival order while memory and slots allow
            ta = now()
            while preparing and preparing[0][1].done() and len(active) < self.max_members:
                req, fut = preparing[0]
                try:
                    h = fut.result()
                except Exception as e:               # rejected at set-up (e.g. an unstable impedance)
                    preparing.pop(0)
                    results.append(Result(req.rid, req.case.steps, req.arrival, now(), now(), 0, error=str(e)))
                    continue
                need = self.backend.footprint(h)
                if need > self.budget:
                    preparing.pop(0)
                    results.append(Result(req.rid, req.case.steps, req.arrival, now(), now(), 0,
                                          error="footprint exceeds the HBM budget"))
                    continue
                if in_use + need > self.budget:
                    break                            # wait for memory to free up
                preparing.pop(0)
                self.backend.admit(h)
                in_use += need
                active.append({"req": req, "h": h, "left": req.case.steps, "admitted": now(), "need": need,
                               "nodes": self.backend.nodes(h)})
            spent["admit_s"] += now() - ta
            peak_mem = max(peak_mem, in_use)
            peak_members = max(peak_members, len(active))
            if not active:
                # idle: wait for the next arrival or a preparation to finish
                tw = now()
                if preparing:
                    wait_futures([preparing[0][1]])      # its outcome is handled at admission
                elif nxt < len(reqs):
                    self.sleep(max(0.0, reqs[nxt].arrival - now()))
                spent["setup_wait_s"] += now() - tw
                continue
            budgets = [min(a["left"], self.chunk) for a in active]
            n = max(budgets)
            ts = now()
            self.backend.step([a["h"] for a in active], budgets, n)
            busy += now() - ts
            node_steps += sum(a["nodes"] * b for a, b in zip(active, budgets))
            still = []
            tr = now()
            for a, b in zip(active, budgets):
                a["left"] -= b
                if a["left"] > 0:
                    still.append(a)
                    continue
                out = self.backend.retire(a["h"])
                in_use -= a["need"]
                req = a["req"]
                res = Result(req.rid, req.case.steps, req.arrival, a["admitted"], now(), a["nodes"],
                             traces=out.get("traces"), watch=out.get("watch"))
                if res.watch is not None and len(res.watch):
                    res.reflection = reflection(res.watch, self.dt_of(req.case), req.case.impedance,
                                                _omegas(req.case))
                results.append(res)
            active = still
            spent["retire_s"] += now() - tr
            if self.report is not None and now() - last_report >= self.report_every:
                last_report = now()
                self.report({"t_s": last_report, "arrived": nxt, "finished": len(results),
                             "active": len(active), "waiting": len(preparing), "bytes_in_use": in_use})
        wall = now()
        ok = [r for r in results if r.error is None]
        lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
        self.stats = {
            "requests": len(results), "served": len(ok), "rejected": len(results) - len(ok),
            "wall_s": wall, "busy_s": busy, "node_stages": 4 * node_steps,
            "throughput": 4 * node_steps / wall if wall > 0 else 0.0,
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_wait_s": float(np.mean([r.wait for r in ok])) if ok else 0.0,
            "peak_members": peak_members, "peak_bytes": peak_mem, **spent,
        }
        return sorted(results, key=lambda r: r.rid)


__all__ = ["Request", "Result", "Server", "GpuBackend", "SimBackend", "reflection"]
