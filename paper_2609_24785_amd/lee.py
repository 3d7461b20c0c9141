"""Python binding of liblee: argument marshalling only.

Every step of the method runs in the library's kernels; PyTorch provides the
device memory (a uint8 tensor handed to lee_bind) and the stream, or, for a
process without torch, hipmem does (Instance.bind_raw).

Live bound instances and batches are closed by an exit hook registered when
the first one binds (after torch is imported, so it runs before torch's own
exit handlers); finalizers make no HIP call while the interpreter shuts down.
"""
from __future__ import annotations

import atexit
import ctypes
import math
import sys
import weakref
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import (BatchOpts, CaseDesc, GhostSummary, ImpedanceDesc, LeeError, Tiling, c_double, c_int64,
                   c_size_t, c_void_p, check, load)


KINDS = {"tile": _lib.SWEEP_TILE, "march": _lib.SWEEP_MARCH}


def make_tiling(kind="tile", vec=0, cols=64, rows=16, waves=1, fused=0) -> Tiling:
    """kind "tile" (cols x rows LDS tiles; fused: ghost fill in the same
    launch) or "march" (vec, rows, waves)."""
    t = Tiling()
    t.kind = KINDS[kind]
    t.vec, t.cols, t.rows, t.waves, t.fused = vec, cols, rows, waves, fused
    return t


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(c_void_p)


def case_desc(case, precision: str = "f32") -> CaseDesc:
    """Marshal a lee_cases.Case into the C description."""
    d = CaseDesc()
    d.nx, d.ny, d.x0, d.y0, d.h = case.nx, case.ny, case.x0, case.y0, case.h
    d.stencil_half = case.H
    d.cfl = case.cfl
    d.filter_sigma = case.filter_sigma
    d.sponge_cells = case.sponge_cells
    d.sponge_sigma = case.sponge_sigma
    d.precision = _lib.F32 if precision == "f32" else _lib.F64
    w = case.wall
    d.wall_kind = _lib.WALL[w.kind]
    d.wall_cx, d.wall_cy, d.wall_nx, d.wall_ny, d.wall_rc = w.cx, w.cy, w.nx, w.ny, w.rc
    ic = case.ic
    if ic is None:
        d.ic_kind = 0
    elif type(ic).__name__ == "Pulse":
        d.ic_kind = 1
        for k, v in enumerate((ic.xs, ic.ys, ic.a, ic.w)):
            d.ic[k] = v
    else:
        d.ic_kind = 2
        for k, v in enumerate((ic.xs, ic.ys, ic.dx, ic.dy, ic.a, ic.alpha, ic.k)):
            d.ic[k] = v
    if case.source is not None:
        s = case.source
        d.src_kind = 1
        for k, v in enumerate((s.xs, s.ys, s.a, s.w, s.omega)):
            d.src[k] = v
    if getattr(case, "radiation", False):
        d.radiation = 1
        d.rad_xc, d.rad_yc = case.rad_center
    d.filter_explicit = 1 if getattr(case, "filter_explicit", False) else 0
    return d


def impedance_desc(imp) -> ImpedanceDesc:
    z = ImpedanceDesc()
    if imp.kind == "rigid":
        z.kind = _lib.Z_RIGID
    elif imp.kind == "poles":
        z.kind = _lib.Z_POLES
        if len(imp.real) > _lib.ADE_MAX_STATES or len(imp.pairs) > _lib.ADE_MAX_STATES // 2:
            raise LeeError(-1, "impedance_desc", "too many pole terms")
        z.n_real, z.n_pair = len(imp.real), len(imp.pairs)
        for k, (lam, a) in enumerate(imp.real):
            z.real_pole[k], z.real_res[k] = lam, a
        for k, (al, be, b, c) in enumerate(imp.pairs):
            z.pair_alpha[k], z.pair_beta[k], z.pair_B[k], z.pair_C[k] = al, be, b, c
    else:
        z.kind = _lib.Z_MSD
        z.R, z.M, z.K = imp.R, imp.M, imp.K
    return z


class Instance:
    """One solve: set-up on the host, fields and lists in caller-owned HBM."""

    def __init__(self, case, precision: str = "f32", device: str = "cuda:0", stream=None,
                 trace_capacity: Optional[int] = None, dft: Optional[tuple] = None, bind: bool = True,
                 watch: Optional[tuple] = None):
        """watch = (x, y, capacity): record p_BP, the ADE's u_n,BP and the
        fluid's u_n at the boundary point of the ghost whose boundary point is
        nearest (x, y) for up to `capacity` steps."""
        self.lib = load()
        self.case = case
        self.precision = precision
        self._h = c_void_p()
        check(self.lib.lee_setup_grid(ctypes.byref(case_desc(case, precision)), ctypes.byref(self._h)),
              "lee_setup_grid")
        self.summary = GhostSummary()
        z = impedance_desc(case.impedance)
        st = self.lib.lee_build_ghosts(self._h, ctypes.byref(z), 4, ctypes.byref(self.summary))
        if st != 0:
            self.close()
            check(st, "lee_build_ghosts")
        if case.probes:
            xy = np.ascontiguousarray(np.array(case.probes, dtype=np.float64).ravel())
            cap = trace_capacity if trace_capacity is not None else max(case.steps, 1)
            om, start, count = dft if dft is not None else (0.0, 0, 0)
            st = self.lib.lee_set_probes(self._h, len(case.probes), _ptr(xy), cap, om, start, count)
            if st != 0:
                self.close()
                check(st, "lee_set_probes")
        self.watch_g = -1
        if watch is not None:
            g = ctypes.c_int32()
            st = self.lib.lee_set_watch(self._h, float(watch[0]), float(watch[1]), int(watch[2]), ctypes.byref(g))
            if st != 0:
                self.close()
                check(st, "lee_set_watch")
            self.watch_g = g.value
        self.buf = None
        self.stream = None
        if bind:
            self.bind(device, stream)

    # ---- device memory ------------------------------------------------------
    def required_bytes(self) -> int:
        n = c_size_t()
        check(self.lib.lee_required_bytes(self._h, ctypes.byref(n)), "lee_required_bytes")
        return n.value

    def bind(self, device: str = "cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the library runs only on the device")
        dev = torch.device(device)
        torch.cuda.set_device(dev)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        nbytes = self.required_bytes()
        self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self.buf.data_ptr()
        aligned = (base + 255) // 256 * 256
        check(self.lib.lee_bind(self._h, c_void_p(aligned), nbytes, c_void_p(self.stream.cuda_stream)),
              "lee_bind")
        _track(self)

    def bind_raw(self, buf, stream):
        """Bind device memory and a stream that the caller made without torch
        (hipmem.DeviceBuffer of at least required_bytes(), hipmem.Stream); the
        caller keeps both alive and frees them after close()."""
        nbytes = self.required_bytes()
        if buf.nbytes < nbytes or buf.ptr % 256:
            raise ValueError("device buffer too small or not 256-byte aligned")
        self.buf, self.stream = buf, stream
        check(self.lib.lee_bind(self._h, c_void_p(buf.ptr), nbytes, c_void_p(stream.handle)), "lee_bind")
        _track(self)

    # ---- stepping -----------------------------------------------------------
    def init_fields(self):
        check(self.lib.lee_init_fields(self._h), "lee_init_fields")

    def rk_stage(self, stage: int):
        check(self.lib.lee_rk_stage(self._h, stage), "lee_rk_stage")

    def step_n(self, n: int):
        check(self.lib.lee_step_n(self._h, n), "lee_step_n")

    def synchronize(self):
        """Wait for the stream; raises if a fused stage's ghost wait ran out."""
        check(self.lib.lee_synchronize(self._h), "lee_synchronize")

    # ---- outputs ------------------------------------------------------------
    def fields(self):
        c = self.case
        p = np.zeros((c.ny, c.nx))
        u = np.zeros_like(p)
        v = np.zeros_like(p)
        check(self.lib.lee_get_fields(self._h, _ptr(p), _ptr(u), _ptr(v)), "lee_get_fields")
        return p, u, v

    def set_fields(self, p=None, u=None, v=None):
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (p, u, v)]
        check(self.lib.lee_set_fields(self._h, *(_ptr(a) for a in arrs)), "lee_set_fields")

    def ade_states(self):
        """Auxiliary states after the last full step, one row per ghost."""
        ns = max(int(self.summary.ade_states), 1)
        out = np.zeros(ns * self.summary.G)
        check(self.lib.lee_get_ade_states(self._h, _ptr(out)), "lee_get_ade_states")
        return out.reshape(-1, ns)

    def set_ade_states(self, x):
        """Overwrite the auxiliary states the next step starts from (rows per
        ghost, as ade_states() returns them)."""
        ns = max(int(self.summary.ade_states), 1)
        a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
        if a.size != ns * self.summary.G:
            raise ValueError(f"expected {ns * self.summary.G} auxiliary states, got {a.size}")
        check(self.lib.lee_set_ade_states(self._h, _ptr(a)), "lee_set_ade_states")

    def rhs(self):
        """The semi-discrete right-hand side at the current state (lee_rhs):
        (p, u, v) planes and the auxiliary states' derivatives, one row per
        ghost."""
        c = self.case
        planes = [np.zeros((c.ny, c.nx)) for _ in range(3)]
        ns = max(int(self.summary.ade_states), 1)
        psi = np.zeros(ns * self.summary.G)
        check(self.lib.lee_rhs(self._h, *(_ptr(a) for a in planes), _ptr(psi) if psi.size else None), "lee_rhs")
        return planes[0], planes[1], planes[2], psi.reshape(-1, ns)

    def probe(self, xy: Sequence[Sequence[float]]):
        xy = np.ascontiguousarray(np.asarray(xy, dtype=np.float64).reshape(-1, 2))
        out = np.zeros((len(xy), 3))
        check(self.lib.lee_probe(self._h, len(xy), _ptr(xy), _ptr(out)), "lee_probe")
        return out

    def traces(self, cap: Optional[int] = None):
        npb = len(self.case.probes)
        if npb == 0:
            return np.zeros((0, 0, 3))
        cap = cap if cap is not None else 1 << 30
        done = c_int64()
        check(self.lib.lee_probe_traces(self._h, None, 0, ctypes.byref(done)), "lee_probe_traces")
        step = self.step
        m = min(step, cap)
        out = np.zeros((max(m, 1), npb, 3))
        check(self.lib.lee_probe_traces(self._h, _ptr(out), m, ctypes.byref(done)), "lee_probe_traces")
        return out[:done.value]

    def watch_traces(self, cap: Optional[int] = None) -> np.ndarray:
        """Recorded (p_BP, u_n,BP of the ADE, u_n read out of the fluid) per
        step of the watched ghost, oldest first."""
        cap = cap if cap is not None else max(self.step, 1)
        out = np.zeros((max(cap, 1), 3))
        n = c_int64()
        check(self.lib.lee_watch_traces(self._h, _ptr(out), cap, ctypes.byref(n)), "lee_watch_traces")
        return out[:n.value]

    def dft(self):
        """Complex DFT amplitudes P_k = (2i/N) sum_n p_k(t_n) exp(-i omega t_n)
        over the window given at construction (lee_probe_dft)."""
        out = np.zeros(2 * len(self.case.probes))
        check(self.lib.lee_probe_dft(self._h, _ptr(out)), "lee_probe_dft")
        return out[0::2] + 1j * out[1::2]

    @property
    def step(self) -> int:
        s = c_int64()
        check(self.lib.lee_get_step(self._h, ctypes.byref(s)), "lee_get_step")
        return s.value

    def export_lists(self):
        G, nnz = self.summary.G, self.summary.nnz
        gi = np.zeros(G, dtype=np.int32)
        cp = np.zeros(G + 1, dtype=np.int32)
        ci = np.zeros(nnz, dtype=np.int32)
        dg = np.zeros(G, dtype=np.int8)
        w = np.zeros(4 * nnz)
        b = np.zeros(2 * G)
        geo = np.zeros(5 * G)
        check(self.lib.lee_export_lists(self._h, *(_ptr(a) for a in (gi, cp, ci, dg, w, b, geo))),
              "lee_export_lists")
        return dict(ghost_idx=gi, cloud_ptr=cp, cloud_idx=ci, degree=dg, weights=w.reshape(-1, 4),
                    beta=b.reshape(-1, 2), geom=geo.reshape(-1, 5))

    def set_tiling(self, kind="tile", vec=0, cols=64, rows=16, waves=1, fused=0):
        t = make_tiling(kind, vec, cols, rows, waves, fused)
        check(self.lib.lee_set_tiling(self._h, ctypes.byref(t)), "lee_set_tiling")

    def set_graph_steps(self, steps: int):
        """Steps per captured hipGraph (0: built-in default, < 0: eager launches)."""
        check(self.lib.lee_set_graph_steps(self._h, steps), "lee_set_graph_steps")

    def set_ghost_wait(self, polls: int):
        """Bound on a fused stage's polls per ghost value (0: default; < 0:
        every wait fails after -polls polls, for testing the error path)."""
        check(self.lib.lee_set_ghost_wait(self._h, polls), "lee_set_ghost_wait")

    def get_tiling(self) -> dict:
        t = Tiling()
        check(self.lib.lee_get_tiling(self._h, ctypes.byref(t)), "lee_get_tiling")
        d = t.as_dict()
        d["kind"] = {v: k for k, v in KINDS.items()}[d["kind"]]
        return d

    def time_kernels(self, n: int):
        a, b, c = c_double(), c_double(), c_double()
        check(self.lib.lee_time_kernels(self._h, n, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
              "lee_time_kernels")
        return a.value, b.value, c.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.lee_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        # no HIP call while the interpreter shuts down: the runtime's own
        # exit handlers may already have run (live objects are closed by the
        # exit hook instead)
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


_live_batches: "weakref.WeakSet" = weakref.WeakSet()
_live_instances: "weakref.WeakSet" = weakref.WeakSet()
_hook = False


def _close_all():
    for b in list(_live_batches):
        b.close()
    for i in list(_live_instances):
        i.close()


def _track(obj):
    global _hook
    (_live_batches if isinstance(obj, Batch) else _live_instances).add(obj)
    if not _hook:
        atexit.register(_close_all)
        _hook = True


class Batch:
    """Bound instances advanced together: one launch per phase over all members."""

    def __init__(self, members: Sequence[Instance], tiling: Optional[dict] = None, persistent_blocks: int = 0,
                 graph_steps: int = 0):
        self.lib = load()
        self.members = list(members)
        arr = (c_void_p * len(members))(*[m._h.value for m in members])
        opts = BatchOpts()
        if tiling is None:
            opts.tiling.kind = -1
        else:
            opts.tiling = make_tiling(**tiling)
        opts.persistent_blocks = persistent_blocks
        opts.graph_steps = graph_steps
        self._h = c_void_p()
        check(self.lib.lee_batch_create(arr, len(members), ctypes.byref(opts), ctypes.byref(self._h)),
              "lee_batch_create")
        _track(self)

    def add(self, inst: "Instance"):
        check(self.lib.lee_batch_add(self._h, inst._h), "lee_batch_add")
        self.members.append(inst)

    def remove(self, inst: "Instance"):
        check(self.lib.lee_batch_remove(self._h, inst._h), "lee_batch_remove")
        self.members.remove(inst)

    def update(self, add: Sequence[Instance] = (), remove: Sequence[Instance] = ()):
        """Removals, then additions at the end, with one rebuild (lee_batch_update)."""
        add, remove = list(add), list(remove)
        a = (c_void_p * max(len(add), 1))(*[m._h.value for m in add])
        r = (c_void_p * max(len(remove), 1))(*[m._h.value for m in remove])
        check(self.lib.lee_batch_update(self._h, a, len(add), r, len(remove)), "lee_batch_update")
        for m in remove:
            self.members.remove(m)
        self.members.extend(add)

    def __len__(self) -> int:
        n = ctypes.c_int32()
        check(self.lib.lee_batch_size(self._h, ctypes.byref(n)), "lee_batch_size")
        return n.value

    def graph_captures(self) -> int:
        """Step graphs captured so far (membership changes keep them unless
        a device list outgrows its capacity)."""
        n = ctypes.c_int64()
        check(self.lib.lee_batch_graph_captures(self._h, ctypes.byref(n)), "lee_batch_graph_captures")
        return n.value

    def set_budget(self, steps: Sequence[int]):
        a = np.ascontiguousarray(np.asarray(steps, dtype=np.int64))
        check(self.lib.lee_batch_set_budget(self._h, _ptr(a)), "lee_batch_set_budget")

    def step_n(self, n: int):
        check(self.lib.lee_batch_step_n(self._h, n), "lee_batch_step_n")

    def synchronize(self):
        check(self.lib.lee_batch_synchronize(self._h), "lee_batch_synchronize")

    def set_tiling(self, kind="tile", vec=0, cols=64, rows=16, waves=1, fused=0):
        t = make_tiling(kind, vec, cols, rows, waves, fused)
        check(self.lib.lee_batch_set_tiling(self._h, ctypes.byref(t)), "lee_batch_set_tiling")

    def get_tiling(self) -> dict:
        t = Tiling()
        check(self.lib.lee_batch_get_tiling(self._h, ctypes.byref(t)), "lee_batch_get_tiling")
        d = t.as_dict()
        d["kind"] = {v: k for k, v in KINDS.items()}[d["kind"]]
        return d

    def set_graph_steps(self, steps: int):
        check(self.lib.lee_batch_set_graph_steps(self._h, steps), "lee_batch_set_graph_steps")

    def init_fields(self):
        """Reset every member to its initial condition (and an unlimited budget)."""
        for m in self.members:
            m.init_fields()

    def time_kernels(self, n: int):
        a, b, c = c_double(), c_double(), c_double()
        check(self.lib.lee_batch_time_kernels(self._h, n, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
              "lee_batch_time_kernels")
        return a.value, b.value, c.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.lee_batch_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def step_members_noalloc(members: Sequence[Instance], steps: int, tiling: Optional[dict] = None):
    """Advance bound instances together as a batch of them would, with the
    library allocating nothing on the device (lee_step_members_noalloc)."""
    lib = load()
    arr = (c_void_p * len(members))(*[m._h.value for m in members])
    t = ctypes.byref(make_tiling(**tiling)) if tiling is not None else None
    check(lib.lee_step_members_noalloc(arr, len(members), t, int(steps)), "lee_step_members_noalloc")


__all__ = ["Instance", "Batch", "LeeError", "case_desc", "impedance_desc", "step_members_noalloc"]
