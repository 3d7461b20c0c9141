"""Oracle driver: builds geometry, clouds, weights and ADE for a case (Python,
FP64) and advances it with the plain C core.  TEST INFRASTRUCTURE ONLY.

Initial state (Sec. 2.1): q0 = [p0, u0, v0] at fluid nodes; ghost, solid and
frame nodes and the auxiliary states start at zero.  The frame of F = 5
nodes around the domain stays zero.  Outer boundary: by default nothing more
than that frame (plus an outer sponge layer when enabled); with
case.radiation, the nodes closer than H to an edge solve the outgoing-wave
equation with one-sided stencils (the paper names one-sided stencils and a
non-reflecting condition on the outer boundary without printing either;
the reading is stated in core.c).

Filter rows: per node and axis, the widest centred filter row that reads no
non-fluid node of the domain (geometry.filter_widths, schemes.filter_rows;
the reading is stated in core.c).  The filter is the damping term of every
stage's right-hand side, or, with case.filter_explicit, applied once after
every step (q <- q - sigma_d (F_x + F_y) q at the fluid nodes).

Sponge reading: sigma_s = sigma_max ((W - e) / W)^2 for a node e < W cells
from the nearest domain edge, zero elsewhere.

Probes: 4 x 4 tensor-product cubic Lagrange interpolation on fluid nodes,
sampled after every full step.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from lee_cases import Case, Monopole, Packet, Pulse
from . import ade as ade_mod
from . import geometry, schemes, weights
from .build import LIB, build

F = 5
_lib = None


class _OcCase(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("F", ctypes.c_int), ("H", ctypes.c_int),
        ("h", ctypes.c_double), ("dt", ctypes.c_double), ("x0", ctypes.c_double), ("y0", ctypes.c_double),
        ("a", ctypes.c_double * 5), ("sigma_d", ctypes.c_double),
        ("sponge_w", ctypes.c_int), ("sponge_smax", ctypes.c_double),
        ("has_src", ctypes.c_int), ("src_x", ctypes.c_double), ("src_y", ctypes.c_double),
        ("src_a", ctypes.c_double), ("src_b", ctypes.c_double), ("src_omega", ctypes.c_double),
        ("fluid", ctypes.c_void_p), ("G", ctypes.c_int),
        ("gidx", ctypes.c_void_p), ("gnx", ctypes.c_void_p), ("gny", ctypes.c_void_p),
        ("cptr", ctypes.c_void_p), ("cidx", ctypes.c_void_p), ("W", ctypes.c_void_p),
        ("lag", ctypes.c_void_p), ("bir", ctypes.c_void_p),
        ("ade_ns", ctypes.c_int), ("ade_A", ctypes.c_double * 64), ("ade_f", ctypes.c_double * 8),
        ("ade_c", ctypes.c_double * 8),
        ("watch_g", ctypes.c_int),
        ("rad_w", ctypes.c_int), ("rad_xc", ctypes.c_double), ("rad_yc", ctypes.c_double),
        ("rad_c", ctypes.c_double * 3), ("rad_b", ctypes.c_double * 21),
        ("fw", ctypes.c_void_p), ("frow", ctypes.c_double * 396),
        ("filter_explicit", ctypes.c_int),
    ]


def _load():
    global _lib
    if _lib is None:
        path = LIB if os.path.exists(LIB) else build()
        _lib = ctypes.CDLL(path)
        _lib.oc_run.restype = ctypes.c_int
        _lib.oc_run.argtypes = [ctypes.POINTER(_OcCase)] + [ctypes.c_void_p] * 4 + [
            ctypes.c_longlong, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_void_p]
    return _lib


def set_threads(n: int = 0) -> int:
    """Threads of the C core's loops (n <= 0: unchanged); returns the count in use."""
    lib = _load()
    lib.oc_set_threads.restype = ctypes.c_int
    lib.oc_set_threads.argtypes = [ctypes.c_int]
    return int(lib.oc_set_threads(int(n)))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def cubic_probe_weights(case: Case, fluid: np.ndarray, x: float, y: float):
    """Origin (i0, j0) and 4x4 weights w[b, a] of the cubic Lagrange stencil
    around (x, y); raises if a stencil node is not a fluid node."""
    def one(c0, n):
        f = (c0 - (case.x0 if n == "x" else case.y0)) / case.h
        i1 = int(math.floor(f))
        i0 = i1 - 1
        t = f - i0
        w = weights.lagrange_at(t, nodes=(0.0, 1.0, 2.0, 3.0))
        return i0, w
    i0, wx = one(x, "x")
    j0, wy = one(y, "y")
    if i0 < 0 or j0 < 0 or i0 + 3 >= case.nx or j0 + 3 >= case.ny:
        raise ValueError("probe stencil leaves the domain")
    if not fluid[j0:j0 + 4, i0:i0 + 4].all():
        raise ValueError("probe stencil touches a non-fluid node")
    return i0, j0, np.outer(wy, wx)


def _check_radiation(c: Case, fluid: np.ndarray):
    """The radiation band (nodes closer than H to an edge) and every node its
    stencils read (6 more) must be fluid, and the centre must lie at least
    one grid step from every band node."""
    reach = c.H + 6
    edge = np.ones_like(fluid)
    edge[reach:c.ny - reach, reach:c.nx - reach] = False
    if c.nx <= 2 * reach or c.ny <= 2 * reach or not np.all(fluid[edge]):
        raise ValueError("radiation condition: the wall comes within reach of the outer band")
    jj, ii = np.nonzero(edge)
    band = np.minimum(np.minimum(ii, jj), np.minimum(c.nx - 1 - ii, c.ny - 1 - jj)) < c.H
    x = c.x0 + ii[band] * c.h - c.rad_center[0]
    y = c.y0 + jj[band] * c.h - c.rad_center[1]
    if np.min(np.hypot(x, y)) < c.h:
        raise ValueError("radiation condition: centre too close to the outer band")


class OracleSolver:
    def __init__(self, case: Case, filter_rows: np.ndarray | None = None):
        """filter_rows (tests only): rows[w, 5 + k] replacing the filter rows
        of schemes.filter_rows(), to show what a different reading does."""
        self.case = case
        c = case
        self.fluid = geometry.fluid_mask(c)
        if c.radiation:
            _check_radiation(c, self.fluid)
        if c.wall.kind != "none":
            self.gidx = geometry.ghost_points(c, self.fluid)
        else:
            self.gidx = np.zeros(0, dtype=np.int64)
        G = len(self.gidx)
        if G:
            self.bx, self.by, self.gnx, self.gny, self.r = geometry.boundary_points(c, self.gidx)
            self.cptr, self.cidx, self.xp, self.yp, self.cut = geometry.clouds(
                c, self.fluid, self.gidx, self.bx, self.by, self.gnx, self.gny)
            self.Ws, self.deg, self.lag, self.bir = weights.ghost_stencils(
                self.xp, self.yp, self.cptr, self.r, self.cut)
            self.W = np.ascontiguousarray(np.concatenate([w.T for w in self.Ws], axis=0))
        else:
            z = np.zeros(0)
            self.bx = self.by = self.gnx = self.gny = self.r = z
            self.cptr = np.zeros(1, dtype=np.int64)
            self.cidx = np.zeros(0, dtype=np.int64)
            self.xp = self.yp = z
            self.cut = np.zeros(0, dtype=bool)
            self.Ws, self.deg = [], np.zeros(0, dtype=np.int64)
            self.lag = self.bir = np.zeros((0, 5))
            self.W = np.zeros((0, 5))
        self.ade = ade_mod.ade_from_impedance(c.impedance, c.dt) if G else ade_mod.ADE("rigid")
        if G:
            ade_mod.check_coupling(c.impedance, c.h, c.filter_sigma > 0.0)
        self.shape = (c.ny + 2 * F, c.nx + 2 * F)
        self.p = np.zeros(self.shape)
        self.u = np.zeros(self.shape)
        self.v = np.zeros(self.shape)
        self.ns = len(self.ade.matrices()[1])        # auxiliary states per ghost
        self.psi = np.zeros(max(self.ns * G, self.ns))
        self.step = 0
        self.watch_g = -1
        self.watch_trace = np.zeros((0, 3))
        self._init_fields()
        self.probe_ij, self.probe_w = self._probes()
        # per node and axis, the half-width of its filter row (schemes, geometry)
        self.filter_w = geometry.filter_widths(self.fluid)
        self.filter_rows = schemes.filter_rows() if filter_rows is None else np.asarray(filter_rows, float)
        self._keep = []
        self._cs = self._make_struct()

    # ---- set-up -----------------------------------------------------------
    def _init_fields(self):
        c = self.case
        x = geometry.node_x(c, np.arange(c.nx))[None, :]
        y = geometry.node_y(c, np.arange(c.ny))[:, None]
        p0 = np.zeros((c.ny, c.nx))
        u0 = np.zeros((c.ny, c.nx))
        v0 = np.zeros((c.ny, c.nx))
        if isinstance(c.ic, Pulse):
            b = math.log(2.0) / (c.ic.w * c.ic.w)
            p0 = c.ic.a * np.exp(-b * ((x - c.ic.xs) ** 2 + (y - c.ic.ys) ** 2))
        elif isinstance(c.ic, Packet):
            k = c.ic
            s = (x - k.xs) * k.dx + (y - k.ys) * k.dy
            p0 = 0.5 * k.a * np.exp(-(k.alpha ** 2) * s * s) * np.cos(2.0 * math.pi * k.k * s)
            u0 = p0 * k.dx
            v0 = p0 * k.dy
        for arr, val in ((self.p, p0), (self.u, u0), (self.v, v0)):
            arr[F:F + c.ny, F:F + c.nx] = np.where(self.fluid, val, 0.0)

    def _probes(self):
        ij, w = [], []
        for (x, y) in self.case.probes:
            i0, j0, ww = cubic_probe_weights(self.case, self.fluid, x, y)
            ij += [i0, j0]
            w.append(ww.ravel())
        return (np.asarray(ij, dtype=np.int64),
                np.ascontiguousarray(np.concatenate(w) if w else np.zeros(0)))

    def _make_struct(self):
        c = self.case
        s = _OcCase()
        s.nx, s.ny, s.F, s.H = c.nx, c.ny, F, c.H
        s.h, s.dt, s.x0, s.y0 = c.h, c.dt, c.x0, c.y0
        a = schemes.drp(c.H)
        for k in range(5):
            s.a[k] = a[k] if k < len(a) else 0.0
        s.sigma_d = c.filter_sigma
        s.filter_explicit = int(bool(c.filter_explicit))
        rows = self.filter_rows.ravel()
        for k in range(len(rows)):
            s.frow[k] = rows[k]
        s.sponge_w = c.sponge_cells
        s.sponge_smax = c.sponge_sigma
        if isinstance(c.source, Monopole):
            m = c.source
            s.has_src = 1
            s.src_x, s.src_y, s.src_a = m.xs, m.ys, m.a
            s.src_b = math.log(2.0) / (m.w * m.w)
            s.src_omega = m.omega
        keep = [np.ascontiguousarray(self.fluid.astype(np.uint8)),
                np.ascontiguousarray(self.gidx, dtype=np.int64),
                np.ascontiguousarray(self.gnx, dtype=np.float64),
                np.ascontiguousarray(self.gny, dtype=np.float64),
                np.ascontiguousarray(self.cptr, dtype=np.int64),
                np.ascontiguousarray(self.cidx, dtype=np.int64),
                np.ascontiguousarray(self.W, dtype=np.float64),
                np.ascontiguousarray(self.lag, dtype=np.float64),
                np.ascontiguousarray(self.bir, dtype=np.float64),
                np.ascontiguousarray(self.filter_w.reshape(-1))]
        self._keep = keep
        s.fw = keep[9].ctypes.data
        s.fluid = keep[0].ctypes.data
        s.G = len(self.gidx)
        s.gidx, s.gnx, s.gny = keep[1].ctypes.data, keep[2].ctypes.data, keep[3].ctypes.data
        s.cptr, s.cidx, s.W = keep[4].ctypes.data, keep[5].ctypes.data, keep[6].ctypes.data
        s.lag, s.bir = keep[7].ctypes.data, keep[8].ctypes.data
        A, f, cv = self.ade.matrices()
        s.ade_ns = len(f)
        for i in range(len(f)):
            s.ade_f[i] = f[i]
            s.ade_c[i] = cv[i]
            for j in range(len(f)):
                s.ade_A[8 * i + j] = A[i][j]
        s.watch_g = -1
        if c.radiation:
            s.rad_w = c.H
            s.rad_xc, s.rad_yc = c.rad_center
            for k in range(3):
                s.rad_c[k] = schemes.DRP7[k]
            for m in range(3):
                for k in range(7):
                    s.rad_b[7 * m + k] = schemes.RAD_ONE_SIDED[m, k]
        return s

    # ---- stepping ---------------------------------------------------------
    def set_watch(self, x: float, y: float) -> int:
        """Record, every step (first stage), p_BP, the ADE's wall velocity
        u_n,BP and the normal velocity read out of the fluid at the boundary
        point (the least-squares fit at P_0, u_n positive into the wall) of
        the ghost whose boundary point is nearest (x, y) (ties: the lowest
        ghost index)."""
        if len(self.gidx) == 0:
            raise ValueError("no ghost points")
        d2 = (self.bx - x) * (self.bx - x) + (self.by - y) * (self.by - y)
        g = int(np.argmin(d2))
        self._cs.watch_g = g
        self.watch_g = g
        return g

    def run(self, nsteps: int) -> np.ndarray:
        """Advance nsteps; returns probe traces [nsteps, nprobes, 3].  With a
        watched ghost, its (p_BP, u_n,BP, fluid u_n) per step are appended to
        self.watch_trace."""
        lib = _load()
        npb = len(self.case.probes)
        trace = np.zeros((max(nsteps, 1), max(npb, 1), 3))
        watch = np.zeros((max(nsteps, 1), 3))
        rc = lib.oc_run(ctypes.byref(self._cs), _ptr(self.p), _ptr(self.u), _ptr(self.v),
                        _ptr(self.psi), self.step, nsteps, npb, _ptr(self.probe_ij),
                        _ptr(self.probe_w), _ptr(trace), _ptr(watch) if self.watch_g >= 0 else None)
        if rc != 0:
            raise MemoryError("oracle core allocation failed")
        self.step += nsteps
        if self.watch_g >= 0:
            self.watch_trace = np.concatenate([self.watch_trace, watch[:nsteps]])
        return trace[:nsteps, :npb]

    # ---- views ------------------------------------------------------------
    def fields(self):
        c = self.case
        sl = (slice(F, F + c.ny), slice(F, F + c.nx))
        return self.p[sl].copy(), self.u[sl].copy(), self.v[sl].copy()

    @property
    def time(self) -> float:
        return self.step * self.case.dt

    def composite_weights(self):
        """Per cloud entry: (w0, wF, wD, wN) and per ghost (beta_D, beta_N) -- the
        ghost values written as single weighted sums, for comparing with an
        implementation that stores them composed."""
        G = len(self.gidx)
        out = np.zeros((len(self.cidx), 4))
        beta = np.zeros((G, 2))
        for g in range(G):
            a, b = self.cptr[g], self.cptr[g + 1]
            W = self.Ws[g]
            L, B = self.lag[g], self.bir[g]
            out[a:b, 0] = W[0]
            out[a:b, 1] = L @ W
            out[a:b, 2] = L[1:] @ W[1:]
            out[a:b, 3] = B[1:] @ W[1:]
            beta[g] = (L[0], B[0])
        return out, beta


def run_case(case: Case, nsteps: int | None = None):
    s = OracleSolver(case)
    tr = s.run(case.steps if nsteps is None else nsteps)
    return s, tr


def relative_l2(a: np.ndarray, ref: np.ndarray, mask: np.ndarray | None = None) -> float:
    if mask is not None:
        a = a[mask]
        ref = ref[mask]
    den = float(np.sqrt(np.sum(ref * ref)))
    num = float(np.sqrt(np.sum((a - ref) ** 2)))
    return num / den if den > 0 else num


def dft_amplitude(trace_p: np.ndarray, case: Case, step_end: int, omega: float, nwin: int):
    """P = (2i/N) sum_n p(t_n) exp(-i omega t_n) over the last N samples, so that
    p(t) = Im(P e^{i omega t}) (Sec. 4.3 / App. C convention)."""
    n = np.arange(step_end - nwin + 1, step_end + 1)
    t = n * case.dt
    ph = np.exp(-1j * omega * t)
    return (2j / nwin) * np.tensordot(ph, trace_p[-nwin:], axes=(0, 0))
