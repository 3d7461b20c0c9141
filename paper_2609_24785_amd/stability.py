"""Spectral stability of the scheme as the library runs it.

The abstract reports a spectral analysis of the linearised operator showing
an instability of the immersed wall where it turns tangent to the grid.
Without a source, one full step of the scheme (four stages of ghost fill,
ADE update and sweep, Sec. 2.2, 2.3 and 3) is a linear map G of the state:
q^n at the fluid nodes (p, u, v, each over the fluid nodes in row-major
order, x fastest) followed, for an impedance wall, by the auxiliary states
of every ghost.  The scheme is stable when the spectral radius of G is at
most 1; above 1, the worst mode grows by that factor every step.

Three tools, all running the library's kernels:
* step_matrix: G column by column on a small grid (one step from each unit
  state); its eigenvalues come from a dense host eigen-solve;
* operator_matrix: the semi-discrete operator L (G is the fourth-order
  Taylor polynomial of dt L) column by column, one right-hand-side
  evaluation per unit state (lee_rhs); the real parts of its eigenvalues are
  growth rates per unit time, free of the time step;
* power_growth: the growth per step of the worst mode by power iteration,
  for grids far too large to assemble: run chunks of steps from a start
  state and renormalise between chunks.

The state is read and written with lee_get_fields / lee_set_fields and the
ADE-state calls; the fluid nodes are those that lee_set_fields keeps.
"""
from __future__ import annotations

import math

import numpy as np

from .lee import Instance


def _check_homogeneous(inst: Instance):
    if inst.case.source is not None:
        raise ValueError("the step map is affine with a source term; analyse the case without it")


def fluid_mask(inst: Instance) -> np.ndarray:
    """bool[ny, nx]: the nodes whose values the scheme advances.  The current
    fields are saved and put back."""
    p, u, v = inst.fields()
    c = inst.case
    inst.set_fields(np.ones((c.ny, c.nx)), None, None)
    m = inst.fields()[0] != 0.0
    inst.set_fields(p, u, v)
    return m


def aux_count(inst: Instance) -> int:
    s = inst.summary
    return 0 if int(s.ade_kind) == 0 else int(s.ade_states) * int(s.G)


class StatePacker:
    """Maps the library's state to the flat vector described above."""

    def __init__(self, inst: Instance):
        self.inst = inst
        self.mask = fluid_mask(inst)
        self.nf = int(self.mask.sum())
        self.naux = aux_count(inst)
        self.n = 3 * self.nf + self.naux

    def put(self, x: np.ndarray):
        c, nf = self.inst.case, self.nf
        planes = []
        for k in range(3):
            a = np.zeros((c.ny, c.nx))
            a[self.mask] = x[k * nf:(k + 1) * nf]
            planes.append(a)
        self.inst.set_fields(*planes)
        if self.naux:
            self.inst.set_ade_states(x[3 * nf:])

    def get(self) -> np.ndarray:
        nf = self.nf
        out = np.empty(self.n)
        for k, a in enumerate(self.inst.fields()):
            out[k * nf:(k + 1) * nf] = a[self.mask]
        if self.naux:
            out[3 * nf:] = self.inst.ade_states().reshape(-1)[:self.naux]
        return out


def step_matrix(inst: Instance) -> np.ndarray:
    """G[n, n], column k = one full step from the k-th unit state."""
    _check_homogeneous(inst)
    sp = StatePacker(inst)
    G = np.empty((sp.n, sp.n))
    e = np.zeros(sp.n)
    for k in range(sp.n):
        e[k] = 1.0
        sp.put(e)
        inst.step_n(1)
        G[:, k] = sp.get()
        e[k] = 0.0
    return G


def operator_matrix(inst: Instance) -> np.ndarray:
    """L[n, n], the semi-discrete operator (the right-hand side with the
    ghosts eliminated), column k the right-hand side at the k-th unit state
    (lee_rhs, through the instance's stage kernels); same state ordering as
    step_matrix.  Its eigenvalues are the growth rates per unit time."""
    _check_homogeneous(inst)
    sp = StatePacker(inst)
    L = np.empty((sp.n, sp.n))
    e = np.zeros(sp.n)
    nf = sp.nf
    for k in range(sp.n):
        e[k] = 1.0
        sp.put(e)
        p, u, v, psi = inst.rhs()
        for m, a in enumerate((p, u, v)):
            L[m * nf:(m + 1) * nf, k] = a[sp.mask]
        if sp.naux:
            L[3 * nf:, k] = psi.reshape(-1)[:sp.naux]
        e[k] = 0.0
    return L


def spectral_abscissa(L: np.ndarray) -> float:
    """Largest real part of the eigenvalues of L (stable when <= 0)."""
    return float(np.max(np.linalg.eigvals(L).real))


def spectral_radius(G: np.ndarray) -> float:
    return float(np.max(np.abs(np.linalg.eigvals(G))))


def power_growth(inst: Instance, x0: np.ndarray, steps: int, chunk: int = 100):
    """Power iteration from the packed state x0: `steps` steps in chunks of
    `chunk`, the state renormalised after each chunk.  Returns (estimate,
    log_norms): the geometric-mean growth per step over the second half of
    the chunks, and the accumulated log-norm after each chunk."""
    _check_homogeneous(inst)
    if steps < 2 * chunk:
        raise ValueError("need at least two chunks")
    sp = StatePacker(inst)
    x = np.asarray(x0, dtype=np.float64)
    if x.shape != (sp.n,):
        raise ValueError(f"start state must have {sp.n} entries")
    x = x / np.linalg.norm(x)
    nch = steps // chunk
    acc, logs = 0.0, []
    for _ in range(nch):
        sp.put(x)
        inst.step_n(chunk)
        x = sp.get()
        nrm = float(np.linalg.norm(x))
        if not math.isfinite(nrm) or nrm == 0.0:
            raise FloatingPointError(f"state norm became {nrm} after {len(logs) + 1} chunks")
        acc += math.log(nrm)
        logs.append(acc)
        x /= nrm
    half = nch // 2
    est = math.exp((logs[-1] - logs[half - 1]) / ((nch - half) * chunk))
    return est, np.asarray(logs)
