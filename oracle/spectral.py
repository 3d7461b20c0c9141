"""Spectral stability of the fully discrete scheme (oracle, FP64).
TEST INFRASTRUCTURE ONLY.

The abstract states that a spectral analysis of the linearised semi-discrete
operator shows the instability that appears when the immersed wall turns
tangent to the grid, reduced but not removed by the normal-stencil
reconstruction.  The body does not say how that analysis was set up.

Reading used here: with the source off, one full step of the scheme is a
linear map G of the state.  The state is q^n at the fluid nodes, the three
fields in the order p, u, v, each over the fluid nodes in row-major order
(x fastest), then, for an impedance wall, the auxiliary states of every ghost
(Sec. 2.3), ghost by ghost.  Ghost, solid and frame nodes are not part of
the state: every stage fills the ghosts again from the current stage value
and the auxiliary states (Sec. 3.2), and the sweep leaves zeros at every
node that is not a fluid node.  G is assembled column by column: step the
oracle once from each unit vector.  Since the ghost fill and the
right-hand side are linear, G is the fourth-order Taylor polynomial of
dt L, with L the semi-discrete operator with the ghosts eliminated (the
two-register scheme on a linear system).  The scheme is stable when the
spectral radius of G does not exceed 1, and the growth per step of the worst
mode is that spectral radius.

The semi-discrete operator L itself (operator_matrix: the right-hand side
at each unit state) gives the growth rates per unit time as the real parts
of its eigenvalues; G = P4(dt L) ties the two assemblies together.

Parity: pinned (tests) against an independent Kronecker-product
construction of L and its Taylor polynomial on wall-free grids, and against
the dissipativity that the central stencil, the selective filter and the
sponge guarantee there.
"""
from __future__ import annotations

import numpy as np

from lee_cases import Case
from .solver import F, OracleSolver


def _solver(case: Case, filter_rows=None) -> OracleSolver:
    # The analysis is of the homogeneous scheme: no source, no probes.
    return OracleSolver(case.replace(ic=None, source=None, probes=(), dft_steps=0), filter_rows)


def state_size(case: Case) -> int:
    s = _solver(case)
    return _layout(s)[2]


def _layout(s: OracleSolver):
    nf = int(s.fluid.sum())
    naux = s.ns * len(s.gidx) if s.ade.kind != "rigid" else 0
    return nf, naux, 3 * nf + naux


def _put(s: OracleSolver, x: np.ndarray):
    c = s.case
    nf, naux, _ = _layout(s)
    sl = (slice(F, F + c.ny), slice(F, F + c.nx))
    for k, arr in enumerate((s.p, s.u, s.v)):
        arr[...] = 0.0
        arr[sl][s.fluid] = x[k * nf:(k + 1) * nf]
    s.psi[...] = 0.0
    if naux:
        s.psi[:naux] = x[3 * nf:]


def _get(s: OracleSolver) -> np.ndarray:
    c = s.case
    nf, naux, n = _layout(s)
    sl = (slice(F, F + c.ny), slice(F, F + c.nx))
    out = np.empty(n)
    for k, arr in enumerate((s.p, s.u, s.v)):
        out[k * nf:(k + 1) * nf] = arr[sl][s.fluid]
    if naux:
        out[3 * nf:] = s.psi[:naux]
    return out


def step_matrix(case: Case, filter_rows=None) -> np.ndarray:
    """G[n, n]: column k is one full step applied to the k-th unit state
    (filter_rows: see OracleSolver)."""
    s = _solver(case, filter_rows)
    n = _layout(s)[2]
    G = np.empty((n, n))
    e = np.zeros(n)
    for k in range(n):
        e[k] = 1.0
        _put(s, e)
        s.run(1)
        G[:, k] = _get(s)
        e[k] = 0.0
    return G


def operator_matrix(case: Case) -> np.ndarray:
    """L[n, n], the semi-discrete operator of the scheme (the right-hand side
    with the ghosts eliminated: every stage fills them linearly from the
    stage value and the auxiliary states), in the state ordering of
    step_matrix; column k is the right-hand side at the k-th unit state
    (oc_rhs).  The step map is the fourth-order Taylor polynomial of dt L;
    the eigenvalues of L are the growth rates per unit time, independent of
    the time step."""
    import ctypes
    from .solver import _load, _ptr
    s = _solver(case)
    lib = _load()
    lib.oc_rhs.restype = ctypes.c_int
    lib.oc_rhs.argtypes = [ctypes.c_void_p] * 5 + [ctypes.c_double] + [ctypes.c_void_p] * 4
    c = s.case
    nf, naux, n = _layout(s)
    sl = (slice(F, F + c.ny), slice(F, F + c.nx))
    rp, ru, rv = (np.zeros(s.shape) for _ in range(3))
    rpsi = np.zeros_like(s.psi)
    L = np.empty((n, n))
    e = np.zeros(n)
    for k in range(n):
        e[k] = 1.0
        _put(s, e)
        if lib.oc_rhs(ctypes.byref(s._cs), _ptr(s.p), _ptr(s.u), _ptr(s.v), _ptr(s.psi), 0.0,
                      _ptr(rp), _ptr(ru), _ptr(rv), _ptr(rpsi)) != 0:
            raise MemoryError("oracle core allocation failed")
        for m, arr in enumerate((rp, ru, rv)):
            L[m * nf:(m + 1) * nf, k] = arr[sl][s.fluid]
        if naux:
            L[3 * nf:, k] = rpsi[:naux]
        e[k] = 0.0
    return L


def spectral_abscissa(L: np.ndarray) -> float:
    """Largest real part of the eigenvalues of L: the growth rate per unit
    time of the worst mode of the semi-discrete scheme (stable when <= 0)."""
    return float(np.max(np.linalg.eigvals(L).real))


def apply_steps(case: Case, x0: np.ndarray, steps: int) -> np.ndarray:
    """The state after `steps` full steps from x0 (same ordering as G)."""
    s = _solver(case)
    _put(s, np.asarray(x0, dtype=np.float64))
    s.run(steps)
    return _get(s)


def spectral_radius(G: np.ndarray) -> float:
    return float(np.max(np.abs(np.linalg.eigvals(G))))


def growth_estimate(G: np.ndarray, x0: np.ndarray, steps: int) -> float:
    """Power-iteration estimate of the spectral radius: the geometric-mean
    growth per step of |G^k x0| over the second half of `steps` steps."""
    x = np.asarray(x0, dtype=np.float64) / np.linalg.norm(x0)
    logs = []
    acc = 0.0
    for _ in range(steps):
        x = G @ x
        nrm = np.linalg.norm(x)
        acc += np.log(nrm)
        logs.append(acc)
        x /= nrm
    half = steps // 2
    return float(np.exp((logs[-1] - logs[half - 1]) / (steps - half)))
