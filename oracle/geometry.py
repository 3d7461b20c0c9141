"""Mask, ghost points, boundary points and elliptical clouds (oracle, FP64).

Follows Sec. 3.1 of the paper:

* mask: a node is fluid when the wall's level set is positive, solid
  otherwise; the equations are advanced at fluid nodes only;
* ghost points: the solid nodes that the difference stencil of some fluid
  node reaches (reading: a fluid node lies within the stencil reach along
  +-x or +-y; the paper states "3 layers" for its 7-point stencil, i.e. the
  stencil reach);
* boundary point BP: projection of the ghost point on the wall along the wall
  normal n, which points from the wall into the fluid; d = |GP - BP|,
  r = d / h (eq. ns-rotation and the text after it);
* cloud: fluid nodes inside the ellipse of eq. ns-ellipse, centred on BP,
  half-axes R_n = 2k along n and R_t = k/2 + 1 along the tangent, in the
  reduced coordinates x' = T (x - x_BP) / h.  For a circle, only the nodes on
  the BP's half of the body (x - c).n >= 0 are kept, so a body thinner than
  the ellipse does not pull in fluid from its far side (reading: the paper's
  bodies are always wider than the ellipse).
* clouds cut by the domain edge (reading; the paper's flat case is periodic
  across the wall's ends, so its walls never meet an outer boundary): when
  the ellipse of a ghost reaches outside the domain, the ghost is treated as
  part of the zero outer frame (all of its weights are zero).  Without this
  the truncated one-sided fits near the corner where an inclined wall meets
  the domain edge drive a fast instability.

All predicates are written as fixed FP64 expressions, evaluated in this order,
so that an independent implementation evaluating the same expressions gets
bit-identical lists.

Parity: pinned in tests by exact counts on hand-checkable grids, by brute-force
re-derivation of the predicates with exact rational arithmetic on small grids,
and by geometric invariants (BP on the wall, |n| = 1, GP = BP - d n).
"""
from __future__ import annotations

import numpy as np

from lee_cases import Case

WINDOW = 14   # candidate cloud window half-size around the ghost node


def node_x(case: Case, i):
    return case.x0 + np.asarray(i, dtype=np.float64) * case.h


def node_y(case: Case, j):
    return case.y0 + np.asarray(j, dtype=np.float64) * case.h


def level_set(case: Case, x, y):
    """phi > 0 in the fluid.  line: (x - c).n ; circle: |x - c|^2 - r_c^2."""
    w = case.wall
    if w.kind == "line":
        return (x - w.cx) * w.nx + (y - w.cy) * w.ny
    if w.kind == "circle":
        dx = x - w.cx
        dy = y - w.cy
        return dx * dx + dy * dy - w.rc * w.rc
    if w.kind == "none":
        return np.ones(np.broadcast(x, y).shape)
    raise ValueError(w.kind)


def fluid_mask(case: Case) -> np.ndarray:
    """bool[ny, nx]: True at fluid nodes (phi > 0; a node exactly on the wall
    is solid)."""
    x = node_x(case, np.arange(case.nx))[None, :]
    y = node_y(case, np.arange(case.ny))[:, None]
    return level_set(case, x, y) > 0.0


def stencil_reach(case: Case) -> int:
    return max(case.H, 5) if case.filter_sigma > 0.0 else case.H


def ghost_points(case: Case, fluid: np.ndarray) -> np.ndarray:
    """Linear indices j*nx + i (ascending) of the solid nodes that some fluid
    node's stencil reaches along x or y."""
    ny, nx = fluid.shape
    R = stencil_reach(case)
    reached = np.zeros_like(fluid)
    for d in range(1, R + 1):
        reached[:, :-d] |= fluid[:, d:]     # fluid at (i+d, j)
        reached[:, d:] |= fluid[:, :-d]     # fluid at (i-d, j)
        reached[:-d, :] |= fluid[d:, :]     # fluid at (i, j+d)
        reached[d:, :] |= fluid[:-d, :]     # fluid at (i, j-d)
    ghost = reached & ~fluid
    jj, ii = np.nonzero(ghost)
    return (jj * nx + ii).astype(np.int64)   # nonzero is row-major: ascending


def boundary_points(case: Case, gidx: np.ndarray):
    """For each ghost: BP (x, y), unit normal n into the fluid, and r = d/h."""
    w = case.wall
    gi = gidx % case.nx
    gj = gidx // case.nx
    xg = node_x(case, gi)
    yg = node_y(case, gj)
    if w.kind == "line":
        phi = (xg - w.cx) * w.nx + (yg - w.cy) * w.ny
        d = -phi
        nxv = np.full(xg.shape, w.nx)
        nyv = np.full(xg.shape, w.ny)
        bx = xg + d * w.nx
        by = yg + d * w.ny
    elif w.kind == "circle":
        dx = xg - w.cx
        dy = yg - w.cy
        rho = np.sqrt(dx * dx + dy * dy)
        if np.any(rho == 0.0):
            raise ValueError("ghost point at the circle centre")
        nxv = dx / rho
        nyv = dy / rho
        bx = w.cx + w.rc * nxv
        by = w.cy + w.rc * nyv
        d = w.rc - rho
    else:
        return (np.zeros(0),) * 5
    r = d / case.h
    return bx, by, nxv, nyv, r


def clouds(case: Case, fluid: np.ndarray, gidx: np.ndarray, bx, by, nxv, nyv, k: int = 4):
    """CSR cloud lists.  Returns (ptr[G+1], idx[nnz], xp[nnz], yp[nnz], cut[G])
    where idx are linear node indices sorted ascending, (xp, yp) the reduced
    rotated coordinates of eq. ns-rotation and cut flags the ghosts whose
    ellipse reaches outside the domain."""
    nx, ny, h = case.nx, case.ny, case.h
    Rn = 2.0 * k
    Rt = k / 2.0 + 1.0
    A = Rt * Rt          # ellipse test scaled by Rn^2 Rt^2:
    B = Rn * Rn          #   Rt^2 x'^2 + Rn^2 y'^2 <= Rn^2 Rt^2
    C = Rn * Rn * Rt * Rt
    w = case.wall
    ptr = [0]
    idx, xps, yps = [], [], []
    cut = np.zeros(len(gidx), dtype=bool)
    for g in range(len(gidx)):
        gi = int(gidx[g] % nx)
        gj = int(gidx[g] // nx)
        jj, ii = np.mgrid[gj - WINDOW:gj + WINDOW + 1, gi - WINDOW:gi + WINDOW + 1]
        jj = jj.ravel()
        ii = ii.ravel()
        x = node_x(case, ii)
        y = node_y(case, jj)
        ddx = x - bx[g]
        ddy = y - by[g]
        xp = (nxv[g] * ddx + nyv[g] * ddy) / h
        yp = (-nyv[g] * ddx + nxv[g] * ddy) / h
        inside = A * xp * xp + B * yp * yp <= C
        indom = (ii >= 0) & (ii < nx) & (jj >= 0) & (jj < ny)
        cut[g] = bool(np.any(inside & ~indom))
        ii, jj, x, y, xp, yp, inside = (a[indom] for a in (ii, jj, x, y, xp, yp, inside))
        keep = inside & fluid[jj, ii]
        if w.kind == "circle":
            keep &= ((x - w.cx) * nxv[g] + (y - w.cy) * nyv[g]) >= 0.0
        lin = jj * nx + ii
        order = np.argsort(lin[keep], kind="stable")
        idx.append(lin[keep][order])
        xps.append(xp[keep][order])
        yps.append(yp[keep][order])
        ptr.append(ptr[-1] + int(keep.sum()))
    cat = (lambda a: np.concatenate(a) if a else np.zeros(0))
    return (np.asarray(ptr, dtype=np.int64), cat(idx).astype(np.int64), cat(xps), cat(yps), cut)


def filter_widths(fluid: np.ndarray) -> np.ndarray:
    """uint8[ny, nx, 2]: for each fluid node, the half-width (0..5) of its
    filter row along x (index 0) and y (index 1): the largest w <= 5 such that
    the nodes i - w .. i + w along that axis hold no non-fluid node inside
    the domain (nodes past the domain edge are the zero frame and count as
    available).  Zero at non-fluid nodes."""
    ny, nx = fluid.shape
    out = np.zeros((ny, nx, 2), dtype=np.uint8)
    solid = ~fluid
    for ax in (0, 1):
        w = np.where(fluid, 5, 0).astype(np.int64)
        for d in range(1, 6):
            near = np.zeros_like(fluid)
            if ax == 0:
                near[:, d:] |= solid[:, :-d]      # non-fluid at (i - d, j)
                near[:, :-d] |= solid[:, d:]      # non-fluid at (i + d, j)
            else:
                near[d:, :] |= solid[:-d, :]      # non-fluid at (i, j - d)
                near[:-d, :] |= solid[d:, :]      # non-fluid at (i, j + d)
            w = np.where(fluid & near, np.minimum(w, d - 1), w)
        out[:, :, ax] = w
    return out


def row_intervals(fluid: np.ndarray):
    """Fluid column intervals per row (for reporting; the oracle itself uses the
    mask directly)."""
    out = []
    for row in fluid:
        edges = np.flatnonzero(np.diff(np.concatenate(([0], row.astype(np.int8), [0]))))
        out.append(list(zip(edges[0::2], edges[1::2])))
    return out
