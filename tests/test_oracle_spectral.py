"""Pins of the oracle's spectral analysis of the step map.

The step matrix G is checked against an operator built independently from
the stencils (Kronecker products of 1-D difference and filter matrices,
eq. DRP_s and the selective filter of Sec. 2.2) and the fourth-order Taylor
polynomial of the two-register scheme, against the dissipativity that the
central stencil, the filter and the sponge guarantee on a wall-free grid,
and against stepping itself (G^k x0 equals k steps from x0, which fails if
the state omits anything a step depends on).
"""
import math

import numpy as np
import pytest

import lee_cases as lc
from oracle import schemes
from oracle import spectral as sp


def _wall_free(nx, ny, H, fs, sponge_cells=0, sponge_sigma=0.0):
    return lc.Case(nx=nx, ny=ny, x0=0.0, y0=0.0, h=0.7, H=H, cfl=0.5,
                   filter_sigma=fs, sponge_cells=sponge_cells,
                   sponge_sigma=sponge_sigma, name="wall-free")


def _diff1(n, a, h):
    """1-D central first derivative with zero values outside [0, n)."""
    D = np.zeros((n, n))
    for i in range(n):
        for k, ak in enumerate(a, start=1):
            if i + k < n:
                D[i, i + k] += ak / h
            if i - k >= 0:
                D[i, i - k] -= ak / h
    return D


def _filt1(n, d):
    Fm = np.zeros((n, n))
    for i in range(n):
        Fm[i, i] += d[0]
        for k in range(1, len(d)):
            if i + k < n:
                Fm[i, i + k] += d[k]
            if i - k >= 0:
                Fm[i, i - k] += d[k]
    return Fm


def _operator(case):
    """Semi-discrete operator of the LEE without mean flow (Sec. 2.1:
    p_t = -(u_x + v_y), u_t = -p_x, v_t = -p_y), state [p; u; v] over the
    nodes in row-major order, plus -(sigma_d/dt)(D_x + D_y) q for the filter
    and -sigma_s(x) q for the sponge."""
    nx, ny, h = case.nx, case.ny, case.h
    a = schemes.drp(case.H)
    Ix, Iy = np.eye(nx), np.eye(ny)
    Dx = np.kron(Iy, _diff1(nx, a, h))
    Dy = np.kron(_diff1(ny, a, h), Ix)
    damp = np.zeros((nx * ny, nx * ny))
    if case.filter_sigma > 0:
        d = schemes.FILTER11
        damp += (case.filter_sigma / case.dt) * (np.kron(Iy, _filt1(nx, d)) + np.kron(_filt1(ny, d), Ix))
    if case.sponge_cells > 0:
        s = np.zeros(nx * ny)
        W = case.sponge_cells
        for j in range(ny):
            for i in range(nx):
                e = min(i, j, nx - 1 - i, ny - 1 - j)
                if e < W:
                    s[j * nx + i] = case.sponge_sigma * ((W - e) / W) ** 2
        damp += np.diag(s)
    Z = np.zeros_like(Dx)
    return np.block([[-damp, -Dx, -Dy], [-Dx, -damp, Z], [-Dy, Z, -damp]])


def _taylor4(A):
    out = np.eye(len(A))
    term = np.eye(len(A))
    for k in range(1, 5):
        term = term @ A / k
        out = out + term
    return out


@pytest.mark.parametrize("H,fs,sw", [(5, 0.2, 3), (3, 0.0, 0), (5, 0.0, 0)])
def test_wall_free_step_matrix_is_taylor_polynomial(H, fs, sw):
    case = _wall_free(13, 11, H, fs, sponge_cells=sw, sponge_sigma=0.4 if sw else 0.0)
    G = sp.step_matrix(case)
    ref = _taylor4(case.dt * _operator(case))
    assert G.shape == ref.shape
    assert np.max(np.abs(G - ref)) < 1e-13 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("H,fs,sw", [(5, 0.2, 3), (3, 0.0, 0), (5, 0.0, 0)])
def test_wall_free_scheme_does_not_grow(H, fs, sw):
    # central stencil: skew part; filter (non-negative symbol, zero-padded
    # principal block of a positive semi-definite Toeplitz matrix) and sponge:
    # non-positive symmetric part; dt |lambda| stays inside the RK4 region.
    case = _wall_free(12, 12, H, fs, sponge_cells=sw, sponge_sigma=0.4 if sw else 0.0)
    G = sp.step_matrix(case)
    rho = sp.spectral_radius(G)
    assert rho <= 1.0 + 1e-12
    if fs > 0:
        assert rho < 1.0 - 1e-6      # the filter damps every mode


def test_flipped_filter_sign_would_grow():
    # the dissipativity pin discriminates: the same operator with the filter
    # term's sign flipped has a growing mode
    case = _wall_free(12, 12, 5, 0.2)
    L = _operator(case)
    L_bad = _operator(case.replace(filter_sigma=0.0)) * 2 - L
    assert sp.spectral_radius(_taylor4(case.dt * L_bad)) > 1.0 + 1e-3
    assert sp.spectral_radius(_taylor4(case.dt * L)) < 1.0


def _small_cylinder(z):
    n = 18
    c0 = -0.5 * (n - 1)
    return lc.Case(nx=n, ny=n, x0=c0, y0=c0, h=1.0, H=5, cfl=0.5, filter_sigma=0.2,
                   wall=lc.Wall("circle", 0.25, 0.125, rc=4.0), impedance=z, name="cyl-18")


MSD = lc.Impedance("msd", R=1.0, M=0.05 * 64.0, K=20.0 / 64.0)


@pytest.mark.parametrize("z", [lc.Impedance(), MSD], ids=["rigid", "msd"])
def test_step_matrix_composes_with_stepping(z):
    case = _small_cylinder(z)
    G = sp.step_matrix(case)
    rng = np.random.default_rng(7)
    x0 = rng.standard_normal(G.shape[0])
    want = x0.copy()
    for _ in range(6):
        want = G @ want
    got = sp.apply_steps(case, x0, 6)
    assert np.max(np.abs(got - want)) < 1e-11 * np.max(np.abs(want))
    if z.kind == "msd":
        # the auxiliary states are part of the state: G couples them both ways
        nf = (G.shape[0] - sp.state_size(case.replace(impedance=lc.Impedance())))
        assert nf > 0
        naux = nf
        assert np.abs(G[-naux:, :-naux]).max() > 0 and np.abs(G[:-naux, -naux:]).max() > 0


def test_power_estimate_converges_to_known_spectrum():
    rng = np.random.default_rng(3)
    n = 40
    lam = np.concatenate([[1.02], rng.uniform(-0.9, 0.9, n - 1)])
    V = rng.standard_normal((n, n))
    A = V @ np.diag(lam) @ np.linalg.inv(V)
    est = sp.growth_estimate(A, rng.standard_normal(n), 600)
    assert abs(est - 1.02) < 1e-9
    assert abs(sp.spectral_radius(A) - 1.02) < 1e-10


def test_growing_modes_sit_at_the_wall():
    # a coarse rigid cylinder (radius 4 cells): the modes that grow are wall
    # modes, the wall-free part of the grid being non-growing (pinned above)
    case = _small_cylinder(lc.Impedance())
    G = sp.step_matrix(case)
    w, V = np.linalg.eig(G)
    s = sp._solver(case)
    nf = int(s.fluid.sum())
    jj, ii = np.nonzero(s.fluid)
    r = np.hypot(case.x0 + ii - case.wall.cx, case.y0 + jj - case.wall.cy)
    grow = np.nonzero(np.abs(w) > 1.0 + 1e-8)[0]
    for k in grow:
        v = np.abs(V[:, k])
        amp = v[:nf] ** 2 + v[nf:2 * nf] ** 2 + v[2 * nf:3 * nf] ** 2
        # most of the mode's energy within 3 cells of the wall
        assert amp[r < case.wall.rc + 3.0].sum() > 0.5 * amp.sum()
