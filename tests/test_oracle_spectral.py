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
    # the paper's setting (no filter) on a coarse rigid cylinder (radius 4
    # cells): the modes that grow are wall modes, the wall-free part of the
    # grid being non-growing (pinned above)
    case = _small_cylinder(lc.Impedance()).replace(filter_sigma=0.0)
    G = sp.step_matrix(case)
    w, V = np.linalg.eig(G)
    s = sp._solver(case)
    nf = int(s.fluid.sum())
    jj, ii = np.nonzero(s.fluid)
    r = np.hypot(case.x0 + ii - case.wall.cx, case.y0 + jj - case.wall.cy)
    grow = np.nonzero(np.abs(w) > 1.0 + 1e-8)[0]
    assert len(grow) > 0
    k = int(np.argmax(np.abs(w)))
    v = np.abs(V[:, k])
    amp = v[:nf] ** 2 + v[nf:2 * nf] ** 2 + v[2 * nf:3 * nf] ** 2
    near = r < case.wall.rc + 3.0
    # the fastest-growing mode: most of its energy within 3 cells of the
    # wall, where fewer than 40% of the fluid nodes lie
    assert near.mean() < 0.4 and amp[near].sum() > 0.6 * amp.sum()


# ---------------------------------------------------------------------------
# The filter next to an immersed wall.  Each axis of a fluid node takes the
# widest centred filter row that reads no non-fluid node of the domain (the
# 11-point selective filter five nodes from the wall, standard centred filters
# of half-width 4..1 closer, none next to it).  Reading the extrapolated ghost
# values instead makes the damping term -(sigma_d/dt) F q anti-dissipative at
# the wall: a mode then grows by the same factor per step at every time
# step, i.e. as sigma_d/dt per unit time.

def _coarse(k, z, cfl):
    n, rc, dx, dy = ((24, 4.0, 0.0, 0.0), (28, 4.0, 0.49, 0.245))[k]
    return lc.coarse_cylinder(n, rc, dx, dy, impedance=z).replace(cfl=cfl)


MSD_COARSE = lc.Impedance("msd", R=0.5, M=1.28, K=10.0 / 64.0)   # the 1024^2 wall in grid units


@pytest.mark.parametrize("z", [lc.Impedance(), MSD_COARSE], ids=["rigid", "msd"])
def test_filtered_wall_does_not_grow(z):
    # shifted coarse cylinder: no growing mode at either time step
    for cfl in (0.5, 0.25):
        rho = sp.spectral_radius(sp.step_matrix(_coarse(1, z, cfl)))
        assert rho <= 1.0 + 1e-9, (cfl, rho)


def test_filter_reduces_tangency_growth():
    # centred coarse cylinder (radius 4 cells): the tangency mode of the
    # scheme keeps a residue, well below the unfiltered scheme's
    for cfl in (0.5, 0.25):
        rho_f = sp.spectral_radius(sp.step_matrix(_coarse(0, lc.Impedance(), cfl)))
        rho_0 = sp.spectral_radius(sp.step_matrix(_coarse(0, lc.Impedance(), cfl).replace(filter_sigma=0.0)))
        assert rho_0 > 1.005 and rho_f - 1.0 < 0.05 * (rho_0 - 1.0), (cfl, rho_f, rho_0)


def _power_growth(case, steps=2000, chunk=100):
    s = sp._solver(case)
    n = sp._layout(s)[2]
    x = np.random.default_rng(1).standard_normal(n)
    x /= np.linalg.norm(x)
    logs = []
    for _ in range(steps // chunk):
        sp._put(s, x)
        s.run(chunk)
        x = sp._get(s)
        nrm = np.linalg.norm(x)
        logs.append(math.log(nrm))
        x /= nrm
    half = len(logs) // 2
    return math.exp(sum(logs[half:]) / ((len(logs) - half) * chunk))


def test_benchmark_wall_does_not_grow():
    # the 1024^2 cylinder-pulse wall (radius 32 cells, centre shifted by
    # 0.3 h, its impedance) on a 128^2 crop of that grid: the worst mode
    # decays at both time steps (the 11-point row at every node grew by
    # 1.0023 per step here)
    h = 1.0 / 64.0
    for cfl in (0.5, 0.25):
        case = lc.Case(nx=128, ny=128, x0=-64 * h, y0=-64 * h, h=h, H=5, cfl=cfl, filter_sigma=0.2,
                       wall=lc.Wall("circle", 0.3 * h, 0.3 * h, rc=0.5),
                       impedance=lc.Impedance("msd", R=0.5, M=0.02, K=10.0))
        assert _power_growth(case) < 1.0, cfl


def test_filter_reading_ghost_values_would_grow():
    # planted reading: the 11-point row at every node, so that next to the
    # wall it reads the extrapolated ghost values; the same coarse cylinder
    # then grows, and by the same factor per step at both time steps
    full = np.tile(schemes.filter_rows()[5], (6, 1))
    rho = [sp.spectral_radius(sp.step_matrix(_coarse(0, lc.Impedance(), cfl), filter_rows=full))
           for cfl in (0.5, 0.25)]
    assert min(rho) > 1.005, rho
    assert abs(rho[0] - rho[1]) < 1e-3 * (rho[0] - 1.0) + 1e-4, rho
    # without any filter the growth per step halves with the step (a rate
    # per unit time): the tangency mode of the scheme itself
    free = [sp.spectral_radius(sp.step_matrix(_coarse(0, lc.Impedance(), cfl).replace(filter_sigma=0.0)))
            for cfl in (0.5, 0.25)]
    g = [math.log(r) / (cfl * 1.0) for r, cfl in zip(free, (0.5, 0.25))]
    assert min(free) > 1.0 and abs(g[0] - g[1]) < 0.25 * g[0], (free, g)


def test_centred_filter_rows():
    rows = schemes.filter_rows()
    k = np.linspace(0.0, math.pi, 37)
    j = np.arange(-5, 6)
    assert np.all(rows[0] == 0.0)
    assert np.array_equal(rows[5, 5:], np.asarray(schemes.FILTER11))
    for w in range(1, 5):
        r = rows[w]
        assert np.all(r[np.abs(j) > w] == 0.0) and np.array_equal(r, r[::-1])
        sym = r @ np.cos(np.outer(j, k))
        assert np.max(np.abs(sym - np.sin(k / 2) ** (2 * w))) < 1e-14
        # it leaves every polynomial of degree below 2w untouched
        for m in range(2 * w):
            assert abs(r @ (j.astype(float) ** m)) < 1e-12
        assert abs(r @ (j.astype(float) ** (2 * w))) > 1e-3
    for w in range(6):
        assert abs(rows[w].sum()) < 1e-15


def _widths_brute(fluid):
    ny, nx = fluid.shape
    out = np.zeros((ny, nx, 2), dtype=np.uint8)
    for jj in range(ny):
        for ii in range(nx):
            if not fluid[jj, ii]:
                continue
            for ax, (di, dj) in enumerate(((1, 0), (0, 1))):
                w = 0
                while w < 5:
                    ok = True
                    for s in (-(w + 1), w + 1):
                        a, b = ii + s * di, jj + s * dj
                        if 0 <= a < nx and 0 <= b < ny and not fluid[b, a]:
                            ok = False
                    if not ok:
                        break
                    w += 1
                out[jj, ii, ax] = w
    return out


def test_filter_widths_brute_force():
    from oracle import geometry
    rng = np.random.default_rng(11)
    masks = [rng.uniform(size=(13, 17)) > p for p in (0.1, 0.3, 0.6)]
    c = lc.coarse_cylinder(24, 4.0, 0.25, 0.125)
    masks.append(geometry.fluid_mask(c))
    f = lc.flat_wall_201(1)
    masks.append(geometry.fluid_mask(f)[60:110, 70:140])
    for m in masks:
        assert np.array_equal(geometry.filter_widths(m), _widths_brute(m))


# ---------------------------------------------------------------------------
# The wall coupling gain h lim sY(s) (1/M for the mass-spring-damper): with
# the filter on, walls up to 1.5 step like the rigid wall; beyond it the
# step map grows, which is why both sides refuse such walls.

def _light_wall(gain, h=1.0):
    M = h / gain
    K = M * 0.09                                      # resonance 0.3 per unit time
    return lc.Impedance("msd", R=2.0 * 0.3 * math.sqrt(K * M), M=M, K=K)


def test_coupling_gain_limit(monkeypatch):
    from oracle import ade as ade_mod
    rigid = sp.spectral_radius(sp.step_matrix(_coarse(1, lc.Impedance(), 0.5)))
    ok = sp.spectral_radius(sp.step_matrix(_coarse(1, _light_wall(1.4), 0.5)))
    assert ok <= max(1.0, rigid) + 1e-9, (ok, rigid)
    with pytest.raises(ade_mod.ImpedanceError):
        sp.step_matrix(_coarse(1, _light_wall(1.6), 0.5))
    # planted: the rules lifted, a wall of gain 2 grows
    monkeypatch.setattr(ade_mod, "COUPLING_MAX", 10.0)
    monkeypatch.setattr(ade_mod, "PEAK_MAX", 100.0)
    bad = sp.spectral_radius(sp.step_matrix(_coarse(1, _light_wall(2.0), 0.5)))
    assert bad > 1.005, bad


def _resonant_wall(peak, wh=1.0, h=1.0):
    # h/M = 0.8, resonance w_res h = wh, peak gain h w_res / R = peak
    M = 1.25 * h
    K = M * (wh / h) ** 2
    return lc.Impedance("msd", R=wh / peak, M=M, K=K)


def test_peak_coupling_gain_limit(monkeypatch):
    from oracle import ade as ade_mod
    rigid = sp.spectral_radius(sp.step_matrix(_coarse(1, lc.Impedance(), 0.5)))
    z = _resonant_wall(2.9)
    assert 2.9 < ade_mod.peak_gain(z) <= 3.0
    ok = sp.spectral_radius(sp.step_matrix(_coarse(1, z, 0.5)))
    assert ok <= max(1.0, rigid) + 1e-9, (ok, rigid)
    with pytest.raises(ade_mod.ImpedanceError):
        sp.step_matrix(_coarse(1, _resonant_wall(3.2), 0.5))
    # planted: the rule lifted, a lightly damped resonance of peak gain 5 grows
    monkeypatch.setattr(ade_mod, "PEAK_MAX", 100.0)
    bad = sp.spectral_radius(sp.step_matrix(_coarse(1, _resonant_wall(5.0, wh=0.5), 0.5)))
    assert bad > 1.002, bad


# ---- the semi-discrete operator L (abstract: spectral analysis of the
# linearised semi-discrete operator) ----------------------------------------

@pytest.mark.parametrize("H,fs,sw", [(5, 0.2, 3), (3, 0.0, 0)])
def test_wall_free_operator_is_the_kronecker_operator(H, fs, sw):
    case = _wall_free(13, 11, H, fs, sponge_cells=sw, sponge_sigma=0.4 if sw else 0.0)
    L = sp.operator_matrix(case)
    ref = _operator(case)
    assert L.shape == ref.shape
    assert np.max(np.abs(L - ref)) < 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("z", [lc.Impedance(), MSD_COARSE], ids=["rigid", "msd"])
@pytest.mark.parametrize("H,fs", [(5, 0.2), (3, 0.0)], ids=["11pt-filter", "paper-scheme"])
def test_step_map_is_taylor_polynomial_of_operator_with_a_wall(z, H, fs):
    # one RHS evaluation per unit state against four stages per unit state:
    # G = P4(dt L) holds with the ghost fill and the auxiliary states in both
    c = lc.coarse_cylinder(20, 4.0, 0.31, 0.17, impedance=z, H=H, filter_sigma=fs)
    G = sp.step_matrix(c)
    L = sp.operator_matrix(c)
    assert np.max(np.abs(G - _taylor4(c.dt * L))) < 1e-13 * max(1.0, np.max(np.abs(G)))
    if z.kind != "rigid":                       # the auxiliary states couple both ways
        nf = (L.shape[0] - 2 * len(sp._solver(c).gidx)) // 3
        assert np.abs(L[3 * nf:, :3 * nf]).max() > 0 and np.abs(L[:3 * nf, 3 * nf:]).max() > 0


def test_operator_does_not_depend_on_the_time_step_without_the_filter():
    # without the filter's sigma_d / dt term the right-hand side has no dt in
    # it (the ADE derivative and the Neumann datum are rates): growth rates
    # per unit time are properties of the space discretisation alone
    c = lc.coarse_cylinder(20, 4.0, 0.31, 0.17, impedance=MSD_COARSE, H=3, filter_sigma=0.0)
    L1 = sp.operator_matrix(c.replace(cfl=0.5))
    L2 = sp.operator_matrix(c.replace(cfl=0.25))
    assert np.max(np.abs(L1 - L2)) <= 1e-15 * np.max(np.abs(L1))


def test_paper_scheme_grows_at_the_wall_and_the_filter_rows_do_not():
    # the semi-discrete growth rate of a coarse shifted cylinder: the paper's
    # scheme (no filter) has growing modes; the filtered scheme with the
    # near-wall rows has none beyond rounding of the eigen-solve
    c = lc.coarse_cylinder(24, 4.0, 0.31, 0.17)
    a_paper = sp.spectral_abscissa(sp.operator_matrix(c.replace(H=3, filter_sigma=0.0)))
    a_filt = sp.spectral_abscissa(sp.operator_matrix(c))
    assert a_paper > 5e-3, a_paper
    assert a_filt < 2e-4, a_filt


@pytest.mark.parametrize("z", [lc.Impedance(), MSD_COARSE], ids=["rigid", "msd"])
def test_explicit_filter_form_does_not_grow(z):
    # the filter once per step (q <- q - sigma F q after the step) with the
    # same near-wall rows: no growing mode on the shifted coarse cylinder at
    # either time step, and the step map is the filter after P4(dt L) with L
    # free of the filter
    for cfl in (0.5, 0.25):
        c = _coarse(1, z, cfl).replace(filter_explicit=True)
        G = sp.step_matrix(c)
        assert sp.spectral_radius(G) <= 1.0 + 1e-9, cfl
    L = sp.operator_matrix(c)
    assert np.allclose(L, sp.operator_matrix(c.replace(filter_sigma=0.0)), rtol=0, atol=0)
