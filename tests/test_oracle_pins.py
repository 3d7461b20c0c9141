"""Pins of the oracle's building blocks against what the paper and mathematics fix.

Every test here checks the oracle against something other than itself:
printed constants, closed forms, exact (rational) arithmetic, invariants.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import lee_cases as lc
from oracle import ade as ade_mod
from oracle import geometry, schemes, weights
from oracle.solver import OracleSolver


# ---------------------------------------------------------------- schemes ---

def test_drp7_printed_coefficients_consistent():
    # Sec. 2.2: a_1..a_3 of the 7-point scheme; consistency sum 2 k a_k = 1 to
    # the 12 printed digits
    a = schemes.DRP7
    assert abs(2 * np.dot(np.arange(1, 4), a) - 1.0) < 1e-11
    kd = np.linspace(1e-3, 1.05, 200)
    err = np.abs(schemes.drp_wavenumber(a, kd) - kd)
    assert err.max() < 1e-3          # dispersion-relation preserving range


def test_drp11_order_and_dispersion():
    a = schemes.DRP11
    k = np.arange(1, 6)
    assert abs(2 * np.dot(k, a) - 1.0) < 1e-14       # consistency
    assert abs(np.dot(k ** 3, a)) < 1e-11            # fourth order
    kd = np.linspace(1e-3, 1.55, 400)
    err = np.abs(schemes.drp_wavenumber(a, kd) - kd)
    assert err.max() < 1e-3          # resolves a wider band than the 7-point set


def test_filter_damping_function():
    d = schemes.FILTER11
    assert abs(schemes.filter_response(d, np.array([0.0]))[0]) < 1e-15
    assert abs(schemes.filter_response(d, np.array([math.pi]))[0] - 1.0) < 1e-12
    kd = np.linspace(0, math.pi, 1000)
    D = schemes.filter_response(d, kd)
    assert D.min() > -1e-12 and D.max() < 1.0 + 1e-12
    assert np.all(D[kd < math.pi / 4] < 1e-4)       # well-resolved waves kept


def test_rk_two_register_is_fourth_order_taylor():
    rng = np.random.default_rng(0)
    for _ in range(20):
        z = complex(*rng.normal(size=2))
        taylor = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
        assert abs(schemes.rk_amplification(z) - taylor) < 1e-13
    assert np.allclose(schemes.RK_C, [0, 0.25, 1 / 3, 0.5])


# ----------------------------------------------------- 1-D extrapolation ---

def test_lagrange_weights_at_r5():
    # closed form: l_j(-5) on nodes 0..4 = (126, -420, 540, -315, 70)
    assert np.allclose(weights.lagrange_at(-5.0), [126, -420, 540, -315, 70], atol=1e-10)


@pytest.mark.parametrize("r", [0.0, 0.37, 1.3, 2.7, 4.9])
def test_ns_ghost_closed_forms(r):
    """eq. ns-ghost: Dirichlet f_GP = (g - sum c_i f_i)/c_0 with c_0 = 24/prod(r+i),
    Neumann with c~_0 = -50/prod(r+i)."""
    prod = (r + 1) * (r + 2) * (r + 3) * (r + 4)
    L = weights.lagrange_at(-r)
    B = weights.birkhoff_at(-r)
    assert abs(L[0] - prod / 24.0) < 1e-10 * max(1, prod)
    assert abs(B[0] + prod / 50.0) < 1e-10 * max(1, prod)
    # c_i / c_0 from the polynomial through (-r, f_GP), (1..4, f_i) evaluated at 0
    nodes = [-r, 1.0, 2.0, 3.0, 4.0]
    c = weights.lagrange_at(0.0, nodes=nodes)            # Q(0) = sum c_i Q(node_i)
    # f_GP = (g - sum_{i>=1} c_i f_i) / c_0 = L0 g + sum_{i>=1} L_i f_i
    assert np.allclose(-c[1:] / c[0], L[1:], rtol=1e-9, atol=1e-9)


def test_birkhoff_reproduces_quartics():
    rng = np.random.default_rng(1)
    for r in (0.2, 3.3, 4.8):
        B = weights.birkhoff_at(-r)
        for _ in range(5):
            q = np.polynomial.Polynomial(rng.normal(size=5))
            lhs = q(-r)
            rhs = B[0] * q.deriv()(0.0) + sum(B[i] * q(float(i)) for i in range(1, 5))
            assert abs(lhs - rhs) < 1e-9 * (1 + abs(lhs))


# --------------------------------------------------------- least squares ---

def _cases_small():
    return [
        lc.Case(nx=40, ny=36, x0=-20.0, y0=-17.0, h=1.0, wall=lc.Wall("line", 0.3, -0.2, *lc.line_normal(30.0))),
        lc.Case(nx=44, ny=44, x0=-22.0, y0=-22.0, h=1.0, wall=lc.Wall("circle", 0.31, 0.17, rc=9.3)),
        lc.Case(nx=64, ny=64, x0=-8.0, y0=-8.0, h=0.25, wall=lc.Wall("circle", 0.07, -0.05, rc=0.61)),
    ]


@pytest.mark.parametrize("case", _cases_small(), ids=["line30", "circle9h", "small-circle"])
def test_composite_weights_reproduce_polynomials(case):
    """Every polynomial of total degree <= 4 sampled on a cloud is reproduced at
    the ghost by all three forms: free, Dirichlet with g = f(BP), Neumann with
    g_n = df/dn(BP); and the read-out gives f(P_i) at BP + i h n."""
    s = OracleSolver(case.replace(impedance=lc.Impedance("rigid")))
    rng = np.random.default_rng(7)
    assert len(s.gidx) > 0
    ex = [(a, b) for d in range(5) for a in range(d + 1) for b in [d - a]]
    coef = rng.normal(size=len(ex))
    x0, y0 = 0.4, -0.3

    def f(x, y):
        return sum(c * ((x - x0) / 3) ** a * ((y - y0) / 3) ** b for c, (a, b) in zip(coef, ex))

    def grad(x, y):
        gx = sum(c * a * ((x - x0) / 3) ** (a - 1) / 3 * ((y - y0) / 3) ** b for c, (a, b) in zip(coef, ex) if a > 0)
        gy = sum(c * b * ((x - x0) / 3) ** a * ((y - y0) / 3) ** (b - 1) / 3 for c, (a, b) in zip(coef, ex) if b > 0)
        return gx, gy

    checked = 0
    for g in range(len(s.gidx)):
        if s.deg[g] != 4:
            continue
        a, b = s.cptr[g], s.cptr[g + 1]
        idx = s.cidx[a:b]
        xc = case.x0 + (idx % case.nx) * case.h
        yc = case.y0 + (idx // case.nx) * case.h
        fc = f(xc, yc)
        W = s.Ws[g]
        nx_, ny_ = s.gnx[g], s.gny[g]
        Pi = [(s.bx[g] + i * case.h * nx_, s.by[g] + i * case.h * ny_) for i in range(5)]
        scale = 1 + np.abs(fc).max()
        assert np.allclose(W @ fc, [f(*P) for P in Pi], atol=1e-8 * scale)
        gx_ = case.x0 + (s.gidx[g] % case.nx) * case.h
        gy_ = case.y0 + (s.gidx[g] // case.nx) * case.h
        fgp = f(gx_, gy_)
        L, B = s.lag[g], s.bir[g]
        read = W @ fc
        free = L @ read
        dirichlet = L[0] * f(*Pi[0]) + L[1:] @ read[1:]
        gxv, gyv = grad(*Pi[0])
        neumann = B[0] * case.h * (gxv * nx_ + gyv * ny_) + B[1:] @ read[1:]
        for val in (free, dirichlet, neumann):
            assert abs(val - fgp) < 1e-6 * scale, (g, val, fgp)
        checked += 1
    assert checked > 10


def _exact_readout(xp, yp, k=4):
    """W = E (V^T V)^{-1} V^T in exact rational arithmetic on the double inputs."""
    ex = weights.monomial_exponents(k)
    X = [Fraction(float(v)) for v in xp]
    Y = [Fraction(float(v)) for v in yp]
    V = [[x ** a * y ** b for (a, b) in ex] for x, y in zip(X, Y)]
    M = len(ex)
    N = len(X)
    A = [[sum(V[n][i] * V[n][j] for n in range(N)) for j in range(M)] for i in range(M)]
    # E rows: monomials at (i, 0)
    E = [[Fraction(i) ** a if b == 0 else Fraction(0) for (a, b) in ex] for i in range(5)]
    # solve A Z = E^T  (Z: M x 5), then W = Z^T V^T
    aug = [A[i][:] + [E[r][i] for r in range(5)] for i in range(M)]
    for c in range(M):
        piv = next(rw for rw in range(c, M) if aug[rw][c] != 0)
        aug[c], aug[piv] = aug[piv], aug[c]
        pv = aug[c][c]
        aug[c] = [v / pv for v in aug[c]]
        for rw in range(M):
            if rw != c and aug[rw][c] != 0:
                fct = aug[rw][c]
                aug[rw] = [v - fct * w for v, w in zip(aug[rw], aug[c])]
    Z = [[aug[i][M + r] for r in range(5)] for i in range(M)]
    W = [[float(sum(Z[i][r] * V[n][i] for i in range(M))) for n in range(N)] for r in range(5)]
    return np.array(W)


def test_least_squares_against_exact_rational_solution():
    case = _cases_small()[0]
    s = OracleSolver(case.replace(impedance=lc.Impedance("rigid")))
    picks = [g for g in range(len(s.gidx)) if s.deg[g] == 4][:3]
    for g in picks:
        a, b = s.cptr[g], s.cptr[g + 1]
        We = _exact_readout(s.xp[a:b], s.yp[a:b])
        assert np.max(np.abs(We - s.Ws[g])) < 1e-9 * (1 + np.abs(We).max())


# -------------------------------------------------------------- geometry ---

def _brute_geometry(case):
    """Ghosts and clouds by plain loops over the whole grid with exact rational
    predicates on the double-valued inputs."""
    Fr = Fraction
    h = Fr(case.h)
    w = case.wall

    def X(i):
        return Fr(case.x0) + i * h

    def Y(j):
        return Fr(case.y0) + j * h

    def phi(x, y):
        if w.kind == "line":
            return (x - Fr(w.cx)) * Fr(w.nx) + (y - Fr(w.cy)) * Fr(w.ny)
        return (x - Fr(w.cx)) ** 2 + (y - Fr(w.cy)) ** 2 - Fr(w.rc) ** 2

    fl = [[phi(X(i), Y(j)) > 0 for i in range(case.nx)] for j in range(case.ny)]
    R = geometry.stencil_reach(case)
    ghosts = []
    for j in range(case.ny):
        for i in range(case.nx):
            if fl[j][i]:
                continue
            hit = False
            for d in range(1, R + 1):
                for (a, b) in ((i + d, j), (i - d, j), (i, j + d), (i, j - d)):
                    if 0 <= a < case.nx and 0 <= b < case.ny and fl[b][a]:
                        hit = True
            if hit:
                ghosts.append(j * case.nx + i)
    return fl, ghosts


@pytest.mark.parametrize("case", _cases_small()[:2], ids=["line30", "circle9h"])
def test_mask_and_ghosts_brute_force(case):
    fl, ghosts = _brute_geometry(case)
    assert np.array_equal(geometry.fluid_mask(case), np.array(fl))
    assert np.array_equal(geometry.ghost_points(case, geometry.fluid_mask(case)), np.array(ghosts))


def test_cloud_lists_brute_force():
    """Clouds re-derived over the whole domain (no window) with the ellipse of
    eq. ns-ellipse in exact arithmetic from the oracle's BP and normal."""
    case = _cases_small()[1]
    s = OracleSolver(case.replace(impedance=lc.Impedance("rigid")))
    Fr = Fraction
    for g in range(0, len(s.gidx), 7):
        bx, by, nx_, ny_ = (Fr(float(v)) for v in (s.bx[g], s.by[g], s.gnx[g], s.gny[g]))
        h = Fr(case.h)
        out = []
        for j in range(case.ny):
            for i in range(case.nx):
                if not s.fluid[j, i]:
                    continue
                dx = Fr(case.x0) + i * h - bx
                dy = Fr(case.y0) + j * h - by
                xp = (nx_ * dx + ny_ * dy) / h
                yp = (-ny_ * dx + nx_ * dy) / h
                if (xp / 8) ** 2 + (yp / 3) ** 2 <= 1:
                    x = Fr(case.x0) + i * h
                    y = Fr(case.y0) + j * h
                    if (x - Fr(case.wall.cx)) * nx_ + (y - Fr(case.wall.cy)) * ny_ >= 0:
                        out.append(j * case.nx + i)
        assert list(s.cidx[s.cptr[g]:s.cptr[g + 1]]) == out


def test_boundary_point_invariants():
    for case in _cases_small():
        s = OracleSolver(case.replace(impedance=lc.Impedance("rigid")))
        gx = case.x0 + (s.gidx % case.nx) * case.h
        gy = case.y0 + (s.gidx // case.nx) * case.h
        assert np.allclose(np.hypot(s.gnx, s.gny), 1.0, atol=1e-14)
        assert np.allclose(np.abs(geometry.level_set(case, s.bx, s.by)), 0.0, atol=1e-12)
        assert np.allclose(gx, s.bx - s.r * case.h * s.gnx, atol=1e-12)
        assert np.allclose(gy, s.by - s.r * case.h * s.gny, atol=1e-12)
        assert s.r.min() >= 0.0 and s.r.max() < 5.0 * math.sqrt(2.0)


def test_horizontal_wall_ghost_count():
    """A horizontal wall between rows: ghosts are exactly the reach R = 5 solid
    rows next to the fluid, nx per row."""
    case = lc.Case(nx=50, ny=40, x0=0.0, y0=0.0, h=1.0, wall=lc.Wall("line", 0.0, 19.5, 0.0, 1.0))
    fl = geometry.fluid_mask(case)
    g = geometry.ghost_points(case, fl)
    assert len(g) == 5 * 50
    assert set(g // 50) == {15, 16, 17, 18, 19}


def test_flat_wall_counts_and_edge_rule():
    case = lc.flat_wall_201()
    s = OracleSolver(case)
    assert len(s.gidx) == 1005
    # clouds cut by the domain edge occur only where the wall meets the edge
    gi = s.gidx % case.nx
    gj = s.gidx // case.nx
    e = np.minimum(np.minimum(gi, gj), np.minimum(case.nx - 1 - gi, case.ny - 1 - gj))
    assert s.cut.sum() > 0 and e[s.cut].max() <= 13
    assert np.all(s.deg[~s.cut] == 4)


# -------------------------------------------------------------------- ADE ---

@pytest.mark.parametrize("imp", [(0.5, 0.02, 10.0), (1.0, 0.01, 5.0), (0.2, 0.025, 1.6), (1.0, 3.2, 0.3125)])
def test_ade_transfer_function_is_admittance(imp):
    R, M, K = imp
    a = ade_mod.ade_from_impedance(lc.Impedance("msd", R=R, M=M, K=K), dt=1e-4)
    A, f, c = (np.array(x, dtype=float) for x in a.matrices())
    for w in (0.3, 1.0, 7.0, 40.0, 300.0):
        H = c @ np.linalg.solve(1j * w * np.eye(2) - A, f)
        Z = R + 1j * (M * w - K / w)
        assert abs(H - 1.0 / Z) < 1e-12 * abs(1.0 / Z)
    # the poles are the roots of M s^2 + R s + K
    roots = np.sort_complex(np.roots([M, R, K]))
    assert np.allclose(np.sort_complex(np.linalg.eigvals(A)), roots, rtol=1e-12)


def test_ade_step_response_closed_form():
    """u_n for a unit pressure step: (e^{s1 t} - e^{s2 t}) / (M (s1 - s2))."""
    R, M, K = 0.5, 0.02, 10.0
    a = ade_mod.ade_from_impedance(lc.Impedance("msd", R=R, M=M, K=K), dt=1e-4)
    A, f, c = (np.array(x, dtype=float) for x in a.matrices())
    s1, s2 = np.roots([M, R, K])
    from scipy.linalg import expm
    for t in (0.01, 0.05, 0.2):
        # exact state for constant forcing: Psi(t) = A^-1 (e^{At} - I) f
        psi = np.linalg.solve(A, (expm(A * t) - np.eye(2)) @ f)
        exact = (np.exp(s1 * t) - np.exp(s2 * t)) / (M * (s1 - s2))
        assert abs(c @ psi - exact.real) < 1e-10 and abs(exact.imag) < 1e-12


def test_ade_rejections():
    with pytest.raises(ade_mod.ImpedanceError):   # critical damping R = 2 sqrt(KM)
        ade_mod.ade_from_impedance(lc.Impedance("msd", R=2 * math.sqrt(10 * 0.02), M=0.02, K=10.0), 1e-3)
    with pytest.raises(ade_mod.ImpedanceError):   # literal flat-wall values at dt = 0.5
        ade_mod.ade_from_impedance(lc.FLAT_IMPEDANCE_LITERAL, 0.5)
    ade_mod.ade_from_impedance(lc.FLAT_IMPEDANCE_GRID, 0.5)
    assert ade_mod.ade_from_impedance(lc.Impedance("rigid"), 0.5).matrices()[2] == [0.0, 0.0]


# A broadband admittance in the multi-pole form of Sec. 2.3: one relaxation
# term and two resonances (5 states), all poles in the left half-plane.
MULTIPOLE = lc.Impedance("poles", real=((-0.5, 0.3),),
                         pairs=((-0.3, 2 * math.pi / 8.0, 0.2, 0.05), (-1.5, 1.2, 0.1, -0.04)))


def _rational(imp, s):
    """Eq. Yrational written out term by term (no direct term)."""
    y = 0j
    for lam, a in imp.real:
        y += a / (s - lam)
    for al, be, b, c in imp.pairs:
        q = complex(b, c)
        sk = complex(al, be)
        y += q / (s - sk) + np.conj(q) / (s - np.conj(sk))
    return y


def test_multipole_transfer_function_is_the_rational_admittance():
    """c (s - A)^-1 f of the auxiliary system (eqs. ADEgeneral, unGeneral)
    equals eq. Yrational at every s off the poles, seeded random terms too."""
    rng = np.random.default_rng(2609)
    imps = [MULTIPOLE]
    for _ in range(4):
        nr, npr = int(rng.integers(0, 3)), int(rng.integers(1, 3))
        imps.append(lc.Impedance("poles", real=tuple((-rng.uniform(0.1, 5), rng.normal()) for _ in range(nr)),
                                 pairs=tuple((-rng.uniform(0.1, 5), rng.uniform(0.1, 9), rng.normal(), rng.normal())
                                             for _ in range(npr))))
    for imp in imps:
        a = ade_mod.ade_from_impedance(imp, dt=1e-3)
        A, f, c = (np.array(x, dtype=float) for x in a.matrices())
        assert len(f) == len(imp.real) + 2 * len(imp.pairs)
        for s in (0.3j, 1.0j, 7.0j, 40.0j, 0.5 + 2.0j):
            H = c @ np.linalg.solve(s * np.eye(len(f)) - A, f)
            Y = _rational(imp, s)
            assert abs(H - Y) < 1e-12 * max(abs(Y), 1e-3), (imp, s)
        want = sorted([complex(l) for l, _ in imp.real] +
                      [complex(al, sg * be) for al, be, _, _ in imp.pairs for sg in (1, -1)],
                      key=lambda z: (z.real, z.imag))
        got = sorted(np.linalg.eigvals(A), key=lambda z: (z.real, z.imag))
        assert np.allclose(got, want, rtol=1e-12)


def test_msd_written_as_poles_steps_like_the_msd():
    """The mass-spring-damper admittance expanded in partial fractions (its
    poles are the roots of M s^2 + R s + K, the residues s_k / (M (s_k - s_j)))
    is the N = 2 or M = 1 case of eq. Yrational: the oracle steps it exactly
    like the MSD kinds, in both regimes."""
    base = lc.small_cylinder(64, 12)
    for R, M, K in ((1.0, 0.2, 10.0), (2.0, 0.2, 1.0)):
        s1, s2 = np.roots([M, R, K])
        if abs(s1.imag) > 0:
            s1 = s1 if s1.imag > 0 else s2
            q = s1 / (M * (s1 - np.conj(s1)))
            poles = lc.Impedance("poles", pairs=((s1.real, s1.imag, q.real, q.imag),))
        else:
            l1, l2 = sorted([s1.real, s2.real], reverse=True)
            poles = lc.Impedance("poles", real=((l1, l1 / (M * (l1 - l2))), (l2, l2 / (M * (l2 - l1)))))
        runs = []
        for imp in (lc.Impedance("msd", R=R, M=M, K=K), poles):
            s = OracleSolver(base.replace(impedance=imp))
            tr = s.run(12)
            runs.append((s.fields(), s.psi.copy(), tr))
        (fa, pa, ta), (fb, pb, tb) = runs
        for x, y in zip(fa, fb):
            assert np.abs(x - y).max() <= 1e-13 * np.abs(x).max()
        assert np.abs(pa - pb).max() <= 1e-12 * max(np.abs(pa).max(), 1e-30)
        assert np.abs(ta - tb).max() <= 1e-13 * np.abs(ta).max()


def test_multipole_rejections():
    with pytest.raises(ade_mod.ImpedanceError):       # a pole in the right half-plane
        ade_mod.ade_from_impedance(lc.Impedance("poles", real=((0.5, 1.0),)), 1e-3)
    with pytest.raises(ade_mod.ImpedanceError):       # more than 8 states
        ade_mod.ade_from_impedance(lc.Impedance("poles", pairs=((-1.0, 1.0, 0.1, 0.0),) * 5), 1e-3)
    with pytest.raises(ade_mod.ImpedanceError):       # no term at all
        ade_mod.ade_from_impedance(lc.Impedance("poles"), 1e-3)
    with pytest.raises(ade_mod.ImpedanceError):       # dt * lambda outside the RK4 region
        ade_mod.ade_from_impedance(lc.Impedance("poles", real=((-100.0, 1.0),)), 0.05)
    ade_mod.ade_from_impedance(MULTIPOLE, 0.25)


def test_msd_peak_gain_closed_form_against_brute_force():
    """max_w |i w Y(i w)| of the mass-spring-damper (closed form in ade.peak_gain)
    against a dense search on the admittance itself, in both pole regimes, and
    its limit 1/M when 2 K M <= R^2."""
    rng = np.random.default_rng(5)
    for _ in range(40):
        R, M, K = (float(np.exp(rng.uniform(np.log(a), np.log(b)))) for a, b in ((0.05, 10), (0.001, 1), (0.5, 100)))
        imp = lc.Impedance("msd", R=R, M=M, K=K)
        g = lambda w: np.abs(1j * w / (M * 1j * w + R + K / (1j * w)))
        w = np.exp(np.linspace(np.log(1e-3), np.log(1e5), 400001))
        k = int(np.argmax(g(w)))
        fine = np.linspace(w[max(k - 1, 0)], w[min(k + 1, len(w) - 1)], 200001)   # around the coarse maximum
        brute = max(float(np.max(g(fine))), float(np.max(g(w))), 1.0 / M)
        got = ade_mod.peak_gain(imp)
        assert got >= brute * (1 - 1e-12) and got - brute <= 1e-9 * brute, (R, M, K, got, brute)
    assert ade_mod.peak_gain(lc.Impedance("msd", R=2.0, M=0.5, K=1.0)) == 2.0        # 2KM = 1 < R^2 = 4
