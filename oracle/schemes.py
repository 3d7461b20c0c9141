"""Difference, filter and time-integration coefficients (oracle, FP64).

* DRP7: the 7-point DRP first derivative printed in Sec. 2.2 (eq. DRP_s):
  a_1..a_3, antisymmetric, a_0 = 0.
* DRP11: the 11-point first derivative.  The paper prints only the 7-point
  set; the 11-point set used here is the optimised 11-point scheme of Bogey &
  Bailly (2004), which is in the paper's bibliography.  Pinned by the
  consistency condition sum 2 k a_k = 1, the fourth-order conditions and the
  dispersion error bound (tests).
* FILTER11: the 11-point selective filter of the same reference, as the
  symmetric stencil D f_i = d_0 f_i + sum_j d_j (f_{i+j} + f_{i-j}).  It is
  applied inside every stage as the damping term -(sigma_d/dt)(D_x + D_y) q.
  Pinned by D(0) = 0 (no damping of a constant) and D(pi) = 1 (full removal
  of the grid-scale mode); beyond these two the coefficient values are
  parity unpinned (recalled from the reference, which is not at hand).
* centred_filter(w): near an immersed wall, where fewer than five fluid
  nodes lie on one side of a node along an axis, that axis takes the
  standard centred filter of the largest half-width w that fits in the fluid
  (w = 0: none): D(k) = sin^{2w}(k/2), i.e. d_j = (-1)^j C(2w, w + j) / 4^w,
  which is the maximal-order centred filter on 2w + 1 nodes with D(pi) = 1.
  filter_rows() tabulates the row of every half-width 0..5.
* RK: the four-stage low-storage Runge-Kutta (Sec. 2.2 cites a low-storage
  fourth-order scheme without printing it).  Reading: the two-register form
  q^(l) = q^n + alpha_l dt RHS(q^(l-1)), alpha = (1/4, 1/3, 1/2, 1), whose
  amplification on a linear system is the fourth-order Taylor polynomial
  (pinned in tests); stage l evaluates the right-hand side at
  t^n + c_l dt with c = (0, 1/4, 1/3, 1/2).
"""
import numpy as np

# Sec. 2.2, eq. DRP_s: a_1, a_2, a_3 of the 7-point scheme.
DRP7 = np.array([0.770882380518, -0.166705904415, 0.020843142770])

# 11-point optimised first derivative (Bogey & Bailly 2004), a_1 .. a_5.
DRP11 = np.array([0.872756993962, -0.286511173973, 0.090320001280,
                  -0.020779405824, 0.002484594688])

# 11-point selective filter (Bogey & Bailly 2004), d_0 .. d_5.
FILTER11 = np.array([0.215044884112, -0.187772883589, 0.123755948787,
                     -0.059227575576, 0.018721609157, -0.002999540835])


def centred_filter(w: int) -> np.ndarray:
    """d_0..d_w of the standard centred filter of half-width w (w >= 1):
    the coefficients of sin^{2w}(k/2) = ((1 - cos k) / 2)^w as
    d_0 + 2 sum_j d_j cos(j k), i.e. d_j = (-1)^j C(2w, w + j) / 4^w."""
    from math import comb
    return np.array([(-1) ** j * comb(2 * w, w + j) / 4.0 ** w for j in range(w + 1)])


def filter_rows() -> np.ndarray:
    """rows[w, 5 + k]: weight of node i + k in the filter row of half-width
    w at node i, for w = 0..5 (w = 5: FILTER11; w = 0: no filter)."""
    rows = np.zeros((6, 11))
    for w in range(1, 6):
        d = FILTER11 if w == 5 else centred_filter(w)
        rows[w, 5] = d[0]
        for j in range(1, w + 1):
            rows[w, 5 + j] = rows[w, 5 - j] = d[j]
    return rows


RK_ALPHA = np.array([0.25, 1.0 / 3.0, 0.5, 1.0])
RK_C = np.array([0.0, 0.25, 1.0 / 3.0, 0.5])


def one_sided7(m: int):
    """First-derivative weights at point m of seven unit-spaced points
    0..6: the derivative of the degree-6 interpolant (exact rationals).  The
    outer boundary's one-sided stencils (Sec. 2.2 names them without
    printing them; reading: the maximal-order set on the same seven points)."""
    from fractions import Fraction
    pts = range(7)
    w = []
    for k in pts:
        # l_k'(m) for the Lagrange basis polynomial l_k on points 0..6
        den = Fraction(1)
        for q in pts:
            if q != k:
                den *= (k - q)
        tot = Fraction(0)
        for skip in pts:
            if skip == k:
                continue
            prod = Fraction(1)
            for q in pts:
                if q != k and q != skip:
                    prod *= (m - q)
            tot += prod
        w.append(tot / den)
    return w


#: one-sided weights for m = 0, 1, 2 nodes on the near side (rows), FP64
RAD_ONE_SIDED = np.array([[float(x) for x in one_sided7(m)] for m in range(3)])


def drp(H: int) -> np.ndarray:
    """a_1..a_H of the central first-derivative stencil of half-width H."""
    if H == 3:
        return DRP7.copy()
    if H == 5:
        return DRP11.copy()
    raise ValueError("H must be 3 or 5")


def drp_wavenumber(a: np.ndarray, kdx: np.ndarray) -> np.ndarray:
    """Effective wavenumber k* dx = 2 sum_k a_k sin(k kdx) of the stencil."""
    k = np.arange(1, len(a) + 1)
    return 2.0 * np.sum(a[None, :] * np.sin(np.outer(kdx, k)), axis=1)


def filter_response(d: np.ndarray, kdx: np.ndarray) -> np.ndarray:
    """Damping function D(k dx) = d_0 + 2 sum_j d_j cos(j k dx)."""
    j = np.arange(1, len(d))
    return d[0] + 2.0 * np.sum(d[None, 1:] * np.cos(np.outer(kdx, j)), axis=1)


def rk_amplification(z: complex) -> complex:
    """Amplification of one step of the two-register scheme on dq/dt = z q/dt,
    applying the stages literally."""
    q = 1.0 + 0j
    qs = q
    for a in RK_ALPHA:
        qs = q + a * z * qs
    return qs
