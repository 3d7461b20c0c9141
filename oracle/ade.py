"""Mass-spring-damper impedance and its auxiliary differential equations (oracle).

Sec. 2.5: Z(s) = M s + R + K / s, Y = 1 / Z = (s / M) / ((s - s1)(s - s2)),
s_{1,2} = -R/(2M) +- sqrt((R/2M)^2 - K/M).

* complex pair (K/M > (R/2M)^2): s1 = -a + i b, residue
  q1 = s1 / (M (s1 - s2)) = B1 + i C1; two real states per boundary point,
  dPsi1/dt = -a Psi1 - b Psi2 + p_BP, dPsi2/dt = -a Psi2 + b Psi1,
  u_n = 2 B1 Psi1 - 2 C1 Psi2 (eq. ADE-un) and
  du_n/dt = 2 B1 dPsi1/dt - 2 C1 dPsi2/dt (eq. ADE-dpdn);
* two real poles: the N = 2, M = 0 case of eq. Yrational (Sec. 2.3):
  dPhi_k/dt = lambda_k Phi_k + p, u_n = sum_k A_k Phi_k, A_k the residues of Y;
* critical damping (double pole): rejected, the partial fractions divide by
  s1 - s2 (reading for the tolerance: |disc| <= 1e-9 K/M);
* rigid wall (Sec. 2.4): all residues zero, u_n = 0, nothing is advanced;
* general multi-pole admittance (Sec. 2.3, eqs. Yrational, ADEgeneral,
  unGeneral) with no direct term: one state Phi_k per real pole,
  dPhi_k/dt = lambda_k Phi_k + p, and two per pole pair,
  dPsi1/dt = alpha Psi1 - beta Psi2 + p, dPsi2/dt = alpha Psi2 + beta Psi1;
  u_n = sum_k A_k Phi_k + sum_k 2 (B_k Psi1_k - C_k Psi2_k).  Every pole must
  lie in the open left half-plane; a direct term Y_inf is not supported
  (its Neumann datum would need dp_BP/dt).

Stability reading: the ADE is advanced by the same RK4 as the field, so its
poles must satisfy |R4(dt s_k)| <= 1 with R4 the RK4 amplification polynomial
(checked at set-up; a violating impedance is rejected).

Coupling reading (the paper states none): the Neumann ghost value takes
h du_n/dt = h s Y(s) p_BP in the frequency domain, which feeds the boundary
pressure back into the stencil with gain h |s Y(s)|.  With the selective
filter on, spectral radii of the step map on coarse cylinders stay at the
rigid wall's while the high-frequency gain h lim_{s -> oo} s Y(s) (h/M for
the MSD) is at most 1.5 (growth from about 1.6) and while the peak gain
h max_w |i w Y(i w)| (about h w_res / R for a lightly damped resonance) is at
most 3.5 (growth from about 4, at w_res h from 0.5 to 2); walls beyond 1.5
or 3 are rejected (check_coupling).  Without the filter the scheme carries
the tangency growth of the wall itself, the coupling only adds to it
smoothly, and nothing is rejected.

u_n is counted positive from the fluid into the wall (Sec. 2.3).

Every kind is handed to the time stepper as one dense linear system
dPsi/dt = A Psi + f p_BP, u_n = c . Psi, with ns = len(f) states per ghost.

Parity: pinned in tests by the frequency response c (i w - A)^-1 f = 1/Z(i w)
in both regimes, the closed-form step response, and the pole eigenvalues; the
multi-pole form by c (i w - A)^-1 f against eq. Yrational evaluated directly
and by the MSD written as poles, which must step exactly like the MSD kinds.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

from lee_cases import Impedance

CRITICAL_TOL = 1e-9
MAX_STATES = 8


class ImpedanceError(ValueError):
    pass


@dataclass(frozen=True)
class ADE:
    kind: str          # "rigid" | "complex" | "real" | "poles"
    a: float = 0.0     # complex: s1 = -a + i b
    b: float = 0.0
    B1: float = 0.0
    C1: float = 0.0
    lam1: float = 0.0  # real: poles and residues
    lam2: float = 0.0
    A1: float = 0.0
    A2: float = 0.0
    real: tuple = ()   # poles: ((lambda_k, A_k), ...)
    pairs: tuple = ()  # poles: ((alpha_k, beta_k, B_k, C_k), ...)

    def matrices(self):
        """(A, f, c) with dPsi/dt = A Psi + f p, u_n = c . Psi."""
        if self.kind == "poles":
            n = len(self.real) + 2 * len(self.pairs)
            A = [[0.0] * n for _ in range(n)]
            f = [0.0] * n
            c = [0.0] * n
            i = 0
            for lam, a in self.real:            # eq. ADEgeneral (a)
                A[i][i] = lam
                f[i] = 1.0
                c[i] = a
                i += 1
            for al, be, B, C in self.pairs:     # eqs. ADEgeneral (b), (c)
                A[i][i], A[i][i + 1] = al, -be
                A[i + 1][i], A[i + 1][i + 1] = be, al
                f[i] = 1.0
                c[i], c[i + 1] = 2.0 * B, -2.0 * C
                i += 2
            return A, f, c
        if self.kind == "complex":
            return ([[-self.a, -self.b], [self.b, -self.a]], [1.0, 0.0],
                    [2.0 * self.B1, -2.0 * self.C1])
        if self.kind == "real":
            return ([[self.lam1, 0.0], [0.0, self.lam2]], [1.0, 1.0], [self.A1, self.A2])
        return ([[0.0, 0.0], [0.0, 0.0]], [0.0, 0.0], [0.0, 0.0])

    def poles(self):
        if self.kind == "poles":
            out = [complex(lam) for lam, _ in self.real]
            for al, be, _, _ in self.pairs:
                out += [complex(al, be), complex(al, -be)]
            return out
        if self.kind == "complex":
            return [complex(-self.a, self.b), complex(-self.a, -self.b)]
        if self.kind == "real":
            return [complex(self.lam1), complex(self.lam2)]
        return []


def rk4_poly(z: complex) -> complex:
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


def admittance(imp: Impedance, s: complex) -> complex:
    """Eq. Yrational at the complex frequency s, term by term (no direct term)."""
    y = 0j
    for lam, a in imp.real:
        y += a / (s - lam)
    for al, be, B, C in imp.pairs:
        q, sk = complex(B, C), complex(al, be)
        y += q / (s - sk) + q.conjugate() / (s - sk.conjugate())
    return y


COUPLING_MAX = 1.5


def coupling_gain(imp: Impedance) -> float:
    """lim_{s -> oo} s Y(s): 1/M for the MSD, sum A_k + 2 sum B_k for a
    multi-pole admittance without direct term, 0 for a rigid wall."""
    if imp.kind == "msd":
        return 1.0 / imp.M
    if imp.kind == "poles":
        return sum(A for _, A in imp.real) + 2.0 * sum(B for _, _, B, _ in imp.pairs)
    return 0.0


PEAK_MAX = 3.0


def peak_gain(imp: Impedance) -> float:
    """max over w > 0 of |i w Y(i w)|.  MSD: |i w Y| = u / |K - M u + i R w|
    with u = w^2, whose square u^2 / ((K - M u)^2 + R^2 u) is largest at
    u* = 2 K^2 / (2 K M - R^2) when 2 K M > R^2, else as u -> oo (1/M).
    Multi-pole: the largest of the limit and of |i w Y(i w)| at w = |s_k| and
    |Im s_k| of every pole and at 2401 log-spaced w from 1e-4 to 1e8."""
    if imp.kind == "msd":
        R, M, K = imp.R, imp.M, imp.K
        if 2.0 * K * M > R * R:
            u = 2.0 * K * K / (2.0 * K * M - R * R)
            return u / math.sqrt((K - M * u) ** 2 + R * R * u)
        return 1.0 / M
    if imp.kind == "poles":
        ws = [10.0 ** (-4.0 + e / 200.0) for e in range(2401)]
        for lam, _ in imp.real:
            ws.append(abs(lam))
        for al, be, _, _ in imp.pairs:
            ws += [abs(complex(al, be)), abs(be)]
        best = abs(coupling_gain(imp))
        for w in ws:
            best = max(best, abs(1j * w * admittance(imp, 1j * w)))
        return best
    return 0.0


def check_coupling(imp: Impedance, h: float, filtered: bool) -> None:
    """Rejects a wall whose high-frequency gain h |lim sY| exceeds
    COUPLING_MAX or whose peak gain h max |i w Y(i w)| exceeds PEAK_MAX in
    the filtered scheme (see the coupling reading above)."""
    if not filtered:
        return
    if h * abs(coupling_gain(imp)) > COUPLING_MAX:
        raise ImpedanceError("wall coupling gain h lim sY(s) > 1.5 with the filter on")
    if h * peak_gain(imp) > PEAK_MAX:
        raise ImpedanceError("wall peak coupling gain h max |i w Y(i w)| > 3 with the filter on")


def ade_from_impedance(imp: Impedance, dt: float) -> ADE:
    if imp.kind == "rigid":
        return ADE("rigid")
    if imp.kind == "poles":
        n = len(imp.real) + 2 * len(imp.pairs)
        if n == 0 or n > MAX_STATES:
            raise ImpedanceError("between 1 and 8 auxiliary states")
        vals = [x for t in imp.real for x in t] + [x for t in imp.pairs for x in t]
        if any(len(t) != 2 for t in imp.real) or any(len(t) != 4 for t in imp.pairs) or \
                not all(math.isfinite(float(x)) for x in vals):
            raise ImpedanceError("pole terms")
        if any(lam >= 0.0 for lam, _ in imp.real) or any(al >= 0.0 or be <= 0.0 for al, be, _, _ in imp.pairs):
            raise ImpedanceError("poles must lie in the open left half-plane (beta > 0 for a pair)")
        ade = ADE("poles", real=tuple((float(l), float(a)) for l, a in imp.real),
                  pairs=tuple(tuple(float(x) for x in t) for t in imp.pairs))
        for s in ade.poles():
            if abs(rk4_poly(dt * s)) > 1.0:
                raise ImpedanceError("ADE pole outside the RK4 stability region")
        return ade
    R, M, K = imp.R, imp.M, imp.K
    if not (R > 0.0 and M > 0.0 and K > 0.0):
        raise ImpedanceError("M, R, K must be positive")
    a = R / (2.0 * M)
    disc = a * a - K / M
    if abs(disc) <= CRITICAL_TOL * (K / M):
        raise ImpedanceError("critical damping: double pole")
    if disc < 0.0:
        b = math.sqrt(-disc)
        s1 = complex(-a, b)
        s2 = complex(-a, -b)
        q1 = s1 / (M * (s1 - s2))
        ade = ADE("complex", a=a, b=b, B1=q1.real, C1=q1.imag)
    else:
        sq = math.sqrt(disc)
        l1 = -a + sq
        l2 = -a - sq
        ade = ADE("real", lam1=l1, lam2=l2, A1=l1 / (M * (l1 - l2)), A2=l2 / (M * (l2 - l1)))
    for s in ade.poles():
        if abs(rk4_poly(dt * s)) > 1.0:
            raise ImpedanceError("ADE pole outside the RK4 stability region")
    return ade
