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
* rigid wall (Sec. 2.4): all residues zero, u_n = 0, nothing is advanced.

Stability reading: the ADE is advanced by the same RK4 as the field, so its
poles must satisfy |R4(dt s_k)| <= 1 with R4 the RK4 amplification polynomial
(checked at set-up; a violating impedance is rejected).

u_n is counted positive from the fluid into the wall (Sec. 2.3).

Parity: pinned in tests by the frequency response c (i w - A)^-1 f = 1/Z(i w)
in both regimes, the closed-form step response, and the pole eigenvalues.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

from lee_cases import Impedance

CRITICAL_TOL = 1e-9


class ImpedanceError(ValueError):
    pass


@dataclass(frozen=True)
class ADE:
    kind: str          # "rigid" | "complex" | "real"
    a: float = 0.0     # complex: s1 = -a + i b
    b: float = 0.0
    B1: float = 0.0
    C1: float = 0.0
    lam1: float = 0.0  # real: poles and residues
    lam2: float = 0.0
    A1: float = 0.0
    A2: float = 0.0

    def matrices(self):
        """(A, f, c) with dPsi/dt = A Psi + f p, u_n = c . Psi."""
        if self.kind == "complex":
            return ([[-self.a, -self.b], [self.b, -self.a]], [1.0, 0.0],
                    [2.0 * self.B1, -2.0 * self.C1])
        if self.kind == "real":
            return ([[self.lam1, 0.0], [0.0, self.lam2]], [1.0, 1.0], [self.A1, self.A2])
        return ([[0.0, 0.0], [0.0, 0.0]], [0.0, 0.0], [0.0, 0.0])

    def poles(self):
        if self.kind == "complex":
            return [complex(-self.a, self.b), complex(-self.a, -self.b)]
        if self.kind == "real":
            return [complex(self.lam1), complex(self.lam2)]
        return []


def rk4_poly(z: complex) -> complex:
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


def ade_from_impedance(imp: Impedance, dt: float) -> ADE:
    if imp.kind == "rigid":
        return ADE("rigid")
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
