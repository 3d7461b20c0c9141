"""Least-squares read-out and 1-D extrapolation weights (oracle, FP64).

Step 1 (Sec. 3.1, eqs. ns-poly2d, ns-vandermonde, ns-LSQ, ns-readout): for a
cloud of N fluid nodes at reduced coordinates (x'_n, y'_n), the polynomial of
total degree k is fitted in the least-squares sense, V a = f, and evaluated at
the normal-stencil points P_i = (i, 0), i = 0..m, m = 4.  Since the fit is
linear in f, the read-out is a matrix W (5 x N) with f(P_i) = sum_n W[i, n] f_n,
W = E V^+ where E holds the monomials at P_i.  The oracle obtains V^+ with
numpy's SVD-based least-squares solver on the column-scaled Vandermonde
matrix; the normal equations of eq. ns-LSQ give the same minimiser but square
the condition number.

Degree fallback (reading; the paper never meets a truncated cloud): if the
cloud has fewer nodes than monomials, or the column-scaled V has
sigma_min / sigma_max < 1e-10, the degree drops to 3, 2, 1; if even degree 1
fails, all weights of that ghost are zero and the ghost is flagged.

Step 2 (Sec. 3.1, eq. ns-ghost): a 1-D polynomial Q of degree m along the
normal, s = 0 at BP and s = -r at the ghost point:

* free:      Q(i) = f(P_i), i = 0..4               -> f_GP = sum_i l_i(-r) f(P_i)
* Dirichlet: Q(0) = g, Q(i) = f(P_i), i = 1..4     -> f_GP = l_0 g + sum_{i>=1} l_i f(P_i)
* Neumann:   Q'(0) = h dg/dn, Q(i) = f(P_i), i>=1  -> f_GP = mu_0 h g_n + sum_{i>=1} mu_i f(P_i)

l_i are the Lagrange basis values at s = -r on the nodes 0..4; mu are the
Birkhoff weights, solved from the five moment conditions.  These are the
same ghost values as eq. ns-ghost (c_0 = 24 / prod(r + i), and
c~_0 = -50 / prod(r + i) for the Neumann form): pinned in tests.

Parity: pinned by polynomial reproduction (all polynomials of total degree
<= 4 are reproduced exactly by every form), by exact rational least squares
on small clouds, and by the closed forms above.
"""
from __future__ import annotations

import numpy as np

M_DEG = 4          # m = k = 4 (Sec. 3.1)
RANK_TOL = 1e-10


def monomial_exponents(k: int):
    """Graded order: degree d = 0..k, alpha = d..0, beta = d - alpha, giving
    1, x', y', x'^2, x'y', y'^2, ... as in eq. ns-vandermonde."""
    out = []
    for d in range(k + 1):
        for a in range(d, -1, -1):
            out.append((a, d - a))
    return out


def vandermonde(xp: np.ndarray, yp: np.ndarray, k: int) -> np.ndarray:
    ex = monomial_exponents(k)
    return np.stack([xp ** a * yp ** b for (a, b) in ex], axis=1)


def readout_matrix(k: int, m: int = M_DEG) -> np.ndarray:
    """E[i, :] = monomials at P_i = (i, 0), i = 0..m."""
    ex = monomial_exponents(k)
    E = np.zeros((m + 1, len(ex)))
    for i in range(m + 1):
        for c, (a, b) in enumerate(ex):
            E[i, c] = float(i) ** a if b == 0 else 0.0
    return E


def scaled_rank_ok(V: np.ndarray) -> bool:
    n = np.sqrt(np.sum(V * V, axis=0))
    if np.any(n == 0.0):
        return False
    s = np.linalg.svd(V / n[None, :], compute_uv=False)
    return s[-1] > RANK_TOL * s[0]


def scaled_sigma_ratio(V: np.ndarray) -> float:
    n = np.sqrt(np.sum(V * V, axis=0))
    if np.any(n == 0.0):
        return 0.0
    s = np.linalg.svd(V / n[None, :], compute_uv=False)
    return float(s[-1] / s[0])


def lsq_readout(xp: np.ndarray, yp: np.ndarray, kmax: int = M_DEG):
    """Returns (W[5, N], degree used).  degree 0 means "no usable fit": W = 0."""
    N = len(xp)
    for k in range(kmax, 0, -1):
        M = (k + 1) * (k + 2) // 2
        if N < M:
            continue
        V = vandermonde(xp, yp, k)
        if not scaled_rank_ok(V):
            continue
        n = np.sqrt(np.sum(V * V, axis=0))
        Vs = V / n[None, :]
        Vs_pinv = np.linalg.lstsq(Vs, np.eye(N), rcond=None)[0]   # M x N
        V_pinv = Vs_pinv / n[:, None]
        return readout_matrix(k) @ V_pinv, k
    return np.zeros((M_DEG + 1, N)), 0


def lagrange_at(s: float, nodes=(0.0, 1.0, 2.0, 3.0, 4.0)) -> np.ndarray:
    """l_j(s) = prod_{q != j} (s - x_q) / (x_j - x_q)."""
    out = np.ones(len(nodes))
    for j, xj in enumerate(nodes):
        for q, xq in enumerate(nodes):
            if q != j:
                out[j] *= (s - xq) / (xj - xq)
    return out


def birkhoff_at(s: float, m: int = M_DEG) -> np.ndarray:
    """mu with Q(s) = mu_0 Q'(0) + sum_{i=1..m} mu_i Q(i) for every Q of degree
    <= m: the moment conditions on the monomials s^p, p = 0..m."""
    A = np.zeros((m + 1, m + 1))
    rhs = np.zeros(m + 1)
    for p in range(m + 1):
        A[p, 0] = 1.0 if p == 1 else 0.0             # d/ds s^p at 0
        for i in range(1, m + 1):
            A[p, i] = float(i) ** p
        rhs[p] = s ** p
    return np.linalg.solve(A, rhs)


def ghost_stencils(xp_all, yp_all, ptr, r, cut=None):
    """Per ghost: W (list of 5 x N arrays), degree, Lagrange l(-r), Birkhoff mu(-r).
    Ghosts flagged in ``cut`` (cloud cut by the domain edge) get degree 0 and
    zero weights."""
    G = len(r)
    Ws, deg = [], np.zeros(G, dtype=np.int64)
    lag = np.zeros((G, M_DEG + 1))
    bir = np.zeros((G, M_DEG + 1))
    for g in range(G):
        a, b = ptr[g], ptr[g + 1]
        if cut is not None and cut[g]:
            Ws.append(np.zeros((M_DEG + 1, b - a)))
            continue
        W, k = lsq_readout(xp_all[a:b], yp_all[a:b])
        Ws.append(W)
        deg[g] = k
        if k > 0:                      # a ghost without a usable fit stays 0
            lag[g] = lagrange_at(-r[g])
            bir[g] = birkhoff_at(-r[g])
    return Ws, deg, lag, bir
