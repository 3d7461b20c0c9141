"""Closed-form and semi-analytic reference solutions used to pin the oracle.

These are independent of the oracle: they come from the governing equations
and the paper's appendices, not from the discretisation.

* free_pulse:       2-D Gaussian pulse from rest in free space, by the Hankel
                    transform of the wave equation (the transform
                    P0(k) = (pi/b) exp(-k^2 / 4b) is the one of App. B).
* image_rigid:      rigid straight wall by the method of images (u_n = 0 and
                    dp/dn = 0 on the wall, Sec. 2.4).
* monopole_from_rest: the harmonic Gaussian monopole of Sec. 4.3 switched on
                    at t = 0 in free space.
* flat_reflection:  App. A: incident packet plus the reflected signal
                    R_c * (signal at the wall), R_c = (Z - 1)/(Z + 1), by FFT.
* msd_Z:            Z(i w) = R + i (M w - K / w) (Sec. 2.5, e^{+iwt}).
* monopole_cylinder: App. C: the harmonic monopole next to a rigid or
                    impedance cylinder, closed form (Graf's addition theorem).
* pulse_cylinder:   App. B: the Gaussian pulse next to the cylinder, by
                    quadrature over frequency of the same modal expansion.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special


def free_pulse(r, t, a, w):
    """p(r, t) of p0 = a exp(-b r^2), u0 = 0, b = ln2 / w^2:
    p = (a / 2b) int_0^inf exp(-xi^2 / 4b) cos(xi t) J0(xi r) xi dxi."""
    b = math.log(2.0) / (w * w)
    kmax = math.sqrt(4.0 * b * 60.0)
    out = []
    for rr in np.atleast_1d(r):
        f = lambda k: math.exp(-k * k / (4 * b)) * math.cos(k * t) * special.j0(k * rr) * k
        val, _ = integrate.quad(f, 0.0, kmax, limit=400, epsabs=1e-14, epsrel=1e-11)
        out.append(a / (2 * b) * val)
    return np.array(out)


def image_rigid(x, y, xs, ys, nx, ny, cx, cy, t, a, w):
    """Pulse at (xs, ys) next to the rigid line through (cx, cy) with unit
    normal (nx, ny): p = p_free(|x - xs|) + p_free(|x - xs'|)."""
    dist = (xs - cx) * nx + (ys - cy) * ny
    xi, yi = xs - 2 * dist * nx, ys - 2 * dist * ny
    r1 = np.hypot(x - xs, y - ys)
    r2 = np.hypot(x - xi, y - yi)
    return free_pulse(r1, t, a, w) + free_pulse(r2, t, a, w)


def monopole_from_rest(r, t, a, w, omega):
    """p(r, t) for p_t + div u = a exp(-b r^2) sin(omega t), u_t = -grad p, zero
    initial state.  In transform space p_tt + k^2 p = S(k) omega cos(omega t):
    p = S(k) omega (cos(omega t) - cos(k t)) / (k^2 - omega^2),
    S(k) = a (pi / b) exp(-k^2 / 4b); back-transformed with J0."""
    b = math.log(2.0) / (w * w)
    kmax = math.sqrt(4.0 * b * 60.0)

    def g(k):
        d = k * k - omega * omega
        if abs(d) < 1e-6 * omega * omega:
            return omega * t * math.sin(omega * t) / (2.0 * omega)
        return omega * (math.cos(omega * t) - math.cos(k * t)) / d

    out = []
    for rr in np.atleast_1d(r):
        f = lambda k: math.exp(-k * k / (4 * b)) * g(k) * special.j0(k * rr) * k
        val, _ = integrate.quad(f, 0.0, kmax, points=[omega] if omega < kmax else None,
                                limit=800, epsabs=1e-14, epsrel=1e-11)
        out.append(a * (math.pi / b) / (2 * math.pi) * val)
    return np.array(out)


def msd_Z(omega, R, M, K):
    return R + 1j * (M * omega - K / omega)


def flat_reflection(F, s_w, s_m, t, R, M, K, n_fft=1 << 16, dt_fft=None, t_span=None, Y=None):
    """App. A.  F(xi): incident profile along the normal coordinate s (fluid at
    s < s_w), p_i = F(s - t).  The signal seen at the wall
    sig(tau) = F(s_w - tau) is filtered by R_c(omega) = (Z - 1)/(Z + 1) with
    Z = R + i (M omega - K / omega) (e^{+i omega t} convention: the FFT of a
    real signal uses exp(-i omega t)), and the pressure at s_m is
    F(s_m - t) + r(t - (s_w - s_m)).  With an admittance function Y(s) (the
    Laplace variable s = i omega) the wall impedance is Z = 1 / Y instead,
    R_c = (1 - Y) / (1 + Y)."""
    if dt_fft is None:
        dt_fft = 0.01
    tau = (np.arange(n_fft) - n_fft // 4) * dt_fft
    sig = F(s_w - tau)
    S = np.fft.rfft(sig)
    om = 2 * np.pi * np.fft.rfftfreq(n_fft, dt_fft)
    Rc = np.ones_like(om, dtype=complex)
    if Y is not None:
        y = np.array([Y(1j * w) for w in om])
        Rc = (1 - y) / (1 + y)
    elif M > 0 or K > 0 or R > 0:
        with np.errstate(divide="ignore", invalid="ignore"):
            Z = msd_Z(om, R, M, K)
            Rc = (Z - 1) / (Z + 1)
        Rc[0] = 1.0                       # K / omega -> inf at omega = 0
    # FFT of sig over tau (tau grid starts at tau[0]): phase of the shift
    refl = np.fft.irfft(S * Rc, n_fft)
    tq = np.asarray(t) - (s_w - s_m)
    rq = np.interp(tq, tau, refl)
    return F(s_m - np.asarray(t)) + rq


# --------------------------------------------------------------------------
# Cylinder references (App. B, App. C)
# --------------------------------------------------------------------------


def _polar(x, y, cx, cy):
    dx, dy = np.asarray(x, float) - cx, np.asarray(y, float) - cy
    return np.hypot(dx, dy), np.arctan2(dy, dx)


def monopole_cylinder(x, y, omega, a_src, w, xs, ys, rc, cx=0.0, cy=0.0, Z=None, nmodes=None):
    """App. C: complex pressure amplitude P (p = Im(P e^{i omega t})) of the
    Gaussian monopole s = a_src exp(-b |x - x_s|^2) sin(omega t) next to a
    cylinder of radius rc centred at (cx, cy), in the e^{+i omega t}
    convention.  Z: the wall impedance at omega (a complex number), None for
    a rigid wall, or the string "free" for no cylinder.  Returns (P, P_free).

    P_free = C H0^(2)(k |x - x_s|), C = (omega / 4) a_src (pi / b) e^{-k^2 / 4b};
    the scattered part, from Graf's re-expansion of H0^(2) about the axis
    and the wall condition P = Z u_n with u_n = -U_r (i omega U_r = -dP/dr),
    is C sum_n eps_n H_n^(2)(k r_s) S_n H_n^(2)(k r) cos(n (theta - theta_s)),
    S_n = -(J_n(ka) + i Z J_n'(ka)) / (H_n^(2)(ka) + i Z H_n^(2)'(ka)),
    truncated at N = ceil(k a) + 40."""
    k = float(omega)
    b = math.log(2.0) / (w * w)
    C = omega / 4.0 * a_src * math.pi / b * math.exp(-k * k / (4.0 * b))
    r, th = _polar(x, y, cx, cy)
    rs, ths = _polar(xs, ys, cx, cy)
    dist = np.hypot(np.asarray(x, float) - xs, np.asarray(y, float) - ys)
    free = C * special.hankel2(0, k * dist)
    if isinstance(Z, str) and Z == "free":
        return free, free
    N = int(math.ceil(k * rc)) + 40 if nmodes is None else int(nmodes)
    n = np.arange(N + 1)
    eps = np.where(n == 0, 1.0, 2.0)
    ka = k * rc
    if Z is None:
        S = -special.jvp(n, ka) / special.h2vp(n, ka)
    else:
        S = -(special.jv(n, ka) + 1j * Z * special.jvp(n, ka)) / (special.hankel2(n, ka) + 1j * Z * special.h2vp(n, ka))
    coef = eps * special.hankel2(n, k * float(rs)) * S
    keep = np.abs(coef) > 0                    # modes whose coefficient underflowed add nothing
    n, coef = n[keep], coef[keep]
    rr = np.atleast_1d(r)
    tt = np.atleast_1d(th)
    scat = np.array([np.sum(coef * special.hankel2(n, k * r1) * np.cos(n * (t1 - ths))) for r1, t1 in zip(rr, tt)])
    return free + C * scat.reshape(np.shape(r)), free


def scattering_coefficients(n, omega, rc, Z, convention):
    """S_n of the cylinder of radius rc at angular frequency omega (k = omega):
    convention "+": e^{+i omega t} (App. C), H^(2) outgoing,
        S_n = -(J_n(ka) + i Z J_n'(ka)) / (H_n^(2)(ka) + i Z H_n^(2)'(ka));
    convention "-": e^{-i omega t} (App. B), H^(1) outgoing,
        S_n = -(i omega J_n(ka) + k Z J_n'(ka)) / (i omega H_n^(1)(ka) + k Z H_n^(1)'(ka)).
    Z None: rigid wall, S_n = -J_n'(ka) / H_n'(ka)."""
    ka = omega * rc
    if convention == "+":
        H, Hp = special.hankel2(n, ka), special.h2vp(n, ka)
        if Z is None:
            return -special.jvp(n, ka) / Hp
        return -(special.jv(n, ka) + 1j * Z * special.jvp(n, ka)) / (H + 1j * Z * Hp)
    H, Hp = special.hankel1(n, ka), special.h1vp(n, ka)
    if Z is None:
        return -special.jvp(n, ka) / Hp
    k = omega
    return -(1j * omega * special.jv(n, ka) + k * Z * special.jvp(n, ka)) / (1j * omega * H + k * Z * Hp)


def cylinder_field(x, y, omega, xs, ys, rc, cx=0.0, cy=0.0, Z=None, convention="+", nmodes=None,
                   incident=True):
    """Unit-strength harmonic field of a point source at (xs, ys) next to the
    cylinder: H0(k |x - x_s|) plus sum_n eps_n H_n(k r_s) S_n H_n(k r)
    cos(n (theta - theta_s)) (Graf's re-expansion about the axis, r < r_s),
    with H = H^(2) for convention "+" and H^(1) for "-".  Modes run to
    N = ceil(k max(r, r_s)) + 40 unless nmodes is given; modes whose
    coefficient underflows to zero add nothing."""
    k = float(omega)
    hank = special.hankel2 if convention == "+" else special.hankel1
    r, th = _polar(x, y, cx, cy)
    rs, ths = _polar(xs, ys, cx, cy)
    rs = float(rs)
    rr = np.atleast_1d(r).astype(float)
    tt = np.atleast_1d(th).astype(float)
    N = int(math.ceil(k * max(rs, float(rr.max())))) + 40 if nmodes is None else int(nmodes)
    n = np.arange(N + 1)
    eps = np.where(n == 0, 1.0, 2.0)
    coef = eps * hank(n, k * rs) * scattering_coefficients(n, k, rc, Z, convention)
    ok = np.isfinite(coef) & (np.abs(coef) > 0)
    n, coef = n[ok], coef[ok]
    Hr = hank(n[None, :], k * rr[:, None])
    term = coef[None, :] * Hr * np.cos(n[None, :] * (tt[:, None] - ths))
    term[~np.isfinite(term)] = 0.0               # an overflowing H_n(k r) times an underflowed coefficient
    out = np.sum(term, axis=1)
    if incident:
        d = np.hypot(np.atleast_1d(np.asarray(x, float)) - xs, np.atleast_1d(np.asarray(y, float)) - ys)
        out = out + hank(0, k * d)
    return out.reshape(np.shape(r))


def monopole_cylinder(x, y, omega, a_src, w, xs, ys, rc, cx=0.0, cy=0.0, Z=None, nmodes=None):
    """App. C: complex pressure amplitude P (p = Im(P e^{i omega t})) of the
    Gaussian monopole s = a_src exp(-b |x - x_s|^2) sin(omega t) next to a
    cylinder of radius rc centred at (cx, cy), in the e^{+i omega t}
    convention.  Z: the wall impedance at omega (a complex number), None for
    a rigid wall, or the string "free" for no cylinder.  Returns (P, P_free):
    P_free = C H0^(2)(k |x - x_s|), C = (omega / 4) a_src (pi / b) e^{-k^2 / 4b},
    and P = C cylinder_field(...) (Graf's re-expansion and the wall condition
    P = Z u_n with u_n = -U_r, i omega U_r = -dP/dr)."""
    k = float(omega)
    b = math.log(2.0) / (w * w)
    C = omega / 4.0 * a_src * math.pi / b * math.exp(-k * k / (4.0 * b))
    dist = np.hypot(np.asarray(x, float) - xs, np.asarray(y, float) - ys)
    free = C * special.hankel2(0, k * dist)
    if isinstance(Z, str) and Z == "free":
        return free, free
    return C * cylinder_field(x, y, omega, xs, ys, rc, cx, cy, Z, "+", nmodes), free


def pulse_cylinder(x, y, t, a, w, xs, ys, rc, cx=0.0, cy=0.0, imp=None, omega_max=None, n_omega=16,
                   incident="closed"):
    """App. B: the Gaussian pulse p0 = a exp(-b |x - x_s|^2) (u0 = 0) released
    next to a cylinder of radius rc, as a quadrature over frequency of the
    cylinder's modal expansion.  Only here the e^{-i omega t} convention is
    used: the initial pulse is the source p0(x) delta(t) of the pressure
    equation, whose transform (omega / 4) P0(k) H0^(1)(k |x - x_s|),
    P0(k) = a (pi / b) e^{-k^2 / 4b}, is the outgoing free field; each
    cylindrical mode takes the scattering coefficient of
    scattering_coefficients(convention "-") with Z(omega) = R - i (M omega - K / omega)
    (imp = (R, M, K); None: rigid), and
    p(x, t) = (1 / pi) Re int_0^inf P(x, omega) e^{-i omega t} d omega.
    The incident part comes from the closed form (free_pulse) unless
    incident == "quadrature"; the integral runs over Gauss-Legendre panels
    of width 1 (n_omega points each) up to omega_max (default: where
    e^{-omega^2 / 4b} < 1e-16).  Returns p[len(t), len(x)]."""
    b = math.log(2.0) / (w * w)
    if omega_max is None:
        omega_max = math.sqrt(4.0 * b * math.log(1e16))
    xg, wg = np.polynomial.legendre.leggauss(n_omega)
    edges = np.arange(0.0, omega_max + 1.0, 1.0)
    om = np.concatenate([0.5 * (e1 - e0) * xg + 0.5 * (e1 + e0) for e0, e1 in zip(edges[:-1], edges[1:])])
    wq = np.concatenate([0.5 * (e1 - e0) * wg for e0, e1 in zip(edges[:-1], edges[1:])])
    x = np.atleast_1d(np.asarray(x, float))
    y = np.atleast_1d(np.asarray(y, float))
    t = np.atleast_1d(np.asarray(t, float))
    quad_inc = incident == "quadrature"
    field = np.zeros((len(om), len(x)), dtype=complex)
    for q, wv in enumerate(om):
        Z = None
        if imp == "free":
            if quad_inc:
                field[q] = special.hankel1(0, wv * np.hypot(x - xs, y - ys))
            continue
        if imp is not None:
            R, M, K = imp
            Z = R - 1j * (M * wv - K / wv)
        field[q] = cylinder_field(x, y, wv, xs, ys, rc, cx, cy, Z, "-", incident=quad_inc)
    amp = (om / 4.0) * a * (math.pi / b) * np.exp(-om * om / (4.0 * b)) * wq
    out = ((np.exp(-1j * np.outer(t, om)) * amp[None, :]) @ field / math.pi).real
    if not quad_inc:
        d = np.hypot(x - xs, y - ys)
        out = out + np.array([[free_pulse(dd, tt, a, w)[0] for dd in d] for tt in t])
    return out
