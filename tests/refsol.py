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
