"""Pins of the cylinder reference solutions (App. B, App. C) themselves.

The references are the modal series of the paper's appendices written out in
tests/refsol.py; before they judge the oracle, they are checked against what
fixes them independently:

* App. C's free field C H0^(2)(k r) is the late-time limit of the monopole
  switched on from rest (a time-domain quadrature of the wave equation), which
  fixes C and the e^{+i omega t} convention;
* App. B's quadrature of the outgoing free field (omega / 4) P0 H0^(1)
  reproduces the closed-form free pulse, which fixes the e^{-i omega t}
  transform pair and the source normalisation;
* Graf's re-expansion sums to H0(k |x - x_s|) inside r_s;
* the total field meets the wall condition at r = a, checked by a
  finite difference of the series in r (rigid: dP/dr = 0; impedance:
  P = Z u_n with u_n from the momentum equation), in both conventions;
* the two appendices' S_n, written for opposite time conventions, are
  complex conjugates of each other for the same physical wall;
* the App. B quadrature is converged in omega_max and the panel order.
"""
import math

import numpy as np
import pytest

from tests import refsol

W = 0.2
A = 1.0


def test_app_c_free_field_is_the_late_time_monopole():
    om = 2.0 * math.pi
    for r in (1.5, 3.0):
        P, free = refsol.monopole_cylinder(r, 0.0, om, A, W, 0.0, 0.0, 0.5, Z="free")
        T = 80.0
        late = refsol.monopole_from_rest(r, T, A, W, om)[0]
        assert abs((P * np.exp(1j * om * T)).imag - late) < 1e-4 * abs(P)


def test_app_b_free_quadrature_is_the_closed_form_pulse():
    t = np.array([2.0, 3.0, 5.0])
    x = np.array([2.0, 1.0, -0.5])
    y = np.array([0.0, 0.0, 1.0])
    q = refsol.pulse_cylinder(x, y, t, A, W, 4.0, 0.0, 0.5, imp="free", incident="quadrature")
    for i, tt in enumerate(t):
        d = np.hypot(x - 4.0, y)
        ref = np.array([refsol.free_pulse(dd, tt, A, W)[0] for dd in d])
        assert np.abs(q[i] - ref).max() < 1e-8


@pytest.mark.parametrize("conv", ["+", "-"])
def test_graf_expansion(conv):
    """sum_n eps_n H_n(k r_s) J_n(k r) cos(n (theta - theta_s)) = H0(k |x - x_s|)
    for r < r_s (the terms fall like (r / r_s)^n once n > k r_s; the
    references sum it only against S_n, which falls much faster)."""
    from scipy import special
    k, rs, ths = 7.3, 2.5, 0.4
    hank = special.hankel2 if conv == "+" else special.hankel1
    for r, th in ((0.6, 1.0), (1.5, -2.2), (1.9, 0.35)):
        n = np.arange(int(math.ceil(k * rs)) + 80)
        eps = np.where(n == 0, 1.0, 2.0)
        s = np.sum(eps * hank(n, k * rs) * special.jv(n, k * r) * np.cos(n * (th - ths)))
        d = math.hypot(r * math.cos(th) - rs * math.cos(ths), r * math.sin(th) - rs * math.sin(ths))
        assert abs(s - hank(0, k * d)) < 1e-10 * abs(hank(0, k * d))


@pytest.mark.parametrize("conv", ["+", "-"])
@pytest.mark.parametrize("Zkind", ["rigid", "msd"])
def test_wall_condition_holds(conv, Zkind):
    om, rc, xs = 9.0, 0.5, 2.0
    R, M, K = 0.7, 0.025, 1.6
    if Zkind == "rigid":
        Z = None
    elif conv == "+":
        Z = R + 1j * (M * om - K / om)
    else:
        Z = R - 1j * (M * om - K / om)
    dr = 1e-5
    for th in (0.0, 0.8, 2.0, math.pi):
        c, s_ = math.cos(th), math.sin(th)
        P = lambda r: complex(refsol.cylinder_field(r * c, r * s_, om, xs, 0.0, rc, Z=Z, convention=conv))
        Pa = P(rc)
        dP = (P(rc + dr) - P(rc - dr)) / (2 * dr)
        if Z is None:
            assert abs(dP) < 1e-6 * abs(Pa) * om
            continue
        # momentum: +: i om U_r = -dP/dr; -: -i om U_r = -dP/dr; u_n = -U_r
        Ur = (-dP / (1j * om)) if conv == "+" else (dP / (1j * om))
        assert abs(Pa - Z * (-Ur)) < 1e-6 * abs(Pa)


def test_appendix_coefficients_are_conjugate():
    n = np.arange(30)
    for om in (3.0, 8.0, 25.0):
        R, M, K = 0.2, 0.025, 1.6
        Zp = R + 1j * (M * om - K / om)
        Sp = refsol.scattering_coefficients(n, om, 0.5, Zp, "+")
        Sm = refsol.scattering_coefficients(n, om, 0.5, np.conj(Zp), "-")
        ok = np.abs(Sp) > 1e-250
        assert np.allclose(Sp[ok], np.conj(Sm[ok]), rtol=1e-10, atol=0)
        assert np.allclose(refsol.scattering_coefficients(n, om, 0.5, None, "+")[ok],
                           np.conj(refsol.scattering_coefficients(n, om, 0.5, None, "-"))[ok], rtol=1e-10, atol=0)


def test_app_b_quadrature_converged():
    ts = np.linspace(4.0, 6.0, 9)
    imp = (0.2, 0.025, 1.6)
    a = refsol.pulse_cylinder([2.0], [0.0], ts, A, W, 4.0, 0.0, 0.5, imp=imp)
    b = refsol.pulse_cylinder([2.0], [0.0], ts, A, W, 4.0, 0.0, 0.5, imp=imp, n_omega=32, omega_max=70.0)
    assert np.abs(a - b).max() < 1e-10 * np.abs(a).max()
    # the impedance wall changes the reflected pulse
    r = refsol.pulse_cylinder([2.0], [0.0], ts, A, W, 4.0, 0.0, 0.5)
    assert np.abs(r - a).max() > 0.1 * np.abs(r).max()
