"""Pins of the oracle's outer radiation condition (Sec. 2.2: one-sided
stencils at the domain edges; Sec. 4.1-4.2: a non-reflecting condition on
the outer boundary).

The one-sided weights are checked by exactness on polynomials; the
condition itself against a run on a domain four times as wide, whose edges
the waves have not reached (a zero frame reflects almost everything); the
band's stability with the spectral analysis of the step map.
"""
import numpy as np
import pytest

import lee_cases as lc
from oracle import schemes
from oracle import spectral as sp
from oracle.solver import OracleSolver


@pytest.mark.parametrize("m", [0, 1, 2])
def test_one_sided_weights_exact_to_degree_six(m):
    w = schemes.RAD_ONE_SIDED[m]
    x = np.arange(7.0)
    for d in range(7):
        want = d * float(m) ** (d - 1) if d > 0 else 0.0
        assert abs(np.dot(w, x ** d) - want) < 1e-9 * max(1.0, abs(want))
    # and not to degree seven: the set is the maximal-order one, no more
    assert abs(np.dot(w, x ** 7) - 7 * float(m) ** 6) > 1e-3


def test_central_part_is_the_printed_7_point_set():
    # the band's central stencil (three nodes each side) is eq. DRP_s
    w = schemes.DRP7
    assert abs(2 * np.dot(np.arange(1, 4), w) - 1.0) < 1e-11


def _pulse(n, L, rad, H=5, fs=0.2):
    h = 2.0 * L / n
    return lc.Case(nx=n, ny=n, x0=-L, y0=-L, h=h, H=H, cfl=0.5, filter_sigma=fs,
                   ic=lc.Pulse(1.0, 0.5, 1e-3, 0.6), radiation=rad, rad_center=(0.0, 0.0),
                   name="free-pulse")


@pytest.mark.parametrize("H,fs", [(5, 0.2), (3, 0.0)])
def test_outgoing_pulse_leaves_without_reflection(H, fs):
    # domain [-8, 8)^2 at h = 1/6; by t = 10 the pulse front has crossed
    # most of the edges; reference: [-32, 32)^2, the same nodes in its centre
    steps = 120
    ref = OracleSolver(_pulse(384, 32.0, False, H, fs))
    ref.run(steps)
    pr = ref.fields()[0][144:240, 144:240]
    errs = {}
    for rad in (False, True):
        s = OracleSolver(_pulse(96, 8.0, rad, H, fs))
        s.run(steps)
        p = s.fields()[0]
        errs[rad] = np.linalg.norm(p - pr) / np.linalg.norm(pr)
    assert errs[False] > 0.3            # the zero frame reflects
    assert errs[True] < 0.03            # the radiation condition lets it out
    assert errs[True] < 0.1 * errs[False]


@pytest.mark.parametrize("H,fs", [(5, 0.2), (3, 0.0), (5, 0.0)])
def test_radiation_band_does_not_grow(H, fs):
    h = 0.125
    n = 2 * (H + 6) + 3
    c = lc.Case(nx=n, ny=n + 1, x0=-0.5 * (n - 1) * h, y0=-0.5 * n * h, h=h, H=H, cfl=0.5,
                filter_sigma=fs, radiation=True, rad_center=(0.01, -0.02), name="band")
    assert sp.spectral_radius(sp.step_matrix(c)) <= 1.0 + 1e-12


def test_rejections():
    c = lc.radiating_cylinder(96)
    with pytest.raises(ValueError):
        OracleSolver(c.replace(wall=lc.Wall("circle", 6.5, 0.0, rc=1.3)))   # wall near the band
    with pytest.raises(ValueError):
        OracleSolver(c.replace(rad_center=(-7.9, 0.0), wall=lc.Wall()))     # centre in the band
    OracleSolver(c)
