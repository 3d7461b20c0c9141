"""The numbers the oracle and the case descriptions take from the paper,
checked against the printed values in tests/golden/paper_values.txt."""
import math

import numpy as np

import lee_cases as lc
from oracle import schemes
from tests.golden import PAPER, paper


def test_fixture_has_citations():
    for key, (val, cite) in PAPER.items():
        assert cite.startswith("Sec.") and math.isfinite(val), key


def test_drp7_is_the_printed_set():
    # Sec. 2.2, eq. DRP_s: the oracle's 7-point coefficients are the printed digits
    printed = np.array([paper("drp7_a1"), paper("drp7_a2"), paper("drp7_a3")])
    assert np.array_equal(schemes.DRP7, printed)


def test_resonances_follow_from_the_printed_walls():
    # omega_res = sqrt(K/M): 40 (Sec. 4.1), 8 (Sec. 4.2), 8 pi (Sec. 4.3)
    assert abs(math.sqrt(paper("flat_K") / paper("flat_M")) - 40.0) < 1e-12
    assert abs(math.sqrt(paper("pulse_K") / paper("pulse_M")) - paper("pulse_omega_res")) < 1e-12
    assert abs(math.sqrt(paper("monopole_K") / paper("monopole_M")) - 8 * math.pi) < 1e-3 * 8 * math.pi


def test_paper_cylinder_pulse_case_is_the_printed_one():
    c = lc.paper_cylinder_pulse()
    assert (c.impedance.kind, c.impedance.R, c.impedance.M, c.impedance.K) == \
        ("msd", paper("pulse_R"), paper("pulse_M"), paper("pulse_K"))
    assert (c.ic.a, c.ic.w) == (paper("pulse_a"), paper("pulse_w"))
    assert c.H == 3 and c.filter_sigma == 0.0          # the paper's scheme has no filter (Sec. 4.3)


def test_paper_monopole_case_is_the_printed_one():
    c = lc.paper_monopole()
    assert (c.impedance.kind, c.impedance.R, c.impedance.M, c.impedance.K) == \
        ("msd", paper("monopole_R"), paper("monopole_M"), paper("monopole_K"))
    assert c.h == paper("monopole_h")
    assert abs(c.dt - paper("monopole_dt")) < 1e-15
    assert (c.source.a, c.source.w) == (paper("monopole_a"), paper("monopole_w"))
    assert abs(c.source.omega - 8 * math.pi) < 1e-15   # omega = omega_res (Sec. 4.3)
