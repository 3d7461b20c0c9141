"""GPU parity of the spectral analysis: the step map assembled through the C
ABI (one library step from every unit state) against the oracle's, entry by
entry, and the power-iteration growth estimate against the oracle's on the
same start state.

Tolerances: FP64 entries within 1e-11 of the largest entry (the two sides
differ in summation order only); FP32 within 1e-4 of the largest entry and
1e-5 in relative Frobenius norm (the FP32 bound of the fields, per entry of
one step).
"""
import sys

import numpy as np
import pytest

import lee_cases as lc
from oracle import spectral as osp

pytestmark = pytest.mark.gpu

MSD = lc.Impedance("msd", R=1.0, M=0.05 * 64.0, K=20.0 / 64.0)


def _mods():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_24785_amd import stability
    from paper_2609_24785_amd.lee import Instance
    return Instance, stability


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cyl(z, n=20, H=5, fs=0.2):
    c0 = -0.5 * (n - 1)
    return lc.Case(nx=n, ny=n + 3, x0=c0, y0=c0 - 1.0, h=1.0, H=H, cfl=0.5, filter_sigma=fs,
                   wall=lc.Wall("circle", 0.25, 0.125, rc=4.0), impedance=z,
                   name=f"cyl-{n}-H{H}")


CASES = [("rigid", lc.Impedance(), 5, 0.2), ("msd", MSD, 5, 0.2), ("paper-scheme", MSD, 3, 0.0)]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name,z,H,fs", CASES, ids=[c[0] for c in CASES])
def test_step_matrix_matches_oracle(prec, name, z, H, fs):
    Instance, stability = _mods()
    case = _cyl(z, H=H, fs=fs)
    _say(f"[stability] step matrix {case.name} {name} prec={prec}")
    inst = Instance(case, prec)
    G = stability.step_matrix(inst)
    inst.close()
    ref = osp.step_matrix(case)
    assert G.shape == ref.shape
    scale = np.abs(ref).max()
    err = np.abs(G - ref).max()
    fro = np.linalg.norm(G - ref) / np.linalg.norm(ref)
    _say(f"[stability] n={G.shape[0]} max|dG|={err:.3e} (scale {scale:.3f}) rel fro {fro:.3e}")
    if prec == "f64":
        assert err <= 1e-11 * scale
        rg, ro = stability.spectral_radius(G), osp.spectral_radius(ref)
        _say(f"[stability] spectral radius gpu {rg:.12f} oracle {ro:.12f}")
        assert abs(rg - ro) <= 1e-9
    else:
        assert err <= 1e-4 * scale and fro <= 1e-5


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_step_matrix_with_radiation_band_matches_oracle(prec):
    # the band's one-sided stencils and outgoing-wave equation are part of
    # the step map too (28 x 31 nodes: the band and the 6 nodes it reads
    # around a cylinder of radius 1.5)
    Instance, stability = _mods()
    n = 28
    case = lc.Case(nx=n, ny=n + 3, x0=-0.5 * (n - 1), y0=-0.5 * (n - 1) - 1.0, h=1.0, H=5, cfl=0.5,
                   filter_sigma=0.2, wall=lc.Wall("circle", 0.25, 0.125, rc=1.5), impedance=MSD,
                   radiation=True, rad_center=(0.1, -0.2), name="cyl-24-radiation")
    _say(f"[stability] step matrix {case.name} prec={prec}")
    inst = Instance(case, prec)
    G = stability.step_matrix(inst)
    inst.close()
    ref = osp.step_matrix(case)
    scale = np.abs(ref).max()
    err = np.abs(G - ref).max()
    _say(f"[stability] n={G.shape[0]} max|dG|={err:.3e} (scale {scale:.3f})")
    if prec == "f64":
        assert err <= 1e-11 * scale
        assert abs(stability.spectral_radius(G) - osp.spectral_radius(ref)) <= 1e-9
    else:
        assert err <= 1e-4 * scale


@pytest.mark.parametrize("name,z,H,fs", CASES[:2], ids=[c[0] for c in CASES[:2]])
def test_power_growth_matches_oracle(name, z, H, fs):
    Instance, stability = _mods()
    case = _cyl(z, H=H, fs=fs)
    _say(f"[stability] power growth {case.name} {name}")
    inst = Instance(case, "f64")
    n = stability.StatePacker(inst).n
    x0 = np.random.default_rng(11).standard_normal(n)
    est, logs = stability.power_growth(inst, x0, 400, chunk=50)
    inst.close()
    G = osp.step_matrix(case)
    ref = osp.growth_estimate(G, x0, 400)
    _say(f"[stability] growth per step gpu {est:.12f} oracle {ref:.12f}")
    assert abs(est - ref) <= 1e-10 * ref


def test_state_round_trip_at_full_size():
    # the packed state of the benchmark grid goes in and comes back unchanged
    Instance, stability = _mods()
    case = lc.cylinder_pulse_1024(10).replace(ic=None, probes=())
    _say(f"[stability] state round trip {case.name} f64")
    inst = Instance(case, "f64")
    sp = stability.StatePacker(inst)
    assert sp.nf == inst.summary.fluid_nodes
    assert sp.naux == inst.summary.ade_states * inst.summary.G
    x = np.random.default_rng(5).standard_normal(sp.n)
    sp.put(x)
    back = sp.get()
    inst.close()
    assert np.array_equal(back, x)


OPER_CASES = CASES + [("fused-two-launch", MSD, 5, 0.2)]


@pytest.mark.parametrize("name,z,H,fs", OPER_CASES, ids=[c[0] for c in OPER_CASES])
def test_semi_discrete_operator_matches_oracle(name, z, H, fs):
    """The semi-discrete operator L through the C ABI (lee_rhs: one
    right-hand-side evaluation of the library's stage kernels per unit state)
    against the oracle's (oc_rhs), entry by entry in FP64, with the same
    growth rate per unit time; the step map of the same instance afterwards
    is still the oracle's (lee_rhs leaves the state and the step sequence as
    they were, and a fused launch takes none of its exchange words)."""
    Instance, stability = _mods()
    case = _cyl(z, H=H, fs=fs)
    _say(f"[stability] semi-discrete operator {case.name} {name} f64")
    inst = Instance(case, "f64")
    if name == "fused-two-launch":
        inst.set_tiling(kind="tile", cols=64, rows=8, fused=0)
    else:
        inst.set_tiling(kind="tile", cols=64, rows=8, fused=1)
    L = stability.operator_matrix(inst)
    ref = osp.operator_matrix(case)
    assert L.shape == ref.shape
    scale = np.abs(ref).max()
    err = np.abs(L - ref).max()
    a_g, a_o = stability.spectral_abscissa(L), osp.spectral_abscissa(ref)
    _say(f"[stability] n={L.shape[0]} max|dL|={err:.3e} (scale {scale:.3f}); abscissa gpu {a_g:.6e} oracle {a_o:.6e}")
    assert err <= 1e-11 * scale
    assert abs(a_g - a_o) <= 1e-9 * scale
    # the instance steps on as if lee_rhs had not been called
    G = stability.step_matrix(inst)
    inst.close()
    Gr = osp.step_matrix(case)
    assert np.abs(G - Gr).max() <= 1e-11 * np.abs(Gr).max()
