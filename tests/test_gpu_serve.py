"""Serving on the device: a request's result is the same alone and in a mix
of requests that arrive while it runs (bit-for-bit: the batch runs the same
per-node arithmetic for every member), and a served result matches the
FP64 oracle within the FP32 bound."""
import numpy as np
import pytest

import lee_cases as lc

pytestmark = pytest.mark.gpu


def _serve():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_24785_amd.serve import GpuBackend, Request, Server
    return GpuBackend, Request, Server


def _run(reqs, chunk=16):
    GpuBackend, Request, Server = _serve()
    be = GpuBackend("f32")
    try:
        srv = Server(be, budget_bytes=8e9, chunk=chunk)
        res = srv.run(reqs)
    finally:
        be.close()
    return res, srv.stats


def test_result_same_alone_and_in_the_mix():
    _, Request, _ = _serve()
    target = lc.small_cylinder(160, 56)
    print("[serve] alone", flush=True)
    alone, _ = _run([Request(0, target, 0.0)])
    mix_cases = [lc.small_cylinder(96, 40), lc.small_cylinder(224, 70).replace(ny=97, y0=-3.5, name="wide"),
                 lc.flat_wall_201(45), lc.small_cylinder(128, 33, impedance=lc.Impedance("rigid"))]
    reqs = [Request(1, mix_cases[0], 0.0), Request(0, target, 0.01), Request(2, mix_cases[1], 0.02),
            Request(3, mix_cases[2], 0.03), Request(4, mix_cases[3], 0.05)]
    print("[serve] mix of 5", flush=True)
    mix, st = _run(reqs, chunk=8)
    assert all(r.error is None for r in mix), [r.error for r in mix]
    got = next(r for r in mix if r.rid == 0)
    ref = alone[0]
    assert got.traces.shape == ref.traces.shape == (56, len(target.probes), 3)
    assert np.array_equal(got.traces, ref.traces)
    assert np.array_equal(got.watch, ref.watch)
    assert st["peak_members"] >= 2


def test_served_result_matches_oracle():
    _, Request, _ = _serve()
    from oracle.solver import OracleSolver
    case = lc.small_cylinder(128, 40)
    print("[serve] vs oracle", flush=True)
    res, _ = _run([Request(0, case, 0.0), Request(1, lc.small_cylinder(96, 25), 0.0)])
    r = res[0]
    ora = OracleSolver(case)
    ora.set_watch(case.ic.xs, case.ic.ys)
    tr = ora.run(case.steps)
    scale = np.abs(tr).max()
    assert np.abs(r.traces - tr).max() <= 1e-4 * scale
    w = ora.watch_trace
    for k in range(3):
        assert np.abs(r.watch[:, k] - w[:, k]).max() <= 1e-4 * np.abs(w[:, k]).max()
    assert r.reflection and len(r.reflection["R_est"]) == 3
    assert len(r.reflection["un_fluid_over_ade"]) == 3
