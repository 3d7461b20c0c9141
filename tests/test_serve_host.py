"""The serving scheduler on a simulated device (no GPU): admission by memory
budget in arrival order, continuous batching, every request served its
steps, latency accounting, the reflection-coefficient estimate."""
import math

import numpy as np
import pytest

import lee_cases as lc
from paper_2609_24785_amd.serve import Request, Server, SimBackend, reflection


class VClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def advance(self, dt):
        self.t += dt

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


def _req(rid, side, steps, arrival):
    case = lc.small_cylinder(side, steps).replace(name=f"r{rid}")
    return Request(rid, case, arrival)


def _serve(reqs, budget=1e12, chunk=10, max_members=64, cost=1e-9):
    clk = VClock()
    be = SimBackend(clk, cost)
    srv = Server(be, budget_bytes=budget, chunk=chunk, max_members=max_members, clock=clk, sleep=clk.sleep)
    return srv.run(reqs), srv, be


def test_every_request_gets_its_steps_and_a_latency():
    reqs = [_req(k, 96 + 16 * (k % 4), 20 + 7 * k, 0.001 * k) for k in range(10)]
    res, srv, be = _serve(reqs)
    assert [r.rid for r in res] == list(range(10))
    for r, q in zip(res, reqs):
        assert r.error is None
        assert int(r.traces[0]) == q.case.steps
        assert r.finished >= r.admitted >= r.arrival
    st = srv.stats
    assert st["served"] == 10 and st["p99_latency_s"] >= st["p50_latency_s"] > 0
    assert st["node_stages"] == 4 * sum(q.case.nx * q.case.ny * q.case.steps for q in reqs)


def test_late_arrivals_join_the_running_batch():
    # a long request starts alone; a short one arrives while it runs and
    # shares launches with it before the long one finishes
    reqs = [_req(0, 160, 200, 0.0), _req(1, 96, 30, 1e-5)]
    res, srv, be = _serve(reqs, chunk=10)
    mixed = [l for l in be.launches if len(l) == 2]
    assert mixed, be.launches[:5]
    first_mixed = be.launches.index(mixed[0])
    assert first_mixed > 0                          # the long one ran alone first
    assert res[1].finished < res[0].finished        # the short one left before it


def test_admission_waits_for_memory_in_arrival_order():
    reqs = [_req(k, 128, 40, 0.0) for k in range(6)]
    one = 36 * 128 * 135
    res, srv, be = _serve(reqs, budget=2.5 * one)
    assert srv.stats["peak_bytes"] <= 2.5 * one
    assert srv.stats["peak_members"] == 2
    adm = [r.admitted for r in res]
    assert adm == sorted(adm)                       # first come, first admitted
    assert all(r.error is None for r in res)


def test_request_larger_than_the_budget_is_rejected():
    reqs = [_req(0, 224, 20, 0.0), _req(1, 96, 20, 0.0)]
    res, srv, be = _serve(reqs, budget=36 * 100 * 110)
    assert res[0].error and "budget" in res[0].error
    assert res[1].error is None


def test_slot_limit():
    reqs = [_req(k, 96, 30, 0.0) for k in range(5)]
    res, srv, be = _serve(reqs, max_members=3)
    assert max(len(l) for l in be.launches) == 3
    assert srv.stats["served"] == 5


def test_reflection_of_a_resistive_relation_is_exact():
    t = np.arange(400) * 0.01
    u = np.exp(-2.0 * t) * np.sin(9.0 * t)
    z0 = 3.0
    # columns: p_BP, the ADE's u_n and the fluid's u_n; the estimate reads
    # the pressure and the fluid's velocity only
    w = np.stack([z0 * u, 0.5 * u, u], axis=1)
    imp = lc.Impedance("msd", R=z0, M=0.1, K=8.1)      # resonance at sqrt(K/M) = 9
    out = reflection(w, 0.01, imp, [4.5, 9.0, 18.0])
    for est, q in zip(out["R_est"], out["un_fluid_over_ade"]):
        assert est[0] == pytest.approx((z0 - 1) / (z0 + 1), abs=1e-12)
        assert est[1] == pytest.approx(0.0, abs=1e-12)
        assert q[0] == pytest.approx(2.0, abs=1e-12) and q[1] == pytest.approx(0.0, abs=1e-12)
    # the exact value at resonance is (R - 1)/(R + 1)
    assert out["R_exact"][1][0] == pytest.approx((z0 - 1) / (z0 + 1), abs=1e-12)
    assert out["R_exact"][1][1] == pytest.approx(0.0, abs=1e-12)


def test_rejected_set_up_is_reported_not_raised():
    """A request the library refuses at set-up (here: an impedance whose ADE
    poles RK4 cannot integrate) comes back with its error; the others run."""
    clk = VClock()

    class Failing(SimBackend):
        def prepare_async(self, case):
            from concurrent.futures import Future
            f = Future()
            if case.name == "bad":
                f.set_exception(RuntimeError("LEE_E_ADE_STIFF"))
            else:
                f.set_result(self.prepare(case))
            return f

    be = Failing(clk)
    srv = Server(be, chunk=10, clock=clk, sleep=clk.sleep)
    reqs = [Request(0, lc.small_cylinder(96, 20).replace(name="bad"), 0.0), _req(1, 96, 20, 0.0)]
    res = srv.run(reqs)
    assert "LEE_E_ADE_STIFF" in res[0].error
    assert res[1].error is None and int(res[1].traces[0]) == 20


def test_progress_reports_follow_the_work():
    # the report callback sees the state after chunks, at most once per
    # report_every seconds of the server's clock, and its counts add up
    reqs = [_req(k, 96, 50, 0.001 * k) for k in range(6)]
    clk = VClock()
    be = SimBackend(clk, 1e-6)
    seen = []
    srv = Server(be, chunk=10, clock=clk, sleep=clk.sleep, report=seen.append, report_every=0.01)
    res = srv.run(reqs)
    assert seen and len(res) == 6
    ts = [r["t_s"] for r in seen]
    assert all(b - a >= 0.01 for a, b in zip(ts, ts[1:]))
    for r in seen:
        assert r["finished"] + r["active"] + r["waiting"] <= r["arrived"] <= 6


def test_reflection_estimate_on_the_flat_wall_matches_the_impedance():
    """The served reflection estimate from the oracle's watched ghost (p_BP and
    the normal velocity read out of the fluid at its boundary point) on the
    201^2 flat wall at 30 deg, 500 steps: a locally-reacting wall relates p
    and u_n by Z at every frequency (single-resonance mass-spring-damper
    wall, Z = R + i (M w - K / w)), so (Z_est - 1)/(Z_est + 1) must reproduce
    (Z - 1)/(Z + 1) wherever the pulse carries energy.  Measured: 0.007 at
    w0/2 and 0.003 at the resonance w0 (40 and 20 points per wavelength),
    0.15 at 2 w0 (10 points per wavelength, where the 11-point scheme with
    its filter no longer resolves the wave)."""
    from oracle.solver import OracleSolver
    from paper_2609_24785_amd.serve import _omegas
    c = lc.flat_wall_201(500)
    o = OracleSolver(c)
    o.set_watch(c.ic.xs, c.ic.ys)
    o.run(c.steps)
    r = reflection(o.watch_trace, c.dt, c.impedance, _omegas(c))
    dev = [math.hypot(a[0] - b[0], a[1] - b[1]) for a, b in zip(r["R_est"], r["R_exact"])]
    assert dev[0] < 0.02 and dev[1] < 0.01, dev
    assert dev[2] < 0.25, dev
    assert abs(complex(*r["R_exact"][1])) < 1e-12      # R = 1: no reflection at resonance
