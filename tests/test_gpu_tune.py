"""The autotuner on the device: it picks a listed configuration, the tuned
instance or batch computes the same fields as the default configuration,
and a cached choice is applied without trials."""
import numpy as np
import pytest

import lee_cases as lc
from oracle.solver import relative_l2

pytestmark = pytest.mark.gpu


def _lee():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_24785_amd import tune
    from paper_2609_24785_amd.lee import Batch, Instance
    return Instance, Batch, tune


def _fields(inst, steps):
    inst.step_n(steps)
    inst.synchronize()
    return inst.fields()


@pytest.mark.parametrize("prec,tol", [("f32", 1e-6), ("f64", 1e-13)])
def test_tuned_instance_matches_default(prec, tol, tmp_path):
    Instance, _, tune = _lee()
    case = lc.small_cylinder(224, 30)
    print(f"[tune] {case.name} {prec}", flush=True)
    cache = tune.TuneCache(str(tmp_path / "t.json"), shipped=False)
    inst = Instance(case, prec)
    choice = tune.tune_instance(inst, cache, steps=16, warmup=4)
    assert not choice["cached"]
    assert {k: choice[k] for k in ("tiling", "graph_steps")} in [
        {k: c[k] for k in ("tiling", "graph_steps")} for c in tune.candidates(prec)]
    assert inst.step == 0                                   # reset after the trials
    got = _fields(inst, 30)
    ref = _fields(Instance(case, prec), 30)
    mask = np.asarray(ref[0] != 0)
    for x, y in zip(got, ref):
        assert relative_l2(x, y, mask) <= tol
    again = tune.tune_instance(Instance(case, prec), cache)
    assert again["cached"] and again["tiling"] == choice["tiling"]


def test_tuned_batch_matches_solo():
    Instance, Batch, tune = _lee()
    cases = [lc.small_cylinder(96, 12), lc.small_cylinder(160, 12), lc.flat_wall_201(12)]
    print("[tune] batch of 3", flush=True)
    mem = [Instance(c, "f32") for c in cases]
    b = Batch(mem)
    choice = tune.tune_batch(b, steps=8, warmup=2)
    assert choice["table"]
    b.step_n(12)
    b.synchronize()
    for m, c in zip(mem, cases):
        ref = _fields(Instance(c, "f32"), 12)
        got = m.fields()
        mask = np.asarray(ref[0] != 0)
        for x, y in zip(got, ref):
            assert relative_l2(x, y, mask) <= 1e-6
