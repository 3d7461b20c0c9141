"""GPU batches: members advanced by one launch per phase over all of them.

Every member of a batch runs the same per-node arithmetic as when it runs
alone, so its fields must be bit-identical to a solo run of the same number
of steps; per-member budgets let finished members idle.
"""
import sys

import numpy as np
import pytest

import lee_cases as lc

pytestmark = pytest.mark.gpu


def _lee():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_24785_amd.lee import Batch, Instance
    return Instance, Batch


def _members():
    return [
        lc.small_cylinder(96, 20),
        lc.small_cylinder(160, 20).replace(wall=lc.Wall("circle", 0.21, -0.13, rc=0.9),
                                           impedance=lc.Impedance("msd", R=2.0, M=0.2, K=0.5)),
        lc.small_cylinder(128, 20, impedance=lc.Impedance("rigid")),
        lc.flat_wall_201(20),
        lc.small_cylinder(224, 20).replace(ny=97, y0=-3.5, probes=((2.5, 0.0),)),
        lc.small_cylinder(112, 20, impedance=lc.Impedance("poles", real=((-0.5, 0.3),),
                                                          pairs=((-0.3, 0.8, 0.2, 0.05),))),
    ]


@pytest.mark.parametrize("prec,fused", [("f32", 1), ("f64", 1), ("f32", 0)])
def test_batch_equals_solo_bitwise(prec, fused):
    """Solo members run the two-launch stage; the batch runs fused or not."""
    Instance, Batch = _lee()
    cases = _members()
    print(f"[batch] {len(cases)} members {prec} fused={fused}", flush=True)
    rows = 16 if prec == "f32" else 8
    solo = []
    for c in cases:
        i = Instance(c, prec)
        i.set_tiling("tile", cols=64, rows=rows, fused=0)
        i.step_n(12)
        i.synchronize()
        solo.append(i.fields())
    mem = [Instance(c, prec) for c in cases]
    b = Batch(mem, tiling=dict(kind="tile", cols=64, rows=rows, fused=fused))
    b.step_n(12)
    b.synchronize()
    for m, ref in zip(mem, solo):
        m.synchronize()
        got = m.fields()
        for x, y in zip(got, ref):
            assert np.array_equal(x, y)


def test_batch_budgets_idle_finished_members():
    Instance, Batch = _lee()
    cases = _members()[:3]
    budgets = [5, 12, 0]
    solo = []
    for c, n in zip(cases, budgets):
        i = Instance(c, "f32")
        if n:
            i.step_n(n)
        i.synchronize()
        solo.append(i.fields())
    mem = [Instance(c, "f32") for c in cases]
    b = Batch(mem, tiling=dict(kind="tile", cols=64, rows=16))
    b.set_budget(budgets)
    b.step_n(12)
    for m, ref in zip(mem, solo):
        m.synchronize()
        for x, y in zip(m.fields(), ref):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("prec,fused", [("f32", 0), ("f32", 1), ("f64", 1)])
def test_membership_changes_keep_graphs(prec, fused):
    """A member leaves and joins again between runs: the batch keeps its
    captured graphs (its padded lists still fit their capacities), and every
    member matches a solo run of the same number of steps bit for bit."""
    Instance, Batch = _lee()
    cases = _members()[:4]
    rows = 16 if prec == "f32" else 8
    steps = [24, 16, 24, 24]                 # member 1 sits out the middle run
    print(f"[batch] membership {prec} fused={fused}", flush=True)
    solo = []
    for c, n in zip(cases, steps):
        i = Instance(c, prec)
        i.set_tiling("tile", cols=64, rows=rows, fused=0)
        i.step_n(n)
        i.synchronize()
        solo.append(i.fields())
    mem = [Instance(c, prec) for c in cases]
    b = Batch(mem, tiling=dict(kind="tile", cols=64, rows=rows, fused=fused), graph_steps=4)
    b.step_n(8)
    b.synchronize()
    captured = b.graph_captures()
    assert captured >= 1
    b.remove(mem[1])
    assert len(b) == 3
    b.step_n(8)
    b.add(mem[1])
    assert len(b) == 4
    b.step_n(8)
    b.synchronize()
    assert b.graph_captures() == captured
    for m, ref in zip(mem, solo):
        m.synchronize()
        for x, y in zip(m.fields(), ref):
            assert np.array_equal(x, y)


def test_batch_capacity_growth_and_trim_recapture():
    """A member that outgrows the padded lists, and removals that leave them
    mostly idle, each drop the captured graphs once (the next run captures
    again); every member still matches its solo run bit for bit."""
    Instance, Batch = _lee()
    small = [lc.small_cylinder(96, 20), lc.small_cylinder(128, 20, impedance=lc.Impedance("rigid"))]
    big = lc.small_cylinder(224, 20).replace(ny=97, y0=-3.5, probes=((2.5, 0.0),))
    print("[batch] capacity growth and trim", flush=True)
    steps = {0: 24, 1: 16, 2: 8}                     # member 1 leaves after 16 steps, the big one joins for 8
    cases = small + [big]
    solo = []
    for k, c in enumerate(cases):
        i = Instance(c, "f32")
        i.set_tiling("tile", cols=64, rows=16, fused=0)
        i.step_n(steps[k])
        i.synchronize()
        solo.append(i.fields())
    mem = [Instance(c, "f32") for c in cases]
    b = Batch(mem[:2], tiling=dict(kind="tile", cols=64, rows=16, fused=0), graph_steps=4)
    b.step_n(8)
    b.synchronize()
    c0 = b.graph_captures()
    b.step_n(8)                                      # same lists: no new capture
    b.synchronize()
    assert b.graph_captures() == c0
    b.remove(mem[1])
    b.add(mem[2])                                    # outgrows the ghost and sweep capacities
    b.step_n(8)
    b.synchronize()
    assert b.graph_captures() == c0 + 1
    for m, ref, n in zip(mem, solo, (24, 16, 8)):
        m.synchronize()
        assert m.step == n
        for x, y in zip(m.fields(), ref):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("prec,fused", [("f32", 1), ("f64", 0)])
def test_update_applies_removals_and_additions_in_one_rebuild(prec, fused):
    """lee_batch_update: two members leave and one joins in one call, then the
    two come back in a second call; every member matches a solo run of the
    same number of steps bit for bit and the same changes made one call at
    a time, and arguments the library refuses (a non-member to remove, a
    member to add) change nothing."""
    from paper_2609_24785_amd._lib import LeeError
    Instance, Batch = _lee()
    cases = _members()[:5]
    rows = 16 if prec == "f32" else 8
    steps = [24, 16, 24, 16, 16]             # 1 and 3 sit out the middle run, 4 joins for it
    print(f"[batch] update {prec} fused={fused}", flush=True)
    solo = []
    for c, n in zip(cases, steps):
        i = Instance(c, prec)
        i.set_tiling("tile", cols=64, rows=rows, fused=0)
        i.step_n(n)
        i.synchronize()
        solo.append(i.fields())
    mem = [Instance(c, prec) for c in cases]
    b = Batch(mem[:4], tiling=dict(kind="tile", cols=64, rows=rows, fused=fused), graph_steps=4)
    b.step_n(8)
    b.synchronize()
    captured = b.graph_captures()
    b.update(add=[mem[4]], remove=[mem[1], mem[3]])
    assert [id(m) for m in b.members] == [id(mem[0]), id(mem[2]), id(mem[4])] and len(b) == 3
    b.step_n(8)
    with pytest.raises(LeeError):
        b.update(remove=[mem[1]])            # not a member
    with pytest.raises(LeeError):
        b.update(add=[mem[0]])               # already a member
    assert len(b) == 3
    b.update(add=[mem[1], mem[3]])
    b.step_n(8)
    b.synchronize()
    assert len(b) == 5
    for m, ref in zip(mem, solo):
        m.synchronize()
        for x, y in zip(m.fields(), ref):
            assert np.array_equal(x, y)
    # the same changes one call at a time give the same fields
    mem2 = [Instance(c, prec) for c in cases]
    b2 = Batch(mem2[:4], tiling=dict(kind="tile", cols=64, rows=rows, fused=fused), graph_steps=4)
    b2.step_n(8)
    b2.remove(mem2[1])
    b2.remove(mem2[3])
    b2.add(mem2[4])
    b2.step_n(8)
    b2.add(mem2[1])
    b2.add(mem2[3])
    b2.step_n(8)
    b2.synchronize()
    assert b.graph_captures() >= captured and b2.graph_captures() >= captured
    for m, m2 in zip(mem, mem2):
        for x, y in zip(m.fields(), m2.fields()):
            assert np.array_equal(x, y)
    b.close()
    b2.close()
