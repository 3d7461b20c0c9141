"""The allocation-free entry point (lee_step_members_noalloc) against the
batch entry point it varies (lee_batch_create + lee_batch_step_n): the same
kernels over the same members give the same fields, traces and auxiliary
states bit for bit, on two calls in a row, the second with fewer members
(the static scratch keeps the first call's contents).
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
    from paper_2609_24785_amd.lee import Batch, Instance, step_members_noalloc
    return Instance, Batch, step_members_noalloc


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cases():
    return [
        lc.small_cylinder(96, 30),
        lc.small_cylinder(160, 30).replace(wall=lc.Wall("circle", 0.21, -0.13, rc=0.9),
                                           impedance=lc.Impedance("msd", R=2.0, M=0.2, K=0.5)),
        lc.small_cylinder(128, 30, impedance=lc.Impedance("rigid")),
        lc.flat_wall_201(30),
        lc.small_cylinder(112, 30, impedance=lc.Impedance("poles", real=((-0.5, 0.3),),
                                                          pairs=((-0.3, 0.8, 0.2, 0.05),))),
    ]


def _state(m):
    return m.fields(), m.ade_states(), m.traces()


def _same(a, b):
    (fa, pa, ta), (fb, pb, tb) = a, b
    for x, y in zip(fa, fb):
        assert np.array_equal(x, y)
    assert np.array_equal(pa, pb)
    assert np.array_equal(ta, tb)


@pytest.mark.parametrize("tiling", [dict(kind="tile", cols=128, rows=8, fused=1),
                                    dict(kind="tile", cols=64, rows=16, fused=0)],
                         ids=["fused-128x8", "two-launch-64x16"])
def test_noalloc_equals_batch_on_two_calls(tiling):
    Instance, Batch, step_members_noalloc = _lee()
    for cases, steps in ((_cases(), 13), (_cases()[1:3], 7)):     # the second call: fewer members
        _say(f"[noalloc] {len(cases)} members, {steps} steps, {tiling}")
        ref = [Instance(c, "f32") for c in cases]
        b = Batch(ref, tiling=tiling)
        b.step_n(steps)
        b.synchronize()
        got = [Instance(c, "f32") for c in cases]
        step_members_noalloc(got, steps, tiling)
        got[0].synchronize()
        for r, g in zip(ref, got):
            assert g.step == r.step == steps
            _same(_state(g), _state(r))
        b.close()
        for m in ref + got:
            m.close()


def test_noalloc_refuses_lists_beyond_its_scratch():
    from paper_2609_24785_amd._lib import LeeError
    Instance, _, step_members_noalloc = _lee()
    big = Instance(lc.flat_wall_201(1).replace(nx=2048, ny=2048, x0=-1024.0, y0=-1024.0), "f32")
    with pytest.raises(LeeError) as e:                # 100 x 8192 tiles of 64 x 8 nodes > 16 MiB of lists
        step_members_noalloc([big] * 100, 1, dict(kind="tile", cols=64, rows=8, fused=0))
    assert e.value.status == -1
    with pytest.raises(LeeError) as e:                # more members than the scratch's table holds
        step_members_noalloc([big] * 1025, 1)
    assert e.value.status == -1
    assert big.step == 0                              # nothing ran
    big.close()
