"""Autotuner host logic: candidates, selection, cache keys (no GPU)."""
import ctypes
import json

import pytest

import lee_cases as lc
from paper_2609_24785_amd import tune


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_every_candidate_is_a_supported_tiling(prec):
    from paper_2609_24785_amd import _lib
    from paper_2609_24785_amd.lee import Instance, make_tiling
    inst = Instance(lc.small_cylinder(96), prec, bind=False)
    lib = _lib.load()
    cands = tune.candidates(prec)
    assert len(cands) >= 6
    assert {c["tiling"]["fused"] for c in cands} == {0, 1}
    for c in cands:
        t = make_tiling(**c["tiling"])
        assert lib.lee_set_tiling(inst._h, ctypes.byref(t)) == 0, c
        assert c["graph_steps"] > 0


def test_select_takes_the_fastest_and_skips_failures():
    cands = [{"tiling": {"cols": c}, "graph_steps": 16} for c in (1, 2, 3, 4)]
    times = {1: 5.0, 2: 3.0, 3: None, 4: float("nan")}

    def measure(c):
        t = times[c["tiling"]["cols"]]
        if t is None:
            raise RuntimeError("rejected")
        return t

    best, table = tune.select(measure, cands)
    assert best["tiling"]["cols"] == 2 and best["step_us"] == 3.0
    assert len(table) == 4
    assert table[2]["step_us"] is None and "rejected" in table[2]["error"]
    assert table[3]["step_us"] is None
    with pytest.raises(RuntimeError):
        tune.select(lambda c: float("inf"), cands)


def test_select_keeps_each_candidates_best_round():
    """Rounds are interleaved and each candidate keeps its best time, so one
    slow trial does not decide the order."""
    cands = [{"tiling": {"cols": c}, "graph_steps": 16} for c in (1, 2)]
    seq = {1: iter([4.0, 9.0, 9.0]), 2: iter([5.0, 3.5, 6.0])}
    calls = []

    def measure(c):
        calls.append(c["tiling"]["cols"])
        return next(seq[c["tiling"]["cols"]])

    best, table = tune.select(measure, cands, rounds=3)
    assert calls == [1, 2, 1, 2, 1, 2]
    assert best["tiling"]["cols"] == 2 and best["step_us"] == 3.5
    assert table[0]["trials"] == [4.0, 9.0, 9.0] and table[0]["step_us"] == 4.0


def test_size_class_groups_nearby_problems():
    a = tune.size_class(1_045_359, 855)
    assert a == tune.size_class(1_000_000, 830)
    assert a != tune.size_class(2_200_000, 855)
    assert a != tune.size_class(1_045_359, 855, members=2)
    assert tune.cache_key("gfx950:sramecc+:xnack-", "f32", a, "v").startswith("gfx950|f32|")


def test_cache_key_separates_kernel_variants():
    # the stencil width, the filter, the radiation band and the wall kind
    # select different kernel code: each gets its own cache entry
    base = lc.cylinder_pulse_1024(10)
    keys = {tune.variant_of(c) for c in (
        base, base.replace(H=3, filter_sigma=0.0), base.replace(filter_sigma=0.0),
        base.replace(radiation=True), base.replace(impedance=lc.Impedance("rigid")),
        base.replace(impedance=lc.Impedance("poles", real=((-1.0, 1.0),))))}
    assert len(keys) == 6
    assert tune.variant_of(base) == tune.variant_of(lc.cylinder_pulse_1024(20).replace(
        impedance=lc.Impedance("msd", R=1.0, M=0.05, K=3.0)))
    # the shipped table answers the benchmark workloads, and only their variant
    for c in (lc.cylinder_pulse_1024(10), lc.monopole_4096(10)):
        from paper_2609_24785_amd.lee import Instance
        s = Instance(c, "f32", bind=False).summary
        assert tune.lookup(c, "f32", s.fluid_nodes, s.G) is not None
        assert tune.lookup(c.replace(radiation=True, rad_center=(0.0, 0.0)), "f32", s.fluid_nodes, s.G) is None


def test_cache_round_trip(tmp_path):
    p = str(tmp_path / "tune.json")
    c = tune.TuneCache(p, shipped=False)
    assert c.get("k") is None
    choice = {"tiling": {"kind": "tile", "cols": 64, "rows": 16, "fused": 1}, "graph_steps": 16, "step_us": 57.9}
    c.put("k", choice)
    assert json.load(open(p))["k"] == choice
    assert tune.TuneCache(p, shipped=False).get("k") == choice
    assert tune.TuneCache(p).get("k") == choice          # the file's entries take precedence


def test_shipped_table_entries_are_candidates():
    import os
    if not os.path.exists(tune.SHIPPED_TABLE):
        pytest.skip("no shipped table")
    base = tune.TuneCache(None).base
    assert base
    for key, v in base.items():
        prec = key.split("|")[1]
        assert {"tiling": v["tiling"], "graph_steps": v["graph_steps"]} in tune.candidates(prec), key
