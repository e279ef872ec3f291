"""The case-batched path (hlbm_create with ncases > 1) against single cases.

Every case of a batch must compute exactly the bits it computes alone (the
single-case path is parity-tested against the oracle), whatever schedule the
autotuner picks; cases stop at their own max_steps; a case whose force turns
non-finite stops and is reported while the others carry on.
"""
import os
import sys

import numpy as np
import pytest

from paper_2006_13631_amd import hlbm
from paper_2006_13631_amd.workloads import preset

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _cases():
    a = preset("tiny_ragged")
    a["max_steps"] = a.pop("steps")                      # 60 steps, odd grid width
    b = preset("tiny_fine_grid")
    b["max_steps"] = b.pop("steps")                      # 40 steps, h_u = 0.2, n = 32
    c = preset("lamina_128x64")
    c.pop("ckpt_every")
    c.pop("steps")
    c["max_steps"] = 90                                  # n = 10
    d = preset("tiny_adjoint", bc=hlbm.BC_PERIODIC)
    d.pop("steps")
    d["max_steps"] = 75
    from paper_2006_13631_amd.workloads import paper_study_cases
    e = {k: v for k, v in paper_study_cases(b=16)[-1].items() if k not in ("eps", "beta_p")}
    e["max_steps"] = 80                                  # the paper's boundaries, 80^2
    return [a, b, c, d, e]


def _solo(cfg, storage):
    g = hlbm.Case(storage=storage, **cfg)
    g.step(cfg["max_steps"])
    return g


def _same(batch_member, solo):
    assert np.array_equal(batch_member.history(), solo.history())
    assert np.array_equal(batch_member.lattice(), solo.lattice())
    assert np.array_equal(batch_member.grid(), solo.grid())


@pytest.mark.parametrize("storage", [hlbm.FP64, hlbm.FP32, hlbm.FP16_DEV])
def test_batch_matches_single_cases_bitwise(storage):
    _say("batch vs single, storage", storage)
    cfgs = _cases()
    batch = hlbm.Batch(cfgs, storage=storage)
    batch.step(max(c["max_steps"] for c in cfgs))
    for i, c in enumerate(cfgs):
        inf = batch[i].info()
        assert inf.step == c["max_steps"] and inf.status == hlbm.STATUS_DONE
        _same(batch[i], _solo(c, storage))


def test_batch_fp64_members_match_the_oracle(oracle):
    """Every member of an FP64 batch (uneven lattices, grids, sub-step
    counts and boundaries, autotuned schedule) against the oracle run of its
    configuration, element by element: lattice, grid and force history
    within 1e-12 of the oracle's largest value."""
    _say("batch members vs oracle")
    cfgs = _cases()
    batch = hlbm.Batch(cfgs, storage=hlbm.FP64)
    batch.tune(trial_steps=4)
    batch.step(max(c["max_steps"] for c in cfgs))
    oracle.set_threads(min(16, len(os.sched_getaffinity(0))))
    try:
        for i, c in enumerate(cfgs):
            o = oracle.Sim(**c)
            o.step(c["max_steps"])
            m = batch[i]
            for name, got, want in (("lattice", m.lattice(), o.lattice()), ("grid", m.grid(), o.grid()),
                                    ("force", m.history(), o.history())):
                assert got.shape == want.shape, (i, name)
                err = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
                _say("case", i, name, err)
                assert err <= 1e-12, (i, name, err)
    finally:
        oracle.set_threads(1)


@pytest.mark.parametrize("schedule", [
    dict(steps_per_graph=4, lattice_threads=128, lattice_rows=1, substep_variant=0, order=1),
    dict(steps_per_graph=16, lattice_threads=256, lattice_rows=2, substep_variant=1, order=0),
    dict(steps_per_graph=1, lattice_threads=64, lattice_rows=4, substep_variant=2, order=1),
    dict(steps_per_graph=8, lattice_threads=192, lattice_rows=2, substep_variant=3, order=0),
    dict(steps_per_graph=4, lattice_threads=128, lattice_rows=2, substep_variant=6, order=1, tail_variant=3),
    # one cooperative launch per run, every phase of a step behind a grid barrier
    dict(steps_per_graph=4, lattice_threads=128, lattice_rows=2, substep_variant=5, order=0, persistent=1),
    dict(steps_per_graph=8, lattice_threads=128, lattice_rows=1, substep_variant=4, order=1, persistent=1,
         persistent_groups=37),
    dict(steps_per_graph=8, lattice_threads=128, lattice_rows=1, substep_variant=7, order=0, persistent=1,
         persistent_groups=1),
    dict(steps_per_graph=4, lattice_threads=256, lattice_rows=4, substep_variant=1, order=1, tail_variant=6,
         persistent=2),
    dict(steps_per_graph=4, lattice_threads=256, lattice_rows=4, substep_variant=2, order=1, persistent=1),
])
def test_schedules_do_not_change_results(schedule):
    _say("schedule", schedule)
    cfgs = _cases()
    batch = hlbm.Batch(cfgs, storage=hlbm.FP32)
    got = batch.tune(schedule=schedule)
    assert got["steps_per_graph"] == schedule["steps_per_graph"]
    # several calls, stopping in the middle of graphs
    for n in (7, 33, 100):
        batch.step(n)
    for i, c in enumerate(cfgs):
        _same(batch[i], _solo(c, hlbm.FP32))


@pytest.mark.parametrize("storage", [hlbm.FP64, hlbm.FP32])
def test_substep_variants_compute_identical_bits(storage):
    """The grid sub-step kernels (tile shape, workgroup size, sub-steps per
    launch) and the stream-collide launch shapes differ only in which
    workgroup and lane compute a node."""
    c = preset("lamina_128x64")
    c.pop("ckpt_every")
    n = c.pop("steps") // 4
    c["max_steps"] = n
    want = hlbm.Case(storage=storage, **c)
    want.step(n)
    shapes = [(128, 1), (256, 2), (64, 4), (192, 1)] * 3
    for v in range(11):
        _say("sub-step variant", v, "stream-collide shape", shapes[v], "storage", storage)
        g = hlbm.Case(storage=storage, **c)
        t = g.tune(variant=v, lattice=shapes[v], order=v % 2)
        assert t["substep_variant"] == v and (t["lattice_threads"], t["lattice_rows"]) == shapes[v]
        assert t["order"] == v % 2
        g.step(n)
        _same(g, want)


def test_single_case_tune_leaves_state_alone():
    _say("single-case tune")
    c = preset("tiny_ragged")
    n = c.pop("steps")
    c["max_steps"] = n
    a = hlbm.Case(storage=hlbm.FP64, **c)
    b = hlbm.Case(storage=hlbm.FP64, **c)
    a.step(n // 2)
    b.step(n // 2)
    lat, grid = a.lattice().copy(), a.grid().copy()
    t = a.tune(trial_steps=2)
    _say("chosen", t)
    assert 0 <= t["substep_variant"] < 11 and t["ms_per_step"] > 0
    assert t["lattice_threads"] in (128, 256) and t["lattice_rows"] in (1, 2, 4)
    assert np.array_equal(a.lattice(), lat) and np.array_equal(a.grid(), grid)
    a.step(n - n // 2)
    b.step(n - n // 2)
    _same(a, b)
    for bad in (dict(variant=11), dict(lattice=(96, 1)), dict(lattice=(128, 3)), dict(order=4)):
        with pytest.raises(hlbm.HlbmError) as e:
            a.tune(**bad)
        assert e.value.code == hlbm.E_ARG


def test_autotune_then_run():
    _say("autotune")
    cfgs = _cases()
    batch = hlbm.Batch(cfgs, storage=hlbm.FP32)
    t = batch.tune(trial_steps=8)
    _say("chosen", t)
    assert t["steps_per_graph"] in (4, 8, 16) and t["ms_per_step"] > 0 and t["lattice_rows"] in (1, 2, 4)
    for m in batch.cases:
        assert m.info().step == 0
    batch.step(200)
    for i, c in enumerate(cfgs):
        _same(batch[i], _solo(c, hlbm.FP32))
    with pytest.raises(hlbm.HlbmError) as e:
        batch.tune(trial_steps=4)
    assert e.value.code == hlbm.E_STATE


def test_unstable_case_stops_alone():
    _say("unstable member")
    cfgs = _cases()
    batch = hlbm.Batch(cfgs, storage=hlbm.FP64)
    g = batch[1].grid()
    g[:] = np.nan                         # the first force of case 1 is not finite
    batch[1].set_grid(g)
    batch.step(100)
    inf = batch[1].info()
    assert inf.status == hlbm.STATUS_UNSTABLE and inf.step < cfgs[1]["max_steps"]
    for i in (0, 2, 3, 4):
        assert batch[i].info().status == hlbm.STATUS_DONE
        _same(batch[i], _solo(cfgs[i], hlbm.FP64))


@pytest.mark.parametrize("storage", [hlbm.FP64, hlbm.FP16_DEV])
def test_persistent_launch_matches_single_cases_bitwise(storage):
    _say("persistent batch vs single, storage", storage)
    cfgs = _cases()
    batch = hlbm.Batch(cfgs, storage=storage)
    got = batch.tune(schedule=dict(steps_per_graph=8, lattice_threads=128, lattice_rows=2, substep_variant=6,
                                   order=0, persistent=1))
    assert got["persistent"] == 1
    batch.step(max(c["max_steps"] for c in cfgs))
    for i, c in enumerate(cfgs):
        assert batch[i].info().status == hlbm.STATUS_DONE
        _same(batch[i], _solo(c, storage))


def test_persistent_unstable_case_stops_alone():
    _say("unstable member, persistent launch")
    cfgs = _cases()
    batch = hlbm.Batch(cfgs, storage=hlbm.FP64)
    batch.tune(schedule=dict(steps_per_graph=8, lattice_threads=128, lattice_rows=2, substep_variant=5, order=0,
                             persistent=1))
    g = batch[1].grid()
    g[:] = np.nan
    batch[1].set_grid(g)
    batch.step(100)
    assert batch[1].info().status == hlbm.STATUS_UNSTABLE
    for i in (0, 2, 3, 4):
        assert batch[i].info().status == hlbm.STATUS_DONE
        _same(batch[i], _solo(cfgs[i], hlbm.FP64))


def test_invalid_persistent_schedule_is_rejected():
    batch = hlbm.Batch(_cases()[:2])
    for bad in (dict(persistent=3), dict(persistent=-1), dict(persistent=1, persistent_groups=-2)):
        with pytest.raises(hlbm.HlbmError) as e:
            batch.tune(schedule=bad)
        assert e.value.code == hlbm.E_ARG


def test_batch_has_no_adjoint():
    b = hlbm.Batch(_cases()[:2])
    rc = hlbm.load().hlbm_adjoint(b.h, 0, hlbm._ptr(np.zeros(2)), 1, hlbm._ptr(np.zeros(3)))
    assert rc == hlbm.E_UNSUPPORTED
