"""Diagnostics on the device. The stop signal: a density that is not
positive (or not a number) anywhere in the lattice stops the case, as a
non-finite force does, and the step reports HLBM_E_UNSTABLE with its
reason; the bad state is set from the host, so every kernel still runs to
its end. Per-launch timing of the grid sub-steps (level 3)."""
import numpy as np
import pytest

from paper_2006_13631_amd import hlbm as H
from paper_2006_13631_amd.workloads import preset

pytestmark = pytest.mark.gpu


def _poison(case, x, y):
    f = case.lattice()
    f[:, y, x] = -1.0  # the nodes that pull from it see a negative density
    case.set_lattice(f)


@pytest.mark.parametrize("storage", [H.FP64, H.FP32])
def test_negative_density_stops_a_lamina_case(storage):
    cfg = preset("tiny_ragged")
    cfg.pop("steps")
    cfg.pop("ckpt_every", None)
    case = H.Case(max_steps=8, storage=storage, **cfg)
    case.step(2)
    _poison(case, 4, 3)  # far from the grid
    with pytest.raises(H.HlbmError) as e:
        case.step(2)
    assert e.value.code == H.E_UNSTABLE and "density" in str(e.value)
    assert case.info().status == H.STATUS_UNSTABLE
    case.close()


def test_negative_density_stops_a_lattice_only_case():
    case = H.Case(nx=40, ny=30, tau=0.8, bc=H.BC_PERIODIC, max_steps=4)
    case.step(1)
    _poison(case, 20, 15)
    with pytest.raises(H.HlbmError) as e:
        case.step(1)
    assert e.value.code == H.E_UNSTABLE and "density" in str(e.value)
    case.close()


def test_healthy_case_is_not_flagged():
    cfg = preset("tiny_ragged")
    n = cfg.pop("steps")
    cfg.pop("ckpt_every", None)
    case = H.Case(max_steps=n, **cfg)
    case.step(n)
    inf = case.info()
    assert inf.status == H.STATUS_DONE
    assert np.all(case.lattice().sum(0) > 0)
    case.close()


@pytest.mark.parametrize("variant,per_step", [(1, 3), (8, 10), (10, 5)])
def test_timing_level3_times_every_substep_launch(variant, per_step):
    """Timing level 3 records each grid sub-step launch of one step of every
    pair (10 sub-steps: three launches of up to four, ten of one, five of
    two) by its own events; the results are those of an untimed run."""
    c = preset("lamina_128x64")
    c.pop("ckpt_every")
    c.pop("steps")
    a = H.Case(max_steps=12, **c)
    b = H.Case(max_steps=12, **c)
    for g in (a, b):
        g.tune(variant=variant)
    b.timing(3)
    a.step(12)
    b.step(12)
    ms, n = b.timing_get(H.K_SUBSTEP_LAUNCH)
    pairs = 6 if b.info().two_step else 12
    assert n == pairs * per_step and ms > 0
    assert np.array_equal(a.grid(), b.grid()) and np.array_equal(a.history(), b.history())
