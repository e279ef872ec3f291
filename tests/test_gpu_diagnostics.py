"""The device-side stop signal: a density that is not positive (or not a
number) anywhere in the lattice stops the case, as a non-finite force does,
and the step reports HLBM_E_UNSTABLE with its reason. The bad state is set
from the host, so every kernel still runs to its end."""
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
