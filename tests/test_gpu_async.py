"""hlbm_step_async enqueues the steps of hlbm_step without waiting for
them: after hlbm_sync, or any call that reads the state, the state and the
force history are those hlbm_step gives, bit for bit; a flag raised on the
device surfaces at hlbm_sync and at the next hlbm_step_async."""
import sys

import numpy as np
import pytest

from paper_2006_13631_amd import hlbm as H
from paper_2006_13631_amd.workloads import preset

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _cfg(name):
    c = preset(name)
    c.pop("steps")
    c.pop("ckpt_every", None)
    return c


@pytest.mark.parametrize("name", ["tiny_ragged", "lamina_256x128"])
def test_async_steps_match_blocking_steps(name):
    _say("async vs blocking", name)
    c = _cfg(name)
    a = H.Case(max_steps=60, **c)
    b = H.Case(max_steps=60, **c)
    for k in (1, 2, 9, 17, 31):  # odd and even counts, below and above the graph length
        a.step(k)
        b.step_async(k)
    b.sync()
    assert np.array_equal(a.lattice(), b.lattice())
    assert np.array_equal(a.grid(), b.grid())
    assert np.array_equal(a.history(), b.history())
    assert b.info().step == 60


def test_reads_wait_for_enqueued_steps():
    _say("reads after async steps")
    c = _cfg("tiny_ragged")
    a = H.Case(max_steps=40, **c)
    b = H.Case(max_steps=40, **c)
    a.step(24)
    b.step_async(16)
    b.step_async(8)
    # no hlbm_sync: the state and history reads wait for the steps
    assert np.array_equal(a.lattice(), b.lattice())
    assert np.array_equal(a.history(), b.history())


def _poison(case, x, y):
    f = case.lattice()
    f[:, y, x] = -1.0  # the nodes that pull from it see a negative density
    case.set_lattice(f)


def test_flag_surfaces_at_sync_and_next_call():
    _say("async density flag")
    c = _cfg("tiny_ragged")
    case = H.Case(max_steps=12, **c)
    case.step(2)
    _poison(case, 4, 3)  # far from the grid
    try:
        case.step_async(2)  # may or may not have seen the flag yet
    except H.HlbmError as e:
        assert e.code == H.E_UNSTABLE
    with pytest.raises(H.HlbmError) as e:
        case.sync()
    assert e.value.code == H.E_UNSTABLE and "density" in str(e.value)
    # the flag copied after those steps is complete: the next call reports it
    with pytest.raises(H.HlbmError) as e:
        case.step_async(1)
    assert e.value.code == H.E_UNSTABLE
    case.close()


def test_async_arguments_checked():
    c = _cfg("tiny_ragged")
    case = H.Case(max_steps=4, **c)
    for bad in (-1, 5):
        with pytest.raises(H.HlbmError) as e:
            case.step_async(bad)
        assert e.value.code == H.E_ARG
    case.sync()  # nothing enqueued: nothing to report
    case.close()
