"""The two-step lattice path (pairs of steps: one launch advances the
lattice away from the grid by two steps, the band near it one step at a
time) gives the same bits as single steps, for every boundary type and
storage, with and without a grid, in graphs and eager launches and across
an odd number of steps; the interface donors computed inside the lattice
launch give the bits of their own launch."""
import os
import sys

import numpy as np
import pytest

from paper_2006_13631_amd import hlbm
from paper_2006_13631_amd.workloads import preset, random_populations

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _make(one_step, **cfg):
    if one_step:
        os.environ["HLBM_ONE_STEP"] = "1"
    try:
        return hlbm.Case(**cfg)
    finally:
        os.environ.pop("HLBM_ONE_STEP", None)


@pytest.mark.parametrize("storage", [hlbm.FP64, hlbm.FP32, hlbm.FP16_DEV])
@pytest.mark.parametrize("bc", [hlbm.BC_PERIODIC_X_WALLS_Y, hlbm.BC_PERIODIC, hlbm.BC_PAPER])
@pytest.mark.parametrize("grid", [True, False])
def test_two_step_matches_single_steps(oracle, storage, bc, grid):
    c = preset("tiny_ragged")
    n = c.pop("steps")
    c.update(bc=bc, storage=storage, max_steps=n)
    if not grid:
        c.update(nux=0, nuy=0, b=0.0)
    _say("two-step vs single", storage, bc, grid)
    a = _make(False, **c)
    b = _make(True, **c)
    assert a.info().two_step == 1 and b.info().two_step == 0
    _, _, w = oracle.d2q9()
    f = random_populations((9, c["ny"], c["nx"]), 7, w, 0.02)
    a.set_lattice(f)
    b.set_lattice(f)
    for k in (1, 2, 9, 3, 17):  # odd and even counts, below and above the graph length
        a.step(k)
        b.step(k)
        assert np.array_equal(a.lattice(), b.lattice()), k
        if grid:
            assert np.array_equal(a.grid(), b.grid()), k
            assert np.array_equal(a.history(), b.history()), k


def test_two_step_off_where_it_cannot_apply():
    c = preset("tiny_ragged")
    c.pop("steps")
    small = hlbm.Case(**dict(c, nx=40, ny=45, nux=0, nuy=0, b=0.0, max_steps=0))
    assert small.info().two_step == 0  # lattice narrower than the tile and its ring


@pytest.mark.parametrize("one_step", [False, True])
@pytest.mark.parametrize("storage", [hlbm.FP64, hlbm.FP32])
def test_donors_in_the_lattice_launch_match_their_own_launch(oracle, one_step, storage):
    """On one stream the lattice launch also computes the grid's interface
    donors; with the grid path on a stream of its own they run as a launch
    of their own. Both give the same bits."""
    c = preset("tiny_ragged")
    n = c.pop("steps")
    c.update(storage=storage, max_steps=n)
    _say("fused donors vs their own launch", storage, "one step" if one_step else "two-step")
    a = _make(one_step, **c)
    os.environ["HLBM_TWO_STREAMS"] = "1"
    try:
        b = _make(one_step, **c)
    finally:
        os.environ.pop("HLBM_TWO_STREAMS", None)
    _, _, w = oracle.d2q9()
    f = random_populations((9, c["ny"], c["nx"]), 9, w, 0.02)
    a.set_lattice(f)
    b.set_lattice(f)
    for k in (1, 2, 9, 17):
        a.step(k)
        b.step(k)
        assert np.array_equal(a.lattice(), b.lattice()), k
        assert np.array_equal(a.grid(), b.grid()), k
        assert np.array_equal(a.history(), b.history()), k
