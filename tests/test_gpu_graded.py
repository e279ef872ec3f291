"""Graded body-fitted grids on the GPU against the FP64 oracle: lattice,
grid and force history element by element (1e-12 relative) for a lamina on
a grid refined toward it, under two boundary types and on both lattice
paths; uniform coordinates given as a graded grid reproduce the uniform
case; the entry point refuses what it does not support."""
import os
import sys

import numpy as np
import pytest

from paper_2006_13631_amd import hlbm
from paper_2006_13631_amd.workloads import graded_nodes

pytestmark = pytest.mark.gpu
TOL = 1e-12
GX = graded_nodes(31, 0.5, 1.25, 1.5, fine=5.0)
GY = graded_nodes(16, 0.5, 1.3, 1.5)
CASE = dict(nx=64, ny=48, nux=31, nuy=16, b=8.0, thickness=0.5, tau=0.8, kc=1.0, beta=20.0)


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _check(o, g, tol=TOL):
    errs = {"lattice": _rel(g.lattice(), o.lattice()), "grid": _rel(g.grid(), o.grid()),
            "force": _rel(g.history(), o.history())}
    _say("graded parity", errs)
    for k, e in errs.items():
        assert e <= tol, (k, e)


@pytest.mark.parametrize("bc,one_step", [(hlbm.BC_PERIODIC_X_WALLS_Y, False), (hlbm.BC_PERIODIC_X_WALLS_Y, True),
                                         (hlbm.BC_PAPER, False)])
def test_graded_grid_parity(oracle, bc, one_step):
    steps = 120
    _say("graded grid", bc, one_step)
    o = oracle.Sim(bc=bc, max_steps=steps, x_nodes=GX, y_nodes=GY, **CASE)
    if one_step:
        os.environ["HLBM_ONE_STEP"] = "1"
    try:
        g = hlbm.Case(bc=bc, max_steps=steps, x_nodes=GX, y_nodes=GY, **CASE)
    finally:
        os.environ.pop("HLBM_ONE_STEP", None)
    for n in (3, 8, 109):
        o.step(n)
        g.step(n)
        _check(o, g)
    inf_o, inf_g = o.info(), g.info()
    assert (inf_g.n_type1, inf_g.n_type2) == (inf_o.n_type1, inf_o.n_type2)


def test_uniform_coordinates_reproduce_the_uniform_case():
    cfg = dict(nx=64, ny=48, nux=24, nuy=16, b=8.0, thickness=1.0, tau=0.8, kc=1.0, beta=20.0, max_steps=80)
    X = np.array([(i - 24 // 2) * 1.0 for i in range(24)])
    Y = np.array([(j - 0.5 * 15) * 1.0 for j in range(16)])
    u = hlbm.Case(**cfg)
    g = hlbm.Case(x_nodes=X, y_nodes=Y, **cfg)
    u.step(80)
    g.step(80)
    for a, b in ((g.lattice(), u.lattice()), (g.grid(), u.grid()), (g.history(), u.history())):
        assert _rel(a, b) <= TOL


def test_graded_refusals():
    with pytest.raises(hlbm.HlbmError) as e:  # rows not symmetric about the lamina
        hlbm.Case(max_steps=4, x_nodes=GX, y_nodes=GY + 0.1, **CASE)
    assert e.value.code == hlbm.E_ARG
    with pytest.raises(hlbm.HlbmError) as e:  # thickness is the slot rows' spacing
        hlbm.Case(max_steps=4, x_nodes=GX, y_nodes=GY, **dict(CASE, thickness=1.0))
    assert e.value.code == hlbm.E_ARG


def test_fp32_graded_tracks_fp64(oracle):
    steps = 120
    o = oracle.Sim(max_steps=steps, x_nodes=GX, y_nodes=GY, **CASE)
    g = hlbm.Case(max_steps=steps, storage=hlbm.FP32, x_nodes=GX, y_nodes=GY, **CASE)
    o.step(steps)
    g.step(steps)
    e = _rel(g.history(), o.history())
    _say("fp32 graded force error", e)
    assert e < 1e-3


def test_coupled_motion_on_a_graded_grid(oracle):
    steps = 150
    mot = dict(mass=40.0, stiffness=0.05, damping=0.0, y0=1.5, v0=0.0, y_max=5.0)
    cfg = dict(CASE, kc=0.0)
    o = oracle.Sim(max_steps=steps, x_nodes=GX, y_nodes=GY, **cfg)
    g = hlbm.Case(max_steps=steps, x_nodes=GX, y_nodes=GY, **cfg)
    o.set_motion(**mot)
    g.set_motion(**mot)
    o.step(steps)
    g.step(steps)
    _check(o, g)
    assert _rel(g.motion_history(), o.motion_history()) <= TOL
