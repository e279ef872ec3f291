"""Parity of the structured refinement levels (HIP library through the C
ABI) with the FP64 CPU oracle: every level's populations, the finest
level's grid and its force history, element by element, after the same
seeded start. FP64 bar: max|gpu - oracle| / max|oracle| <= 1e-12 per array.
"""
import os
import sys

import numpy as np
import pytest

from paper_2006_13631_amd import hlbm
from paper_2006_13631_amd.workloads import random_populations

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _pair(oracle, nx0, ny0, boxes, bc0, storage=hlbm.FP64, seed=None, **fine):
    o = oracle.MultiLevel(nx0, ny0, boxes, bc0=bc0, **fine)
    g = hlbm.MultiLevel(nx0, ny0, boxes, bc0=bc0, storage=storage, **fine)
    assert g.shapes == o.shapes
    assert np.allclose(g.taus, o.taus, rtol=0, atol=0)
    if seed is not None:
        _, _, w = oracle.d2q9()
        for l, (nx, ny) in enumerate(o.shapes):
            f = random_populations((9, ny, nx), seed + l, w, 0.02)
            o.set_level(l, f)
            g.set_level(l, f)
    return o, g


def _check(o, g, tol=TOL):
    errs = {f"level{l}": _rel(g.level(l), o.level(l)) for l in range(o.nlevels)}
    if o.finest.nnode:
        errs["grid"] = _rel(g.grid(), o.finest.grid())
        ho, hg = o.history(), g.history()
        assert ho.shape == hg.shape
        errs["force"] = _rel(hg, ho)
    _say("multilevel parity", errs)
    for k, e in errs.items():
        assert e <= tol, (k, e)


@pytest.mark.parametrize("bc0,boxes", [
    (hlbm.BC_PERIODIC_X_WALLS_Y, [(5, 4, 19, 15)]),
    (hlbm.BC_PERIODIC, [(4, 5, 20, 16), (3, 4, 26, 19)]),
    (hlbm.BC_PAPER, [(6, 3, 17, 18), (2, 5, 19, 28)]),
])
def test_lattice_levels(oracle, bc0, boxes):
    _say("lattice levels", bc0, boxes)
    o, g = _pair(oracle, 26, 22, boxes, bc0, seed=11, tau=0.85)
    for n in (1, 2, 4):  # odd and even numbers of level-0 steps
        o.step(n)
        g.step(n)
        _check(o, g)


def test_graph_replay_matches_eager_launches(oracle):
    boxes = [(4, 5, 20, 16), (3, 4, 26, 19)]
    _, g = _pair(oracle, 26, 22, boxes, hlbm.BC_PERIODIC, seed=5, tau=0.8)
    os.environ["HLBM_NO_GRAPHS"] = "1"
    try:
        _, e = _pair(oracle, 26, 22, boxes, hlbm.BC_PERIODIC, seed=5, tau=0.8)
    finally:
        del os.environ["HLBM_NO_GRAPHS"]
    g.step(3)
    e.step(3)
    for l in range(3):
        assert np.array_equal(g.level(l), e.level(l)), l


LAMINA = dict(nux=48, nuy=12, b=12, tau=0.8, kc=1.0, beta=20)


@pytest.mark.parametrize("bc0,nx0,ny0,boxes", [
    (hlbm.BC_PERIODIC_X_WALLS_Y, 48, 40, [(10, 12, 38, 28)]),
    (hlbm.BC_PAPER, 48, 40, [(10, 12, 38, 28)]),
    (hlbm.BC_PERIODIC_X_WALLS_Y, 40, 32, [(6, 8, 34, 24), (4, 6, 52, 26)]),
])
def test_lamina_on_the_finest_level(oracle, bc0, nx0, ny0, boxes):
    _say("lamina on finest level", bc0, boxes)
    per = 2 ** len(boxes)  # finest steps per level-0 step
    total = 48 // per      # level-0 steps: 48 finest steps
    o, g = _pair(oracle, nx0, ny0, boxes, bc0, max_steps=total * per, **LAMINA)
    o.step(3)
    g.step(3)
    _check(o, g)
    o.step(total - 3)
    g.step(total - 3)
    _check(o, g)


def test_tuned_shape_keeps_the_bits(oracle):
    boxes = [(10, 12, 38, 28)]
    o, g = _pair(oracle, 48, 40, boxes, hlbm.BC_PERIODIC_X_WALLS_Y, max_steps=40, **LAMINA)
    t = g.tune(2)
    _say("schedule", t)
    o.step(4)
    g.step(4)
    _check(o, g)


def test_fp32_levels_track_the_oracle(oracle):
    boxes = [(10, 12, 38, 28)]
    o, g = _pair(oracle, 48, 40, boxes, hlbm.BC_PERIODIC_X_WALLS_Y, storage=hlbm.FP32, max_steps=40,
                 **LAMINA)
    o.step(20)
    g.step(20)
    _, _, w = oracle.d2q9()
    for l in range(2):
        dev_o = o.level(l) - w[:, None, None]
        dev_g = g.level(l) - w[:, None, None]
        e = np.max(np.abs(dev_g - dev_o)) / np.max(np.abs(dev_o))
        _say("fp32 level", l, e)
        assert e < 1e-3


def test_fp16_deviation_levels_track_the_oracle(oracle):
    boxes = [(10, 12, 38, 28)]
    o, g = _pair(oracle, 48, 40, boxes, hlbm.BC_PERIODIC_X_WALLS_Y, storage=hlbm.FP16_DEV, max_steps=40,
                 **LAMINA)
    o.step(20)
    g.step(20)
    _, _, w = oracle.d2q9()
    for l in range(2):
        dev_o = o.level(l) - w[:, None, None]
        dev_g = g.level(l) - w[:, None, None]
        e = np.max(np.abs(dev_g - dev_o)) / np.max(np.abs(dev_o))
        _say("fp16 level", l, e)
        assert e < 2e-2
