"""Pins of the hybrid method on a graded body-fitted grid (columns and rows
at given coordinates, spacing growing away from the lamina, as the paper
refines its grid toward the body). The finite-volume matrices of graded
grids are pinned with the closed forms in test_oracle_mesh; here the
coupling: a fluid at rest stays at rest and a uniform flow stays uniform
while the graded grid oscillates through the lattice; a mirror-symmetric
graded grid feels no x-force; and uniform coordinates given through the
graded path reproduce the uniform grid's run.
"""
import numpy as np

from oracle import oracle as O
from paper_2006_13631_amd.workloads import graded_nodes

GX = graded_nodes(31, 0.5, 1.25, 1.5, fine=5.0)   # odd: mirror-symmetric columns
GY = graded_nodes(16, 0.5, 1.3, 1.5)
BASE = dict(nx=64, ny=48, nux=31, nuy=16, b=8.0, thickness=0.5, tau=0.8, kc=1.0, beta=20.0)


def test_rest_state_with_moving_graded_grid():
    s = O.Sim(max_steps=60, flags=O.FLAG_NO_BODY, x_nodes=GX, y_nodes=GY, **BASE)
    _, _, w = O.d2q9()
    s.step(60)
    inf = s.info()
    assert abs(inf.y) > 0.1 and inf.n_type1 > 0 and inf.n_type2 == 0
    assert np.max(np.abs(s.lattice() - w[:, None, None])) < 1e-15
    assert np.max(np.abs(s.grid() - w[:, None])) < 1e-15


def test_uniform_flow_preserved_on_graded_grid():
    s = O.Sim(max_steps=40, flags=O.FLAG_NO_BODY, bc=O.BC_PERIODIC, x_nodes=GX, y_nodes=GY,
              **dict(BASE, tau=0.7))
    e = O.feq(1.0, 0.03, -0.02)
    s.set_lattice(np.broadcast_to(e[:, None, None], (9, 48, 64)).copy())
    s.set_grid(np.broadcast_to(e[:, None], (9, s.nnode)).copy())
    s.step(40)
    assert s.info().n_type1 > 0
    assert np.max(np.abs(s.lattice() - e[:, None, None])) < 1e-14
    assert np.max(np.abs(s.grid() - e[:, None])) < 1e-14


def test_symmetric_graded_grid_gives_no_x_force():
    s = O.Sim(max_steps=120, x_nodes=GX, y_nodes=GY, **BASE)
    s.step(120)
    h = s.history()
    assert np.abs(h[:, 1]).max() > 1e-4
    assert np.abs(h[:, 0]).max() <= 1e-12 * np.abs(h[:, 1]).max()


def test_uniform_coordinates_reproduce_the_uniform_grid():
    cfg = dict(nx=64, ny=48, nux=24, nuy=16, b=8.0, thickness=1.0, tau=0.8, kc=1.0, beta=20.0, max_steps=80)
    u = O.Sim(**cfg)
    X = np.array([(i - 24 // 2) * 1.0 for i in range(24)])
    Y = np.array([(j - 0.5 * 15) * 1.0 for j in range(16)])
    g = O.Sim(x_nodes=X, y_nodes=Y, **cfg)
    u.step(80)
    g.step(80)
    for a, b in ((g.lattice(), u.lattice()), (g.grid(), u.grid()), (g.history(), u.history())):
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_graded_coordinates_checked():
    import pytest
    with pytest.raises(ValueError):  # rows not symmetric about the lamina
        O.Sim(max_steps=1, x_nodes=GX, y_nodes=GY + 0.1, **BASE)
    with pytest.raises(ValueError):  # grid wider than the lattice
        O.Sim(max_steps=1, x_nodes=GX * 4, y_nodes=GY, **BASE)
