"""Pins of the oracle's hybrid coupling: interface exchange (Eqs.
(postcollision2_s), (postcollision2_u)), node classification, the moving grid
and its refill (Sec. Refill procedure), the wall force and the fit of the
hydrodynamic function (Sec. 2.1).
"""
import math

import numpy as np
import pytest

from paper_2006_13631_amd.workloads import preset


def _sim(oracle, cfg, steps=None, **kw):
    c = dict(cfg)
    c.update(kw)
    n = c.pop("steps")
    c.pop("ckpt_every", None)
    return oracle.Sim(max_steps=steps or n, **c), n


def test_rest_state_with_moving_grid(oracle):
    """No body, grid oscillating: the fluid stays at rest on both grids."""
    cfg = dict(nx=64, ny=48, nux=24, nuy=16, h_u=1.0, b=8.0, thickness=1.0, tau=0.8, kc=1.0,
               beta=20.0, steps=60)
    s, n = _sim(oracle, cfg, flags=oracle.FLAG_NO_BODY)
    _, _, w = oracle.d2q9()
    s.step(n)
    inf = s.info()
    assert abs(inf.y) > 0.1 and inf.n_type1 > 0 and inf.n_type2 == 0
    assert np.max(np.abs(s.lattice() - w[:, None, None])) < 1e-15
    assert np.max(np.abs(s.grid() - w[:, None])) < 1e-15


def test_uniform_flow_preserved(oracle):
    """Uniform flow on a doubly periodic lattice with an oscillating grid
    (no body) stays uniform: every interpolation (bilinear, barycentric)
    reproduces a constant and the finite-volume stencils sum to zero."""
    cfg = dict(nx=64, ny=48, nux=24, nuy=16, h_u=1.0, b=8.0, thickness=1.0, tau=0.7, kc=1.0,
               beta=20.0, steps=40)
    s, n = _sim(oracle, cfg, flags=oracle.FLAG_NO_BODY, bc=oracle.BC_PERIODIC)
    e = oracle.feq(1.0, 0.03, -0.02)
    s.set_lattice(np.broadcast_to(e[:, None, None], (9, 48, 64)).copy())
    s.set_grid(np.broadcast_to(e[:, None], (9, s.nnode)).copy())
    s.step(n)
    assert s.info().n_type1 > 0
    assert np.max(np.abs(s.lattice() - e[:, None, None])) < 1e-14
    assert np.max(np.abs(s.grid() - e[:, None])) < 1e-14


def test_classification_guarantees(oracle):
    """Fictitious rectangle inset by 2 units: every discretization node pulls
    only from discretization or interpolation nodes; every lattice
    interpolation node lies in a triangle with no outer grid node; every outer
    grid node's four lattice donors are discretization nodes."""
    cfg = preset("lamina_256x128")
    s, _ = _sim(oracle, cfg, steps=10)
    m = s.mesh()
    x, y, typ = m.nodes()
    tri, _ = m.triangles()
    A, om = s.info().A, s.info().omega
    for k in (0, 7, 25, 51, 77):
        yk = A * math.sin(om * k)
        st = s.status(k)
        ny, nx = st.shape
        disc = st == 0
        # neighbours of disc nodes are disc or interpolation (never unused)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                sh = np.roll(np.roll(st, -dy, 0), -dx, 1)
                assert not np.any(disc & (sh == 2))
        # interpolation nodes: enclosing triangle without interface vertex
        for (j, i) in zip(*np.nonzero(st == 1)):
            t, lam = m.locate(i - nx // 2, j - (0.5 * (ny - 1) + yk))
            assert t >= 0
            assert not np.any(typ[tri[t]] == oracle.NODE_INTERFACE)
        # outer grid nodes: donors are disc
        for p in np.nonzero(typ == oracle.NODE_INTERFACE)[0]:
            X = nx // 2 + x[p]
            Y = 0.5 * (ny - 1) + yk + y[p]
            for dx in (0, 1):
                for dy in (0, 1):
                    assert disc[int(math.floor(Y)) + dy, int(math.floor(X)) + dx]


def test_refill_types_lamina(oracle):
    """Spacing 1 > per-step displacement: type 2 never occurs and exactly one
    grid row per step is refilled from the lattice (type 1)."""
    cfg = preset("lamina_256x128")
    s, _ = _sim(oracle, cfg, steps=200)
    s.step(200)
    inf = s.info()
    assert inf.n_type2 == 0
    assert inf.n_type1 == 200 * cfg["nux"]
    assert inf.n_type3 == 200 * (cfg["nux"] * cfg["nuy"] - cfg["nux"] - inf.n_wall)


def test_refill_type2_on_fine_grid(oracle):
    """Grid spacing 0.2 below the per-step displacement (up to 0.225): nodes
    land inside the old lamina and keep their previous values (type 2)."""
    cfg = preset("tiny_fine_grid")
    s, n = _sim(oracle, cfg)
    s.step(n)
    inf = s.info()
    assert inf.u_max > cfg["h_u"] and inf.n_type2 > 0
    assert np.all(np.isfinite(s.grid()))


def test_symmetric_grid_gives_no_drag(oracle):
    """Odd grid width: the grid, the lattice and the motion are mirror
    symmetric about the lamina's centre line, so F_x vanishes to rounding."""
    cfg = preset("tiny_ragged", nx=76)
    s, n = _sim(oracle, cfg)
    s.step(n)
    h = s.history()
    assert np.max(np.abs(h[:, 1])) > 1e-3
    assert np.max(np.abs(h[:, 0])) < 1e-12 * np.max(np.abs(h[:, 1]))


# ---- force (stress integral on the wall polygon) ----------------------
def _lamina_mesh(oracle, b=6.0):
    return oracle.Mesh.lamina(16, 10, 1.0, b)


def test_force_uniform_pressure_is_zero(oracle):
    m = _lamina_mesh(oracle)
    f = np.broadcast_to(oracle.feq(1.3, 0.0, 0.0)[:, None], (9, m.nnode)).copy()
    assert np.max(np.abs(m.force(f))) < 1e-14


def test_force_linear_pressure_exact(oracle):
    """p' = c_s^2 (rho - 1) linear in space: the trapezoid rule is exact and
    the force equals minus the pressure gradient times the body area b*T."""
    b, T = 6.0, 1.0
    m = _lamina_mesh(oracle, b)
    x, y, _ = m.nodes()
    for gx, gy in ((0.0, 0.01), (0.02, 0.0), (-0.01, 0.005)):
        rho = 1.0 + gx * x + gy * y
        f = np.array([oracle.feq(r, 0.0, 0.0) for r in rho]).T.copy()
        F = m.force(f)
        want = -(1.0 / 3.0) * np.array([gx, gy]) * b * T
        assert np.max(np.abs(F - want)) < 1e-14


def test_force_constant_stress_is_zero(oracle):
    """A uniform viscous stress integrates to zero around a closed polygon."""
    m = _lamina_mesh(oracle)
    cx, cy, w = oracle.d2q9()
    fneq = 1e-3 * w * (cx * cy)  # pure shear non-equilibrium part
    f = (oracle.feq(1.0, 0.0, 0.0) + fneq)[:, None] * np.ones(m.nnode)[None, :]
    assert np.max(np.abs(m.force(f))) < 1e-15


def test_force_shear_stress_value(oracle):
    """sigma_xy = -sum c_x c_y f^neq; on the top face (n = +y) alone it gives
    F_x = sigma_xy * b; with a stress that differs between the two faces the
    net force is b * (sigma_top - sigma_bottom)."""
    b = 6.0
    m = _lamina_mesh(oracle, b)
    x, y, _ = m.nodes()
    cx, cy, w = oracle.d2q9()
    unit = w * cx * cy  # sum_i c_x c_y (w c_x c_y) = 4 * (1/36) = 1/9
    amp = np.where(y > 0, 2e-3, 5e-4)
    f = oracle.feq(1.0, 0.0, 0.0)[:, None] + unit[:, None] * amp[None, :]
    F = m.force(f)
    sxy_top, sxy_bot = -2e-3 / 9.0, -5e-4 / 9.0
    # end faces (n = +-x) see sigma_xx = 0 and pick up sigma_xy n_x in F_y:
    # half top, half bottom value at each end -> cancels between the ends
    assert abs(F[0] - b * (sxy_top - sxy_bot)) < 1e-15
    assert abs(F[1]) < 1e-15


# ---- fit ----------------------------------------------------------------
def test_fit_recovers_synthetic_harmonic(oracle):
    om, A, b = 0.061359, 2.5, 32.0
    n = 600
    t = np.arange(1, n + 1)
    for F0, phi in ((3.0, 0.4), (11.0, -1.2), (0.5, 2.9)):
        F = F0 * np.sin(om * t + phi)
        hist = np.c_[np.zeros(n), F]
        th = oracle.fit_theta(hist, om, A, b)
        norm = 0.25 * math.pi * om * om * b * b * A
        want = F0 * complex(math.cos(phi), math.sin(phi)) / norm
        assert abs(th - want) < 1e-12 * abs(want)
    # a constant offset outside the model biases the fit only through the
    # window's incomplete cancellation; a pure offset over whole periods is
    # invisible
    T = 2 * math.pi / om
    F = np.full(n, 0.7)
    th = oracle.fit_theta(np.c_[np.zeros(n), F], om, A, b)
    assert abs(th) < 0.05 * 0.7 / (0.25 * math.pi * om * om * b * b * A)
