"""Pins of the oracle's finite-volume sub-step (Eq.(ulbe)) and its wall rule.

* conservation: on a doubly periodic grid the control-volume weighted mass
  and momentum are invariant (streaming fluxes cancel pairwise, collision
  conserves rho and rho u at every node);
* the rest state is a fixed point;
* a Taylor-Green vortex decays at 4 nu k^2 with the paper's grid viscosity
  nu = c_s^2 tau_u (Sec. 3), converging at second order in the spacing;
* Stokes' oscillating plate on a channel grid whose wall nodes carry the
  imposed-velocity rule.
"""
import math

import numpy as np
import pytest


def _tg_state(oracle, m, N, U=0.01):
    x, y, _ = m.nodes()
    k = 2 * math.pi / N
    ux = -U * np.cos(k * x) * np.sin(k * y)
    uy = U * np.sin(k * x) * np.cos(k * y)
    p = -0.25 * U * U * (np.cos(2 * k * x) + np.cos(2 * k * y))
    rho = 1 + 3 * p
    return np.array([oracle.feq(rho[i], ux[i], uy[i]) for i in range(m.nnode)]).T.copy()


def test_conservation_periodic(oracle):
    from paper_2006_13631_amd.workloads import random_populations
    m = oracle.Mesh.periodic(7, 6, 1.0)
    _, _, _, V = m.stencil()
    cx, cy, w = oracle.d2q9()
    f = random_populations((9, m.nnode), seed=11, base=w, spread=0.2)
    mass0 = (f.sum(0) * V).sum()
    mx0 = ((cx[:, None] * f).sum(0) * V).sum()
    my0 = ((cy[:, None] * f).sum(0) * V).sum()
    for _ in range(10):
        f = m.substep(f, 0.1, 0.05)
    assert abs((f.sum(0) * V).sum() - mass0) < 1e-13 * mass0
    assert abs(((cx[:, None] * f).sum(0) * V).sum() - mx0) < 1e-13
    assert abs(((cy[:, None] * f).sum(0) * V).sum() - my0) < 1e-13


def test_rest_state_fixed(oracle):
    cx, cy, w = oracle.d2q9()
    for m in (oracle.Mesh.periodic(5, 5, 1.0), oracle.Mesh.channel(4, 6, 1.0)):
        f = np.broadcast_to(w[:, None], (9, m.nnode)).copy()
        z = np.zeros(m.nnode)
        g = f
        for _ in range(8):
            g = m.substep(g, 0.3, 0.25, uwx=z, uwy=z)
        assert np.max(np.abs(g - f)) < 1e-15


def _tg_rate(oracle, N, tau_u, n):
    m = oracle.Mesh.periodic(N, N, 1.0)
    f = _tg_state(oracle, m, N)
    cx, cy, _ = oracle.d2q9()

    def energy(f):
        r = f.sum(0)
        return ((((cx[:, None] * f).sum(0) / r) ** 2) + (((cy[:, None] * f).sum(0) / r) ** 2)).sum()

    for _ in range(10 * n):
        f = m.substep(f, tau_u, 1.0 / n)
    e0 = energy(f)
    steps = 2 * N
    for _ in range(steps * n):
        f = m.substep(f, tau_u, 1.0 / n)
    k = 2 * math.pi / N
    return -math.log(energy(f) / e0) / steps / (4 * (tau_u / 3.0) * k * k)


def test_taylor_green_grid_viscosity(oracle):
    r16 = _tg_rate(oracle, 16, 0.1, 10)
    r32 = _tg_rate(oracle, 32, 0.1, 10)
    assert abs(r32 - 1) < 0.03, (r16, r32)
    assert abs(r16 - 1) / abs(r32 - 1) > 3.0  # second order


def _stokes_channel(oracle, period, ny, n=4, tau_u=0.3):
    m = oracle.Mesh.channel(4, ny, 1.0)
    x, y, t = m.nodes()
    cx, _, w = oracle.d2q9()
    om = 2 * math.pi / period
    U = 0.01
    f = np.broadcast_to(w[:, None], (9, m.nnode)).copy()
    bottom = (t == oracle.NODE_WALL) & (y < 0.5)
    zero = np.zeros(m.nnode)
    steps = 5 * period
    for k in range(steps):
        for s in range(n):
            uwx = np.where(bottom, U * math.cos(om * (k + (s + 1) / n)), 0.0)
            f = m.substep(f, tau_u, 1.0 / n, uwx=uwx, uwy=zero)
    r = f.sum(0)
    ux = (cx[:, None] * f).sum(0) / r
    nu = tau_u / 3.0
    delta = math.sqrt(2 * nu / om)
    col = np.abs(x) < 1e-12
    eta = y[col] / delta
    exact = U * np.exp(-eta) * np.cos(om * steps - eta)
    return np.linalg.norm(ux[col] - exact) / np.linalg.norm(exact), delta


def test_stokes_second_problem_grid(oracle):
    """Wall nodes move tangentially with U cos(omega t) (imposed-velocity
    wall rule); the far wall rests more than 10 delta away."""
    e1, d1 = _stokes_channel(oracle, 400, 48)
    e2, d2 = _stokes_channel(oracle, 1600, 96)
    assert 10 * d1 < 47 and 10 * d2 < 95
    # about 2 % with the plate's layer resolved by 3.6 nodes, second-order
    # convergence when the resolution doubles
    assert e1 < 0.03 and e2 < 0.01 and e2 < e1 / 3, (e1, e2)
