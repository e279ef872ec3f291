"""Pins of the oracle's structured lattice (Eqs. (LBE) and (local_eq)).

Each check compares the oracle with something other than itself: exact moment
identities of the D2Q9 equilibrium, conservation laws, the analytic decay of a
Taylor-Green vortex, the exact Couette profile of halfway bounce-back and
Stokes' oscillating-plate solution.
"""
import math

import numpy as np
import pytest


def test_equilibrium_moments(oracle):
    """Zeroth, first and second moments of Eq.(local_eq) are rho, rho u and
    rho c_s^2 I + rho u u exactly (this fixes the weights and each term)."""
    cx, cy, w = oracle.d2q9()
    assert abs(w.sum() - 1.0) < 1e-15
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho = rng.uniform(0.8, 1.2)
        ux, uy = rng.uniform(-0.2, 0.2, 2)
        f = oracle.feq(rho, ux, uy)
        assert abs(f.sum() - rho) < 1e-14
        assert abs((cx * f).sum() - rho * ux) < 1e-15
        assert abs((cy * f).sum() - rho * uy) < 1e-15
        cs2 = 1.0 / 3.0
        assert abs((cx * cx * f).sum() - (rho * cs2 + rho * ux * ux)) < 1e-14
        assert abs((cx * cy * f).sum() - rho * ux * uy) < 1e-15
        assert abs((cy * cy * f).sum() - (rho * cs2 + rho * uy * uy)) < 1e-14


def test_rest_state_is_fixed_point(oracle):
    _, _, w = oracle.d2q9()
    A = np.broadcast_to(w[:, None, None], (9, 12, 10)).copy()
    for bc in (oracle.BC_PERIODIC, oracle.BC_PERIODIC_X_WALLS_Y):
        B = A
        for _ in range(10):
            B = oracle.lattice_step(B, 0.7, bc=bc)
        assert np.max(np.abs(A - B)) < 1e-15


def test_conservation_random_state(oracle):
    """Stream + BGK conserve total mass and momentum on a periodic lattice,
    and total mass with resting bounce-back walls."""
    from paper_2006_13631_amd.workloads import random_populations
    cx, cy, w = oracle.d2q9()
    A = random_populations((9, 20, 24), seed=3, base=w, spread=0.3)
    for tau in (0.55, 0.8, 1.7):
        B = oracle.lattice_step(A, tau, bc=oracle.BC_PERIODIC)
        for f0, f1 in ((A, B),):
            assert abs(f1.sum() - f0.sum()) < 1e-12 * f0.sum()
            assert abs((cx[:, None, None] * f1).sum() - (cx[:, None, None] * f0).sum()) < 1e-13
            assert abs((cy[:, None, None] * f1).sum() - (cy[:, None, None] * f0).sum()) < 1e-13
        B = oracle.lattice_step(A, tau, bc=oracle.BC_PERIODIC_X_WALLS_Y)
        assert abs(B.sum() - A.sum()) < 1e-12 * A.sum()


def _taylor_green(oracle, N, tau, steps, U=0.01):
    """Taylor-Green vortex on an N^2 periodic lattice; returns the measured
    decay rate of the kinetic energy and the analytic 4 nu k^2."""
    k = 2 * math.pi / N
    x = np.arange(N)
    X, Y = np.meshgrid(x, x, indexing="xy")
    ux = -U * np.cos(k * X) * np.sin(k * Y)
    uy = U * np.sin(k * X) * np.cos(k * Y)
    p = -0.25 * U * U * (np.cos(2 * k * X) + np.cos(2 * k * Y))
    rho = 1.0 + 3.0 * p
    cx, cy, w = oracle.d2q9()
    f = np.zeros((9, N, N))
    for j in range(N):
        for i in range(N):
            f[:, j, i] = oracle.feq(rho[j, i], ux[j, i], uy[j, i])

    def energy(f):
        r = f.sum(0)
        vx = (cx[:, None, None] * f).sum(0) / r
        vy = (cy[:, None, None] * f).sum(0) / r
        return (vx * vx + vy * vy).sum()

    # skip a short start-up transient of the non-equilibrium part
    for _ in range(20):
        f = oracle.lattice_step(f, tau, bc=oracle.BC_PERIODIC)
    e0 = energy(f)
    for _ in range(steps):
        f = oracle.lattice_step(f, tau, bc=oracle.BC_PERIODIC)
    e1 = energy(f)
    nu = (tau - 0.5) / 3.0
    return -math.log(e1 / e0) / steps, 4 * nu * k * k


def test_taylor_green_decay(oracle):
    """Kinetic energy decays as exp(-4 nu k^2 t) with nu = c_s^2 (tau - 1/2)
    (text after Eq.(local_eq)); rate error < 1 % at N = 64 and second order
    in the resolution."""
    errs = []
    for N in (16, 32, 64):
        rate, exact = _taylor_green(oracle, N, 0.8, steps=N * 4)
        errs.append(abs(rate / exact - 1.0))
    assert errs[-1] < 0.01
    order = math.log(errs[0] / errs[1], 2), math.log(errs[1] / errs[2], 2)
    assert min(order) > 1.7, (errs, order)


def test_couette_exact(oracle):
    """Plane Couette flow with halfway bounce-back walls (top wall moving at
    U) is reproduced exactly: u_x(y) = U (y + 1/2) / ny."""
    nx, ny, U, tau = 4, 16, 0.05, 1.0
    _, _, w = oracle.d2q9()
    cx, _, _ = oracle.d2q9()
    f = np.broadcast_to(w[:, None, None], (9, ny, nx)).copy()
    for _ in range(20000):
        f = oracle.lattice_step(f, tau, bc=oracle.BC_PERIODIC_X_WALLS_Y, u_top=U)
    r = f.sum(0)
    ux = (cx[:, None, None] * f).sum(0) / r
    exact = U * (np.arange(ny) + 0.5) / ny
    assert np.max(np.abs(ux - exact[:, None])) < 1e-12


def _stokes_lattice(oracle, period, ny, periods=5):
    tau = 0.8
    nu = (tau - 0.5) / 3.0
    om = 2 * math.pi / period
    U = 0.01
    cx, _, w = oracle.d2q9()
    f = np.broadcast_to(w[:, None, None], (9, ny, 3)).copy()
    steps = periods * period
    for t in range(steps):
        # wall velocity at the time the populations reach the wall
        f = oracle.lattice_step(f, tau, bc=oracle.BC_PERIODIC_X_WALLS_Y,
                                u_bot=U * math.cos(om * (t + 0.5)))
    r = f.sum(0)
    ux = ((cx[:, None, None] * f).sum(0) / r)[:, 0]
    delta = math.sqrt(2 * nu / om)
    eta = (np.arange(ny) + 0.5) / delta
    exact = U * np.exp(-eta) * np.cos(om * steps - eta)
    return np.linalg.norm(ux - exact) / np.linalg.norm(exact), delta


def test_stokes_second_problem_lattice(oracle):
    """Stokes' oscillating plate: u = U exp(-eta) cos(omega t - eta),
    eta = y / delta, delta = sqrt(2 nu / omega); depth > 10 delta."""
    e1, d1 = _stokes_lattice(oracle, 400, 48)
    e2, d2 = _stokes_lattice(oracle, 1600, 96)
    assert 10 * d1 < 48 and 10 * d2 < 96
    assert e1 < 0.02 and e2 < e1, (e1, e2)


# ---- the paper's outer boundaries: no-slip x walls, outflow y ends ----------

def test_paper_boundaries_stream_as_defined(oracle):
    """Pure streaming (tau -> infinity) on a random state: interior
    populations shift along c_i; at an x wall the incoming population is the
    node's own opposite one (halfway bounce-back at rest); at a y end the
    incoming population equals that of the next row in (zero normal
    gradient); at the four corners the wall decides."""
    from paper_2006_13631_amd.workloads import random_populations
    cx, cy, w = oracle.d2q9()
    opp = [int(np.flatnonzero((cx == -cx[i]) & (cy == -cy[i]))[0]) for i in range(9)]
    ny, nx = 7, 9
    A = random_populations((9, ny, nx), seed=11, base=w, spread=0.3)
    B = oracle.lattice_step(A, 1e300, bc=oracle.BC_PAPER)
    for i in range(9):
        for y in range(ny):
            for x in range(nx):
                xs, ys = x - cx[i], y - cy[i]
                if not 0 <= xs < nx:
                    want = A[opp[i], y, x]
                elif not 0 <= ys < ny:
                    want = B[i, y + cy[i], x]   # the next row in
                else:
                    want = A[i, ys, xs]
                assert B[i, y, x] == want, (i, y, x)


def test_paper_boundaries_rest_and_uniform_rows(oracle):
    """The rest state is a fixed point, and a state that does not vary
    along y stays so exactly (the outflow ends then act like periodic ones)."""
    from paper_2006_13631_amd.workloads import random_populations
    _, _, w = oracle.d2q9()
    A = np.broadcast_to(w[:, None, None], (9, 12, 10)).copy()
    B = A
    for _ in range(10):
        B = oracle.lattice_step(B, 0.7, bc=oracle.BC_PAPER)
    assert np.max(np.abs(A - B)) < 1e-15
    row = random_populations((9, 1, 10), seed=5, base=w, spread=0.05)
    A = np.repeat(row, 8, axis=1)
    for _ in range(25):
        A = oracle.lattice_step(A, 0.9, bc=oracle.BC_PAPER)
    assert np.max(np.abs(A - A[:, :1, :])) == 0.0


def _channel_shear_decay(oracle, nx, tau=0.8, steps=None, U=1e-4):
    """u_y(x) = U sin(pi (x + 1/2) / nx) between the no-slip x walls (at
    x = -1/2 and nx - 1/2), uniform along y: decays as exp(-nu k^2 t),
    k = pi / nx. Returns the relative error of the measured rate."""
    cx, cy, w = oracle.d2q9()
    nu = (tau - 0.5) / 3.0
    k = math.pi / nx
    x = np.arange(nx) + 0.5
    uy = U * np.sin(k * x)
    f = np.zeros((9, 4, nx))
    for i in range(9):
        f[i] = w[i] * (1.0 + 3.0 * cy[i] * uy + 4.5 * (cy[i] * uy) ** 2 - 1.5 * uy ** 2)[None, :]
    steps = steps or int(round(0.5 / (nu * k * k)))
    amp0 = None
    for t in range(steps + 1):
        if t == steps // 4:
            r = f.sum(0)
            amp0 = ((cy[:, None, None] * f).sum(0) / r)[0] @ np.sin(k * x)
        if t < steps:
            f = oracle.lattice_step(f, tau, bc=oracle.BC_PAPER)
    r = f.sum(0)
    amp1 = ((cy[:, None, None] * f).sum(0) / r)[0] @ np.sin(k * x)
    rate = -math.log(amp1 / amp0) / (steps - steps // 4)
    return abs(rate - nu * k * k) / (nu * k * k)


def test_paper_boundaries_channel_shear_decay(oracle):
    """No-slip walls in x: the slowest shear mode of the channel decays at the
    viscous rate nu (pi/nx)^2, to second order in the resolution."""
    e16 = _channel_shear_decay(oracle, 16)
    e32 = _channel_shear_decay(oracle, 32)
    assert e32 < 1e-2
    assert e16 / e32 > 3.0
