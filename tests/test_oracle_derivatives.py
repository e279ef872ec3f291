"""Pins of the oracle's complex-step build, the exact-derivative reference of
the adjoint.

The complex-step build runs the oracle's source with A, omega and tau (and
everything computed from them) held as complex numbers while every discrete
decision follows the real part. These tests tie it to the real build:
zero perturbation reproduces the real build bit for bit, and its derivatives
agree with central differences of the real build wherever the force history
is smooth in the parameters.
"""
import math

import numpy as np
import pytest

from paper_2006_13631_amd.workloads import preset, random_populations


def _cfg(name):
    c = preset(name)
    n = c.pop("steps")
    c.pop("ckpt_every", None)
    return c, n


def _run(O, n, c, **kw):
    cc = dict(c)
    cc.update(kw)
    s = O.Sim(max_steps=n, **cc)
    s.step(n)
    return s


def test_zero_perturbation_reproduces_real_build(oracle):
    c, n = _cfg("tiny_ragged")
    r = _run(oracle, n, c)
    z = oracle.SimCS(0.0, 0.0, 0.0, max_steps=n, **c)
    z.step(n)
    hre, him = z.history()
    lre, lim = z.lattice()
    gre, gim = z.grid()
    assert np.array_equal(hre, r.history()) and not him.any()
    assert np.array_equal(lre, r.lattice()) and not lim.any()
    assert np.array_equal(gre, r.grid()) and not gim.any()


def test_complex_step_matches_central_differences(oracle):
    """A = KC b / (2 pi), omega = 2 pi nu beta / b^2, nu = (tau - 1/2)/3:
    central differences in (KC, beta, tau) at relative step 1e-6 against the
    complex-step derivatives combined by the chain rule."""
    c, n = _cfg("tiny_adjoint")
    inf = oracle.Sim(max_steps=1, **c).info()
    h = 1e-30
    d = {}
    for key, hv in (("A", (h, 0, 0)), ("omega", (0, h, 0)), ("tau", (0, 0, h))):
        z = oracle.SimCS(*hv, max_steps=n, **c)
        z.step(n)
        d[key] = z.history()[1] / h
    w = np.random.default_rng(3).standard_normal((n, 2))
    J = lambda H: float(np.sum(w * H))
    b, tau, om = c["b"], c["tau"], inf.omega
    cs = {"kc": J(d["A"]) * b / (2 * math.pi),
          "beta": J(d["omega"]) * om / c["beta"],
          "tau": J(d["tau"]) + J(d["omega"]) * om / (tau - 0.5)}
    for key, want in cs.items():
        e = 1e-6 * c[key]
        fd = (J(_run(oracle, n, c, **{key: c[key] + e}).history())
              - J(_run(oracle, n, c, **{key: c[key] - e}).history())) / (2 * e)
        assert abs(fd - want) <= 1e-6 * abs(want), (key, fd, want)


def test_complex_step_along_initial_state(oracle):
    """Directional derivative along a random start of both grids (a
    dot-product pin for the adjoint with respect to the state)."""
    c, n = _cfg("tiny_adjoint")
    n = 20
    _, _, wq = oracle.d2q9()
    f0 = random_populations((9, c["ny"], c["nx"]), seed=31, base=wq, spread=0.01)
    g0 = random_populations((9, 33 * 16), seed=32, base=wq, spread=0.01)
    vl = np.random.default_rng(33).standard_normal(f0.shape) * wq[:, None, None]
    vg = np.random.default_rng(34).standard_normal(g0.shape) * wq[:, None]
    h = 1e-30
    z = oracle.SimCS(max_steps=n, **c)
    z.set_lattice(f0, h * vl)
    z.set_grid(g0, h * vg)
    z.step(n)
    w = np.random.default_rng(35).standard_normal((n, 2))
    cs = float(np.sum(w * z.history()[1])) / h

    def J(eps):
        s = oracle.Sim(max_steps=n, **c)
        s.set_lattice(f0 + eps * vl)
        s.set_grid(g0 + eps * vg)
        s.step(n)
        return float(np.sum(w * s.history()))
    e = 1e-6
    fd = (J(e) - J(-e)) / (2 * e)
    assert abs(fd - cs) <= 1e-6 * abs(cs), (fd, cs)


def test_symmetric_turning_point_is_a_tie(oracle):
    """tiny_ragged's period is exactly 54 steps, so y_13 = y_14 in FP64 and
    the grid does not move in step 13: the top row then lies exactly on the
    old grid's edge (type 3 by the closed-interval rule). Any change of omega
    breaks the tie, so the history jumps there (derivatives of this case are
    one-sided; derivative tests use tiny_adjoint)."""
    c, n = _cfg("tiny_ragged")
    om = oracle.Sim(max_steps=1, **c).info().omega
    A = c["kc"] * c["b"] / (2 * math.pi)
    assert A * math.sin(om * 13) == A * math.sin(om * 14)
    base = _run(oracle, 16, c).info()
    up = _run(oracle, 16, c, beta=c["beta"] * (1 + 1e-9)).info()
    assert up.n_type1 - base.n_type1 == 33 and base.n_type3 - up.n_type3 == 33
