"""Physics context for the oracle: the hydrodynamic function of a lamina in
the nearly incompressible regime, against the semianalytical Theta of Eqs.
(hydro_gamma) + (hydro_delta). The paper's own method lands within a few per
cent of it (Fig. results); a confined 8b x 8b domain adds a few per cent more
(Table sensitivity). This is context, not parity: it guards against gross
errors (a wrong sign, a lost wall term) that the unit pins could miss.

It takes about two minutes on one core; the oracle's per-node loops run on
every core the process may use (which leaves its bits unchanged).
"""
import math
import os

from physics_refs import theta_semianalytical


def _cores():
    return max(1, len(os.sched_getaffinity(0)))


def test_theta_near_semianalytical(oracle):
    b, beta, eps, tau, N = 32.0, 20.0, 0.05, 0.56, 256
    kc = 2 * math.pi * eps
    nu = (tau - 0.5) / 3
    period = 2 * math.pi / (2 * math.pi * nu * beta / b ** 2)
    steps = int(4 * period) + 2
    s = oracle.Sim(N, N, 64, 32, 1.0, b, 1.0, tau, kc, beta, max_steps=steps)
    oracle.set_threads(_cores())
    try:
        s.step(steps)
    finally:
        oracle.set_threads(1)
    inf = s.info()
    th = oracle.fit_theta(s.history(), inf.omega, inf.A, b)
    ref = theta_semianalytical(beta, eps)
    assert abs(th.real / ref.real - 1) < 0.05, (th, ref)
    assert abs(th.imag / ref.imag - 1) < 0.10, (th, ref)
