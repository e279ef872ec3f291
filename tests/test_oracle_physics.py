"""Physics context for the oracle: the hydrodynamic function of a lamina in
the nearly incompressible regime, against the semianalytical Theta of Eqs.
(hydro_gamma) + (hydro_delta). The paper's own method lands within a few per
cent of it (Fig. results); a confined 8b x 8b domain adds a few per cent more
(Table sensitivity). This is context, not parity: it guards against gross
errors (a wrong sign, a lost wall term) that the unit pins could miss.

It takes about two minutes on one core, so it runs only with HLBM_SLOW=1.
"""
import math
import os

import pytest

from physics_refs import theta_semianalytical

pytestmark = pytest.mark.skipif(os.environ.get("HLBM_SLOW") != "1",
                                reason="two-minute oracle run; set HLBM_SLOW=1")


def test_theta_near_semianalytical(oracle):
    b, beta, eps, tau, N = 32.0, 20.0, 0.05, 0.56, 256
    kc = 2 * math.pi * eps
    nu = (tau - 0.5) / 3
    period = 2 * math.pi / (2 * math.pi * nu * beta / b ** 2)
    steps = int(4 * period) + 2
    s = oracle.Sim(N, N, 64, 32, 1.0, b, 1.0, tau, kc, beta, max_steps=steps)
    s.step(steps)
    inf = s.info()
    th = oracle.fit_theta(s.history(), inf.omega, inf.A, b)
    ref = theta_semianalytical(beta, eps)
    assert abs(th.real / ref.real - 1) < 0.05, (th, ref)
    assert abs(th.imag / ref.imag - 1) < 0.10, (th, ref)
