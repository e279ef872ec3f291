"""Closed forms the paper prints, used as references by the tests.

* semianalytical hydrodynamic function Theta = Gamma + Delta,
  Eqs.(hydro_tot), (hydro_gamma), (hydro_delta) of Sec. 2.1;
* harmonic-regime bound beta < 2.6 eps^-1.6, Eq.(betalimit);
* cost indicator G = (1 + chi s' n) / g, Eq.(speedup).
"""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def theta_semianalytical(beta: float, eps: float) -> complex:
    gamma = 1.02 + 2.45 * beta ** -0.5 - 1j * 2.49 * beta ** -0.5
    delta = -1j * 0.879 * beta ** 0.75 * eps ** 2
    return gamma + delta


def beta_limit(eps: float) -> float:
    return 2.6 * eps ** -1.6


def cost_indicator(chi: float, s_prime: float, n: float, g: float) -> float:
    return (1.0 + chi * s_prime * n) / g


def read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line.split())
    return rows
