"""Reference values the paper compares its results with (reporting only).

The semianalytical hydrodynamic function of a thin lamina oscillating with
small finite amplitude, Theta = Gamma(beta) + Delta(beta, epsilon), from the
fits the paper quotes (Sec. 2.1, Eqs. (hydro_tot), (hydro_gamma),
(hydro_delta)), and the bound beta < 2.6 epsilon^-1.6 within which the force
is expected to stay harmonic (Eq.(betalimit)).
"""
from __future__ import annotations


def theta_semianalytical(beta: float, eps: float) -> complex:
    """Gamma(beta) = 1.02 + 2.45 beta^-1/2 - 2.49 i beta^-1/2 and
    Delta(beta, eps) = -0.879 i beta^3/4 eps^2."""
    gamma = complex(1.02 + 2.45 * beta ** -0.5, -2.49 * beta ** -0.5)
    return gamma + complex(0.0, -0.879 * beta ** 0.75 * eps * eps)


def beta_limit(eps: float) -> float:
    """Upper bound of beta for a harmonic force at amplitude ratio eps."""
    return 2.6 * eps ** -1.6
