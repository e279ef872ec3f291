"""torch.autograd bridge to the GPU adjoint.

``lamina_forces(A, omega, tau, cfg)`` runs the hybrid method on the GPU for
the given amplitude, angular frequency and relaxation time and returns the
force history F(t_{k+1}), k = 0 .. steps-1, as a float64 tensor; its backward
calls the library's discrete adjoint (``hlbm_adjoint``), so gradients with
respect to A, omega and tau come from the GPU adjoint kernels.

``theta(hist, A, omega, b)`` is the hydrodynamic function of Eq.(force_phasor)
from the single-harmonic least-squares fit of F_y over [t0 T, t1 T)
(Sec. 2.1), written in torch so that its own dependence on omega (fit basis)
and on A, omega (normalisation (pi/4) rho omega^2 L^2 A) is differentiated by
torch. The window's sample set is a discrete decision and is held fixed.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import hlbm

_GRID_KEYS = ("nx", "ny", "nux", "nuy", "h_u", "b", "thickness", "n_sub", "bc", "flags")


def config_for(A: float, omega: float, tau: float, base: dict) -> dict:
    """Library configuration naming (A, omega, tau): KC = 2 pi A / b and
    beta = omega b^2 / (2 pi nu) with nu = (tau - 1/2)/3."""
    b = float(base["b"])
    nu = (tau - 0.5) / 3.0
    c = {k: base[k] for k in _GRID_KEYS if k in base}
    c.update(tau=float(tau), kc=2.0 * math.pi * A / b, beta=omega * b * b / (2.0 * math.pi * nu))
    return c


class _LaminaForces(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, omega, tau, base, steps, storage, ckpt_every):
        c = config_for(float(A), float(omega), float(tau), base)
        case = hlbm.Case(max_steps=steps, storage=storage, ckpt_every=ckpt_every, **c)
        case.step(steps)
        ctx.case = case
        return torch.from_numpy(case.history().copy())

    @staticmethod
    def backward(ctx, g_hist):
        g = ctx.case.adjoint(g_hist.detach().to(torch.float64).cpu().numpy())
        out = [torch.tensor(v, dtype=torch.float64) for v in g]
        return out[0], out[1], out[2], None, None, None, None


def lamina_forces(A, omega, tau, base: dict, steps: int, storage=hlbm.FP64, ckpt_every: int = 200):
    """Force history (steps, 2) of the lamina case ``base`` (grid sizes, b,
    boundary) moving with amplitude A and angular frequency omega at
    relaxation time tau. A, omega, tau: 0-d float64 tensors."""
    ckpt = max(1, min(int(ckpt_every), int(steps)))
    return _LaminaForces.apply(A, omega, tau, base, int(steps), storage, ckpt)


def theta(hist: torch.Tensor, A, omega, b: float, t0: float = 1.0, t1: float = 4.0) -> torch.Tensor:
    """Theta = (a_s + i a_c) / ((pi/4) omega^2 b^2 A) from F_y(t) ~ a_s sin(omega
    t) + a_c cos(omega t) over t0 T <= t < t1 T, t = k + 1, T = 2 pi / omega.
    Returns a complex128 tensor."""
    om = float(omega.detach()) if torch.is_tensor(omega) else float(omega)
    T = 2.0 * math.pi / om
    t = np.arange(1, hist.shape[0] + 1, dtype=np.float64)
    sel = np.nonzero((t >= t0 * T) & (t < t1 * T))[0]
    if sel.size < 2:
        raise ValueError("fit window holds fewer than two samples")
    tt = torch.from_numpy(t[sel])
    F = hist[torch.from_numpy(sel), 1]
    sn, cs = torch.sin(omega * tt), torch.cos(omega * tt)
    ss, sc, cc = (sn * sn).sum(), (sn * cs).sum(), (cs * cs).sum()
    sf, cf = (sn * F).sum(), (cs * F).sum()
    det = ss * cc - sc * sc
    norm = 0.25 * math.pi * omega * omega * b * b * A
    a_s = (sf * cc - cf * sc) / det / norm
    a_c = (cf * ss - sf * sc) / det / norm
    return torch.complex(a_s, a_c)
