"""torch.autograd bridge: Theta fit in torch and its gradient through the GPU
adjoint.

The reference derivative of Theta is the complex-step one: the oracle's
complex-step history (A, omega or tau carrying i h) pushed through the same
single-harmonic fit written in plain numpy complex arithmetic, applied to
Re Theta = a_s / norm and Im Theta = a_c / norm separately.
"""
import math
import sys

import numpy as np
import pytest
import torch

from paper_2006_13631_amd.workloads import preset

H = 1e-30


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _fit_np(Fy, omega, A, b, omega_re, t0=1.0, t1=4.0):
    """(a_s / norm, a_c / norm) in numpy; the window follows Re(omega)."""
    t = np.arange(1, Fy.shape[0] + 1, dtype=np.float64)
    T = 2 * math.pi / omega_re
    sel = (t >= t0 * T) & (t < t1 * T)
    t, F = t[sel], Fy[sel]
    sn, cs = np.sin(omega * t), np.cos(omega * t)
    ss, sc, cc = np.sum(sn * sn), np.sum(sn * cs), np.sum(cs * cs)
    sf, cf = np.sum(sn * F), np.sum(cs * F)
    det = ss * cc - sc * sc
    norm = 0.25 * math.pi * omega * omega * b * b * A
    return (sf * cc - cf * sc) / det / norm, (cf * ss - sf * sc) / det / norm


def test_torch_fit_matches_oracle_fit(oracle):
    from paper_2006_13631_amd.autograd import theta
    c = preset("lamina_128x64")
    c.pop("steps")
    c.pop("ckpt_every")
    s = oracle.Sim(max_steps=250, **c)
    s.step(250)
    inf = s.info()
    h = s.history()
    want = oracle.fit_theta(h, inf.omega, inf.A, c["b"])
    got = theta(torch.from_numpy(h), torch.tensor(inf.A, dtype=torch.float64),
                torch.tensor(inf.omega, dtype=torch.float64), c["b"])
    assert abs(complex(got) - want) <= 1e-13 * abs(want)
    re, im = _fit_np(h[:, 1], inf.omega, inf.A, c["b"], inf.omega)
    assert abs(complex(re, im) - want) <= 1e-13 * abs(want)


@pytest.mark.gpu
@pytest.mark.timeout(600)
def test_theta_gradient_through_gpu_adjoint(oracle):
    from paper_2006_13631_amd import hlbm
    from paper_2006_13631_amd.autograd import lamina_forces, theta
    _say("autograd Theta gradient, lamina_128x64, 250 steps")
    c = preset("lamina_128x64")
    c.pop("steps")
    c.pop("ckpt_every")
    n = 250
    inf = oracle.Sim(max_steps=1, **c).info()
    A0, om0, tau0 = inf.A, inf.omega, c["tau"]
    # complex-step reference
    ref = np.zeros((2, 3))
    for k, hv in enumerate(((H, 0, 0), (0, H, 0), (0, 0, H))):
        z = oracle.SimCS(*hv, max_steps=n, **c)
        z.step(n)
        hre, him = z.history()
        Fy = hre[:, 1] + 1j * him[:, 1]
        re, im = _fit_np(Fy, om0 + 1j * hv[1], A0 + 1j * hv[0], c["b"], om0)
        ref[0, k] = re.imag / H
        ref[1, k] = im.imag / H
    # GPU forward + adjoint through torch
    got = np.zeros((2, 3))
    for part in (0, 1):
        A = torch.tensor(A0, dtype=torch.float64, requires_grad=True)
        om = torch.tensor(om0, dtype=torch.float64, requires_grad=True)
        tau = torch.tensor(tau0, dtype=torch.float64, requires_grad=True)
        hist = lamina_forces(A, om, tau, c, n, storage=hlbm.FP64, ckpt_every=100)
        th = theta(hist, A, om, c["b"])
        (th.real if part == 0 else th.imag).backward()
        got[part] = [A.grad.item(), om.grad.item(), tau.grad.item()]
    rel = np.abs(got - ref) / np.abs(ref)
    _say("torch+adjoint", got, "\ncomplex step", ref, "\nrel", rel)
    assert np.all(rel <= 1e-8), rel
