"""Seeded synthetic workloads: named lamina configurations and random fields.

This module only states sizes, parameters and seeded random numbers. It holds
none of the method's arithmetic, so both the GPU library's tests and the CPU
oracle can take their inputs from it.

The configurations follow the problem statement of the paper (Sec. Problem
statement): a lamina of width ``b`` and thickness 1 in a D2Q9 lattice, moving
as y = A sin(omega t) with KC = 2 pi A / b and beta = omega b^2 / (2 pi nu).
"""
from __future__ import annotations

import math

import numpy as np

# name -> parameters (lattice nx*ny, body-fitted grid nux*nuy, lamina width b,
# relaxation time tau, KC, beta, number of structured steps)
PRESETS = {
    # plain run with oracle parity: 256x128 lattice, 64x32 grid, 2000 steps
    "lamina_256x128": dict(nx=256, ny=128, nux=64, nuy=32, h_u=1.0, b=32.0, thickness=1.0,
                           tau=0.8, kc=0.5, beta=100.0, steps=2000),
    # sweep scale: 2048^2 lattice, 512x128 grid, 20000 steps
    "lamina_2048": dict(nx=2048, ny=2048, nux=512, nuy=128, h_u=1.0, b=128.0, thickness=1.0,
                        tau=0.55, kc=1.0, beta=1000.0, steps=20000),
    # differentiation case: 1024^2 lattice, 256x64 grid, 4000 steps, window 200
    "lamina_1024": dict(nx=1024, ny=1024, nux=256, nuy=64, h_u=1.0, b=64.0, thickness=1.0,
                        tau=0.6, kc=0.8, beta=500.0, steps=4000, ckpt_every=200),
    # 128x64 copy of the differentiation case (same KC, tau and lamina speed)
    "lamina_128x64": dict(nx=128, ny=64, nux=64, nuy=16, h_u=1.0, b=16.0, thickness=1.0,
                          tau=0.6, kc=0.8, beta=125.0, steps=4000, ckpt_every=200),
    # precision at scale: 4096^2 lattice, 1024x256 grid, 100000 steps
    "lamina_4096": dict(nx=4096, ny=4096, nux=1024, nuy=256, h_u=1.0, b=256.0, thickness=1.0,
                        tau=0.52, kc=3.0, beta=2000.0, steps=100000),
    # the same lattice, grid and KC at a viscosity and frequency plain BGK
    # sustains (U = 0.059, Ma = 0.10, Re = 450): period 13107 steps, fit
    # window [T, 4T) inside 52429 steps
    "lamina_4096_stable": dict(nx=4096, ny=4096, nux=1024, nuy=256, h_u=1.0, b=256.0, thickness=1.0,
                               tau=0.6, kc=3.0, beta=150.0, steps=52429),
    # small cases for tests: several tiles, ragged sizes, odd grid width
    "tiny_ragged": dict(nx=77, ny=45, nux=33, nuy=16, h_u=1.0, b=12.0, thickness=1.0,
                        tau=0.7, kc=0.6, beta=40.0, steps=60),
    # tiny_ragged with beta 41: its period (52.7 steps) is not an even
    # integer, so no step has y_{k+1} = y_k exactly and the force history is
    # smooth in A, omega and tau at this point (derivative tests)
    "tiny_adjoint": dict(nx=77, ny=45, nux=33, nuy=16, h_u=1.0, b=12.0, thickness=1.0,
                         tau=0.7, kc=0.6, beta=41.0, n_sub=5, steps=60),
    # grid spacing 0.2 below the largest per-step displacement (0.225): some
    # nodes land inside the old lamina
    "tiny_fine_grid": dict(nx=48, ny=48, nux=90, nuy=44, h_u=0.2, b=8.0, thickness=0.2,
                           tau=0.8, kc=1.8, beta=10.0, n_sub=32, steps=40),
}


def preset(name: str, **overrides) -> dict:
    cfg = dict(PRESETS[name])
    cfg.update(overrides)
    return cfg


def batch_cases(seed: int = 0, n_kc: int = 8, n_beta: int = 8):
    """64 (KC, beta) cases on a log grid, KC in [0.1, 4], beta in [50, 5000],
    each with a lattice edge drawn uniformly from {256, 512, 768, 1024} and a
    lamina of width edge/8 in a 4b x b grid."""
    rng = np.random.default_rng(seed)
    kcs = np.geomspace(0.1, 4.0, n_kc)
    betas = np.geomspace(50.0, 5000.0, n_beta)
    sizes = rng.choice([256, 512, 768, 1024], n_kc * n_beta)
    cases = []
    for i, kc in enumerate(kcs):
        for j, beta in enumerate(betas):
            n = int(sizes[i * n_beta + j])
            b = n // 8
            cases.append(dict(nx=n, ny=n, nux=4 * b, nuy=b, h_u=1.0, b=float(b), thickness=1.0,
                              kc=float(kc), beta=float(beta)))
    return cases


def sweep_cases(seed: int = 0, periods: float = 10.0, mach: float = 0.05):
    """The parametric sweep as runnable configurations: batch_cases(seed) with
    tau chosen to hold the lattice Mach number U sqrt(3) at ``mach``, where
    U = A omega = KC nu beta / b, i.e. tau = min(0.9, 1/2 + 3 nu*) with
    nu* = (mach / sqrt(3)) b / (KC beta), but not below 0.52 (such cases run
    above ``mach`` and are flagged), and ``periods`` oscillation periods of
    T = b^2 / (nu beta) steps each. Returns (configs, flagged)."""
    out, flagged = [], []
    u_star = mach / math.sqrt(3.0)
    for c in batch_cases(seed):
        nu_star = u_star * c["b"] / (c["kc"] * c["beta"])
        tau = min(0.9, 0.5 + 3.0 * nu_star)
        flag = tau < 0.52
        if flag:
            tau = 0.52
        nu = (tau - 0.5) / 3.0
        period = c["b"] ** 2 / (nu * c["beta"])
        cfg = dict(c, tau=tau, max_steps=int(math.ceil(periods * period)))
        out.append(cfg)
        flagged.append(flag)
    return out, flagged


# the paper's parameter grid (Sec. Problem statement)
STUDY_EPS = (0.02, 0.03, 0.04, 0.05, 0.075, 0.1)
STUDY_BETA = (20, 50, 100, 150, 200, 250, 300)


def paper_study_cases(b: int = 64, waves: float = 4.0, periods: float = 4.0, tau_max: float = 0.9):
    """The (epsilon, beta) study of the paper as runnable configurations:
    every pair of the grid with beta < 2.6 epsilon^-1.6 (Eq.(betalimit); 35
    pairs), on a 5L x 5L lattice with the paper's outer boundaries (bc 2),
    lamina L = b, body-fitted grid 4L x L, KC = 2 pi epsilon, and enough
    steps for the fit window [T, 4T). The paper keeps tau between 0.7 and 0.9
    with L = 800 lattice units; at a small L that would make the acoustic
    wavelength c_s T shorter than the domain, so here the viscosity is chosen
    per case for c_s T = waves x 5L, i.e. nu = c_s L / (5 waves beta), with
    tau at most tau_max. Each configuration also carries its eps and beta_p
    (the paper's beta) for reporting."""
    out = []
    cs = 1.0 / math.sqrt(3.0)
    for eps in STUDY_EPS:
        for beta in STUDY_BETA:
            if not beta < 2.6 * eps ** -1.6:
                continue
            tau = min(tau_max, 0.5 + 3.0 * cs * b / (5.0 * waves * beta))
            nu = (tau - 0.5) / 3.0
            period = b * b / (nu * beta)
            out.append(dict(nx=5 * b, ny=5 * b, nux=4 * b, nuy=b, h_u=1.0, b=float(b), thickness=1.0, tau=tau,
                            kc=2.0 * math.pi * eps, beta=float(beta), bc=2,
                            max_steps=int(math.ceil(periods * period)) + 1, eps=eps, beta_p=beta))
    return out


def paper_levels(b: int = 800, nlevels: int = 4, eps: float = 0.1, beta: float = 50.0, tau: float = 0.8,
                 margin: int = 16, pad: int = 8) -> dict:
    """The paper's structured refinement (Sec. Problem statement): a 5L x 5L
    domain, ``nlevels`` levels with the lamina (width L = b at the finest
    resolution, relaxation time tau there) on the finest. Level 0 spans the
    domain with spacing 2^(nlevels-1); each box is centred in its level,
    ``margin`` nodes clear of the finer level on every side; the finest
    level holds the 4b x b body-fitted grid, its motion amplitude A and
    ``pad`` nodes on each side. Returns nx0, ny0, bc0 (2: the paper's outer
    boundaries), boxes and the finest level's configuration."""
    kc = 2.0 * math.pi * eps
    A = kc * b / (2.0 * math.pi)
    W = -(-(4 * b + 2 * pad) // 2)
    H = int(math.ceil((b + 2.0 * A + 2 * pad) / 2.0))
    sizes = [(W, H)]  # box widths in cells, finest box first
    for _ in range(nlevels - 2):
        W, H = -(-(W + 2 * margin) // 2), -(-(H + 2 * margin) // 2)
        sizes.append((W, H))
    sizes.reverse()
    n0 = (5 * b) // 2 ** (nlevels - 1) + 1
    boxes, nx, ny = [], n0, n0
    for W, H in sizes:
        if W + 2 * margin + 1 > nx or H + 2 * margin + 1 > ny:
            raise ValueError("the levels do not fit the 5L x 5L domain")
        x0, y0 = (nx - 1 - W) // 2, (ny - 1 - H) // 2
        boxes.append((x0, y0, x0 + W, y0 + H))
        nx, ny = 2 * W + 1, 2 * H + 1
    fine = dict(nux=4 * b, nuy=b, h_u=1.0, b=float(b), thickness=1.0, tau=tau, kc=kc, beta=beta)
    return dict(nx0=n0, ny0=n0, bc0=2, boxes=boxes, fine=fine, finest=(nx, ny))


def graded_nodes(n: int, h_min: float, ratio: float, h_max: float, fine: float = 0.0) -> np.ndarray:
    """Node coordinates of a graded grid line centred at 0: spacing h_min
    out to |x| = fine, then growing by `ratio` per cell up to h_max. Odd n:
    a node sits at 0 (grid columns); even n: the two middle nodes sit at
    +-h_min/2 (grid rows around the lamina, whose thickness is h_min).
    Symmetric about 0."""
    odd = n % 2 == 1
    half = []
    x = 0.0 if odd else 0.5 * h_min
    h = h_min
    m = n // 2 + (1 if odd else 0)
    for _ in range(m):
        half.append(x)
        if x + 0.5 * h_min > fine:
            h = min(h * ratio, h_max)
        x += h
    half = np.array(half)
    if odd:
        return np.concatenate([-half[:0:-1], half])
    return np.concatenate([-half[::-1], half])


def random_populations(shape, seed: int, base: np.ndarray, spread: float = 0.02) -> np.ndarray:
    """base * (1 + u), u uniform in [-spread, spread]; base broadcasts over the
    trailing axes of ``shape`` (first axis = population index)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(-spread, spread, size=shape)
    b = np.asarray(base, dtype=np.float64).reshape((shape[0],) + (1,) * (len(shape) - 1))
    return b * (1.0 + u)


def random_field(shape, seed: int, lo: float, hi: float) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)
