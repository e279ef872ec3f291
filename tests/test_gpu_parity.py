"""Parity of the HIP library (through the C ABI) with the FP64 CPU oracle.

Both sides start from the same seeded inputs (workloads module) and are
compared element by element. FP64 bar (the parity norm of the design notes):
    max|f_gpu - f_oracle| / max|f_oracle| <= 1e-12 over lattice and grid, and
    max_k|F_gpu - F_oracle| / max_k|F_oracle| <= 1e-12 over the force history.
The same differences are also measured against the flow's signal, the
largest deviation from the rest state, max|f_oracle - w_i| (a hundred to a
few thousand times smaller than max|f| in these cases), with the bar
1e-10: the FP64 differences stay at rounding level relative to what the
flow carries, not only relative to the rest weights. A part whose largest
deviation is below 1e-8 max|f| (still at rest to rounding, e.g. the
lattice in the first steps of a large case) has no signal to compare with;
there only the first bar applies.
"""
import math
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2006_13631_amd import hlbm
from paper_2006_13631_amd.workloads import preset, random_populations

pytestmark = pytest.mark.gpu
TOL = 1e-12
TOL_DEV = 1e-10
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _pair(oracle, cfg, steps=None, storage=hlbm.FP64, **kw):
    c = dict(cfg)
    c.update(kw)
    n = c.pop("steps")
    c.pop("ckpt_every", None)
    cap = steps if steps is not None else n
    o = oracle.Sim(max_steps=cap, **c)
    g = hlbm.Case(max_steps=cap, storage=storage, **c)
    return o, g, cap


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _rel_dev(a, b):
    """max|a - b| relative to the largest deviation of b from the rest
    state w_i (populations first: [9, ...]); None where that deviation is
    below 1e-8 max|b| (no flow signal above rounding)."""
    dev = float(np.max(np.abs(b - W.reshape((9,) + (1,) * (b.ndim - 1)))))
    if dev < 1e-8 * float(np.max(np.abs(b))):
        return None
    return float(np.max(np.abs(a - b)) / dev)


def _check_state(o, g, tol=TOL, hist=True, tol_dev=TOL_DEV):
    lo, lg = o.lattice(), g.lattice()
    errs = {"lattice": _rel(lg, lo)}
    devs = {"lattice": _rel_dev(lg, lo)}
    if o.nnode:
        go, gg = o.grid(), g.grid()
        errs["grid"] = _rel(gg, go)
        devs["grid"] = _rel_dev(gg, go)
        if hist:
            ho, hg = o.history(), g.history()
            assert ho.shape == hg.shape
            errs["force"] = _rel(hg, ho)
    _say("parity errors", errs, "relative to the deviation from rest", devs)
    for k, e in errs.items():
        assert e <= tol, (k, e)
    for k, e in devs.items():
        assert e is None or e <= tol_dev, (k, "relative to the deviation", e)
    return errs


def _sparse(nbr, M):
    N = nbr.shape[0]
    rows = np.repeat(np.arange(N), nbr.shape[1])
    cols = nbr.ravel()
    keep = cols >= 0
    return sp.csr_matrix((M.ravel()[keep], (rows[keep], cols[keep])), shape=(N, N))


@pytest.mark.parametrize("name", ["lamina_256x128", "tiny_ragged", "tiny_fine_grid", "lamina_128x64"])
def test_stencil_matches_oracle(oracle, name):
    _say("stencil", name)
    cfg = preset(name)
    o, g, _ = _pair(oracle, cfg, steps=1)
    nbr_g, S_g, C_g = g.stencil(8)
    nbr_o, S_o, C_o, _ = o.mesh().stencil()
    assert abs(_sparse(nbr_g, C_g) - _sparse(nbr_o, C_o)).max() < 1e-13
    smax = np.abs(S_o).max()  # S scales as 1/h_u
    for q in range(9):
        assert abs(_sparse(nbr_g, S_g[:, q, :]) - _sparse(nbr_o, S_o[:, q, :])).max() < 1e-13 * smax
    assert g.info().n_classes < 200


@pytest.mark.parametrize("bc", [hlbm.BC_PERIODIC_X_WALLS_Y, hlbm.BC_PERIODIC, hlbm.BC_PAPER])
def test_lattice_only_random_state(oracle, bc):
    """Eq.(LBE) alone on a ragged 77 x 45 lattice from a random state."""
    _say("lattice only bc", bc)
    nx, ny = 77, 45
    _, _, w = oracle.d2q9()
    f0 = random_populations((9, ny, nx), seed=5, base=w, spread=0.05)
    g = hlbm.Case(nx, ny, tau=0.62, bc=bc)
    g.set_lattice(f0)
    g.step(25)
    f = f0
    for _ in range(25):
        f = oracle.lattice_step(f, 0.62, bc=bc)
    assert _rel(g.lattice(), f) <= TOL


def test_lamina_256x128_full_run(oracle):
    """The 256 x 128 lamina case, 2000 steps: force history and final
    distributions of both grids."""
    _say("lamina_256x128 2000 steps")
    o, g, n = _pair(oracle, preset("lamina_256x128"))
    for _ in range(4):
        o.step(n // 4)
        g.step(n // 4)
        _check_state(o, g)
    io, ig = o.info(), g.info()
    assert (ig.n_type1, ig.n_type2, ig.n_type3) == (io.n_type1, io.n_type2, io.n_type3)
    th_o = oracle.fit_theta(o.history(), io.omega, io.A, 32.0)
    th_g = g.theta()
    _say("theta", th_g, th_o)
    assert abs(th_g - th_o) <= 1e-11 * abs(th_o)


def test_ragged_random_state(oracle):
    """Odd grid width, ragged lattice, random start on both grids."""
    _say("tiny_ragged random state")
    cfg = preset("tiny_ragged")
    o, g, n = _pair(oracle, cfg)
    _, _, w = oracle.d2q9()
    fl = random_populations((9, cfg["ny"], cfg["nx"]), seed=21, base=w, spread=0.01)
    fg = random_populations((9, o.nnode), seed=22, base=w, spread=0.01)
    for s in (o, g):
        s.set_lattice(fl)
        s.set_grid(fg)
    o.step(n)
    g.step(n)
    _check_state(o, g)


def test_fine_grid_with_type2_refill(oracle):
    """Grid spacing 0.2 below the per-step displacement: type-2 refill."""
    _say("tiny_fine_grid")
    o, g, n = _pair(oracle, preset("tiny_fine_grid"))
    o.step(n)
    g.step(n)
    _check_state(o, g)
    assert g.info().n_type2 == o.info().n_type2 > 0


def test_periodic_lattice_with_body(oracle):
    _say("periodic bc with lamina")
    o, g, n = _pair(oracle, preset("tiny_ragged"), bc=hlbm.BC_PERIODIC)
    o.step(n)
    g.step(n)
    _check_state(o, g)


def test_paper_boundaries_with_body(oracle):
    """No-slip x walls and outflow y ends around the lamina, random start on
    both grids (ragged lattice, odd grid width)."""
    _say("paper boundaries with lamina")
    cfg = preset("tiny_ragged")
    o, g, n = _pair(oracle, cfg, bc=hlbm.BC_PAPER)
    _, _, w = oracle.d2q9()
    fl = random_populations((9, cfg["ny"], cfg["nx"]), seed=31, base=w, spread=0.01)
    fg = random_populations((9, o.nnode), seed=32, base=w, spread=0.01)
    for s in (o, g):
        s.set_lattice(fl)
        s.set_grid(fg)
    o.step(n)
    g.step(n)
    _check_state(o, g)


def test_paper_study_case(oracle):
    """A case of the paper's (epsilon, beta) study at a small size: 5L x 5L
    domain with the paper's boundaries, grid 4L x L."""
    from paper_2006_13631_amd.workloads import paper_study_cases
    c = [c for c in paper_study_cases(b=16) if c["eps"] == 0.1 and c["beta_p"] == 20][0]
    cfg = {k: v for k, v in c.items() if k not in ("eps", "beta_p", "max_steps")}
    _say("paper study case", cfg)
    o, g, _ = _pair(oracle, dict(cfg, steps=300))
    o.step(300)
    g.step(300)
    _check_state(o, g)


def test_uniform_flow_no_body_invariant(oracle):
    """GPU alone: uniform flow stays uniform with an oscillating grid."""
    _say("uniform flow")
    g = hlbm.Case(64, 48, 24, 16, 1.0, 8.0, 1.0, 0.7, 1.0, 20.0, bc=hlbm.BC_PERIODIC,
                  flags=hlbm.FLAG_NO_BODY, max_steps=40)
    e = oracle.feq(1.0, 0.03, -0.02)
    g.set_lattice(np.broadcast_to(e[:, None, None], (9, 48, 64)).copy())
    g.set_grid(np.broadcast_to(e[:, None], (9, g.nnode)).copy())
    g.step(40)
    assert np.max(np.abs(g.lattice() - e[:, None, None])) < 1e-14
    assert np.max(np.abs(g.grid() - e[:, None])) < 1e-14


@pytest.mark.timeout(600)
def test_lamina_2048_first_steps(oracle):
    """The 2048^2 lamina case at full size, in the configuration the
    benchmark times, over its first steps (whole-array comparison)."""
    _say("lamina_2048 3 steps")
    o, g, _ = _pair(oracle, preset("lamina_2048"), steps=3)
    o.step(3)
    g.step(3)
    _check_state(o, g)


def _host_threads():
    import os
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    return min(n, int(env)) if env.isdigit() and int(env) > 0 else n


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name,steps,schedule", [
    # the schedule the autotuner picks for the 2048^2 FP64 benchmark line
    ("lamina_2048", 202, dict(variant=1, lattice=(128, 1), order=3)),
    # and for the 4096^2 FP64 precision line
    ("lamina_4096", 26, dict(variant=9, lattice=(256, 1), order=2)),
])
def test_full_size_in_benchmark_configuration(oracle, name, steps, schedule):
    """The benchmark workloads at full size in the launch configuration the
    benchmark times: its tuned schedule, pairs of steps on the two-step
    lattice path, and 8 steps per HIP graph replayed from several buffer
    arrangements, ending on a pair. Over 202 steps the 2048^2 grid moves
    about 20 lattice units, through every kind of refill. Whole-array
    comparison. The oracle runs its per-node loops on every host core,
    which leaves its bits unchanged."""
    _say(name, steps, "steps, schedule", schedule)
    oracle.set_threads(_host_threads())
    try:
        o, g, _ = _pair(oracle, preset(name), steps=steps)
        t = g.tune(**schedule)
        assert t["substep_variant"] == schedule["variant"]
        assert g.info().two_step == 1
        o.step(steps)
        g.step(steps)
        _check_state(o, g)
    finally:
        oracle.set_threads(1)


@pytest.mark.parametrize("storage,tol", [(hlbm.FP32, 2e-3), (hlbm.FP16_DEV, 3e-2)])
def test_reduced_precision_theta(storage, tol):
    """FP32 and FP16-deviation storage against the FP64 run of the
    256 x 128 lamina case: relative error of Theta."""
    _say("precision", storage)
    cfg = preset("lamina_256x128")
    ref = hlbm.case_from_preset(cfg)
    ref.step(cfg["steps"])
    low = hlbm.case_from_preset(cfg, storage=storage)
    low.step(cfg["steps"])
    t64, tlo = ref.theta(), low.theta()
    _say("theta f64", t64, "reduced", tlo, "rel", abs(tlo - t64) / abs(t64))
    assert abs(tlo - t64) <= tol * abs(t64)


def test_fp32_state_full_run(oracle):
    """FP32 storage and arithmetic against the FP64 oracle over the whole
    2 000 steps of the 256 x 128 lamina case. Bar: the differences stay
    below N u_32 max|f| (N = 2 000 steps, u_32 = 2^-24): rounding that
    accumulates at most linearly, not an error that grows with the flow."""
    cfg = preset("lamina_256x128")
    n = cfg["steps"]
    _say("fp32 full run", n)
    o, g, _ = _pair(oracle, cfg, storage=hlbm.FP32)
    o.step(n)
    g.step(n)
    bound = n * 2.0 ** -24
    errs = {"lattice": _rel(g.lattice(), o.lattice()), "grid": _rel(g.grid(), o.grid()),
            "force": _rel(g.history(), o.history())}
    devs = {"lattice": _rel_dev(g.lattice(), o.lattice()), "grid": _rel_dev(g.grid(), o.grid())}
    _say("errors", errs, "relative to the deviation from rest", devs, "bound", bound)
    assert max(errs["lattice"], errs["grid"]) <= bound, errs


@pytest.mark.parametrize("storage,tol", [(hlbm.FP32, 2e-6), (hlbm.FP16_DEV, 2e-4)])
@pytest.mark.parametrize("name", ["tiny_ragged", "lamina_256x128"])
def test_reduced_precision_state(oracle, storage, tol, name):
    """FP32 and FP16-deviation storage against the FP64 oracle over the first
    steps: largest deviation of either grid relative to max|f|."""
    _say("reduced precision state", name, storage)
    o, g, _ = _pair(oracle, preset(name), steps=20, storage=storage)
    o.step(20)
    g.step(20)
    errs = {"lattice": _rel(g.lattice(), o.lattice()), "grid": _rel(g.grid(), o.grid())}
    _say("errors", errs)
    assert max(errs.values()) <= tol, errs
