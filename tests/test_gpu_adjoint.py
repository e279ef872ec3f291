"""The GPU discrete adjoint (through the C ABI) against the oracle's
complex-step derivatives and against central differences of the GPU forward.

J = sum_k w_k . F(t_{k+1}) with seeded random weights w. Compared: dJ/dA,
dJ/domega, dJ/dtau (A, omega, tau independent) and the adjoint of the
initial state along seeded random directions of the lattice and of the grid
(each against the complex-step derivative along that direction). The
complex-step derivative is exact to rounding and follows the same discrete
decisions as the forward run, so the FP64 bar is rounding-level:
|gpu - oracle| <= 1e-9 |oracle| per number.
"""
import math
import os
import sys

import numpy as np
import pytest

from paper_2006_13631_amd import hlbm
from paper_2006_13631_amd.workloads import preset, random_populations

pytestmark = pytest.mark.gpu
TOL = 1e-9
H = 1e-30


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _cfg(name, **kw):
    c = preset(name, **kw)
    c.pop("steps")
    c.pop("ckpt_every", None)
    return c


def _weights(n, seed=11):
    return np.random.default_rng(seed).standard_normal((n, 2))


def _oracle_derivatives(oracle, c, n, w, f0=None, g0=None, dirs=()):
    """Complex-step dJ/dA, dJ/domega, dJ/dtau and dJ along each (lattice,
    grid) direction pair in dirs."""
    out = []
    runs = [((H, 0, 0), None), ((0, H, 0), None), ((0, 0, H), None)] + [((0, 0, 0), d) for d in dirs]
    for hv, d in runs:
        z = oracle.SimCS(*hv, max_steps=n, **c)
        if f0 is not None:
            z.set_lattice(f0, None if d is None else H * d[0])
            z.set_grid(g0, None if d is None else H * d[1])
        z.step(n)
        out.append(float(np.sum(w * z.history()[1])) / H)
    return np.array(out)


def _gpu_derivatives(c, n, w, f0=None, g0=None, dirs=(), ckpt=8, storage=hlbm.FP64):
    g = hlbm.Case(max_steps=n, ckpt_every=ckpt, storage=storage, **c)
    if f0 is not None:
        g.set_lattice(f0)
        g.set_grid(g0)
    g.step(n)
    grad = g.adjoint(w)
    out = list(grad)
    if dirs:
        lam_l, lam_g = g.adjoint_lattice(), g.adjoint_grid()
        for dl, dg in dirs:
            out.append(float(np.sum(lam_l * dl) + np.sum(lam_g * dg)))
    return np.array(out), g


def _compare(gpu, ref, tol=TOL, names=("A", "omega", "tau", "dir0", "dir1")):
    rel = np.abs(gpu - ref) / np.maximum(np.abs(ref), 1e-300)
    _say("gpu", gpu, "\noracle", ref, "\nrel", rel)
    for k, r in enumerate(rel):
        assert r <= tol, (names[k], gpu[k], ref[k], r)


def _random_state(oracle, c, seed):
    _, _, wq = oracle.d2q9()
    nn = c["nux"] * c["nuy"]
    f0 = random_populations((9, c["ny"], c["nx"]), seed=seed, base=wq, spread=0.01)
    g0 = random_populations((9, nn), seed=seed + 1, base=wq, spread=0.01)
    rng = np.random.default_rng(seed + 2)
    dirs = [(rng.standard_normal(f0.shape) * wq[:, None, None], np.zeros(g0.shape)),
            (np.zeros(f0.shape), rng.standard_normal(g0.shape) * wq[:, None])]
    return f0, g0, dirs


@pytest.mark.parametrize("n", [1, 3, 20])
def test_adjoint_few_steps_random_state(oracle, n):
    """Random start, few steps: parameters and both initial-state directions."""
    _say("adjoint tiny_adjoint random state, steps", n)
    c = _cfg("tiny_adjoint")
    f0, g0, dirs = _random_state(oracle, c, 40 + n)
    w = _weights(n)
    ref = _oracle_derivatives(oracle, c, n, w, f0, g0, dirs)
    gpu, _ = _gpu_derivatives(c, n, w, f0, g0, dirs, ckpt=8)
    _compare(gpu, ref)


def test_adjoint_full_run_from_rest(oracle):
    """Whole run from rest, several checkpoint windows and a ragged last one."""
    _say("adjoint full run tiny_adjoint")
    c = _cfg("tiny_adjoint")
    n = preset("tiny_adjoint")["steps"]
    w = _weights(n, 12)
    ref = _oracle_derivatives(oracle, c, n, w)
    gpu, _ = _gpu_derivatives(c, n, w, ckpt=8)
    _compare(gpu, ref)


def test_adjoint_at_a_tie(oracle):
    """tiny_ragged's grid stands still in step 13 (y_13 = y_14 exactly), so
    the top row lands exactly on old grid nodes. The value is the same in
    every triangle around such a node, its derivative along omega is not:
    the two sides may hold different triangles, and J is only one-sided
    differentiable in omega there. Along A the step stays zero (y_14 - y_13
    = A (sin 14 omega - sin 13 omega) = 0 for every A), and tau does not move
    the grid, so those two derivatives still agree to rounding."""
    _say("adjoint at a tie, tiny_ragged")
    c = _cfg("tiny_ragged")
    n = preset("tiny_ragged")["steps"]
    w = _weights(n, 12)
    ref = _oracle_derivatives(oracle, c, n, w)
    gpu, _ = _gpu_derivatives(c, n, w, ckpt=7)
    _compare(gpu[[0, 2]], ref[[0, 2]], names=("A", "tau"))


def test_adjoint_fine_grid_type2(oracle):
    """h_u = 0.2: many grid nodes per lattice cell, type-2 refills."""
    _say("adjoint tiny_fine_grid")
    c = _cfg("tiny_fine_grid")
    n = 16
    w = _weights(n, 13)
    ref = _oracle_derivatives(oracle, c, n, w)
    gpu, _ = _gpu_derivatives(c, n, w, ckpt=5)
    _compare(gpu, ref)


def _graded_cfg():
    """A lamina on a grid refined toward it (spacing 0.5 near the lamina,
    several grid rows per lattice cell, growing to 1.5)."""
    from paper_2006_13631_amd.workloads import graded_nodes
    return dict(nx=64, ny=48, nux=31, nuy=16, b=8.0, thickness=0.5, tau=0.8, kc=1.0, beta=20.0,
                x_nodes=graded_nodes(31, 0.5, 1.25, 1.5, fine=5.0), y_nodes=graded_nodes(16, 0.5, 1.3, 1.5))


@pytest.mark.parametrize("bc", [hlbm.BC_PERIODIC_X_WALLS_Y, hlbm.BC_PAPER])
def test_adjoint_graded_grid(oracle, bc):
    """Graded grid, random start: parameters and both initial-state
    directions over several checkpoint windows (the derivatives of the
    interpolation weights in y_k follow each cell's own height)."""
    _say("adjoint graded grid, bc", bc)
    c = dict(_graded_cfg(), bc=bc)
    n = 24
    f0, g0, dirs = _random_state(oracle, c, 71)
    w = _weights(n, 15)
    ref = _oracle_derivatives(oracle, c, n, w, f0, g0, dirs)
    gpu, _ = _gpu_derivatives(c, n, w, f0, g0, dirs, ckpt=7)
    _compare(gpu, ref)


def test_adjoint_graded_grid_from_rest(oracle):
    """Graded grid from rest over 150 steps (the grid moves through its
    fine rows and the lamina sheds vorticity)."""
    _say("adjoint graded grid from rest")
    c = _graded_cfg()
    n = 150
    w = _weights(n, 16)
    ref = _oracle_derivatives(oracle, c, n, w)
    gpu, _ = _gpu_derivatives(c, n, w, ckpt=32)
    _compare(gpu, ref)


def test_adjoint_periodic_bc(oracle):
    _say("adjoint periodic bc")
    c = _cfg("tiny_adjoint", bc=hlbm.BC_PERIODIC)
    n = 30
    w = _weights(n, 14)
    ref = _oracle_derivatives(oracle, c, n, w)
    gpu, _ = _gpu_derivatives(c, n, w, ckpt=16)
    _compare(gpu, ref)


def test_adjoint_paper_boundaries(oracle):
    """The paper's outer boundaries (no-slip x walls, outflow y ends), random
    start: parameters, the grid direction, a lattice direction over the
    whole lattice and one confined to the two rows at each outflow end and
    the wall columns (the rows whose sources have two readers or none)."""
    _say("adjoint, paper boundaries")
    c = _cfg("tiny_adjoint", bc=hlbm.BC_PAPER)
    n = 30
    f0, g0, dirs = _random_state(oracle, c, 61)
    _, _, wq = oracle.d2q9()
    rng = np.random.default_rng(64)
    edge = np.zeros(f0.shape)
    edge[:, [0, 1, -2, -1], :] = rng.standard_normal((9, 4, c["nx"])) * wq[:, None, None]
    edge[:, :, [0, -1]] = rng.standard_normal((9, c["ny"], 2)) * wq[:, None, None]
    dirs = dirs + [(edge, np.zeros(g0.shape))]
    w = _weights(n, 17)
    ref = _oracle_derivatives(oracle, c, n, w, f0, g0, dirs)
    gpu, _ = _gpu_derivatives(c, n, w, f0, g0, dirs, ckpt=8)
    _compare(gpu, ref, names=("A", "omega", "tau", "lattice", "grid", "edges"))


@pytest.mark.timeout(900)
def test_adjoint_lamina_128x64_copy(oracle):
    """The 128 x 64 copy of the differentiation case as specified: all 4000
    steps, twenty 200-step checkpoint windows (the oracle's complex-step runs
    use every host core)."""
    _say("adjoint lamina_128x64, 4000 steps")
    c = _cfg("lamina_128x64")
    n = 4000
    w = _weights(n, 15)
    oracle.lib_cs().or_set_threads(min(16, len(os.sched_getaffinity(0))))
    try:
        ref = _oracle_derivatives(oracle, c, n, w)
    finally:
        oracle.lib_cs().or_set_threads(1)
    gpu, g = _gpu_derivatives(c, n, w, ckpt=200)
    assert g.info().step == 4000
    _compare(gpu, ref)


def test_adjoint_matches_gpu_central_differences():
    """Central differences of the GPU forward in (KC, beta, tau), relative
    step 1e-6, against the adjoint combined by A = KC b/(2 pi),
    omega = 2 pi nu beta / b^2, nu = (tau - 1/2)/3."""
    _say("adjoint vs GPU central differences")
    c = _cfg("tiny_adjoint")
    n = 60
    w = _weights(n, 16)
    gpu, case = _gpu_derivatives(c, n, w, ckpt=20)
    inf = case.info()
    b, tau, om = c["b"], c["tau"], inf.omega
    want = {"kc": gpu[0] * b / (2 * math.pi), "beta": gpu[1] * om / c["beta"],
            "tau": gpu[2] + gpu[1] * om / (tau - 0.5)}

    def J(**kw):
        cc = dict(c)
        cc.update(kw)
        g = hlbm.Case(max_steps=n, **cc)
        g.step(n)
        return float(np.sum(w * g.history()))
    for key, v in want.items():
        e = 1e-6 * c[key]
        fd = (J(**{key: c[key] + e}) - J(**{key: c[key] - e})) / (2 * e)
        _say(key, "fd", fd, "adjoint", v)
        assert abs(fd - v) <= 1e-6 * abs(v), (key, fd, v)


def test_adjoint_is_reproducible_and_leaves_forward_state():
    _say("adjoint reproducibility")
    c = _cfg("tiny_adjoint")
    w = _weights(30, 17)
    g = hlbm.Case(max_steps=60, ckpt_every=8, **c)
    g.step(30)
    a1 = g.adjoint(w)
    a2 = g.adjoint(w)
    assert np.array_equal(a1, a2)
    g.step(30)
    ref = hlbm.Case(max_steps=60, **c)
    ref.step(60)
    assert np.array_equal(g.history(), ref.history())
    assert np.array_equal(g.lattice(), ref.lattice())


def test_adjoint_timing_records_substep_launches():
    """With timing on, hlbm_adjoint times the lattice adjoint and the first
    reverse sub-step launch of every step by their own events, and the
    gradient is the untimed one bit for bit."""
    _say("adjoint timing")
    c = _cfg("tiny_adjoint")
    w = _weights(30, 17)
    g = hlbm.Case(max_steps=30, ckpt_every=8, **c)
    g.step(30)
    a0 = g.adjoint(w)
    g.timing(1)
    a1 = g.adjoint(w)
    ms, n = g.timing_get(hlbm.K_ADJ_SUBSTEPS)
    ms_l, n_l = g.timing_get(hlbm.K_ADJ_STREAM_COLLIDE)
    g.timing(0)
    assert np.array_equal(a0, a1)
    assert n == 30 and n_l == 30 and ms > 0 and ms_l > 0


def test_adjoint_errors():
    c = _cfg("tiny_adjoint")
    g = hlbm.Case(max_steps=10, **c)
    g.step(4)
    with pytest.raises(hlbm.HlbmError) as e:
        g.adjoint(np.ones((4, 2)))
    assert e.value.code == hlbm.E_STATE
    g = hlbm.Case(max_steps=10, ckpt_every=4, **c)
    g.step(4)
    with pytest.raises(hlbm.HlbmError) as e:
        g.adjoint(np.ones((3, 2)))
    assert e.value.code == hlbm.E_ARG
    with pytest.raises(hlbm.HlbmError) as e:
        g.adjoint_lattice()
    assert e.value.code == hlbm.E_STATE
    g.set_grid(g.grid())
    with pytest.raises(hlbm.HlbmError) as e:
        g.adjoint(np.ones((4, 2)))
    assert e.value.code == hlbm.E_STATE


@pytest.mark.parametrize("storage,tol", [(hlbm.FP32, 2e-3), (hlbm.FP16_DEV, 5e-2)])
def test_reduced_precision_adjoint(storage, tol):
    """FP32 and FP16-deviation storage: the adjoint (in FP32 arithmetic)
    against the FP64 adjoint of the same run."""
    _say("reduced precision adjoint", storage)
    c = _cfg("lamina_128x64")
    n = 400
    w = _weights(n, 18)
    g64, _ = _gpu_derivatives(c, n, w, ckpt=100)
    glo, _ = _gpu_derivatives(c, n, w, ckpt=100, storage=storage)
    rel = np.abs(glo - g64) / np.abs(g64)
    _say("f64", g64, "reduced", glo, "rel", rel)
    assert np.all(rel <= tol), rel
