"""The oracle's per-node loops may run on several host threads: nodes are
independent within a step (each writes only its own populations and reads
the previous step's), and every reduction (wall force, Theta fit) stays
serial, so the results must be bitwise identical for any thread count."""
import numpy as np

from oracle import oracle as O


def _run(threads, cs=False):
    O.set_threads(threads)
    O.lib_cs().or_set_threads(threads)
    kw = dict(nx=80, ny=48, nux=40, nuy=10, b=10.0, tau=0.8, kc=0.3, beta=10.0,
              bc=O.BC_PERIODIC_X_WALLS_Y, max_steps=40)
    s = O.SimCS(1e-20, 0.0, 0.0, **kw) if cs else O.Sim(**kw)
    s.step(40)
    return s.lattice(), s.grid(), s.history()


def test_serial_by_default():
    assert O.set_threads(0) == 1


def test_thread_count_does_not_change_results():
    try:
        one = _run(1)
        many = _run(4)
    finally:
        O.set_threads(1)
        O.lib_cs().or_set_threads(1)
    for a, b in zip(one, many):
        assert np.array_equal(a, b)


def test_thread_count_does_not_change_complex_step_results():
    try:
        one = _run(1, cs=True)
        many = _run(3, cs=True)
    finally:
        O.set_threads(1)
        O.lib_cs().or_set_threads(1)
    for a, b in zip(one, many):
        assert np.array_equal(a, b)
