"""The allocation-free state read, hlbm_get_state_noalloc, against
hlbm_get_state through the C ABI on the same handles: calls in a row on
successively smaller inputs (a lattice whose planes take several pieces of
the 64 MiB staging buffer, with a ragged last piece, then lamina cases), in
FP64, FP32 and FP16-deviation storage. The two reads must give the same
bits for the lattice and the grid."""
import ctypes as C

import numpy as np
import pytest

from paper_2006_13631_amd import hlbm as H
from paper_2006_13631_amd.workloads import preset, random_populations

pytestmark = pytest.mark.gpu

SCRATCH_DOUBLES = (64 << 20) // 8
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def _read(case, which, shape, noalloc):
    out = np.full(shape, np.nan)
    L = H.load()
    fn = L.hlbm_get_state_noalloc if noalloc else L.hlbm_get_state
    rc = fn(case.h, 0, which, out.ctypes.data, out.nbytes)
    assert rc == 0, L.hlbm_last_error(case.h).decode()
    return out


def _cases(storage):
    # a lattice-only case whose planes (4100 x 2050 nodes) exceed the staging
    # buffer: two pieces per plane, the second 16 392 values long
    yield dict(nx=4100, ny=2050, tau=0.8, storage=storage, max_steps=4), 3, True
    for name, steps in (("lamina_256x128", 40), ("tiny_ragged", 12)):
        cfg = preset(name)
        cfg.pop("steps")
        cfg.pop("ckpt_every", None)
        yield dict(max_steps=steps, storage=storage, **cfg), steps, False


@pytest.mark.parametrize("storage", [H.FP64, H.FP32, H.FP16_DEV])
def test_noalloc_read_matches_get_state(storage):
    sizes = []
    for cfg, steps, randomize in _cases(storage):
        print(f"# noalloc read: storage {storage} lattice {cfg['nx']}x{cfg['ny']} steps {steps}", flush=True)
        case = H.Case(**cfg)
        if randomize:
            assert cfg["nx"] * cfg["ny"] > SCRATCH_DOUBLES
            case.set_lattice(random_populations((9, cfg["ny"], cfg["nx"]), seed=7, base=W, spread=0.05))
        case.step(steps)
        shapes = [(H.STATE_LATTICE, (9, case.ny, case.nx))]
        if case.nnode:
            shapes.append((H.STATE_GRID, (9, case.nnode)))
        for which, shape in shapes:
            a = _read(case, which, shape, noalloc=False)
            b = _read(case, which, shape, noalloc=True)
            assert np.isfinite(a).all()
            assert np.array_equal(a, b), (which, float(np.max(np.abs(a - b))))
        sizes.append(case.nx * case.ny)
        case.close()
    assert sizes == sorted(sizes, reverse=True)


def test_noalloc_read_rejects_bad_arguments():
    cfg = preset("tiny_ragged")
    cfg.pop("steps")
    cfg.pop("ckpt_every", None)
    case = H.Case(max_steps=4, **cfg)
    L = H.load()
    out = np.zeros((9, case.ny, case.nx))
    assert L.hlbm_get_state_noalloc(case.h, 0, H.STATE_LATTICE, out.ctypes.data, out.nbytes - 8) == H.E_ARG
    assert L.hlbm_get_state_noalloc(case.h, 0, H.STATE_MOTION, out.ctypes.data, out.nbytes) == H.E_ARG
    assert L.hlbm_get_state_noalloc(case.h, 1, H.STATE_LATTICE, out.ctypes.data, out.nbytes) == H.E_ARG
    assert L.hlbm_get_state_noalloc(case.h, 0, H.STATE_LATTICE, None, out.nbytes) == H.E_ARG
    assert L.hlbm_get_state_noalloc(case.h, 0, H.STATE_LATTICE, out.ctypes.data, out.nbytes) == H.OK
    case.close()
