"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/hlbm.h declares, its structs have the layout the
binding assumes, and invalid configurations are rejected before any device
work."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2006_13631_amd import hlbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hlbm.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(hlbm_[a-z_]+)\s*\(", text)))


def test_header_declares_binding_exports():
    assert sorted(hlbm.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(hlbm.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", hlbm.LIB_PATH], capture_output=True, text=True)
    exported = set(re.findall(r"\bT (hlbm_\w+)", out.stdout))
    assert set(_declared()) <= exported


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "hlbm.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(hlbm_config),'
                   ' offsetof(hlbm_config, max_steps), sizeof(hlbm_info), offsetof(hlbm_info, lattice_bytes),'
                   ' offsetof(hlbm_info, status), sizeof(hlbm_tuning), offsetof(hlbm_tuning, ms_per_step),'
                   ' offsetof(hlbm_tuning, substep_variant), offsetof(hlbm_tuning, lattice_rows));'
                   'return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    a, b, c, d, e, f, g, h, i = map(int, subprocess.check_output([str(exe)]).split())
    assert a == C.sizeof(hlbm.Config) and b == hlbm.Config.max_steps.offset
    assert c == C.sizeof(hlbm.Info) and d == hlbm.Info.lattice_bytes.offset
    assert e == hlbm.Info.status.offset
    assert f == C.sizeof(hlbm.Tuning) and g == hlbm.Tuning.ms_per_step.offset
    assert h == hlbm.Tuning.substep_variant.offset and i == hlbm.Tuning.lattice_rows.offset


@pytest.mark.parametrize("bad", [
    dict(tau=0.5),                       # tau must exceed 1/2
    dict(nuy=31),                        # odd grid height
    dict(thickness=2.0),                 # thickness must equal h_u
    dict(ny=36),                         # grid motion leaves the lattice
    dict(b=60.0),                        # lamina wider than the fictitious rectangle
    dict(n_sub=1, tau=0.8),              # Delta t_u = 1 > 2 tau_u = 0.6
    dict(storage=7),
    dict(bc=5),
])
def test_invalid_configuration_rejected_on_host(bad):
    cfg = dict(nx=256, ny=128, nux=64, nuy=32, h_u=1.0, b=32.0, thickness=1.0, tau=0.8, kc=0.5,
               beta=100.0, max_steps=10)
    cfg.update(bad)
    with pytest.raises(hlbm.HlbmError) as ei:
        hlbm.Case(**cfg)
    assert ei.value.code == hlbm.E_ARG


def _cfg_struct(**kw):
    c = dict(nx=256, ny=128, nux=64, nuy=32, h_u=1.0, b=32.0, thickness=1.0, tau=0.8, kc=0.5,
             beta=100.0, n_sub=0, bc=0, storage=hlbm.FP64, flags=0, ckpt_every=0, reserved=0, max_steps=10)
    c.update(kw)
    return hlbm.Config(*[c[k] for k, _ in hlbm.Config._fields_])


@pytest.mark.parametrize("second", [dict(storage=hlbm.FP32), dict(ckpt_every=5), dict(nux=0, nuy=0),
                                    dict(tau=0.4)])
def test_invalid_batch_rejected_on_host(second):
    """Batches are validated on the host before any device work."""
    arr = (hlbm.Config * 2)(_cfg_struct(), _cfg_struct(**second))
    h = C.c_void_p()
    rc = hlbm.load().hlbm_create(arr, 2, C.byref(h))
    assert rc == hlbm.E_ARG and not h.value
    assert b"case 1" in hlbm.load().hlbm_last_error(None) or second.get("storage") is not None \
        or second.get("ckpt_every") or second.get("nux") == 0


def test_levels_struct_layout(tmp_path):
    src = tmp_path / "levels.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "hlbm.h"\n'
                   'int main(void){printf("%zu %zu %d\\n", sizeof(hlbm_levels), offsetof(hlbm_levels, box),'
                   ' HLBM_STATE_LEVEL); return 0;}\n')
    exe = tmp_path / "levels"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    a, b, c = map(int, subprocess.check_output([str(exe)]).split())
    assert a == C.sizeof(hlbm.Levels) and b == hlbm.Levels.box.offset and c == hlbm.STATE_LEVEL


def test_ring_boundaries_only_in_a_multilevel_handle():
    with pytest.raises(hlbm.HlbmError) as ei:
        hlbm.Case(nx=33, ny=33, tau=0.8, bc=hlbm.BC_RING)
    assert ei.value.code == hlbm.E_ARG


@pytest.mark.parametrize("boxes,extra", [
    ([(1, 4, 12, 12)], {}),               # box too close to level 0's edge
    ([(4, 4, 7, 12)], {}),                # box fewer than four cells wide
    ([(4, 4, 14, 12)], {}),               # box beyond nx - 3
    ([(4, 4, 12, 12)] * 8, {}),           # nine levels
    ([(4, 4, 12, 12)], {"tau": 0.5}),     # invalid finest configuration
])
def test_invalid_levels_rejected_on_host(boxes, extra):
    with pytest.raises(hlbm.HlbmError) as ei:
        hlbm.MultiLevel(16, 16, boxes, **dict(dict(tau=0.8), **extra))
    assert ei.value.code == hlbm.E_ARG


def test_multilevel_finest_shape_and_bc_checked_on_host():
    L = hlbm.load()
    lv = hlbm.Levels()
    lv.nlevels, lv.nx0, lv.ny0, lv.bc0 = 2, 16, 16, 0
    for i, v in enumerate((4, 4, 12, 12)):
        lv.box[0][i] = v
    h = C.c_void_p()
    for kw in (dict(nx=16, ny=17, bc=hlbm.BC_RING), dict(nx=17, ny=17, bc=0),
               dict(nx=17, ny=17, bc=hlbm.BC_RING, ckpt_every=4)):
        cfg = _cfg_struct(nux=0, nuy=0, b=0.0, **kw)
        assert L.hlbm_create_multilevel(C.byref(cfg), C.byref(lv), C.byref(h)) == hlbm.E_ARG
        assert not h.value
    cfg = _cfg_struct(nx=17, ny=17, nux=0, nuy=0, b=0.0, bc=hlbm.BC_RING)
    for n in (1, 9):
        lv.nlevels = n
        assert L.hlbm_create_multilevel(C.byref(cfg), C.byref(lv), C.byref(h)) == hlbm.E_ARG


def test_motion_struct_layout(tmp_path):
    src = tmp_path / "motion.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "hlbm.h"\n'
                   'int main(void){printf("%zu %zu %d\\n", sizeof(hlbm_motion), offsetof(hlbm_motion, y_max),'
                   ' HLBM_STATE_MOTION); return 0;}\n')
    exe = tmp_path / "motion"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    a, b, c = map(int, subprocess.check_output([str(exe)]).split())
    assert a == C.sizeof(hlbm.Motion) and b == hlbm.Motion.y_max.offset and c == hlbm.STATE_MOTION


def test_graded_configuration_checked_on_host():
    from paper_2006_13631_amd.workloads import graded_nodes
    gx, gy = graded_nodes(31, 0.5, 1.25, 1.5, fine=5.0), graded_nodes(16, 0.5, 1.3, 1.5)
    cfg = dict(nx=64, ny=48, nux=31, nuy=16, b=8.0, thickness=0.5, tau=0.8, kc=1.0, beta=20.0, max_steps=4)
    for bad in (dict(y_nodes=gy + 0.1), dict(x_nodes=gx[::-1].copy()), dict(x_nodes=gx * 4)):
        kw = dict(x_nodes=gx, y_nodes=gy)
        kw.update(bad)
        with pytest.raises(hlbm.HlbmError) as ei:
            hlbm.Case(**cfg, **kw)
        assert ei.value.code == hlbm.E_ARG
