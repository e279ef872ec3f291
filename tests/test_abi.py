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
