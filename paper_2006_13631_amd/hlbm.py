"""Thin ctypes binding of ``libhlbm.so`` (include/hlbm.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels. There is no fallback; a missing library raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhlbm.so")

OK, E_ARG, E_NOMEM, E_HIP, E_UNSTABLE, E_STATE, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
BC_PERIODIC_X_WALLS_Y, BC_PERIODIC, BC_PAPER, BC_RING = 0, 1, 2, 3
FP64, FP32, FP16_DEV = 0, 1, 2
FLAG_NO_BODY = 1
STATE_LATTICE, STATE_GRID, STATE_ADJ_LATTICE, STATE_ADJ_GRID = 0, 1, 2, 3
STATE_MOTION = 4
STATE_LEVEL = 16
MAX_LEVELS = 8
(K_STREAM_COLLIDE, K_LATTICE_FROM_GRID, K_GRID_SUBSTEPS, K_REFILL, K_FORCE, K_STEP,
 K_ADJ_STREAM_COLLIDE, K_ADJOINT, K_SUBSTEP_LAUNCH, K_ADJ_SUBSTEPS) = range(10)
STORAGE = {"f64": FP64, "f32": FP32, "f16dev": FP16_DEV}

EXPORTS = ("hlbm_create", "hlbm_step", "hlbm_force", "hlbm_adjoint", "hlbm_get_state",
           "hlbm_set_state", "hlbm_info_get", "hlbm_get_stencil", "hlbm_timing",
           "hlbm_timing_get", "hlbm_tune", "hlbm_destroy", "hlbm_last_error",
           "hlbm_create_multilevel", "hlbm_level_shape", "hlbm_set_motion", "hlbm_create_graded",
           "hlbm_create_mesh", "hlbm_set_deformation",
           "hlbm_get_state_noalloc", "hlbm_step_async", "hlbm_sync")
STATUS_RUNNING, STATUS_DONE, STATUS_UNSTABLE = 0, 1, 2


class HlbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class Config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nux", C.c_int32), ("nuy", C.c_int32),
                ("h_u", C.c_double), ("b", C.c_double), ("thickness", C.c_double),
                ("tau", C.c_double), ("kc", C.c_double), ("beta", C.c_double),
                ("n_sub", C.c_int32), ("bc", C.c_int32), ("storage", C.c_int32),
                ("flags", C.c_int32), ("ckpt_every", C.c_int32), ("reserved", C.c_int32),
                ("max_steps", C.c_int64)]


class Info(C.Structure):
    _fields_ = [(n, C.c_double) for n in
                ("nu", "tau_u", "dt_u", "A", "omega", "period", "u_max", "mach", "reynolds", "eps")] + \
               [(n, C.c_int32) for n in
                ("n_sub", "nnode", "ntri", "n_interface", "n_wall", "n_wall_edges", "beta_limit_ok",
                 "n_classes")] + \
               [("step", C.c_int64), ("y", C.c_double), ("n_type1", C.c_int64),
                ("n_type2", C.c_int64), ("n_type3", C.c_int64), ("lattice_bytes", C.c_int64),
                ("status", C.c_int32), ("two_step", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("steps_per_graph", C.c_int32), ("lattice_threads", C.c_int32),
                ("lattice_rows", C.c_int32), ("substep_variant", C.c_int32), ("order", C.c_int32),
                ("tail_variant", C.c_int32), ("persistent", C.c_int32), ("persistent_groups", C.c_int32),
                ("ms_per_step", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Motion(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("mass", "stiffness", "damping", "y0", "v0", "y_max")]


class Levels(C.Structure):
    _fields_ = [("nlevels", C.c_int32), ("nx0", C.c_int32), ("ny0", C.c_int32), ("bc0", C.c_int32),
                ("box", (C.c_int32 * 4) * (MAX_LEVELS - 1))]


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it with paper_2006_13631_amd/build.py")
    L = C.CDLL(path)
    vp, d, i32, i64 = C.c_void_p, C.c_double, C.c_int32, C.c_int64
    dp = C.POINTER(C.c_double)
    L.hlbm_create.argtypes = [C.POINTER(Config), i32, C.POINTER(vp)]
    L.hlbm_step.argtypes = [vp, i64]
    L.hlbm_step_async.argtypes = [vp, i64]
    L.hlbm_sync.argtypes = [vp]
    L.hlbm_force.argtypes = [vp, i32, dp, i64, C.POINTER(i64), d, d, dp]
    L.hlbm_adjoint.argtypes = [vp, i32, dp, i64, dp]
    L.hlbm_get_state.argtypes = [vp, i32, i32, vp, C.c_size_t]
    L.hlbm_set_state.argtypes = [vp, i32, i32, vp, C.c_size_t]
    L.hlbm_get_state_noalloc.argtypes = [vp, i32, i32, vp, C.c_size_t]
    L.hlbm_info_get.argtypes = [vp, i32, C.POINTER(Info)]
    L.hlbm_get_stencil.argtypes = [vp, i32, C.POINTER(C.c_int32), dp, dp]
    L.hlbm_timing.argtypes = [vp, i32]
    L.hlbm_timing_get.argtypes = [vp, i32, dp, C.POINTER(i64)]
    L.hlbm_tune.argtypes = [vp, i32, C.POINTER(Tuning)]
    L.hlbm_create_multilevel.argtypes = [C.POINTER(Config), C.POINTER(Levels), C.POINTER(vp)]
    L.hlbm_level_shape.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i32), dp]
    L.hlbm_set_motion.argtypes = [vp, i32, C.POINTER(Motion)]
    L.hlbm_set_deformation.argtypes = [vp, C.c_double, C.c_double]
    L.hlbm_create_graded.argtypes = [C.POINTER(Config), dp, dp, C.POINTER(vp)]
    L.hlbm_create_mesh.argtypes = [C.POINTER(Config), i32, dp, C.POINTER(i32), i32, C.POINTER(i32),
                                   C.POINTER(vp)]
    L.hlbm_destroy.argtypes = [vp]
    L.hlbm_destroy.restype = None
    L.hlbm_last_error.argtypes = [vp]
    L.hlbm_last_error.restype = C.c_char_p
    _lib = L
    return L


def _ptr(a, t=C.c_double):
    return a.ctypes.data_as(C.POINTER(t))


class Case:
    """One lamina case on the GPU."""

    def __init__(self, nx, ny, nux=0, nuy=0, h_u=1.0, b=0.0, thickness=1.0, tau=0.8, kc=0.0,
                 beta=0.0, n_sub=0, bc=BC_PERIODIC_X_WALLS_Y, storage=FP64, flags=0,
                 ckpt_every=0, max_steps=0, x_nodes=None, y_nodes=None, mesh=None):
        L = load()
        if isinstance(storage, str):
            storage = STORAGE[storage]
        self.cfg = Config(nx, ny, nux, nuy, h_u, b, thickness, tau, kc, beta, n_sub, bc, storage,
                          flags, ckpt_every, 0, max_steps)
        h = C.c_void_p()
        if mesh is not None:  # any triangulation: (xy [n, 2], node types [n], triangles [m, 3])
            xy = np.ascontiguousarray(mesh[0], dtype=np.float64)
            ty = np.ascontiguousarray(mesh[1], dtype=np.int32)
            tri = np.ascontiguousarray(mesh[2], dtype=np.int32)
            if xy.ndim != 2 or xy.shape[1] != 2 or ty.shape != (len(xy),) or tri.ndim != 2 or tri.shape[1] != 3:
                raise HlbmError(E_ARG, "mesh needs xy [n, 2], types [n] and triangles [m, 3]")
            rc = L.hlbm_create_mesh(C.byref(self.cfg), len(xy), _ptr(xy), _ptr(ty, C.c_int32), len(tri),
                                    _ptr(tri, C.c_int32), C.byref(h))
        elif x_nodes is not None or y_nodes is not None:  # graded grid
            gx = np.ascontiguousarray(x_nodes, dtype=np.float64)
            gy = np.ascontiguousarray(y_nodes, dtype=np.float64)
            if gx.shape != (nux,) or gy.shape != (nuy,):
                raise HlbmError(E_ARG, "x_nodes and y_nodes need nux and nuy entries")
            rc = L.hlbm_create_graded(C.byref(self.cfg), _ptr(gx), _ptr(gy), C.byref(h))
        else:
            rc = L.hlbm_create(C.byref(self.cfg), 1, C.byref(h))
        if rc != 0:
            raise HlbmError(rc, L.hlbm_last_error(None).decode())
        self.h = h
        self.nx, self.ny = nx, ny
        self.nnode = self.info().nnode

    def _check(self, rc):
        if rc != 0:
            raise HlbmError(rc, load().hlbm_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            load().hlbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        self._check(load().hlbm_step(self.h, n))

    def step_async(self, n=1):
        """Enqueue n steps without waiting (hlbm_step_async)."""
        self._check(load().hlbm_step_async(self.h, n))

    def sync(self):
        """Wait for the enqueued steps (hlbm_sync)."""
        self._check(load().hlbm_sync(self.h))

    def info(self) -> Info:
        i = Info()
        self._check(load().hlbm_info_get(self.h, 0, C.byref(i)))
        return i

    def lattice(self):
        out = np.zeros((9, self.ny, self.nx))
        self._check(load().hlbm_get_state(self.h, 0, STATE_LATTICE, out.ctypes.data, out.nbytes))
        return out

    def set_lattice(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        self._check(load().hlbm_set_state(self.h, 0, STATE_LATTICE, f.ctypes.data, f.nbytes))

    def grid(self):
        out = np.zeros((9, self.nnode))
        self._check(load().hlbm_get_state(self.h, 0, STATE_GRID, out.ctypes.data, out.nbytes))
        return out

    def set_grid(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        self._check(load().hlbm_set_state(self.h, 0, STATE_GRID, f.ctypes.data, f.nbytes))

    def history(self):
        n = C.c_int64()
        self._check(load().hlbm_force(self.h, 0, None, 0, C.byref(n), 0.0, 0.0, None))
        out = np.zeros((max(n.value, 1), 2))
        self._check(load().hlbm_force(self.h, 0, _ptr(out), n.value, C.byref(n), 0.0, 0.0, None))
        return out[:n.value]

    def theta(self, t0=1.0, t1=4.0):
        th = np.zeros(2)
        self._check(load().hlbm_force(self.h, 0, None, 0, None, t0, t1, _ptr(th)))
        return complex(th[0], th[1])

    def stencil(self, kmax=8):
        nbr = np.zeros((self.nnode, kmax), np.int32)
        S = np.zeros((self.nnode, 9, kmax))
        Cm = np.zeros((self.nnode, kmax))
        self._check(load().hlbm_get_stencil(self.h, kmax, _ptr(nbr, C.c_int32), _ptr(S), _ptr(Cm)))
        return nbr, S, Cm

    def tune(self, trial_steps=4, variant=None, lattice=None, order=None):
        """Pick the stream-collide launch shape and order and the grid
        sub-step kernel variant by timing each (state untouched), or apply
        ``variant`` (-1 = default), ``lattice`` = (threads, rows) and
        ``order`` (bit 0: single-step rows banded by XCD; bit 1: two-step
        tiles in staggered runs per XCD; default 2) as given. Returns the
        schedule."""
        t = Tuning()
        if variant is not None or lattice is not None or order is not None:
            t.substep_variant = -1 if variant is None else variant
            if lattice is not None:
                t.lattice_threads, t.lattice_rows = lattice
            t.order = 2 if order is None else order
            trial_steps = 0
        self._check(load().hlbm_tune(self.h, trial_steps, C.byref(t)))
        return t.as_dict()

    def timing(self, level=1):
        """1: every kernel of the step; 2: the stream-collide alone; 3: the
        grid sub-step launches of each step alone, each by its own events; 0: off."""
        self._check(load().hlbm_timing(self.h, int(level)))

    def timing_get(self, kernel):
        ms = C.c_double()
        cnt = C.c_int64()
        self._check(load().hlbm_timing_get(self.h, kernel, C.byref(ms), C.byref(cnt)))
        return ms.value, cnt.value

    def adjoint(self, dJ_dF):
        """dJ/d(A, omega, tau) for J = sum_k dJ_dF[k] . F(t_{k+1}); dJ_dF has
        one (x, y) row per step taken."""
        g = np.zeros(3)
        dJ = np.ascontiguousarray(dJ_dF, dtype=np.float64).reshape(-1, 2)
        self._check(load().hlbm_adjoint(self.h, 0, _ptr(dJ), dJ.shape[0], _ptr(g)))
        return g

    def set_motion(self, mass, stiffness, damping=0.0, y0=0.0, v0=0.0, y_max=1.0):
        """Two-way coupled motion M y'' + C y' + K y = F_y (before the first step)."""
        m = Motion(mass, stiffness, damping, y0, v0, y_max)
        self._check(load().hlbm_set_motion(self.h, 0, C.byref(m)))

    def set_deformation(self, B, phi=0.0):
        """Bending B sin(omega t + phi) (2x/b)^2 of the lamina on a given
        triangulation, the grid following it (before the first step)."""
        self._check(load().hlbm_set_deformation(self.h, float(B), float(phi)))

    def motion_history(self):
        """(y, v) after each step of a coupled case, entry k at t = k+1."""
        n = self.info().step
        out = np.zeros((n, 2))
        self._check(load().hlbm_get_state(self.h, 0, STATE_MOTION, out.ctypes.data, out.nbytes))
        return out

    def adjoint_lattice(self):
        """dJ/d(lattice at t_0) from the last adjoint."""
        out = np.zeros((9, self.ny, self.nx))
        self._check(load().hlbm_get_state(self.h, 0, STATE_ADJ_LATTICE, out.ctypes.data, out.nbytes))
        return out

    def adjoint_grid(self):
        """dJ/d(grid at t_0) from the last adjoint."""
        out = np.zeros((9, self.nnode))
        self._check(load().hlbm_get_state(self.h, 0, STATE_ADJ_GRID, out.ctypes.data, out.nbytes))
        return out


def level_shape(box):
    """Node counts of the level covering node box (x0, y0, x1, y1)."""
    x0, y0, x1, y1 = box
    return 2 * (x1 - x0) + 1, 2 * (y1 - y0) + 1


class MultiLevel(Case):
    """Nested structured refinement levels on the GPU, the finest carrying
    the lamina case. ``boxes[l] = (x0, y0, x1, y1)``: node box of level l
    covered by level l+1. Keyword arguments configure the finest level in
    its own lattice units (as for :class:`Case`, without nx, ny, bc). The
    history, theta, info and grid are the finest level's; ``step(n)``
    advances level 0 by n steps."""

    def __init__(self, nx0, ny0, boxes, bc0=BC_PERIODIC_X_WALLS_Y, storage=FP64, **fine):
        L = load()
        if isinstance(storage, str):
            storage = STORAGE[storage]
        if not 1 <= len(boxes) <= MAX_LEVELS - 1:
            raise HlbmError(E_ARG, f"2 .. {MAX_LEVELS} levels")
        nx, ny = level_shape(boxes[-1])
        self.cfg = Config(nx, ny, fine.get("nux", 0), fine.get("nuy", 0), fine.get("h_u", 1.0),
                          fine.get("b", 0.0), fine.get("thickness", 1.0), fine.get("tau", 0.8),
                          fine.get("kc", 0.0), fine.get("beta", 0.0), fine.get("n_sub", 0), BC_RING,
                          storage, fine.get("flags", 0), 0, 0, fine.get("max_steps", 0))
        lv = Levels()
        lv.nlevels, lv.nx0, lv.ny0, lv.bc0 = len(boxes) + 1, nx0, ny0, bc0
        for l, b in enumerate(boxes):
            for i in range(4):
                lv.box[l][i] = int(b[i])
        h = C.c_void_p()
        rc = L.hlbm_create_multilevel(C.byref(self.cfg), C.byref(lv), C.byref(h))
        if rc != 0:
            raise HlbmError(rc, L.hlbm_last_error(None).decode())
        self.h = h
        self.nx, self.ny = nx, ny
        self.nlevels = len(boxes) + 1
        self.boxes = [tuple(b) for b in boxes]
        self.shapes, self.taus = [], []
        for l in range(self.nlevels):
            a, b_, t = C.c_int32(), C.c_int32(), C.c_double()
            self._check(L.hlbm_level_shape(self.h, l, C.byref(a), C.byref(b_), C.byref(t)))
            self.shapes.append((a.value, b_.value))
            self.taus.append(t.value)
        self.nnode = self.info().nnode

    def level(self, l):
        nx, ny = self.shapes[l]
        out = np.zeros((9, ny, nx))
        self._check(load().hlbm_get_state(self.h, 0, STATE_LEVEL + l, out.ctypes.data, out.nbytes))
        return out

    def set_level(self, l, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        self._check(load().hlbm_set_state(self.h, 0, STATE_LEVEL + l, f.ctypes.data, f.nbytes))


class _Member:
    """One case of a batch (reads and writes go to that case)."""

    def __init__(self, batch, cid, nx, ny, nnode):
        self.batch, self.cid, self.nx, self.ny, self.nnode = batch, cid, nx, ny, nnode

    def _check(self, rc):
        self.batch._check(rc)

    def info(self) -> Info:
        i = Info()
        self._check(load().hlbm_info_get(self.batch.h, self.cid, C.byref(i)))
        return i

    def history(self):
        n = C.c_int64()
        h = self.batch.h
        self._check(load().hlbm_force(h, self.cid, None, 0, C.byref(n), 0.0, 0.0, None))
        out = np.zeros((max(n.value, 1), 2))
        self._check(load().hlbm_force(h, self.cid, _ptr(out), n.value, C.byref(n), 0.0, 0.0, None))
        return out[:n.value]

    def theta(self, t0=1.0, t1=4.0):
        th = np.zeros(2)
        self._check(load().hlbm_force(self.batch.h, self.cid, None, 0, None, t0, t1, _ptr(th)))
        return complex(th[0], th[1])

    def lattice(self):
        out = np.zeros((9, self.ny, self.nx))
        self._check(load().hlbm_get_state(self.batch.h, self.cid, STATE_LATTICE, out.ctypes.data, out.nbytes))
        return out

    def grid(self):
        out = np.zeros((9, self.nnode))
        self._check(load().hlbm_get_state(self.batch.h, self.cid, STATE_GRID, out.ctypes.data, out.nbytes))
        return out

    def set_lattice(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        self._check(load().hlbm_set_state(self.batch.h, self.cid, STATE_LATTICE, f.ctypes.data, f.nbytes))

    def set_grid(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        self._check(load().hlbm_set_state(self.batch.h, self.cid, STATE_GRID, f.ctypes.data, f.nbytes))


class Batch:
    """Many lamina cases advanced together by the case-batched kernels.
    ``configs``: list of keyword dicts as for :class:`Case` (each with its
    own max_steps); all share one storage type."""

    def __init__(self, configs, storage=FP64):
        L = load()
        if isinstance(storage, str):
            storage = STORAGE[storage]
        arr = (Config * len(configs))()
        for i, c in enumerate(configs):
            c = dict(c)
            arr[i] = Config(c["nx"], c["ny"], c.get("nux", 0), c.get("nuy", 0), c.get("h_u", 1.0),
                            c.get("b", 0.0), c.get("thickness", 1.0), c.get("tau", 0.8), c.get("kc", 0.0),
                            c.get("beta", 0.0), c.get("n_sub", 0), c.get("bc", BC_PERIODIC_X_WALLS_Y),
                            storage, c.get("flags", 0), 0, 0, c.get("max_steps", 0))
        h = C.c_void_p()
        rc = L.hlbm_create(arr, len(configs), C.byref(h))
        if rc != 0:
            raise HlbmError(rc, L.hlbm_last_error(None).decode())
        self.h = h
        self.cases = []
        for i, c in enumerate(configs):
            m = _Member(self, i, c["nx"], c["ny"], 0)
            m.nnode = m.info().nnode
            self.cases.append(m)

    def _check(self, rc):
        if rc != 0:
            raise HlbmError(rc, load().hlbm_last_error(self.h).decode())

    def __len__(self):
        return len(self.cases)

    def __getitem__(self, i):
        return self.cases[i]

    def step(self, n):
        self._check(load().hlbm_step(self.h, n))

    def tune(self, trial_steps=16, schedule=None):
        """Autotune (trial_steps > 0) or apply ``schedule`` (dict) as given."""
        t = Tuning(steps_per_graph=8, lattice_threads=128, lattice_rows=2, substep_variant=-1, order=1,
                   tail_variant=-1)
        if schedule:
            for k, v in schedule.items():
                setattr(t, k, v)
            trial_steps = 0
        self._check(load().hlbm_tune(self.h, trial_steps, C.byref(t)))
        return t.as_dict()

    def close(self):
        if getattr(self, "h", None):
            load().hlbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def case_from_preset(cfg: dict, **overrides) -> Case:
    c = dict(cfg)
    c.update(overrides)
    steps = c.pop("steps", 0)
    c.setdefault("max_steps", steps)
    return Case(**c)
