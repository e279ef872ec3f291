"""ctypes binding of the FP64 CPU oracle (``liboracle.so``) and of its
complex-step build (``liboracle_cs.so``).

TEST INFRASTRUCTURE: only the test suite, the smoke check and the CPU-baseline
leg of the benchmark import this module. It never backs the GPU library.

The complex-step build runs the same source with every quantity that depends
continuously on (A, omega, tau) held as a complex number. Adding i*h to one
parameter gives Im(output)/h = d(output)/d(parameter) with no cancellation
error (Squire and Trapp, SIAM Review 40, 1998), while every discrete decision
(cells, triangles, refill types, node status) follows the real part.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hlbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_CS = os.path.join(_HERE, "liboracle_cs.so")

BC_PERIODIC_X_WALLS_Y = 0
BC_PERIODIC = 1
BC_PAPER = 2
BC_RING = 3
ML_PLANT_NO_RESCALE = 256
ML_PLANT_SAME_TAU = 512
FLAG_NO_BODY = 1
# planted mistakes in the lattice-grid exchange (tests show the pins catch them)
PLANT_S_FACTOR = 2       # 1 - 1/tau_s in place of Eq.(postcollision2_s)'s 2(tau_s-1)/(2tau_s-1)
PLANT_NO_KNEQ = 4        # the (1 - 1/(2 tau_s)) rescale of f^neq,s dropped
PLANT_SWAP_BILIN_Y = 8   # bilinear weights mirrored in y
PLANT_SWAP_BILIN_X = 16  # bilinear weights mirrored in x
PLANT_BARY = 32          # barycentric weights in a rotated vertex order
NODE_INTERIOR, NODE_INTERFACE, NODE_WALL = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no contraction of a*b+c), once as
    plain doubles and once as the complex-step variant."""
    for out, extra in ((_LIB, []), (_LIB_CS, ["-DOR_COMPLEX_STEP"])):
        if force or not os.path.exists(out):
            cmd = ["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-Wall", "-fPIC", "-fopenmp", *extra,
                   "-shared", "-o", out + ".tmp", _SRC, "-lm"]
            subprocess.check_call(cmd)
            os.replace(out + ".tmp", out)
    return _LIB


class Config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nux", C.c_int32), ("nuy", C.c_int32),
                ("h_u", C.c_double), ("b", C.c_double), ("thickness", C.c_double),
                ("tau", C.c_double), ("kc", C.c_double), ("beta", C.c_double),
                ("n_sub", C.c_int32), ("bc", C.c_int32), ("flags", C.c_int32),
                ("max_steps", C.c_int64)]


class Info(C.Structure):
    _fields_ = [(n, C.c_double) for n in
                ("nu", "tau_u", "dt_u", "A", "omega", "period", "u_max", "mach", "reynolds", "eps")] + \
               [(n, C.c_int32) for n in
                ("n_sub", "nnode", "ntri", "n_interface", "n_wall", "n_wall_edges", "beta_limit_ok")] + \
               [("step", C.c_int64), ("y", C.c_double),
                ("n_type1", C.c_int64), ("n_type2", C.c_int64), ("n_type3", C.c_int64)]


_lib = None
_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_I = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_U8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        vp = C.c_void_p
        L.or_feq.argtypes = [C.c_double, C.c_double, C.c_double, _D]
        L.or_d2q9.argtypes = [_I, _I, _D]
        L.or_lattice_step.argtypes = [_D, _D, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                      C.c_double, C.c_double, vp]
        for f in ("or_mesh_lamina",):
            getattr(L, f).argtypes = [C.c_int32, C.c_int32, C.c_double, C.c_double]
            getattr(L, f).restype = vp
        for f in ("or_mesh_periodic", "or_mesh_channel"):
            getattr(L, f).argtypes = [C.c_int32, C.c_int32, C.c_double]
            getattr(L, f).restype = vp
        L.or_mesh_free.argtypes = [vp]
        for f in ("or_mesh_nnode", "or_mesh_ntri", "or_mesh_kmax"):
            getattr(L, f).argtypes = [vp]
            getattr(L, f).restype = C.c_int32
        L.or_mesh_nodes.argtypes = [vp, _D, _D, _I]
        L.or_mesh_triangles.argtypes = [vp, _I, _D]
        L.or_mesh_stencil.argtypes = [vp, C.c_int32, _I, _D, _D, _D]
        L.or_mesh_locate.argtypes = [vp, C.c_double, C.c_double, _D]
        L.or_mesh_locate.restype = C.c_int32
        L.or_fv_substep.argtypes = [vp, _D, vp, vp, _D, C.c_double, C.c_double, vp, vp]
        L.or_mesh_force.argtypes = [vp, _D, _D]
        L.or_create.argtypes = [C.POINTER(Config), C.POINTER(vp)]
        L.or_destroy.argtypes = [vp]
        L.or_step.argtypes = [vp, C.c_int64]
        L.or_info_get.argtypes = [vp, C.POINTER(Info)]
        L.or_sim_mesh.argtypes = [vp]
        L.or_sim_mesh.restype = vp
        for f in ("or_get_lattice", "or_set_lattice", "or_get_mesh", "or_set_mesh"):
            getattr(L, f).argtypes = [vp, _D]
        L.or_history.argtypes = [vp, _D, C.c_int64]
        L.or_history.restype = C.c_int64
        L.or_lattice_status.argtypes = [vp, C.c_int64, C.c_int32, C.c_int32]
        L.or_lattice_status.restype = C.c_int32
        L.or_set_walls.argtypes = [vp, C.c_double, C.c_double]
        L.or_create_wallband.argtypes = [C.POINTER(Config), C.c_int32, C.c_double, C.c_double,
                                         C.c_double, C.c_double, C.POINTER(vp)]
        for f in ("or_probe_bilinear", "or_probe_grid"):
            getattr(L, f).argtypes = [vp, C.c_double, C.c_double, _D]
        L.or_fit_theta.argtypes = [_D, C.c_int64, C.c_double, C.c_double, C.c_double,
                                   C.c_double, C.c_double, _D]
        L.or_set_threads.argtypes = [C.c_int32]
        L.or_set_threads.restype = C.c_int32
        L.or_set_motion.argtypes = [vp] + [C.c_double] * 6
        L.or_create_graded.argtypes = [C.POINTER(Config), _D, _D, C.POINTER(vp)]
        L.or_create_mesh.argtypes = [C.POINTER(Config), C.c_int32, _D, _I, C.c_int32, _I, C.POINTER(vp)]
        L.or_set_deformation.argtypes = [vp, C.c_double, C.c_double]
        L.or_mesh_lamina_coords.argtypes = [C.c_int32, C.c_int32, _D, _D, C.c_double]
        L.or_mesh_lamina_coords.restype = vp
        L.or_motion_history.argtypes = [vp, _D, C.c_int64]
        L.or_motion_history.restype = C.c_int64
        L.or_ml_create.argtypes = [C.POINTER(Config), C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                   C.c_double, C.c_double, _I, C.c_int32, C.POINTER(vp)]
        L.or_ml_destroy.argtypes = [vp]
        L.or_ml_step.argtypes = [vp, C.c_int64]
        L.or_ml_level_shape.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                        C.POINTER(C.c_double)]
        L.or_ml_get_level.argtypes = [vp, C.c_int32, _D]
        L.or_ml_set_level.argtypes = [vp, C.c_int32, _D]
        L.or_ml_finest.argtypes = [vp]
        L.or_ml_finest.restype = vp
        L.or_ml_steps.argtypes = [vp]
        L.or_ml_steps.restype = C.c_int64
        _lib = L
    return _lib


_lib_cs = None


def lib_cs():
    global _lib_cs
    if _lib_cs is None:
        if not os.path.exists(_LIB_CS):
            build()
        L = C.CDLL(_LIB_CS)
        vp = C.c_void_p
        L.or_create.argtypes = [C.POINTER(Config), C.POINTER(vp)]
        L.or_create_graded.argtypes = [C.POINTER(Config), _D, _D, C.POINTER(vp)]
        L.or_destroy.argtypes = [vp]
        L.or_step.argtypes = [vp, C.c_int64]
        L.or_info_get.argtypes = [vp, C.POINTER(Info)]
        L.or_set_threads.argtypes = [C.c_int32]
        L.or_set_threads.restype = C.c_int32
        L.or_cs_perturb.argtypes = [vp, C.c_double, C.c_double, C.c_double]
        for f in ("or_cs_get_lattice", "or_cs_get_mesh"):
            getattr(L, f).argtypes = [vp, _D, _D]
        for f in ("or_cs_set_lattice", "or_cs_set_mesh"):
            getattr(L, f).argtypes = [vp, _D, vp]
        L.or_cs_history.argtypes = [vp, _D, _D, C.c_int64]
        L.or_cs_history.restype = C.c_int64
        _lib_cs = L
    return _lib_cs


def set_threads(n: int) -> int:
    """Host threads of the oracle's per-node loops (1 unless set; n <= 0
    queries). Results do not depend on it."""
    return lib().or_set_threads(n)


def d2q9():
    cx = np.zeros(9, np.int32)
    cy = np.zeros(9, np.int32)
    w = np.zeros(9)
    lib().or_d2q9(cx, cy, w)
    return cx, cy, w


def feq(rho: float, ux: float, uy: float) -> np.ndarray:
    out = np.zeros(9)
    lib().or_feq(rho, ux, uy, out)
    return out


def lattice_step(A: np.ndarray, tau: float, bc: int = BC_PERIODIC, u_bot: float = 0.0,
                 u_top: float = 0.0, disc: np.ndarray | None = None) -> np.ndarray:
    """One Eq.(LBE) step on a [9][ny][nx] array; returns the new array."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    _, ny, nx = A.shape
    B = A.copy()  # a ring-fed lattice (bc 3) leaves its ring as it was
    dptr = None
    if disc is not None:
        disc = np.ascontiguousarray(disc, dtype=np.uint8)
        dptr = disc.ctypes.data_as(C.c_void_p)
    lib().or_lattice_step(A, B, nx, ny, bc, tau, u_bot, u_top, dptr)
    return B


class Mesh:
    """A triangular grid with its finite-volume matrices."""

    def __init__(self, ptr, owned=True):
        if not ptr:
            raise ValueError("mesh construction rejected its arguments")
        self.ptr = ptr
        self.owned = owned
        L = lib()
        self.nnode = L.or_mesh_nnode(ptr)
        self.ntri = L.or_mesh_ntri(ptr)
        self.kmax = L.or_mesh_kmax(ptr)

    @classmethod
    def lamina(cls, nux, nuy, h=1.0, b=0.0):
        return cls(lib().or_mesh_lamina(nux, nuy, h, b))

    @classmethod
    def lamina_coords(cls, X, Y, b=0.0):
        X = np.ascontiguousarray(X, dtype=np.float64)
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        return cls(lib().or_mesh_lamina_coords(len(X), len(Y), X, Y, b))

    @classmethod
    def periodic(cls, nx, ny, h=1.0):
        return cls(lib().or_mesh_periodic(nx, ny, h))

    @classmethod
    def channel(cls, nx, ny, h=1.0):
        return cls(lib().or_mesh_channel(nx, ny, h))

    def __del__(self):
        if getattr(self, "owned", False) and self.ptr and _lib is not None:
            _lib.or_mesh_free(self.ptr)
            self.ptr = None

    def nodes(self):
        x = np.zeros(self.nnode)
        y = np.zeros(self.nnode)
        t = np.zeros(self.nnode, np.int32)
        lib().or_mesh_nodes(self.ptr, x, y, t)
        return x, y, t

    def triangles(self):
        tri = np.zeros((self.ntri, 3), np.int32)
        txy = np.zeros((self.ntri, 3, 2))
        lib().or_mesh_triangles(self.ptr, tri, txy)
        return tri, txy

    def stencil(self):
        k = self.kmax
        nbr = np.zeros((self.nnode, k), np.int32)
        S = np.zeros((self.nnode, 9, k))
        Cm = np.zeros((self.nnode, k))
        V = np.zeros(self.nnode)
        lib().or_mesh_stencil(self.ptr, k, nbr, S, Cm, V)
        return nbr, S, Cm, V

    def locate(self, px, py):
        lam = np.zeros(3)
        t = lib().or_mesh_locate(self.ptr, px, py, lam)
        return t, lam

    def substep(self, f, tau_u, dt_u, star_eq=None, star_neq=None, uwx=None, uwy=None):
        f = np.ascontiguousarray(f, dtype=np.float64)
        out = np.empty_like(f)
        keep = []

        def p(a):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dtype=np.float64)
            keep.append(a)
            return a.ctypes.data_as(C.c_void_p)
        lib().or_fv_substep(self.ptr, f, p(star_eq), p(star_neq), out, tau_u, dt_u, p(uwx), p(uwy))
        return out

    def force(self, f):
        F = np.zeros(2)
        lib().or_mesh_force(self.ptr, np.ascontiguousarray(f, dtype=np.float64), F)
        return F


class Sim:
    """The hybrid method, advanced step by step on the CPU."""

    def __init__(self, nx, ny, nux=0, nuy=0, h_u=1.0, b=0.0, thickness=1.0, tau=0.8, kc=0.0,
                 beta=0.0, n_sub=0, bc=BC_PERIODIC_X_WALLS_Y, flags=0, max_steps=0, x_nodes=None,
                 y_nodes=None, mesh=None):
        self.cfg = Config(nx, ny, nux, nuy, h_u, b, thickness, tau, kc, beta, n_sub, bc, flags,
                          max_steps)
        h = C.c_void_p()
        if mesh is not None:  # any triangulation: (xy [n, 2], node types [n], triangles [m, 3])
            xy = np.ascontiguousarray(mesh[0], dtype=np.float64)
            ty = np.ascontiguousarray(mesh[1], dtype=np.int32)
            tri = np.ascontiguousarray(mesh[2], dtype=np.int32)
            if xy.ndim != 2 or xy.shape[1] != 2 or ty.shape != (len(xy),) or tri.ndim != 2 or tri.shape[1] != 3:
                raise ValueError("mesh needs xy [n, 2], types [n] and triangles [m, 3]")
            rc = lib().or_create_mesh(C.byref(self.cfg), len(xy), xy, ty, len(tri), tri, C.byref(h))
        elif x_nodes is not None or y_nodes is not None:  # graded grid
            gx = np.ascontiguousarray(x_nodes, dtype=np.float64)
            gy = np.ascontiguousarray(y_nodes, dtype=np.float64)
            if gx.shape != (nux,) or gy.shape != (nuy,):
                raise ValueError("x_nodes and y_nodes need nux and nuy entries")
            rc = lib().or_create_graded(C.byref(self.cfg), gx, gy, C.byref(h))
        else:
            rc = lib().or_create(C.byref(self.cfg), C.byref(h))
        if rc != 0:
            raise ValueError(f"or_create rejected the configuration (code {rc})")
        self.ptr = h
        self.nx, self.ny = nx, ny
        inf = self.info()
        self.nnode = inf.nnode

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.or_destroy(self.ptr)
            self.ptr = None

    def step(self, n=1):
        rc = lib().or_step(self.ptr, n)
        if rc != 0:
            raise RuntimeError(f"or_step failed (code {rc})")

    def info(self) -> Info:
        i = Info()
        lib().or_info_get(self.ptr, C.byref(i))
        return i

    def mesh(self) -> Mesh:
        m = Mesh(lib().or_sim_mesh(self.ptr), owned=False)
        m._owner = self  # the case owns the mesh: keep it alive with the view
        return m

    def lattice(self):
        out = np.zeros((9, self.ny, self.nx))
        lib().or_get_lattice(self.ptr, out)
        return out

    def set_lattice(self, f):
        lib().or_set_lattice(self.ptr, np.ascontiguousarray(f, dtype=np.float64))

    def grid(self):
        out = np.zeros((9, self.nnode))
        lib().or_get_mesh(self.ptr, out)
        return out

    def set_grid(self, f):
        lib().or_set_mesh(self.ptr, np.ascontiguousarray(f, dtype=np.float64))

    def history(self):
        n = lib().or_history(self.ptr, np.zeros(2), 0)
        out = np.zeros((max(n, 1), 2))
        lib().or_history(self.ptr, out, n)
        return out[:n]

    def set_deformation(self, B, phi=0.0):
        """Prescribed bending B sin(omega t + phi) (2x/b)^2 of the lamina on a
        given triangulation (before the first step)."""
        rc = lib().or_set_deformation(self.ptr, B, phi)
        if rc != 0:
            raise ValueError(f"or_set_deformation rejected the arguments (code {rc})")

    def set_motion(self, mass, stiffness, damping=0.0, y0=0.0, v0=0.0, y_max=1.0):
        """Two-way coupled motion M y'' + C y' + K y = F_y (before the first step)."""
        rc = lib().or_set_motion(self.ptr, mass, stiffness, damping, y0, v0, y_max)
        if rc != 0:
            raise ValueError(f"or_set_motion rejected the arguments (code {rc})")

    def motion_history(self):
        n = lib().or_motion_history(self.ptr, np.zeros(2), 0)
        out = np.zeros((max(n, 1), 2))
        lib().or_motion_history(self.ptr, out, n)
        return out[:n]

    @classmethod
    def wallband(cls, nx, ny, nband, tau, U, omega, x_off=0.0, y_wall=0.0, n_sub=0, flags=0,
                 max_steps=0):
        """A static grid band of nband rows on a wall oscillating tangentially
        with U cos(omega t), the lattice above it (or_create_wallband)."""
        self = cls.__new__(cls)
        self.cfg = Config(nx, ny, 0, 0, 1.0, 0.0, 1.0, tau, 0.0, 0.0, n_sub,
                          BC_PERIODIC_X_WALLS_Y, flags, max_steps)
        h = C.c_void_p()
        rc = lib().or_create_wallband(C.byref(self.cfg), nband, x_off, y_wall, U, omega, C.byref(h))
        if rc != 0:
            raise ValueError(f"or_create_wallband rejected the configuration (code {rc})")
        self.ptr = h
        self.nx, self.ny = nx, ny
        self.nnode = self.info().nnode
        return self

    def set_walls(self, u_bot, u_top):
        """Tangential x-velocities of the lattice's y walls (bc 0)."""
        if lib().or_set_walls(self.ptr, u_bot, u_top) != 0:
            raise ValueError("moving walls need bc BC_PERIODIC_X_WALLS_Y")

    def probe_bilinear(self, X, Y):
        """(rho, ux, uy, f^neq[9]) bilinear from the lattice's pre-collision
        populations at t_{k+1}, at lattice position (X, Y)."""
        out = np.zeros(12)
        lib().or_probe_bilinear(self.ptr, X, Y, out)
        return out

    def probe_grid(self, X, Y):
        """(rho, ux, uy, f^neq[9]) barycentric from the grid at its current
        offset, at lattice position (X, Y)."""
        out = np.zeros(12)
        if lib().or_probe_grid(self.ptr, X, Y, out) != 0:
            raise ValueError("no grid triangle holds the point")
        return out

    def status(self, k):
        return np.array([[lib().or_lattice_status(self.ptr, k, x, y) for x in range(self.nx)]
                         for y in range(self.ny)], dtype=np.int32)


class _FinestView(Sim):
    """The finest level of a :class:`MultiLevel`, owned by it."""

    def __init__(self, ptr, nx, ny, owner):
        self.ptr = C.c_void_p(ptr)
        self._owner = owner
        self.nx, self.ny = nx, ny
        self.nnode = self.info().nnode

    def __del__(self):
        pass  # freed with its owner

    def step(self, n=1):
        raise RuntimeError("the finest level advances with its MultiLevel")


def level_shape(box):
    """Node counts of the level covering node box (x0, y0, x1, y1)."""
    x0, y0, x1, y1 = box
    return 2 * (x1 - x0) + 1, 2 * (y1 - y0) + 1


class MultiLevel:
    """Nested structured refinement levels with a hybrid case on the finest.

    ``boxes[l] = (x0, y0, x1, y1)``: node box of level l covered by level
    l+1. ``fine`` holds the finest level's configuration (tau, body, grid)
    in its own lattice units; its lattice size follows from the last box."""

    def __init__(self, nx0, ny0, boxes, bc0=BC_PERIODIC_X_WALLS_Y, u_bot=0.0, u_top=0.0, flags=0,
                 **fine):
        nx, ny = level_shape(boxes[-1])
        fine = dict(fine)
        fine.setdefault("tau", 0.8)
        self.cfg = Config(nx, ny, fine.get("nux", 0), fine.get("nuy", 0), fine.get("h_u", 1.0),
                          fine.get("b", 0.0), fine.get("thickness", 1.0), fine["tau"],
                          fine.get("kc", 0.0), fine.get("beta", 0.0), fine.get("n_sub", 0), BC_RING,
                          fine.get("flags", 0), fine.get("max_steps", 0))
        box = np.ascontiguousarray(np.array(boxes, dtype=np.int32).reshape(-1))
        h = C.c_void_p()
        rc = lib().or_ml_create(C.byref(self.cfg), len(boxes) + 1, nx0, ny0, bc0, u_bot, u_top, box,
                                flags, C.byref(h))
        if rc != 0:
            raise ValueError(f"or_ml_create rejected the configuration (code {rc})")
        self.ptr = h
        self.nlevels = len(boxes) + 1
        self.boxes = [tuple(b) for b in boxes]
        self.shapes = []
        self.taus = []
        for l in range(self.nlevels):
            a, b_, t = C.c_int32(), C.c_int32(), C.c_double()
            lib().or_ml_level_shape(self.ptr, l, C.byref(a), C.byref(b_), C.byref(t))
            self.shapes.append((a.value, b_.value))
            self.taus.append(t.value)
        self.finest = _FinestView(lib().or_ml_finest(self.ptr), nx, ny, self)

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.or_ml_destroy(self.ptr)
            self.ptr = None

    def step(self, n=1):
        rc = lib().or_ml_step(self.ptr, n)
        if rc != 0:
            raise RuntimeError(f"or_ml_step failed (code {rc})")

    def steps(self):
        return lib().or_ml_steps(self.ptr)

    def level(self, l):
        nx, ny = self.shapes[l]
        out = np.zeros((9, ny, nx))
        lib().or_ml_get_level(self.ptr, l, out)
        return out

    def set_level(self, l, f):
        nx, ny = self.shapes[l]
        f = np.ascontiguousarray(f, dtype=np.float64)
        if f.shape != (9, ny, nx):
            raise ValueError(f"level {l} holds (9, {ny}, {nx}) populations")
        lib().or_ml_set_level(self.ptr, l, f)

    def history(self):
        return self.finest.history()


class SimCS:
    """The complex-step build of :class:`Sim`.

    ``SimCS(h_A, h_omega, h_tau, **cfg)`` adds i*h to A, omega and tau_s
    (tau_u = tau_s - 1/2 follows). After ``step``, ``history()`` returns the
    real force history and its imaginary part; divided by h the latter is
    the exact derivative of the history along that direction. ``x_nodes``
    and ``y_nodes`` give a graded grid, as for :class:`Sim`."""

    def __init__(self, h_A=0.0, h_omega=0.0, h_tau=0.0, *, nx, ny, nux=0, nuy=0, h_u=1.0,
                 b=0.0, thickness=1.0, tau=0.8, kc=0.0, beta=0.0, n_sub=0,
                 bc=BC_PERIODIC_X_WALLS_Y, flags=0, max_steps=0, x_nodes=None, y_nodes=None):
        self.cfg = Config(nx, ny, nux, nuy, h_u, b, thickness, tau, kc, beta, n_sub, bc, flags,
                          max_steps)
        h = C.c_void_p()
        if x_nodes is not None or y_nodes is not None:  # graded grid
            gx = np.ascontiguousarray(x_nodes, dtype=np.float64)
            gy = np.ascontiguousarray(y_nodes, dtype=np.float64)
            if gx.shape != (nux,) or gy.shape != (nuy,):
                raise ValueError("x_nodes and y_nodes need nux and nuy entries")
            rc = lib_cs().or_create_graded(C.byref(self.cfg), gx, gy, C.byref(h))
        else:
            rc = lib_cs().or_create(C.byref(self.cfg), C.byref(h))
        if rc != 0:
            raise ValueError(f"or_create rejected the configuration (code {rc})")
        self.ptr = h
        self.nx, self.ny = nx, ny
        lib_cs().or_cs_perturb(self.ptr, h_A, h_omega, h_tau)
        i = Info()
        lib_cs().or_info_get(self.ptr, C.byref(i))
        self.nnode = i.nnode

    def __del__(self):
        if getattr(self, "ptr", None) and _lib_cs is not None:
            _lib_cs.or_destroy(self.ptr)
            self.ptr = None

    def step(self, n=1):
        rc = lib_cs().or_step(self.ptr, n)
        if rc != 0:
            raise RuntimeError(f"or_step failed (code {rc})")

    def info(self) -> Info:
        i = Info()
        lib_cs().or_info_get(self.ptr, C.byref(i))
        return i

    def history(self):
        z = np.zeros(2)
        n = lib_cs().or_cs_history(self.ptr, z, z, 0)
        re = np.zeros((max(n, 1), 2))
        im = np.zeros((max(n, 1), 2))
        lib_cs().or_cs_history(self.ptr, re, im, n)
        return re[:n], im[:n]

    def lattice(self):
        re = np.zeros((9, self.ny, self.nx))
        im = np.zeros_like(re)
        lib_cs().or_cs_get_lattice(self.ptr, re, im)
        return re, im

    def grid(self):
        re = np.zeros((9, self.nnode))
        im = np.zeros_like(re)
        lib_cs().or_cs_get_mesh(self.ptr, re, im)
        return re, im

    def set_lattice(self, re, im=None):
        im = None if im is None else np.ascontiguousarray(im, dtype=np.float64)
        lib_cs().or_cs_set_lattice(self.ptr, np.ascontiguousarray(re, dtype=np.float64),
                                   None if im is None else im.ctypes.data_as(C.c_void_p))

    def set_grid(self, re, im=None):
        im = None if im is None else np.ascontiguousarray(im, dtype=np.float64)
        lib_cs().or_cs_set_mesh(self.ptr, np.ascontiguousarray(re, dtype=np.float64),
                                None if im is None else im.ctypes.data_as(C.c_void_p))


def fit_theta(hist, omega, A, b, t0=1.0, t1=4.0):
    hist = np.ascontiguousarray(hist, dtype=np.float64).reshape(-1, 2)
    out = np.zeros(2)
    rc = lib().or_fit_theta(hist, hist.shape[0], omega, A, b, t0, t1, out)
    if rc != 0:
        raise ValueError("fit window holds fewer than two samples")
    return complex(out[0], out[1])
