"""Plain CPU FP64 oracle of the D3Q19 BGK lattice Boltzmann method.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it to check and to time the GPU library.  The product
path never imports it.  The arithmetic lives in ``lbm_oracle.c`` (plain C,
FP64, one global grid, Sec. 2.1 of Feichtinger et al.) and in ``conv.py``
(the surrogate's FP64 convolution reference); this module only marshals
numpy arrays through ctypes.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")
_lib = None

FACES = ("-x", "+x", "-y", "+y", "-z", "+z")


def set_threads(n):
    """OpenMP threads of the oracle's step (timing on one and on all cores)."""
    _load().orc_set_threads(int(n))


def max_threads():
    return int(_load().orc_max_threads())


def build(force=False):
    """Compile the C oracle with gcc (OpenMP over z planes)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.orc_create.restype = P
        lib.orc_create.argtypes = [ip, ip, dp, ctypes.c_double, ctypes.c_double, dp]
        lib.orc_destroy.argtypes = [P]
        lib.orc_set_geometry.argtypes = [P, ctypes.c_void_p]
        lib.orc_set_equilibrium.argtypes = [P, dp, dp]
        lib.orc_step.argtypes = [P, ctypes.c_long]
        lib.orc_macroscopic.argtypes = [P, dp, dp]
        lib.orc_sums.argtypes = [P, dp, dp]
        lib.orc_residual.argtypes = [P]
        lib.orc_residual.restype = ctypes.c_double
        lib.orc_get_state.argtypes = [P, dp]
        lib.orc_set_state.argtypes = [P, dp, dp, dp]
        lib.orc_steps.argtypes = [P]
        lib.orc_steps.restype = ctypes.c_long
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_max_threads.restype = ctypes.c_int
        lib.orc_velocity.argtypes = [ctypes.c_int, ip]
        lib.orc_weight.argtypes = [ctypes.c_int]
        lib.orc_weight.restype = ctypes.c_double
        lib.orc_set_face.argtypes = [P, ctypes.c_int, ctypes.c_int, dp, ctypes.c_double]
        lib.orc_set_face.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class OracleLBM:
    """One global FP64 lattice; arrays are numpy, cell index (z, y, x).

    dims = (nx, ny, nz); walls = per-axis flag (True: half-way bounce-back
    walls on both faces, False: periodic); wall_u = {face: (ux, uy, uz)};
    open_faces = {face: ("velocity", (ux, uy, uz)) | ("pressure", rho) |
    "wall"}, faces of one axis ("-x"/"+x", "-y"/"+y" or "-z"/"+z"): open faces
    by non-equilibrium extrapolation (a face not named keeps what `walls`
    says; that axis must not be periodic then).  open_x is the older name.
    """

    def __init__(self, dims, walls=(False, False, False), wall_u=None, tau=0.6,
                 rho0=1.0, force=(0.0, 0.0, 0.0), open_x=None, open_faces=None):
        lib = _load()
        self.dims = tuple(int(d) for d in dims)
        self.rho0 = float(rho0)
        self.force = tuple(float(v) for v in force)
        d = (ctypes.c_int * 3)(*self.dims)
        w = (ctypes.c_int * 3)(*[1 if v else 0 for v in walls])
        uw = np.zeros(18)
        for face, vel in (wall_u or {}).items():
            k = FACES.index(face)
            uw[3 * k:3 * k + 3] = vel
        g = np.asarray(force, dtype=np.float64)
        self._h = lib.orc_create(d, w, _dptr(uw), float(tau), float(rho0), _dptr(g))
        if not self._h:
            raise ValueError("oracle: invalid parameters")
        self._lib = lib
        for face, spec in dict(open_x or {}, **(open_faces or {})).items():
            side = FACES.index(face)
            if spec == "wall":
                kind, u, rho = 1, np.zeros(3), 0.0
            elif spec[0] == "velocity":
                kind, u, rho = 2, np.asarray(spec[1], dtype=np.float64), 0.0
            elif spec[0] == "pressure":
                kind, u, rho = 3, np.zeros(3), float(spec[1])
            else:
                raise ValueError("oracle: bad open face %r" % (spec,))
            if lib.orc_set_face(self._h, side, kind, _dptr(u), rho) != 0:
                raise ValueError("oracle: bad open face")
        nx, ny, nz = self.dims
        self.shape = (nz, ny, nx)
        self.ncell = nx * ny * nz

    def close(self):
        if self._h:
            self._lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_geometry(self, solid=None):
        if solid is None:
            self._lib.orc_set_geometry(self._h, None)
        else:
            s = np.ascontiguousarray(solid, dtype=np.uint8).reshape(self.shape)
            self._keep = s
            self._lib.orc_set_geometry(self._h, s.ctypes.data)

    def set_equilibrium(self, rho, u):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.shape)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape((3,) + self.shape)
        self._lib.orc_set_equilibrium(self._h, _dptr(rho), _dptr(u))

    def step(self, n=1):
        self._lib.orc_step(self._h, int(n))

    @property
    def steps(self):
        return self._lib.orc_steps(self._h)

    def macroscopic(self):
        rho = np.empty(self.shape)
        u = np.empty((3,) + self.shape)
        self._lib.orc_macroscopic(self._h, _dptr(rho), _dptr(u))
        return rho, u

    def sums(self):
        m = np.zeros(1)
        p = np.zeros(3)
        self._lib.orc_sums(self._h, _dptr(m), _dptr(p))
        return float(m[0]), p

    def residual(self):
        return self._lib.orc_residual(self._h)

    def get_state(self):
        f = np.empty((19,) + self.shape)
        self._lib.orc_get_state(self._h, _dptr(f))
        return f

    def set_state(self, f, rho=None, u=None):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape((19,) + self.shape)
        r = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64)
        v = None if u is None else np.ascontiguousarray(u, dtype=np.float64)
        self._lib.orc_set_state(self._h, _dptr(f), None if r is None else _dptr(r),
                                None if v is None else _dptr(v))


def velocities():
    """The oracle's D3Q19 direction table, as numpy (19, 3)."""
    lib = _load()
    out = np.zeros((19, 3), dtype=np.int64)
    e = (ctypes.c_int * 3)()
    for i in range(19):
        lib.orc_velocity(i, e)
        out[i] = list(e)
    return out


def weights():
    """The oracle's D3Q19 lattice weights, as numpy (19,)."""
    lib = _load()
    return np.array([lib.orc_weight(i) for i in range(19)])
