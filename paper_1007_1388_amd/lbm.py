"""ctypes binding of the C ABI in include/lbm.h (same names, argument marshalling only).

Every step of the method runs in the HIP library liblbm_hip.so.  This module
loads it on first use and raises ``LBMLibraryMissing`` when it is absent:
there is no CPU fallback.  PyTorch supplies device memory (its caching
allocator, through the lbm_params allocator hook) and the stream.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm_hip.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ESTATE, LBM_EUNSTABLE = range(6)
LBM_F64, LBM_F32, LBM_F16S, LBM_BF16S = range(4)
LBM_PERIODIC, LBM_WALL, LBM_VELOCITY, LBM_PRESSURE = 0, 1, 2, 3
PRECISIONS = {"f64": LBM_F64, "f32": LBM_F32, "f16s": LBM_F16S, "bf16s": LBM_BF16S}
STORAGE_DTYPE = {LBM_F64: np.float64, LBM_F32: np.float32, LBM_F16S: np.uint16, LBM_BF16S: np.uint16}
FACES = ("-x", "+x", "-y", "+y", "-z", "+z")


class LBMLibraryMissing(RuntimeError):
    pass


class LBMError(RuntimeError):
    def __init__(self, status, where, detail=""):
        self.status = status
        super().__init__("%s: status %d (%s) %s" % (where, status, _STATUS_NAMES.get(status, "?"), detail))


_STATUS_NAMES = {0: "ok", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ESTATE", 5: "EUNSTABLE"}

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class lbm_aabb(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int32 * 3), ("hi", ctypes.c_int32 * 3)]


class lbm_params(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 3), ("face", ctypes.c_int32 * 6),
                ("wall_u", (ctypes.c_double * 3) * 6), ("tau", ctypes.c_double),
                ("rho0", ctypes.c_double), ("force", ctypes.c_double * 3),
                ("precision", ctypes.c_int32), ("fp64_math", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN),
                ("alloc_user", ctypes.c_void_p), ("row_pad", ctypes.c_int32),
                ("face_rho", ctypes.c_double * 6)]


class lbm_schedule(ctypes.Structure):
    _fields_ = [("fused_exchange", ctypes.c_int32), ("item_cells", ctypes.c_int32),
                ("wg_size", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("graph_steps", ctypes.c_int32), ("nontemporal", ctypes.c_int32),
                ("cells_per_lane", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class lbm_info(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int64), ("n_fluid", ctypes.c_int64), ("n_blocks", ctypes.c_int32),
                ("n_items", ctypes.c_int32), ("steps", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("bytes_per_update", ctypes.c_double), ("storage_bytes", ctypes.c_int32),
                ("has_obstacles", ctypes.c_int32)]

    def as_dict(self):
        return {k: (float(getattr(self, k)) if k == "bytes_per_update" else int(getattr(self, k)))
                for k, _ in self._fields_}


# The exported symbols of include/lbm.h, in declaration order.
SYMBOLS = ["lbm_create_blocks", "lbm_set_geometry", "lbm_set_equilibrium", "lbm_step", "lbm_step_persistent",
           "lbm_step_timed", "lbm_macroscopic", "lbm_residual", "lbm_residual_mark", "lbm_residual_since_mark",
           "lbm_sums", "lbm_sums_noalloc", "lbm_get_state", "lbm_set_state", "lbm_average_two_steps",
           "lbm_get_schedule", "lbm_set_schedule", "lbm_set_host_blocks", "lbm_step_host_timed",
           "lbm_balance_host_blocks", "lbm_autotune", "lbm_info_get", "lbm_destroy",
           "lbm_strerror", "lbm_last_error", "lbm_bw_probe", "lbm_hbm_probe"]

_lib = None


def load(path=LIB_PATH):
    """Load liblbm_hip.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise LBMLibraryMissing("HIP library %s is not built; run python -m paper_1007_1388_amd.build" % path)
    try:
        import torch  # noqa: F401  (loads the HIP runtime that the library binds to)
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    st = ctypes.c_int
    sig = {
        "lbm_create_blocks": [ctypes.POINTER(lbm_params), ctypes.POINTER(lbm_aabb), ctypes.c_int32,
                              ctypes.POINTER(ctypes.c_void_p)],
        "lbm_set_geometry": [P, P],
        "lbm_set_equilibrium": [P, dp, dp],
        "lbm_step": [P, ctypes.c_int64],
        "lbm_step_persistent": [P, ctypes.c_int64, ctypes.c_int32],
        "lbm_step_timed": [P, ctypes.c_int64, dp, dp],
        "lbm_macroscopic": [P, P, P, ctypes.c_int32],
        "lbm_residual": [P, dp],
        "lbm_residual_mark": [P],
        "lbm_residual_since_mark": [P, dp, ctypes.POINTER(ctypes.c_int64)],
        "lbm_sums": [P, dp, dp],
        "lbm_sums_noalloc": [P, dp, dp],
        "lbm_get_state": [P, P, ctypes.c_int32],
        "lbm_set_state": [P, P, ctypes.c_int32],
        "lbm_average_two_steps": [P],
        "lbm_get_schedule": [P, ctypes.POINTER(lbm_schedule)],
        "lbm_set_schedule": [P, ctypes.POINTER(lbm_schedule)],
        "lbm_set_host_blocks": [P, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_int32],
        "lbm_step_host_timed": [P, ctypes.c_int64, dp, dp, dp, dp],
        "lbm_balance_host_blocks": [P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), dp, dp],
        "lbm_autotune": [P, ctypes.c_char_p, ctypes.c_int32, ctypes.POINTER(lbm_schedule)],
        "lbm_info_get": [P, ctypes.POINTER(lbm_info)],
        "lbm_destroy": [P],
        "lbm_bw_probe": [P, P, ctypes.c_size_t, ctypes.c_int32, P, dp],
        "lbm_hbm_probe": [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P, ctypes.c_size_t, ctypes.c_int32,
                          ctypes.c_int32, P, dp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = st
    lib.lbm_strerror.argtypes = [ctypes.c_int]
    lib.lbm_strerror.restype = ctypes.c_char_p
    lib.lbm_last_error.argtypes = []
    lib.lbm_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status, where):
    if status != LBM_OK:
        detail = load().lbm_last_error().decode(errors="replace")
        raise LBMError(status, where, detail)


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---------------------------------------------------------------- C names ---

def lbm_create_blocks(params, blocks):
    lib = load()
    arr = (lbm_aabb * len(blocks))()
    for k, (lo, hi) in enumerate(blocks):
        arr[k].lo[:] = list(lo)
        arr[k].hi[:] = list(hi)
    h = ctypes.c_void_p()
    _check(lib.lbm_create_blocks(ctypes.byref(params), arr, len(blocks), ctypes.byref(h)),
           "lbm_create_blocks")
    return h


def lbm_set_geometry(ctx, solid):
    if solid is None:
        _check(load().lbm_set_geometry(ctx, None), "lbm_set_geometry")
    else:
        s = np.ascontiguousarray(solid, dtype=np.uint8)
        _check(load().lbm_set_geometry(ctx, s.ctypes.data), "lbm_set_geometry")


def lbm_set_equilibrium(ctx, rho, u):
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    _check(load().lbm_set_equilibrium(ctx, _dptr(rho), _dptr(u)), "lbm_set_equilibrium")


def lbm_step(ctx, n):
    _check(load().lbm_step(ctx, int(n)), "lbm_step")


def lbm_step_persistent(ctx, n, steps_per_launch):
    _check(load().lbm_step_persistent(ctx, int(n), int(steps_per_launch)), "lbm_step_persistent")


def lbm_step_timed(ctx, n):
    """n steps with per-launch HIP events: (mean sweep ms, mean exchange ms)."""
    a = ctypes.c_double()
    b = ctypes.c_double()
    _check(load().lbm_step_timed(ctx, int(n), ctypes.byref(a), ctypes.byref(b)), "lbm_step_timed")
    return a.value, b.value


def lbm_macroscopic(ctx, rho, u, dst_is_device):
    _check(load().lbm_macroscopic(ctx, rho, u, int(dst_is_device)), "lbm_macroscopic")


def lbm_residual(ctx):
    r = ctypes.c_double()
    _check(load().lbm_residual(ctx, ctypes.byref(r)), "lbm_residual")
    return r.value


def lbm_residual_mark(ctx):
    _check(load().lbm_residual_mark(ctx), "lbm_residual_mark")


def lbm_residual_since_mark(ctx):
    r = ctypes.c_double()
    n = ctypes.c_int64()
    _check(load().lbm_residual_since_mark(ctx, ctypes.byref(r), ctypes.byref(n)), "lbm_residual_since_mark")
    return r.value, n.value


def lbm_sums(ctx):
    m = ctypes.c_double()
    p = (ctypes.c_double * 3)()
    _check(load().lbm_sums(ctx, ctypes.byref(m), p), "lbm_sums")
    return m.value, np.array(list(p))


def lbm_sums_noalloc(ctx):
    """lbm_sums with the reduction scratch in the library's static device array."""
    m = ctypes.c_double()
    p = (ctypes.c_double * 3)()
    _check(load().lbm_sums_noalloc(ctx, ctypes.byref(m), p), "lbm_sums_noalloc")
    return m.value, np.array(p[:])


def lbm_get_state(ctx, out, as_fp64):
    _check(load().lbm_get_state(ctx, out.ctypes.data, int(as_fp64)), "lbm_get_state")


def lbm_set_state(ctx, f, as_fp64):
    _check(load().lbm_set_state(ctx, f.ctypes.data, int(as_fp64)), "lbm_set_state")


def lbm_average_two_steps(ctx):
    _check(load().lbm_average_two_steps(ctx), "lbm_average_two_steps")


def lbm_get_schedule(ctx):
    s = lbm_schedule()
    _check(load().lbm_get_schedule(ctx, ctypes.byref(s)), "lbm_get_schedule")
    return s


def lbm_set_schedule(ctx, s):
    _check(load().lbm_set_schedule(ctx, ctypes.byref(s)), "lbm_set_schedule")


def lbm_set_host_blocks(ctx, ids, threads=0):
    ids = [int(j) for j in ids]
    arr = (ctypes.c_int32 * max(1, len(ids)))(*ids)
    _check(load().lbm_set_host_blocks(ctx, arr if ids else None, len(ids), int(threads)), "lbm_set_host_blocks")


def lbm_step_host_timed(ctx, n):
    """n heterogeneous steps: mean (GPU sweep, host sweep, exchange, step) ms."""
    v = [ctypes.c_double() for _ in range(4)]
    _check(load().lbm_step_host_timed(ctx, int(n), *[ctypes.byref(x) for x in v]), "lbm_step_host_timed")
    return tuple(x.value for x in v)


def lbm_balance_host_blocks(ctx, threads=0, trial_steps=20):
    """Static load balance: (host Block count k, ms per step GPU alone, ms per step of the split tried)."""
    k = ctypes.c_int32()
    a = ctypes.c_double()
    b = ctypes.c_double()
    _check(load().lbm_balance_host_blocks(ctx, int(threads), int(trial_steps), ctypes.byref(k), ctypes.byref(a),
                                          ctypes.byref(b)), "lbm_balance_host_blocks")
    return k.value, a.value, b.value


def lbm_autotune(ctx, cache_path=None, trial_steps=10):
    s = lbm_schedule()
    cp = cache_path.encode() if cache_path else None
    _check(load().lbm_autotune(ctx, cp, int(trial_steps), ctypes.byref(s)), "lbm_autotune")
    return s


def lbm_info_get(ctx):
    i = lbm_info()
    _check(load().lbm_info_get(ctx, ctypes.byref(i)), "lbm_info_get")
    return i


def lbm_destroy(ctx):
    _check(load().lbm_destroy(ctx), "lbm_destroy")


def lbm_strerror(status):
    return load().lbm_strerror(int(status)).decode()


def lbm_bw_probe(dst_ptr, src_ptr, nbytes, reps, stream):
    ms = ctypes.c_double()
    _check(load().lbm_bw_probe(dst_ptr, src_ptr, int(nbytes), int(reps), stream, ctypes.byref(ms)),
           "lbm_bw_probe")
    return ms.value


def lbm_hbm_probe(kind, unroll, nontemporal, a_ptr, b_ptr, nbytes, grid, reps, stream):
    """Mean milliseconds per pass of an HBM access pattern (0 read, 1 write,
    2 copy); see lbm.h."""
    ms = ctypes.c_double()
    _check(load().lbm_hbm_probe(int(kind), int(unroll), int(nontemporal), a_ptr, b_ptr, int(nbytes), int(grid),
                                int(reps), stream, ctypes.byref(ms)), "lbm_hbm_probe")
    return ms.value


# ----------------------------------------------------------- convenience ---

def make_params(dims, walls=(False, False, False), wall_u=None, tau=0.6, rho0=1.0,
                force=(0.0, 0.0, 0.0), precision="f32", fp64_math=False, stream=None, row_pad=0,
                open_x=None, open_faces=None):
    """open_faces = {face: ("velocity", (ux, uy, uz)) | ("pressure", rho) |
    "wall"}, faces of one axis ("-x"/"+x", "-y"/"+y" or "-z"/"+z"): open faces
    (non-equilibrium extrapolation); a face of that axis not named keeps what
    `walls` says for it (which must then be True).  open_x: the older name."""
    p = lbm_params()
    p.dims[:] = [int(d) for d in dims]
    for k in range(3):
        f = LBM_WALL if walls[k] else LBM_PERIODIC
        p.face[2 * k] = f
        p.face[2 * k + 1] = f
    for face, vel in (wall_u or {}).items():
        for a in range(3):
            p.wall_u[FACES.index(face)][a] = float(vel[a])
    for face, spec in dict(open_x or {}, **(open_faces or {})).items():
        k = FACES.index(face)
        if spec == "wall":
            p.face[k] = LBM_WALL
        elif spec[0] == "velocity":
            p.face[k] = LBM_VELOCITY
            for a in range(3):
                p.wall_u[k][a] = float(spec[1][a])
        elif spec[0] == "pressure":
            p.face[k] = LBM_PRESSURE
            p.face_rho[k] = float(spec[1])
        else:
            raise ValueError("bad open face %r" % (spec,))
    p.tau = float(tau)
    p.rho0 = float(rho0)
    p.force[:] = [float(v) for v in force]
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.fp64_math = 1 if fp64_math else 0
    p.stream = stream
    p.row_pad = int(row_pad)
    return p


class _TorchAllocator:
    """lbm_params allocator hook backed by torch's caching allocator."""

    def __init__(self, stream_ptr):
        import torch
        self.torch = torch
        self.device = torch.cuda.current_device()
        self.stream = stream_ptr
        self.alloc = ALLOC_FN(self._alloc)
        self.free = FREE_FN(self._free)

    def _alloc(self, nbytes, user):
        try:
            return self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
        except Exception:
            return None

    def _free(self, ptr, user):
        try:
            self.torch.cuda.caching_allocator_delete(ptr)
        except Exception:
            pass


class Lattice:
    """One lbm_ctx: a Patch split into Blocks on the current GPU.

    Arrays are numpy with cell index (z, y, x) and vector fields (3, z, y, x).
    """

    def __init__(self, dims, blocks=None, walls=(False, False, False), wall_u=None, tau=0.6,
                 rho0=1.0, force=(0.0, 0.0, 0.0), precision="f32", fp64_math=False,
                 stream=None, torch_alloc=True, row_pad=0, open_x=None, open_faces=None):
        load()
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the lattice runs only on the HIP device")
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        self.dims = tuple(int(d) for d in dims)
        nx, ny, nz = self.dims
        self.shape = (nz, ny, nx)
        self.ncell = nx * ny * nz
        if blocks is None:
            blocks = [((0, 0, 0), self.dims)]
        self.blocks = [tuple(map(tuple, b)) for b in blocks]
        self.params = make_params(dims, walls, wall_u, tau, rho0, force, precision, fp64_math, stream,
                                  row_pad, open_x, open_faces)
        self._alloc = None
        if torch_alloc:
            self._alloc = _TorchAllocator(stream)
            self.params.dev_alloc = self._alloc.alloc
            self.params.dev_free = self._alloc.free
        self.precision = self.params.precision
        self.ctx = lbm_create_blocks(self.params, self.blocks)

    def close(self):
        if getattr(self, "ctx", None):
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_geometry(self, solid=None):
        lbm_set_geometry(self.ctx, None if solid is None else np.asarray(solid).reshape(self.shape))

    def set_equilibrium(self, rho, u):
        lbm_set_equilibrium(self.ctx, np.asarray(rho).reshape(self.shape),
                            np.asarray(u).reshape((3,) + self.shape))

    def step(self, n=1):
        lbm_step(self.ctx, n)

    def step_persistent(self, n, steps_per_launch=100):
        """n steps as persistent launches (grid barrier per step, fused exchange)."""
        lbm_step_persistent(self.ctx, n, steps_per_launch)

    def step_timed(self, n):
        """Advance n steps launch by launch; returns (sweep ms, exchange ms)
        per launch, from HIP events on the context's stream."""
        return lbm_step_timed(self.ctx, n)

    def macroscopic(self):
        rho = np.empty(self.shape)
        u = np.empty((3,) + self.shape)
        lbm_macroscopic(self.ctx, rho.ctypes.data, u.ctypes.data, 0)
        return rho, u

    def macroscopic_device(self):
        import torch
        rho = torch.empty(self.shape, dtype=torch.float64, device="cuda")
        u = torch.empty((3,) + self.shape, dtype=torch.float64, device="cuda")
        lbm_macroscopic(self.ctx, rho.data_ptr(), u.data_ptr(), 1)
        return rho, u

    def residual(self):
        return lbm_residual(self.ctx)

    def residual_mark(self):
        """Snapshot the current velocity field for residual_since_mark."""
        lbm_residual_mark(self.ctx)

    def residual_since_mark(self):
        """(||u^n - u^mark|| / ||u^n||, steps since the mark)."""
        return lbm_residual_since_mark(self.ctx)

    def sums(self):
        return lbm_sums(self.ctx)

    def get_state(self, as_fp64=True):
        dt = np.float64 if as_fp64 else STORAGE_DTYPE[self.precision]
        f = np.empty((19,) + self.shape, dtype=dt)
        lbm_get_state(self.ctx, f, as_fp64)
        return f

    def set_state(self, f, as_fp64=True):
        dt = np.float64 if as_fp64 else STORAGE_DTYPE[self.precision]
        lbm_set_state(self.ctx, np.ascontiguousarray(f, dtype=dt).reshape((19,) + self.shape), as_fp64)

    def average_two_steps(self):
        """Replace the state by the mean of this step's and the previous
        step's (removes period-two components of a state set from outside)."""
        lbm_average_two_steps(self.ctx)

    @property
    def schedule(self):
        return lbm_get_schedule(self.ctx).as_dict()

    def set_schedule(self, **kw):
        s = lbm_get_schedule(self.ctx)
        for k, v in kw.items():
            setattr(s, k, int(v))
        lbm_set_schedule(self.ctx, s)

    def autotune(self, cache_path=None, trial_steps=10):
        return lbm_autotune(self.ctx, cache_path, trial_steps).as_dict()

    def set_host_blocks(self, ids, threads=0):
        """Run the Blocks with these BlockIDs on the host CPU (Sec. 4.5); [] returns all to the GPU."""
        lbm_set_host_blocks(self.ctx, ids, threads)

    def step_host_timed(self, n):
        """n steps with host Blocks: mean (GPU sweep, host sweep, exchange, whole step) in ms."""
        return lbm_step_host_timed(self.ctx, n)

    def balance_host_blocks(self, threads=0, trial_steps=20):
        """Static load balance between the GPU and the host CPU; returns
        (k, ms GPU alone, ms with the split tried), the last k Blocks on the host."""
        return lbm_balance_host_blocks(self.ctx, threads, trial_steps)

    def info(self):
        return lbm_info_get(self.ctx).as_dict()
