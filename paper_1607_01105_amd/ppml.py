"""ctypes binding of the C ABI in ``include/ppml.h``.

Argument marshalling only: every step of the method runs in the HIP kernels
of ``csrc/libppml.so``.  PyTorch supplies device memory (``torch.empty`` on
the GPU) and the HIP stream.  If the library is missing this module raises;
there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "csrc", "libppml.so")
LIB_EXACT_PATH = os.path.join(HERE, "csrc", "libppml_exact.so")

PPML_OK, PPML_EINVAL, PPML_ENOMEM, PPML_EHIP, PPML_ENONFINITE, PPML_EBUDGET, PPML_ESTATE = 0, -1, -2, -3, -4, -5, -6
PPML_FP32, PPML_FP64 = 0, 1
PPML_PERIODIC, PPML_OUTFLOW, PPML_REFLECT, PPML_INFLOW = 0, 1, 2, 3
PPML_RHO, PPML_MX, PPML_MY, PPML_MZ, PPML_ETOT, PPML_EINT = 0, 1, 2, 3, 4, 5
PPML_POT_NONE, PPML_POT_LOG, PPML_POT_UNIFORM, PPML_POT_HALO = 0, 1, 2, 3
PPML_FLAG_FIRST_ORDER, PPML_FLAG_ISOTHERMAL = 1, 2

BC = {"periodic": PPML_PERIODIC, "outflow": PPML_OUTFLOW, "reflect": PPML_REFLECT, "inflow": PPML_INFLOW}
PREC = {"fp32": PPML_FP32, "f32": PPML_FP32, "fp64": PPML_FP64, "f64": PPML_FP64}
POT = {None: PPML_POT_NONE, "none": PPML_POT_NONE, "log": PPML_POT_LOG, "uniform": PPML_POT_UNIFORM,
       "halo": PPML_POT_HALO}


class ppml_desc(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32), ("prec", C.c_int32), ("n", C.c_int64 * 3),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("gamma", C.c_double), ("cfl", C.c_double),
        ("bc_lo", C.c_int32 * 3), ("bc_hi", C.c_int32 * 3), ("vacuum_ratio", C.c_double),
        ("potential", C.c_int32), ("flags", C.c_int32), ("pot", C.c_double * 8),
        ("tile", C.c_int32), ("self_gravity", C.c_int32), ("inflow", (C.c_double * 5) * 6),
        ("grav_G", C.c_double), ("iso_cs", C.c_double),
    ]


class PPMLError(RuntimeError):
    def __init__(self, status, detail):
        super().__init__(f"ppml status {status}: {detail}")
        self.status = status


# functions exported by the library, as declared in include/ppml.h
EXPORTS = (
    "ppml_state_bytes", "ppml_scratch_bytes", "ppml_create", "ppml_set_primitive", "ppml_set_conserved",
    "ppml_step", "ppml_get_time", "ppml_max_speeds", "ppml_get_conserved", "ppml_totals", "ppml_sync",
    "ppml_destroy", "ppml_strerror", "ppml_last_error", "ppml_version", "ppml_set_timing", "ppml_get_timing",
    "ppml_batch_create", "ppml_batch_admit", "ppml_batch_retire", "ppml_batch_step", "ppml_batch_sync",
    "ppml_batch_info", "ppml_batch_destroy", "ppml_tile_count", "ppml_tile_shape", "ppml_batch_set_tile",
    "ppml_get_potential", "ppml_get_timing_split", "ppml_step_noalloc",
)

_libs: dict[str, C.CDLL] = {}


def load(path: str | None = None) -> C.CDLL:
    """Load the HIP library (after torch, so both share one HIP runtime)."""
    path = path or LIB_PATH
    if path in _libs:
        return _libs[path]
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run __graft_entry__.build())")
    import torch  # noqa: F401  -- loads the HIP runtime the library binds to

    lib = C.CDLL(path)
    dp = C.POINTER(C.c_double)
    vp = C.c_void_p
    D = C.POINTER(ppml_desc)
    lib.ppml_state_bytes.restype = C.c_size_t
    lib.ppml_state_bytes.argtypes = [D]
    lib.ppml_scratch_bytes.restype = C.c_size_t
    lib.ppml_scratch_bytes.argtypes = [D]
    lib.ppml_create.argtypes = [D, vp, vp, vp, C.POINTER(vp)]
    lib.ppml_set_primitive.argtypes = [vp, dp, dp, dp, dp, dp]
    lib.ppml_set_conserved.argtypes = [vp, C.POINTER(dp), C.c_double, C.c_double]
    lib.ppml_step.argtypes = [vp, C.c_int32, C.c_double, C.c_double]
    lib.ppml_get_time.argtypes = [vp, dp, dp, C.POINTER(C.c_int64)]
    lib.ppml_max_speeds.argtypes = [vp, dp, dp]
    lib.ppml_get_conserved.argtypes = [vp, C.c_int32, dp]
    lib.ppml_totals.argtypes = [vp, dp]
    lib.ppml_sync.argtypes = [vp]
    lib.ppml_destroy.argtypes = [vp]
    lib.ppml_set_timing.argtypes = [vp, C.c_int32]
    lib.ppml_get_timing.argtypes = [vp, dp, dp, C.POINTER(C.c_int64)]
    lib.ppml_get_timing_split.argtypes = [vp, dp, C.POINTER(C.c_int64)]
    lib.ppml_get_potential.argtypes = [vp, dp]
    lib.ppml_batch_create.argtypes = [C.c_int32, C.c_size_t, vp, C.POINTER(vp)]
    lib.ppml_batch_admit.argtypes = [vp, vp, C.POINTER(C.c_int32)]
    lib.ppml_batch_retire.argtypes = [vp, C.c_int32]
    lib.ppml_batch_step.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.c_double, C.c_double, C.c_int32]
    lib.ppml_batch_sync.argtypes = [vp]
    lib.ppml_batch_info.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_size_t)]
    lib.ppml_batch_destroy.argtypes = [vp]
    lib.ppml_tile_count.argtypes = [C.c_int32]
    lib.ppml_tile_shape.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.ppml_batch_set_tile.argtypes = [vp, C.c_int32, C.c_int32]
    lib.ppml_step_noalloc.argtypes = [D, vp, C.c_double, C.c_double, C.c_int32, C.c_double, C.c_double, vp, dp,
                                      C.POINTER(C.c_int64)]
    lib.ppml_strerror.restype = C.c_char_p
    lib.ppml_strerror.argtypes = [C.c_int]
    lib.ppml_last_error.restype = C.c_char_p
    lib.ppml_last_error.argtypes = []
    lib.ppml_version.restype = C.c_int
    for name in EXPORTS:
        if name not in ("ppml_state_bytes", "ppml_scratch_bytes", "ppml_strerror", "ppml_last_error", "ppml_version"):
            getattr(lib, name).restype = C.c_int
    _libs[path] = lib
    return lib


def _check(lib, rc):
    if rc != PPML_OK:
        raise PPMLError(rc, lib.ppml_last_error().decode())
    return rc


def make_desc(ndim, n, lo, hi, gamma, cfl, bc="periodic", prec="fp64", vacuum_ratio=1e-5, potential=None,
              first_order=False, tile=0, inflow=None, self_gravity=None, isothermal=None):
    """Descriptor of a grid; self_gravity = G > 0 turns on the self-gravity
    potential (Sec. 2.5) with that gravitational constant; isothermal = cs > 0
    selects the isothermal variant p = cs^2 rho (Sec. 4)."""
    d = ppml_desc()
    d.ndim = int(ndim)
    d.prec = PREC[prec] if isinstance(prec, str) else int(prec)
    n = list(n) + [1] * (3 - len(n))
    lo = list(lo) + [0.0] * (3 - len(lo))
    hi = list(hi) + [1.0] * (3 - len(hi))
    for a in range(3):
        d.n[a] = int(n[a]) if a < ndim else 1
        d.lo[a] = float(lo[a])
        d.hi[a] = float(hi[a])
    if isinstance(bc, str):
        bcs = [(bc, bc)] * 3
    else:
        bcs = [tuple(b) if not isinstance(b, str) else (b, b) for b in bc] + [("periodic", "periodic")] * 3
    for a in range(3):
        d.bc_lo[a] = BC[bcs[a][0]] if a < ndim else PPML_PERIODIC
        d.bc_hi[a] = BC[bcs[a][1]] if a < ndim else PPML_PERIODIC
    d.gamma = float(gamma)
    d.cfl = float(cfl)
    d.vacuum_ratio = float(vacuum_ratio)
    d.potential = POT[potential[0]] if potential else PPML_POT_NONE
    d.flags = (PPML_FLAG_FIRST_ORDER if first_order else 0) | (PPML_FLAG_ISOTHERMAL if isothermal is not None else 0)
    d.iso_cs = float(isothermal) if isothermal is not None else 0.0
    d.tile = int(tile)
    d.self_gravity = 1 if self_gravity is not None else 0
    d.grav_G = float(self_gravity) if self_gravity is not None else 0.0
    for face, st in (inflow or {}).items():  # face 2*axis+side -> (rho, vx, vy, vz, p)
        for q in range(5):
            d.inflow[int(face)][q] = float(st[q])
    if potential:
        for i, v in enumerate(potential[1:]):
            d.pot[i] = float(v)
    return d


# ---- thin wrappers with the C names -------------------------------------
def ppml_state_bytes(desc, lib=None) -> int:
    return int((lib or load()).ppml_state_bytes(C.byref(desc)))


def ppml_scratch_bytes(desc, lib=None) -> int:
    return int((lib or load()).ppml_scratch_bytes(C.byref(desc)))


def ppml_create(desc, state_ptr: int, scratch_ptr: int, stream: int, lib=None):
    lib = lib or load()
    h = C.c_void_p()
    _check(lib, lib.ppml_create(C.byref(desc), C.c_void_p(state_ptr), C.c_void_p(scratch_ptr),
                                C.c_void_p(stream), C.byref(h)))
    return h


def ppml_step_noalloc(desc, state_ptr: int, nsteps: int, rho_mean0=0.0, t0=0.0, dt_fixed=0.0, t_stop=0.0,
                      stream: int = 0, sync=True, lib=None):
    """Allocation-free stepping of a state already on the device (see the
    header): returns (t, steps) when sync, else None."""
    lib = lib or load()
    t, n = C.c_double(), C.c_int64()
    _check(lib, lib.ppml_step_noalloc(C.byref(desc), C.c_void_p(state_ptr), float(rho_mean0), float(t0), int(nsteps),
                                      float(dt_fixed), float(t_stop), C.c_void_p(stream),
                                      C.byref(t) if sync else None, C.byref(n) if sync else None))
    return (t.value, n.value) if sync else None


def ppml_tile_count(ndim, lib=None) -> int:
    lib = lib or load()
    rc = lib.ppml_tile_count(int(ndim))
    if rc < 0:
        _check(lib, rc)
    return int(rc)


def ppml_tile_shape(ndim, variant, lib=None) -> tuple[int, int]:
    lib = lib or load()
    tx, ty = C.c_int32(), C.c_int32()
    _check(lib, lib.ppml_tile_shape(int(ndim), int(variant), C.byref(tx), C.byref(ty)))
    return tx.value, ty.value


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, n):
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64)).reshape(-1)
    if a.size != n:
        raise ValueError("array size does not match the grid")
    return a


class Grid:
    """One grid on the current GPU; state and scratch are torch tensors."""

    def __init__(self, ndim, n, lo, hi, gamma, cfl, bc="periodic", prec="fp64", vacuum_ratio=1e-5,
                 potential=None, device="cuda", stream=None, exact=False, first_order=False, lib_path=None, tile=0,
                 inflow=None, self_gravity=None, isothermal=None):
        import torch

        self.lib = load(lib_path or (LIB_EXACT_PATH if exact else LIB_PATH))
        self.desc = make_desc(ndim, n, lo, hi, gamma, cfl, bc, prec, vacuum_ratio, potential, first_order, tile,
                              inflow, self_gravity, isothermal)
        self.ndim = int(ndim)
        self.ncell = int(self.desc.n[0] * self.desc.n[1] * self.desc.n[2])
        sb = ppml_state_bytes(self.desc, self.lib)
        kb = ppml_scratch_bytes(self.desc, self.lib)
        if sb == 0 or kb == 0:
            raise PPMLError(PPML_EINVAL, self.lib.ppml_last_error().decode())
        self.device = torch.device(device)
        self.state = torch.empty(sb, dtype=torch.uint8, device=self.device)
        self.scratch = torch.empty(kb, dtype=torch.uint8, device=self.device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        self.h = ppml_create(self.desc, self.state.data_ptr(), self.scratch.data_ptr(), self.stream.cuda_stream,
                             self.lib)

    @classmethod
    def from_problem(cls, prob, prec="fp64", exact=False, vacuum_ratio=1e-5, **kw):
        kw.setdefault("inflow", getattr(prob, "inflow", None))
        kw.setdefault("self_gravity", getattr(prob, "self_gravity", None))
        kw.setdefault("isothermal", getattr(prob, "isothermal", None))
        g = cls(prob.ndim, prob.n, prob.lo, prob.hi, prob.gamma, prob.cfl, bc=prob.bc, prec=prec,
                vacuum_ratio=vacuum_ratio, potential=prob.potential, exact=exact, **kw)
        g.set_primitive(prob.rho, prob.vx, prob.vy, prob.vz, prob.p)
        return g

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.ppml_destroy(h)
            self.h = None

    @property
    def shape(self):
        return (int(self.desc.n[2]), int(self.desc.n[1]), int(self.desc.n[0]))

    def set_primitive(self, rho, vx=None, vy=None, vz=None, p=None):
        arrs = [_f64(a, self.ncell) for a in (rho, vx, vy, vz, p)]
        _check(self.lib, self.lib.ppml_set_primitive(self.h, *[_dp(a) for a in arrs]))

    def set_conserved(self, fields, rho_mean0=0.0, t=0.0):
        arrs = [_f64(f, self.ncell) if f is not None else None for f in fields]
        P = C.POINTER(C.c_double)
        ptrs = (P * 6)(*[(_dp(a) if a is not None else P()) for a in arrs])
        _check(self.lib, self.lib.ppml_set_conserved(self.h, ptrs, float(rho_mean0), float(t)))

    def step(self, nsteps=1, dt_fixed=0.0, t_stop=0.0):
        _check(self.lib, self.lib.ppml_step(self.h, int(nsteps), float(dt_fixed), float(t_stop)))

    def time(self):
        t, dt = C.c_double(), C.c_double()
        s = C.c_int64()
        _check(self.lib, self.lib.ppml_get_time(self.h, C.byref(t), C.byref(dt), C.byref(s)))
        return t.value, dt.value, s.value

    def max_speeds(self):
        v, c = C.c_double(), C.c_double()
        _check(self.lib, self.lib.ppml_max_speeds(self.h, C.byref(v), C.byref(c)))
        return v.value, c.value

    def get(self, field) -> np.ndarray:
        names = {"rho": 0, "mx": 1, "my": 2, "mz": 3, "Et": 4, "e": 5}
        f = names[field] if isinstance(field, str) else int(field)
        out = np.empty(self.shape, dtype=np.float64)
        _check(self.lib, self.lib.ppml_get_conserved(self.h, f, _dp(out)))
        return out

    def conserved(self):
        return [self.get(f) if (f in (0, 4, 5) or f - 1 < self.ndim) else np.zeros(self.shape) for f in range(6)]

    def totals(self) -> np.ndarray:
        out = np.zeros(6)
        _check(self.lib, self.lib.ppml_totals(self.h, _dp(out)))
        return out

    def sync(self):
        _check(self.lib, self.lib.ppml_sync(self.h))

    def set_timing(self, cap):
        _check(self.lib, self.lib.ppml_set_timing(self.h, int(cap)))

    def get_timing(self):
        a, b = C.c_double(), C.c_double()
        n = C.c_int64()
        _check(self.lib, self.lib.ppml_get_timing(self.h, C.byref(a), C.byref(b), C.byref(n)))
        return a.value, b.value, n.value

    def get_timing_split(self):
        """(ms gravity solve, ms Eulerian kernel, ms Lagrangian kernel, steps timed)."""
        ms = (C.c_double * 3)()
        n = C.c_int64()
        _check(self.lib, self.lib.ppml_get_timing_split(self.h, ms, C.byref(n)))
        return ms[0], ms[1], ms[2], n.value

    def potential(self) -> np.ndarray:
        """Self-gravity potential of the current state, shell included:
        shape (nz+2, ny+2, nx+2), FP64."""
        nz, ny, nx = self.shape
        out = np.empty((nz + 2, ny + 2, nx + 2), dtype=np.float64)
        _check(self.lib, self.lib.ppml_get_potential(self.h, _dp(out)))
        return out

    def run_to(self, t_stop, chunk=64, max_steps=10 ** 7):
        """Step until t_stop (CFL steps, the last one clipped)."""
        taken = 0
        while taken < max_steps:
            self.step(chunk, 0.0, t_stop)
            t, _, s = self.time()
            taken = s
            if t >= t_stop:
                break
        return self.time()


class Batch:
    """Many grids stepped together by the batched kernels (include/ppml.h,
    ppml_batch_*).  Grids must be created on the batch's stream (pass
    ``stream=batch.stream``) and have their state set before admission."""

    def __init__(self, capacity, budget_bytes=0, device="cuda", stream=None, exact=False):
        import torch

        self.lib = load(LIB_EXACT_PATH if exact else LIB_PATH)
        self.exact = exact
        self.device = torch.device(device)
        # a dedicated stream: HIP graphs cannot be captured on the NULL stream
        self.stream = stream or torch.cuda.Stream(self.device)
        self.capacity = int(capacity)
        h = C.c_void_p()
        _check(self.lib, self.lib.ppml_batch_create(self.capacity, C.c_size_t(int(budget_bytes)),
                                                    C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.grids = {}

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.ppml_batch_destroy(h)
            self.h = None

    def new_grid(self, prob, prec="fp32", vacuum_ratio=1e-5, stream=None):
        """A grid for this batch (same library), state set; on the batch's
        stream unless another is given (its state transfer then overlaps the
        batch's kernels)."""
        return Grid.from_problem(prob, prec=prec, exact=self.exact, vacuum_ratio=vacuum_ratio, device=self.device,
                                 stream=stream or self.stream)

    def side_stream(self):
        """A second stream on the batch's device, for preparing grids while the
        batch steps."""
        import torch

        return torch.cuda.Stream(self.device)

    def admit(self, grid) -> int:
        s = C.c_int32()
        _check(self.lib, self.lib.ppml_batch_admit(self.h, grid.h, C.byref(s)))
        self.grids[s.value] = grid
        return s.value

    def retire(self, slot):
        _check(self.lib, self.lib.ppml_batch_retire(self.h, int(slot)))
        return self.grids.pop(int(slot))

    def step(self, nsteps, steps_per_slot=None, dt_fixed=0.0, t_stop=0.0, graph=True):
        arr = None
        if steps_per_slot is not None:
            a = np.zeros(self.capacity, dtype=np.int32)
            for s, k in (steps_per_slot.items() if isinstance(steps_per_slot, dict) else enumerate(steps_per_slot)):
                a[int(s)] = int(k)
            self._steps = a
            arr = a.ctypes.data_as(C.POINTER(C.c_int32))
        _check(self.lib, self.lib.ppml_batch_step(self.h, int(nsteps), arr, float(dt_fixed), float(t_stop),
                                                  int(bool(graph))))

    def sync(self):
        _check(self.lib, self.lib.ppml_batch_sync(self.h))

    def info(self):
        n = C.c_int32()
        b = C.c_size_t()
        _check(self.lib, self.lib.ppml_batch_info(self.h, C.byref(n), C.byref(b)))
        return n.value, b.value

    def set_tile(self, ndim, variant):
        """Tile shape of the launches for grids of ndim dimensions (before any
        such grid is admitted)."""
        _check(self.lib, self.lib.ppml_batch_set_tile(self.h, int(ndim), int(variant)))

