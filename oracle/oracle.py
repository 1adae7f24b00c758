"""ctypes wrapper of the FP64 C oracle (``ppml_oracle.c``).

TEST INFRASTRUCTURE: see the package docstring.  Arrays are numpy float64
in C order ``[z][y][x]`` (interior cells only).

Field order of the conserved state (Sec. 2, eqs. (1)-(4)): rho, rho*vx,
rho*vy, rho*vz, rho*E, rho*eps.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ppml_oracle.c")
_LIB = os.path.join(_HERE, "libppml_oracle.so")

FIELDS = ("rho", "mx", "my", "mz", "Et", "e")
BC = {"periodic": 0, "outflow": 1, "reflect": 2, "inflow": 3}
POT = {None: 0, "none": 0, "log": 1, "uniform": 2, "halo": 3}

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c11"]


def lib_path() -> str:
    return _LIB


def build(src: str = _SRC, out: str = _LIB, extra: list[str] | None = None) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    cmd = ["gcc", *CFLAGS, *(extra or []), src, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


_cache: dict[str, C.CDLL] = {}


def load_library(path: str | None = None) -> C.CDLL:
    path = path or _LIB
    if path in _cache:
        return _cache[path]
    if not os.path.exists(path):
        if path == _LIB:
            build()
        else:
            raise FileNotFoundError(path)
    lib = C.CDLL(path)
    dp = C.POINTER(C.c_double)
    lp = C.POINTER(C.c_long)
    ip = C.POINTER(C.c_int)
    lib.og_create.restype = C.c_void_p
    lib.og_create.argtypes = [C.c_int, lp, dp, dp, C.c_double, C.c_double, ip, ip, C.c_double, C.c_int, dp, C.c_int]
    lib.og_destroy.argtypes = [C.c_void_p]
    lib.og_set_primitive.argtypes = [C.c_void_p, dp, dp, dp, dp, dp]
    lib.og_set_inflow.restype = None
    lib.og_set_inflow.argtypes = [C.c_void_p, C.c_int] + [C.c_double] * 5
    lib.og_set_conserved.argtypes = [C.c_void_p, C.POINTER(dp), C.c_double, C.c_double]
    lib.og_get.argtypes = [C.c_void_p, C.c_int, dp]
    lib.og_totals.argtypes = [C.c_void_p, dp]
    lib.og_time.restype = C.c_double
    lib.og_time.argtypes = [C.c_void_p]
    lib.og_rho_mean0.restype = C.c_double
    lib.og_rho_mean0.argtypes = [C.c_void_p]
    lib.og_dt.restype = C.c_double
    lib.og_dt.argtypes = [C.c_void_p]
    lib.og_max_speeds.argtypes = [C.c_void_p, dp, dp]
    lib.og_step.argtypes = [C.c_void_p, C.c_double]
    lib.og_run.restype = C.c_long
    lib.og_run.argtypes = [C.c_void_p, C.c_long, C.c_double, C.c_double, dp]
    lib.og_last_max_z_euler.restype = C.c_double
    lib.og_last_max_z_euler.argtypes = [C.c_void_p]
    lib.og_last_max_z_lagr.restype = C.c_double
    lib.og_last_max_z_lagr.argtypes = [C.c_void_p]
    lib.og_reconstruct_line.argtypes = [dp, C.c_long, dp, dp, dp, dp, dp]
    lib.og_avg_left.restype = C.c_double
    lib.og_avg_left.argtypes = [C.c_double] * 4
    lib.og_max_threads.restype = C.c_int
    lib.og_max_threads.argtypes = []
    lib.og_set_threads.restype = None
    lib.og_set_threads.argtypes = [C.c_int]
    lib.og_set_isothermal.restype = C.c_int
    lib.og_set_isothermal.argtypes = [C.c_void_p, C.c_double]
    lib.og_set_self_gravity.restype = C.c_int
    lib.og_set_self_gravity.argtypes = [C.c_void_p, C.c_double]
    lib.og_multipole_moments.restype = None
    lib.og_multipole_moments.argtypes = [C.c_void_p, dp]
    lib.og_multipole_value.restype = C.c_double
    lib.og_multipole_value.argtypes = [dp, C.c_double, C.c_double, C.c_double, C.c_double]
    lib.og_sine_transform.restype = None
    lib.og_sine_transform.argtypes = [dp, C.c_long, dp]
    lib.og_potential.restype = C.c_int
    lib.og_potential.argtypes = [C.c_void_p, dp]
    lib.og_avg_right.restype = C.c_double
    lib.og_avg_right.argtypes = [C.c_double] * 4
    _cache[path] = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def max_threads(lib: C.CDLL | None = None) -> int:
    """Threads the oracle's OpenMP loops use."""
    return int((lib or load_library()).og_max_threads())


def set_threads(n: int, lib: C.CDLL | None = None) -> None:
    """Threads for the oracle's OpenMP loops from now on (timing only)."""
    (lib or load_library()).og_set_threads(int(n))


def reconstruct_line(q, lib: C.CDLL | None = None):
    """Parabolas (qL, qR, q6) of cells 2..n-3 of the line q (Appendix, steps 1-3)."""
    lib = lib or load_library()
    q = _f64(q)
    n = q.size
    qL, qR, q6, dm, qI = (np.full(n, np.nan) for _ in range(5))
    lib.og_reconstruct_line(_dp(q), n, _dp(qL), _dp(qR), _dp(q6), _dp(dm), _dp(qI))
    return qL, qR, q6


def sine_transform(x, lib: C.CDLL | None = None) -> np.ndarray:
    """y_j = sum_k x_k sin(pi j k / (n+1)), j, k = 1..n (Sec. 2.5, stages 2-3)."""
    lib = lib or load_library()
    x = _f64(x)
    y = np.empty_like(x)
    lib.og_sine_transform(_dp(x), x.size, _dp(y))
    return y


def multipole_value(mom, G, x, y, z, lib: C.CDLL | None = None) -> float:
    """Two-term multipole potential at (x, y, z) of the moments
    mom = (M, Ix, Iy, Iz, Ixy, Ixz, Iyz) (Sec. 2.5, stage 1)."""
    lib = lib or load_library()
    m = _f64(mom)
    return lib.og_multipole_value(_dp(m), float(G), float(x), float(y), float(z))


def avg_left(qL, qR, q6, z, lib: C.CDLL | None = None) -> float:
    return (lib or load_library()).og_avg_left(qL, qR, q6, z)


def avg_right(qL, qR, q6, z, lib: C.CDLL | None = None) -> float:
    return (lib or load_library()).og_avg_right(qL, qR, q6, z)


class Oracle:
    """One grid of the FP64 oracle.

    ``n`` is (nx[, ny[, nz]]); ``lo``/``hi`` the domain extents per axis;
    ``bc`` a boundary name or a per-axis list of (lo, hi) names;
    ``potential`` None, ("log", v0, rc, q, cx, cy, cz) or ("uniform", gx, gy, gz);
    ``inflow`` maps a face (2 * axis + side, side 0 low / 1 high) with an
    "inflow" boundary to its ghost state (rho, vx, vy, vz, p);
    ``self_gravity`` = G > 0 adds the force of the potential of the gas's own
    mass (Sec. 2.5; 3-D, cubic cells); ``isothermal`` = cs > 0 selects the
    isothermal variant p = cs^2 rho (Sec. 4).
    """

    def __init__(self, ndim, n, lo, hi, gamma, cfl, bc="periodic", vacuum_ratio=1e-5,
                 potential=None, first_order=False, lib: C.CDLL | str | None = None, inflow=None,
                 self_gravity=None, isothermal=None):
        self.lib = lib if isinstance(lib, C.CDLL) else load_library(lib)
        self.ndim = int(ndim)
        n = list(n) + [1] * (3 - len(n))
        lo = list(lo) + [0.0] * (3 - len(lo))
        hi = list(hi) + [1.0] * (3 - len(hi))
        self.n = tuple(int(v) for v in n)
        if isinstance(bc, str):
            bcs = [(bc, bc)] * 3
        else:
            bcs = [tuple(b) if not isinstance(b, str) else (b, b) for b in bc]
            bcs += [("periodic", "periodic")] * (3 - len(bcs))
        blo = (C.c_int * 3)(*[BC[b[0]] for b in bcs])
        bhi = (C.c_int * 3)(*[BC[b[1]] for b in bcs])
        pot = np.zeros(8)
        kind = 0
        if potential is not None:
            kind = POT[potential[0]]
            vals = list(potential[1:])
            pot[: len(vals)] = vals
        self._pot = pot
        self.gamma = float(gamma)
        self.h = [(hi[a] - lo[a]) / n[a] for a in range(3)]
        self.g = self.lib.og_create(
            self.ndim, (C.c_long * 3)(*self.n), (C.c_double * 3)(*lo), (C.c_double * 3)(*hi),
            float(gamma), float(cfl), blo, bhi, float(vacuum_ratio), kind, _dp(pot), int(bool(first_order)))
        if not self.g:
            raise ValueError("og_create failed")
        for face, st in (inflow or {}).items():
            self.lib.og_set_inflow(self.g, int(face), *[float(v) for v in st])
        if isothermal is not None:
            if self.lib.og_set_isothermal(self.g, float(isothermal)) != 0:
                raise ValueError("isothermal sound speed must be > 0")
        if self_gravity is not None:
            if self.lib.og_set_self_gravity(self.g, float(self_gravity)) != 0:
                raise ValueError("self-gravity needs a 3-D grid of cubic cells")

    def __del__(self):
        g = getattr(self, "g", None)
        if g:
            self.lib.og_destroy(g)
            self.g = None

    @property
    def shape(self):
        nx, ny, nz = self.n
        return (nz, ny, nx)

    def _arr(self, a):
        if a is None:
            return None
        a = _f64(a)
        if a.size != self.n[0] * self.n[1] * self.n[2]:
            raise ValueError("array size does not match grid")
        return a

    def set_primitive(self, rho, vx=None, vy=None, vz=None, p=None):
        arrs = [self._arr(x) for x in (rho, vx, vy, vz, p)]
        self._keep = arrs
        ptrs = [(_dp(a) if a is not None else None) for a in arrs]
        self.lib.og_set_primitive(self.g, *ptrs)

    def set_conserved(self, fields, rho_mean0=0.0, t=0.0):
        arrs = [self._arr(f) for f in fields]
        P = C.POINTER(C.c_double)
        ptrs = (P * 6)(*[(_dp(a) if a is not None else P()) for a in arrs])
        self.lib.og_set_conserved(self.g, ptrs, float(rho_mean0), float(t))

    def get(self, field) -> np.ndarray:
        f = FIELDS.index(field) if isinstance(field, str) else int(field)
        out = np.empty(self.shape, dtype=np.float64)
        self.lib.og_get(self.g, f, _dp(out))
        return out

    def conserved(self) -> list[np.ndarray]:
        return [self.get(f) for f in range(6)]

    def totals(self) -> np.ndarray:
        out = np.zeros(6)
        self.lib.og_totals(self.g, _dp(out))
        return out

    @property
    def t(self) -> float:
        return self.lib.og_time(self.g)

    @property
    def rho_mean0(self) -> float:
        return self.lib.og_rho_mean0(self.g)

    def dt(self) -> float:
        return self.lib.og_dt(self.g)

    def max_speeds(self):
        vm, cm = C.c_double(), C.c_double()
        self.lib.og_max_speeds(self.g, C.byref(vm), C.byref(cm))
        return vm.value, cm.value

    def step(self, tau: float):
        self.lib.og_step(self.g, float(tau))

    def run(self, nsteps: int, dt_fixed: float = 0.0, t_stop: float = 0.0) -> np.ndarray:
        taus = np.zeros(max(int(nsteps), 1))
        k = self.lib.og_run(self.g, int(nsteps), float(dt_fixed), float(t_stop), _dp(taus))
        return taus[:k].copy()

    @property
    def last_max_z_euler(self) -> float:
        return self.lib.og_last_max_z_euler(self.g)

    @property
    def last_max_z_lagr(self) -> float:
        return self.lib.og_last_max_z_lagr(self.g)

    def potential(self) -> np.ndarray:
        """Self-gravity potential of the current state on the interior cells
        and the one-cell shell around them: shape (nz+2, ny+2, nx+2)."""
        nx, ny, nz = self.n
        out = np.empty((nz + 2, ny + 2, nx + 2))
        if self.lib.og_potential(self.g, _dp(out)) != 0:
            raise ValueError("self-gravity is off")
        return out

    def moments(self) -> np.ndarray:
        """(M, Ix, Iy, Iz, Ixy, Ixz, Iyz) of the cell masses (Sec. 2.5, stage 1)."""
        out = np.zeros(7)
        self.lib.og_multipole_moments(self.g, _dp(out))
        return out

    def primitive(self):
        r = self.get("rho")
        out = {"rho": r, "vx": self.get("mx") / r, "vy": self.get("my") / r, "vz": self.get("mz") / r,
               "p": (self.gamma - 1.0) * self.get("e")}
        return out
