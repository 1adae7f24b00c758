"""Seeded synthetic inputs (primitive variables rho, v, p at cell centres).

This module holds no arithmetic of the method: it only draws and lays out
initial data, so that the GPU path and the CPU oracle can start from the
same arrays.  Every generator returns a :class:`Problem` whose arrays are
float64 numpy arrays in C order ``[z][y][x]`` (interior cells only).

Generators and the paper's workloads they stand in for:

* :func:`riemann_1d`     -- seeded 1-D Riemann problems (shock tubes of the
  verification section, random left/right states).
* :func:`shock_tube`     -- the three shock tubes of the paper's Table
  "Initial state of the shock tube problem".
* :func:`periodic_modes` -- 3-D (or 2-D) periodic box with a random-mode
  density field and a central high-pressure sphere (Sedov-like blast in a
  structured medium; the paper's blast and vacuum tests are 3-D boxes of
  this kind).
* :func:`disk`           -- rotating gaseous disk in a fixed logarithmic
  potential (stand-in for the galactic-disk simulations; the paper's
  equilibrium procedure and self-gravity are not reproduced).
* :func:`aksenov`        -- smooth periodic Aksenov test (closed-form
  solution).
* :func:`advected_profile` -- smooth density advected by a uniform flow.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Problem:
    name: str
    ndim: int
    n: tuple            # (nx, ny, nz); 1 for unused axes
    lo: tuple
    hi: tuple
    gamma: float
    cfl: float
    bc: list            # per axis (lo, hi) names: "periodic" | "outflow" | "reflect" | "inflow"
    rho: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    p: np.ndarray
    potential: tuple | None = None   # ("log", v0, rc, q, cx, cy, cz) | ("uniform", gx, gy, gz)
    nsteps: int | None = None
    t_stop: float | None = None
    inflow: dict | None = None       # face (2 * axis + side) -> ghost state (rho, vx, vy, vz, p)
    self_gravity: float | None = None  # G of the self-gravity potential (Sec. 2.5), or None
    isothermal: float | None = None    # sound speed of the isothermal variant (p = cs^2 rho), or None

    @property
    def shape(self):
        return (self.n[2], self.n[1], self.n[0])

    @property
    def cells(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    def centres(self, axis: int) -> np.ndarray:
        h = (self.hi[axis] - self.lo[axis]) / self.n[axis]
        return self.lo[axis] + (np.arange(self.n[axis]) + 0.5) * h


def _grid(ndim, n, lo, hi):
    n = tuple(list(n) + [1] * (3 - len(n)))
    lo = tuple(list(lo) + [-0.5] * (3 - len(lo)))
    hi = tuple(list(hi) + [0.5] * (3 - len(hi)))
    return n, lo, hi


def _mesh(n, lo, hi):
    xs = [lo[a] + (np.arange(n[a]) + 0.5) * (hi[a] - lo[a]) / n[a] for a in range(3)]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    return X, Y, Z


def riemann_states(seed: int):
    """Left and right (rho, u, p): rho, p ~ U[0.1, 1], u ~ U[-1, 1], drawn in
    the order rho_L, u_L, p_L, rho_R, u_R, p_R from numpy's PCG64."""
    rng = np.random.default_rng(seed)
    rL = rng.uniform(0.1, 1.0)
    uL = rng.uniform(-1.0, 1.0)
    pL = rng.uniform(0.1, 1.0)
    rR = rng.uniform(0.1, 1.0)
    uR = rng.uniform(-1.0, 1.0)
    pR = rng.uniform(0.1, 1.0)
    return (rL, uL, pL), (rR, uR, pR)


def _two_state_1d(name, left, right, n, lo, hi, x0, gamma, cfl, bc, t_stop):
    x = lo + (np.arange(n) + 0.5) * (hi - lo) / n
    L = x < x0
    rho = np.where(L, left[0], right[0]).astype(np.float64).reshape(1, 1, n)
    u = np.where(L, left[1], right[1]).astype(np.float64).reshape(1, 1, n)
    p = np.where(L, left[2], right[2]).astype(np.float64).reshape(1, 1, n)
    z = np.zeros_like(rho)
    return Problem(name, 1, (n, 1, 1), (lo, -0.5, -0.5), (hi, 0.5, 0.5), gamma, cfl,
                   [(bc, bc), ("periodic", "periodic"), ("periodic", "periodic")],
                   rho, u, z.copy(), z.copy(), p, None, None, t_stop)


def riemann_1d(seed: int, n: int = 512, lo: float = 0.0, hi: float = 1.0, x0: float = 0.5,
               gamma: float = 1.4, cfl: float = 0.4, t_stop: float = 0.15, bc: str = "outflow") -> Problem:
    left, right = riemann_states(seed)
    return _two_state_1d(f"riemann1d_s{seed}_n{n}", left, right, n, lo, hi, x0, gamma, cfl, bc, t_stop)


def isothermal_riemann(seed: int, n: int = 512, cs: float = 1.0, cfl: float = 0.4, t_stop: float = 0.15,
                       gamma: float = 1.4) -> Problem:
    """1-D Riemann problem of the isothermal variant (p = cs^2 rho) on [0, 1]:
    rho_L, u_L, rho_R, u_R drawn in that order (rho ~ U[0.1, 1], u ~ U[-1, 1]),
    interface at 0.5, outflow, CFL 0.4, t = 0.15.  The pressure array holds
    cs^2 rho; gamma only sets the carried energy densities."""
    rng = np.random.default_rng(seed)
    rL, uL, rR, uR = rng.uniform(0.1, 1.0), rng.uniform(-1.0, 1.0), rng.uniform(0.1, 1.0), rng.uniform(-1.0, 1.0)
    prob = _two_state_1d(f"iso_riemann1d_s{seed}_n{n}", (rL, uL, cs * cs * rL), (rR, uR, cs * cs * rR), n, 0.0, 1.0,
                         0.5, gamma, cfl, "outflow", t_stop)
    prob.isothermal = cs
    return prob


def isothermal_wave(n: int = 128, amp: float = 1e-3, cs: float = 0.7, cfl: float = 0.4, gamma: float = 1.4) -> Problem:
    """Right-moving isothermal sound wave on the periodic unit interval:
    rho = 1 + amp sin(2 pi x), u = cs amp sin(2 pi x) (the linear simple wave),
    p = cs^2 rho; after t = 1 / cs it has travelled once round the interval."""
    x = (np.arange(n) + 0.5) / n
    d = amp * np.sin(2.0 * math.pi * x)
    rho = (1.0 + d).reshape(1, 1, n)
    u = (cs * d).reshape(1, 1, n)
    z = np.zeros_like(rho)
    prob = Problem(f"iso_wave_n{n}", 1, (n, 1, 1), (0.0, -0.5, -0.5), (1.0, 0.5, 0.5), gamma, cfl,
                   [("periodic", "periodic")] * 3, rho, u, z.copy(), z.copy(), cs * cs * rho, None, None, 1.0 / cs)
    prob.isothermal = cs
    return prob


# The paper's Table "Initial state of the shock tube problem":
# (rho_L, v_L, p_L, rho_R, v_R, p_R, x0, t).  Copied in tests/golden too.
SHOCK_TUBES = (
    (1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 0.5, 0.2),
    (1.0, -2.0, 0.4, 1.0, 2.0, 0.4, 0.5, 0.15),
    (1.0, 0.0, 1000.0, 1.0, 0.0, 0.01, 0.5, 0.012),
)


def shock_tube(k: int, n: int = 100, gamma: float = 1.4, cfl: float = 0.2) -> Problem:
    rL, uL, pL, rR, uR, pR, x0, t = SHOCK_TUBES[k]
    return _two_state_1d(f"shocktube{k + 1}_n{n}", (rL, uL, pL), (rR, uR, pR), n, 0.0, 1.0, x0,
                         gamma, cfl, "outflow", t)


def blast_waves(n: int = 2400, gamma: float = 1.4, cfl: float = 0.4, t_stop: float = 0.038) -> Problem:
    """Two interacting blast waves (the paper's Colella-Woodward test): unit
    density at rest on [0, 1], p = 1000 for x < 0.1, 0.01 for 0.1 < x < 0.9,
    100 for x > 0.9, reflecting walls, 2400 cells.  The paper does not state
    its output time; t = 0.038 is the time of the original test."""
    x = (np.arange(n) + 0.5) / n
    p = np.where(x < 0.1, 1000.0, np.where(x < 0.9, 0.01, 100.0)).reshape(1, 1, n)
    rho = np.ones((1, 1, n))
    z = np.zeros((1, 1, n))
    return Problem(f"blast_waves_n{n}", 1, (n, 1, 1), (0.0, -0.5, -0.5), (1.0, 0.5, 0.5), gamma, cfl,
                   [("reflect", "reflect"), ("periodic", "periodic"), ("periodic", "periodic")],
                   rho, z.copy(), z.copy(), z.copy(), p, None, None, t_stop)


def sedov(n: int = 100, gamma: float = 5.0 / 3.0, cfl: float = 0.3, e0: float = 0.6, r0: float = 0.02,
          p_bg: float = 1e-5, t_stop: float = 0.05) -> Problem:
    """Sedov blast (the paper's test): [-1/2, 1/2]^3, rho = 1, p = 1e-5, the
    thermal energy E0 = 0.6 put into the cells whose centres lie within
    r = 0.02 of the centre (at least the 8 central cells: at 100^3 the sphere
    is about two cells wide), periodic boundaries (the shock stays inside
    the box until t = 0.05)."""
    n3, lo, hi = _grid(3, (n, n, n), (-0.5,) * 3, (0.5,) * 3)
    X, Y, Z = _mesh(n3, lo, hi)
    r = np.sqrt(X * X + Y * Y + Z * Z)
    h = 1.0 / n
    inside = r <= max(r0, math.sqrt(3.0) * h / 2 * 1.0000001)
    vol = float(np.count_nonzero(inside)) * h ** 3
    p = np.full(n3[::-1], p_bg)
    p[inside] = (gamma - 1.0) * e0 / vol
    rho = np.ones(n3[::-1])
    zero = np.zeros(n3[::-1])
    return Problem(f"sedov_n{n}", 3, n3, lo, hi, gamma, cfl, [("periodic", "periodic")] * 3, rho, zero.copy(),
                   zero.copy(), zero.copy(), p, None, None, t_stop)


def kelvin_helmholtz(n: int = 256, gamma: float = 1.4, cfl: float = 0.4, t_stop: float = 1.0) -> Problem:
    """Kelvin-Helmholtz instability (the paper's test): [-1/2, 1/2]^2, p = 2.5,
    rho = 2 and v_x = 0.5 where |y| <= 0.25 + 0.01 (1 + cos(8 pi x)), else
    rho = 1 and v_x = -0.5; v_y = 0; periodic; 256^2."""
    n3, lo, hi = _grid(2, (n, n), (-0.5, -0.5), (0.5, 0.5))
    X, Y, Z = _mesh(n3, lo, hi)
    inner = np.abs(Y) <= 0.25 + 0.01 * (1.0 + np.cos(8.0 * math.pi * X))
    rho = np.where(inner, 2.0, 1.0)
    vx = np.where(inner, 0.5, -0.5)
    zero = np.zeros_like(rho)
    p = np.full_like(rho, 2.5)
    return Problem(f"kelvin_helmholtz_n{n}", 2, n3, lo, hi, gamma, cfl, [("periodic", "periodic")] * 3, rho, vx,
                   zero.copy(), zero.copy(), p, None, None, t_stop)


def rayleigh_taylor(n: tuple = (100, 600), g: float = 0.1, gamma: float = 1.4, cfl: float = 0.2,
                    p_top: float = 0.15, amp: float = 1e-2, band: float = 0.01, waves: int = 1,
                    t_stop: float | None = None) -> Problem:
    """Rayleigh-Taylor instability (the paper's test, under a repaired
    reading): [-0.25, 0.25] x [-1.5, 1.5], rho = 2 for |y| <= 0.75 and 1
    outside, gamma = 1.4, uniform gravity g = 0.1 along -y (the potential
    g y), and the pressure of hydrostatic equilibrium
    p(y) = p_top + g * (mass per unit area above y), continuous and positive
    (p_top = 0.15 at the top wall).  The heavy slab then lies over light gas
    at y = -0.75 (unstable) and under it at y = +0.75 (stable).  The printed
    perturbation, restricted to a band of half-width 0.01 around both
    interfaces, with one mode that is periodic in x:
    v_y = amp (1 + cos(2 pi y)) cos(2 pi waves x / 0.5).  Periodic in x,
    reflecting walls at y = -1.5 and 1.5; 100 x 600 cells as printed."""
    n3, lo, hi = _grid(2, tuple(n), (-0.25, -1.5), (0.25, 1.5))
    X, Y, Z = _mesh(n3, lo, hi)
    rho = np.where(np.abs(Y) <= 0.75, 2.0, 1.0)
    # mass per unit area between y and the top wall
    above = np.where(Y >= 0.75, 1.0 * (1.5 - Y),
                     np.where(Y >= -0.75, 0.75 + 2.0 * (0.75 - Y), 0.75 + 3.0 + 1.0 * (-0.75 - Y)))
    p = p_top + g * above
    vy = np.where(np.abs(np.abs(Y) - 0.75) <= band,
                  amp * (1.0 + np.cos(2.0 * math.pi * Y)) * np.cos(2.0 * math.pi * waves * X / 0.5), 0.0)
    zero = np.zeros_like(rho)
    bc = [("periodic", "periodic"), ("reflect", "reflect"), ("periodic", "periodic")]
    return Problem(f"rayleigh_taylor_{n3[0]}x{n3[1]}", 2, n3, lo, hi, gamma, cfl, bc, rho, zero.copy(), vy,
                   zero.copy(), p, ("uniform", 0.0, g, 0.0), None, t_stop)


def _mode_set(kmax: float, ndim: int):
    r = int(math.floor(kmax))
    ks = []
    rng3 = range(-r, r + 1)
    for kz in (rng3 if ndim == 3 else [0]):
        for ky in (rng3 if ndim >= 2 else [0]):
            for kx in rng3:
                nrm = math.sqrt(kx * kx + ky * ky + kz * kz)
                if 1.0 <= nrm <= kmax:
                    ks.append((kx, ky, kz))
    return ks


def random_modes(rng, X, Y, Z, ndim, nmodes=8, kmax=4.0, amp=0.1):
    """1 + amp * sum_m cos(2 pi k_m . x + phi_m), integer k_m uniform on
    {1 <= |k| <= kmax}, phi_m ~ U[0, 2 pi)."""
    ks = _mode_set(kmax, ndim)
    idx = rng.integers(0, len(ks), size=nmodes)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=nmodes)
    f = np.ones(X.shape)
    for m in range(nmodes):
        kx, ky, kz = ks[idx[m]]
        f += amp * np.cos(2.0 * math.pi * (kx * X + ky * Y + kz * Z) + phi[m])
    return f


def periodic_modes(n: int | tuple = 256, seed: int = 0, ndim: int = 3, gamma: float = 5.0 / 3.0,
                   cfl: float = 0.3, nsteps: int = 100, sphere_p: float = 100.0, sphere_r: float = 0.1,
                   random_pressure: bool = False, sphere_centre=None) -> Problem:
    """Periodic unit box: rho = random modes, p = 1 (or random modes) with a
    high-pressure sphere, u = 0."""
    if isinstance(n, int):
        n = (n,) * ndim
    n3, lo, hi = _grid(ndim, n, (0.0,) * ndim, (1.0,) * ndim)
    X, Y, Z = _mesh(n3, lo, hi)
    rng = np.random.default_rng(seed)
    rho = random_modes(rng, X, Y, Z, ndim)
    p = random_modes(rng, X, Y, Z, ndim) if random_pressure else np.ones(X.shape)
    if sphere_p is not None and sphere_p > 0:
        c = sphere_centre if sphere_centre is not None else (0.5, 0.5, 0.5)
        d2 = (X - c[0]) ** 2
        if ndim >= 2:
            d2 = d2 + (Y - c[1]) ** 2
        if ndim >= 3:
            d2 = d2 + (Z - c[2]) ** 2
        p = np.where(d2 <= sphere_r * sphere_r, sphere_p, p)
    z = np.zeros(X.shape)
    bc = [("periodic", "periodic")] * 3
    return Problem(f"periodic{ndim}d_{'x'.join(map(str, n))}_s{seed}", ndim, n3, lo, hi, gamma, cfl, bc,
                   np.ascontiguousarray(rho), z.copy(), z.copy(), z.copy(), np.ascontiguousarray(p),
                   None, nsteps, None)


def disk(nx: int = 512, ny: int = 512, nz: int = 64, seed: int = 0, v0: float = 1.0, rc: float = 0.02,
         rd: float = 0.2, cs: float = 0.05, gamma: float = 5.0 / 3.0, cfl: float = 0.2, nsteps: int = 500,
         rho_floor: float = 1e-3, noise: float = 0.01, isothermal: bool = False, hz: float | None = None) -> Problem:
    """Rotating gas disk in Phi = v0^2/2 ln(rc^2 + x^2 + y^2 + z^2), box
    [-1/2,1/2]^2 x [-nz hz/2, nz hz/2] with in-plane cells h = 1/nx and
    vertical cells hz (default h, cubic cells): surface density exp(-R/rd),
    vertical Gaussian of scale height max(cs/v0 sqrt(R^2+rc^2), 2 hz), flat
    rotation v = v0 R / sqrt(R^2 + rc^2), p = rho cs^2 / gamma, 1% lognormal
    density noise, outflow boundaries.  isothermal=True runs the paper's
    isothermal approximation instead (p = cs^2 rho, the variant of Sec. 4).
    A reduced disk keeps the vertical resolution of the full one with a
    coarser plane: e.g. 128 x 128 x 32 with hz = 1/512."""
    h = 1.0 / nx
    hz = h if hz is None else float(hz)
    lo = (-0.5, -0.5 * ny * h, -0.5 * nz * hz)
    hi = (0.5, 0.5 * ny * h, 0.5 * nz * hz)
    n3 = (nx, ny, nz)
    X, Y, Z = _mesh(n3, lo, hi)
    R = np.sqrt(X * X + Y * Y)
    sigma = np.exp(-R / rd)
    H = np.maximum((cs / v0) * np.sqrt(R * R + rc * rc), 2.0 * hz)
    rho = sigma / (math.sqrt(2.0 * math.pi) * H) * np.exp(-Z * Z / (2.0 * H * H))
    rho = np.maximum(rho, rho_floor)
    rng = np.random.default_rng(seed)
    rho = rho * np.exp(noise * rng.standard_normal(rho.shape))
    vphi = v0 * R / np.sqrt(R * R + rc * rc)
    with np.errstate(invalid="ignore", divide="ignore"):
        cx = np.where(R > 0, -Y / R, 0.0)
        cy = np.where(R > 0, X / R, 0.0)
    vx = vphi * cx
    vy = vphi * cy
    vz = np.zeros(X.shape)
    p = rho * cs * cs / gamma
    bc = [("outflow", "outflow")] * 3
    pot = ("log", v0, rc, 1.0, 0.0, 0.0, 0.0)
    if isothermal:
        p = rho * cs * cs
    iso = "_iso" if isothermal else ""
    prob = Problem(f"disk_{nx}x{ny}x{nz}_s{seed}{iso}", 3, n3, lo, hi, gamma, cfl, bc,
                   np.ascontiguousarray(rho), np.ascontiguousarray(vx), np.ascontiguousarray(vy), vz,
                   np.ascontiguousarray(p), pot, nsteps, None)
    prob.isothermal = cs if isothermal else None
    return prob


def gravity_sphere(n: int | tuple = 32, L: float = 2.0, G: float = 1.0, rho_floor: float = 1e-3,
                   p0: float = 0.05, gamma: float = 5.0 / 3.0, cfl: float = 0.3, seed: int | None = None,
                   noise: float = 0.0) -> Problem:
    """The density of the Poisson verification problem (Sec. 2.5; 2r^3 - 3r^2 + 1
    inside r = 1, the reading under which the printed potential solves it) as
    a self-gravitating gas ball at rest on [-L, L]^3 (cubic cells), over a
    uniform floor density, at uniform pressure p0 (so it starts to collapse);
    outflow boundaries.  noise > 0 multiplies the density by a seeded
    lognormal factor."""
    n3 = (n, n, n) if isinstance(n, int) else tuple(n)
    h = 2.0 * L / n3[0]
    lo = tuple(-0.5 * n3[a] * h for a in range(3))
    hi = tuple(0.5 * n3[a] * h for a in range(3))
    X, Y, Z = _mesh(n3, lo, hi)
    r = np.sqrt(X * X + Y * Y + Z * Z)
    rho = np.where(r <= 1.0, 2.0 * r ** 3 - 3.0 * r ** 2 + 1.0, 0.0) + rho_floor
    if noise > 0.0:
        rho = rho * np.exp(noise * np.random.default_rng(seed).standard_normal(rho.shape))
    z = np.zeros(X.shape)
    p = np.full(X.shape, p0)
    nm = "x".join(str(v) for v in n3)
    prob = Problem(f"gravity_sphere_{nm}", 3, n3, lo, hi, gamma, cfl, [("outflow", "outflow")] * 3,
                   np.ascontiguousarray(rho), z, z.copy(), z.copy(), p)
    prob.self_gravity = G
    return prob


def galaxy_disk(n: int = 256, seed: int = 0, v0: float = 1.0, r0: float = 0.05, rh_over_r0: float = 78.55 / 1.6,
                rd: float = 0.1, cs: float = 0.05, G: float = 1.0, cfl: float = 0.2, rho_floor: float = 1e-3,
                noise: float = 1e-4, gamma: float = 5.0 / 3.0, halo: str = "paper") -> Problem:
    """The configuration of the paper's galactic-disk runs (Sec. 4) with
    synthetic data: a self-gravitating isothermal gas disk in a fixed dark
    matter halo, on an n^3 mesh of the box [-1/2, 1/2]^3.  halo = "paper":
    the paper's halo density rho0 / (1 + (r/r0)^2) out to rh (its ratio
    rh / r0 = 78.55 / 1.6), rho0 set so that the circular speed tends to v0;
    halo = "log": the logarithmic potential of the disk workload with core r0.
    The disk has surface density exp(-R/rd), a Gaussian vertical profile of
    scale height max(cs/v0 sqrt(R^2+r0^2), 2h), the halo's rotation curve (the
    disk's own gravity is not balanced, so the disk contracts and, at Toomre Q
    below 1, fragments), p = cs^2 rho (isothermal), a floor density and a
    seeded lognormal density perturbation of rms 1e-4 as in the paper; G = 1,
    outflow boundaries, CFL 0.2 (the paper's)."""
    h = 1.0 / n
    lo, hi = (-0.5,) * 3, (0.5,) * 3
    n3 = (n, n, n)
    X, Y, Z = _mesh(n3, lo, hi)
    R = np.sqrt(X * X + Y * Y)
    H = np.maximum((cs / v0) * np.sqrt(R * R + r0 * r0), 2.0 * h)
    rho = np.exp(-R / rd) / (math.sqrt(2.0 * math.pi) * H) * np.exp(-Z * Z / (2.0 * H * H))
    rho = np.maximum(rho, rho_floor)
    rho = rho * np.exp(noise * np.random.default_rng(seed).standard_normal(rho.shape))
    if halo == "paper":
        # circular speed of the halo: v^2 = G M(R) / R = v0^2 (1 - atan(u) / u), u = R / r0
        u = R / r0
        with np.errstate(invalid="ignore", divide="ignore"):
            vphi = v0 * np.sqrt(np.where(u > 0, 1.0 - np.arctan(u) / np.where(u > 0, u, 1.0), 0.0))
        pot = ("halo", v0 * v0 / (4.0 * math.pi * r0 * r0), r0, r0 * rh_over_r0, 0.0, 0.0, 0.0)
    else:
        vphi = v0 * R / np.sqrt(R * R + r0 * r0)
        pot = ("log", v0, r0, 1.0, 0.0, 0.0, 0.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        cx = np.where(R > 0, -Y / R, 0.0)
        cy = np.where(R > 0, X / R, 0.0)
    prob = Problem(f"galaxy_disk_{n}_s{seed}_{halo}", 3, n3, lo, hi, gamma, cfl, [("outflow", "outflow")] * 3,
                   np.ascontiguousarray(rho), np.ascontiguousarray(vphi * cx), np.ascontiguousarray(vphi * cy),
                   np.zeros(X.shape), np.ascontiguousarray(rho * cs * cs), pot)
    prob.isothermal = cs
    prob.self_gravity = G
    return prob


def aksenov(n: int, cfl: float = 0.2) -> Problem:
    """rho = 1 + 0.5 cos x on [0, 2 pi], u = 0, gamma = 3 and p = rho^3 / 3
    (sound speed equal to rho), periodic."""
    L = 2.0 * math.pi
    x = (np.arange(n) + 0.5) * L / n
    rho = (1.0 + 0.5 * np.cos(x)).reshape(1, 1, n)
    p = rho ** 3 / 3.0
    z = np.zeros_like(rho)
    return Problem(f"aksenov_n{n}", 1, (n, 1, 1), (0.0, -0.5, -0.5), (L, 0.5, 0.5), 3.0, cfl,
                   [("periodic", "periodic")] * 3, rho, z.copy(), z.copy(), z.copy(), p, None, None,
                   0.5 * math.pi)


def advected_profile(ndim: int, n: int, u0=(1.0, 0.5, 0.25), p0: float = 1.0, amp: float = 0.2,
                     gamma: float = 1.4, cfl: float = 0.4, t_stop: float = 1.0) -> Problem:
    """rho = 1 + amp sin(2 pi (x + y + z)) on the periodic unit box, uniform
    velocity u0 and pressure p0: the exact solution is a translation."""
    n3, lo, hi = _grid(ndim, (n,) * ndim, (0.0,) * ndim, (1.0,) * ndim)
    X, Y, Z = _mesh(n3, lo, hi)
    arg = X.copy()
    if ndim >= 2:
        arg = arg + Y
    if ndim >= 3:
        arg = arg + Z
    rho = 1.0 + amp * np.sin(2.0 * math.pi * arg)
    ones = np.ones(X.shape)
    vx = u0[0] * ones
    vy = (u0[1] if ndim >= 2 else 0.0) * ones
    vz = (u0[2] if ndim >= 3 else 0.0) * ones
    return Problem(f"advect{ndim}d_n{n}", ndim, n3, lo, hi, gamma, cfl, [("periodic", "periodic")] * 3,
                   rho, vx, vy, vz, p0 * ones, None, None, t_stop)


def uniform(ndim: int, n: int | tuple, rho0=1.0, v0=(0.3, -0.2, 0.1), p0=0.7, gamma=1.4, cfl=0.4,
            bc="periodic") -> Problem:
    if isinstance(n, int):
        n = (n,) * ndim
    n3, lo, hi = _grid(ndim, n, (0.0,) * ndim, (1.0,) * ndim)
    shp = (n3[2], n3[1], n3[0])
    ones = np.ones(shp)
    return Problem(f"uniform{ndim}d", ndim, n3, lo, hi, gamma, cfl, [(bc, bc)] * 3, rho0 * ones,
                   v0[0] * ones, (v0[1] if ndim >= 2 else 0.0) * ones, (v0[2] if ndim >= 3 else 0.0) * ones,
                   p0 * ones, None, None, None)


def supersonic_inflow(n: int = 400, left=(1.0, 3.0, 1.0), right=(0.5, 3.0, 0.4), gamma: float = 1.4,
                      cfl: float = 0.4, t_stop: float = 0.1) -> Problem:
    """1-D gas moving at Mach ~4 through [0, 1]: the interior holds the right
    state (rho, u, p), the inflow face at x = 0 feeds the left state, outflow
    at x = 1.  Every wave of the Riemann problem between the two states moves
    to the right, so on [0, 1] the solution is that Riemann problem's, with
    the discontinuity starting at x = 0."""
    x = (np.arange(n) + 0.5) / n
    shp = (1, 1, n)
    z = np.zeros(shp)
    return Problem(f"supersonic_inflow_n{n}", 1, (n, 1, 1), (0.0, -0.5, -0.5), (1.0, 0.5, 0.5), gamma, cfl,
                   [("inflow", "outflow"), ("periodic", "periodic"), ("periodic", "periodic")],
                   np.full(shp, right[0]), np.full(shp, right[1]), z.copy(), z.copy(), np.full(shp, right[2]),
                   None, None, t_stop, {0: (left[0], left[1], 0.0, 0.0, left[2])})


def inflow_channel(ndim: int, n: int | tuple, seed: int, gamma: float = 1.4, cfl: float = 0.4) -> Problem:
    """Inflow at x = 0 (a fixed supersonic stream) into random blocks, outflow
    at x = 1, reflecting walls on the other axes: a wind tunnel without an
    obstacle.  The inflow state differs from every interior state."""
    p = blocks(ndim, n, seed, gamma=gamma, cfl=cfl)
    p.name = f"inflow_channel{ndim}d"
    p.bc = [("inflow", "outflow")] + [("reflect", "reflect")] * (ndim - 1) + [("periodic", "periodic")] * (3 - ndim)
    p.inflow = {0: (1.4, 3.0, 0.2 if ndim >= 2 else 0.0, -0.1 if ndim >= 3 else 0.0, 1.0)}
    return p


def random_smooth(ndim: int, n: int | tuple, seed: int, gamma=1.4, cfl=0.4, bc="periodic",
                  vel_amp=0.3) -> Problem:
    """Random-mode density and pressure, random-mode velocity components."""
    if isinstance(n, int):
        n = (n,) * ndim
    n3, lo, hi = _grid(ndim, n, (0.0,) * ndim, (1.0,) * ndim)
    X, Y, Z = _mesh(n3, lo, hi)
    rng = np.random.default_rng(seed)
    rho = random_modes(rng, X, Y, Z, ndim, amp=0.1)
    p = random_modes(rng, X, Y, Z, ndim, amp=0.1)
    vs = []
    for a in range(3):
        if a < ndim:
            vs.append(vel_amp * (random_modes(rng, X, Y, Z, ndim, amp=0.1) - 1.0) * 10.0 / 8.0)
        else:
            vs.append(np.zeros(X.shape))
    return Problem(f"smooth{ndim}d_s{seed}", ndim, n3, lo, hi, gamma, cfl, [(bc, bc)] * 3,
                   rho, vs[0], vs[1], vs[2], p, None, None, None)


def blocks(ndim: int, n: int | tuple, seed: int, gamma=1.4, cfl=0.4, bc="periodic") -> Problem:
    """Piecewise-constant random blocks (discontinuities everywhere): exercises
    every limiter branch."""
    if isinstance(n, int):
        n = (n,) * ndim
    n3, lo, hi = _grid(ndim, n, (0.0,) * ndim, (1.0,) * ndim)
    shp = (n3[2], n3[1], n3[0])
    rng = np.random.default_rng(seed)

    def field(lo_, hi_):
        nb = [max(1, s // 4) for s in shp]
        coarse = rng.uniform(lo_, hi_, size=nb)
        f = coarse
        for ax, s in enumerate(shp):
            f = np.repeat(f, int(math.ceil(s / nb[ax])), axis=ax)
        return np.ascontiguousarray(f[: shp[0], : shp[1], : shp[2]])

    rho = field(0.2, 2.0)
    p = field(0.2, 2.0)
    vs = [field(-0.5, 0.5) if a < ndim else np.zeros(shp) for a in range(3)]
    return Problem(f"blocks{ndim}d_s{seed}", ndim, n3, lo, hi, gamma, cfl, [(bc, bc)] * 3,
                   rho, vs[0], vs[1], vs[2], p, None, None, None)


def batch_mix(seed: int = 0, n1d: int = 128, n2d: int = 128, steps: int = 200,
              n1_range=(64, 4096), n2_range=(32, 256)) -> list:
    """Independent grids of uneven sizes for one batched launch: n1d 1-D
    Riemann problems (states drawn as in riemann_states, gamma 1.4, CFL 0.4,
    outflow) with log-uniform sizes in n1_range, and n2d 2-D periodic boxes
    with log-uniform sides in n2_range, density and pressure 1 + 0.1 * 8
    random modes (separate draws), u = 0, gamma 5/3, CFL 0.3."""
    rng = np.random.default_rng(seed)
    probs = []
    for i in range(n1d):
        n = int(round(math.exp(rng.uniform(math.log(n1_range[0]), math.log(n1_range[1])))))
        left = (rng.uniform(0.1, 1.0), rng.uniform(-1.0, 1.0), rng.uniform(0.1, 1.0))
        right = (rng.uniform(0.1, 1.0), rng.uniform(-1.0, 1.0), rng.uniform(0.1, 1.0))
        p = _two_state_1d(f"batch1d_{i}_n{n}", left, right, n, 0.0, 1.0, 0.5, 1.4, 0.4, "outflow", None)
        p.nsteps = steps
        probs.append(p)
    for i in range(n2d):
        nx = int(round(math.exp(rng.uniform(math.log(n2_range[0]), math.log(n2_range[1])))))
        ny = int(round(math.exp(rng.uniform(math.log(n2_range[0]), math.log(n2_range[1])))))
        n3, lo, hi = _grid(2, (nx, ny), (0.0, 0.0), (1.0, 1.0))
        X, Y, Z = _mesh(n3, lo, hi)
        rho = random_modes(rng, X, Y, Z, 2)
        pr = random_modes(rng, X, Y, Z, 2)
        z = np.zeros(X.shape)
        probs.append(Problem(f"batch2d_{i}_{nx}x{ny}", 2, n3, lo, hi, 5.0 / 3.0, 0.3, [("periodic", "periodic")] * 3,
                             np.ascontiguousarray(rho), z.copy(), z.copy(), z.copy(), np.ascontiguousarray(pr), None,
                             steps, None))
    return probs


@dataclasses.dataclass
class Request:
    """One simulation request of a served trace (built lazily: a 192^3 state
    is large)."""
    rid: int
    arrival: float      # seconds after the start of the trace
    ndim: int
    n: int
    steps: int
    seed: int
    centre: tuple

    @property
    def cells(self) -> int:
        return self.n ** self.ndim

    def problem(self) -> Problem:
        p = periodic_modes(self.n, seed=self.seed, ndim=self.ndim, sphere_p=100.0, sphere_r=0.1,
                           sphere_centre=self.centre, nsteps=self.steps)
        p.name = f"req{self.rid}_{self.ndim}d_{self.n}"
        return p


def served_trace(seed: int, n_requests: int, rate: float, n2_range=(64, 512), n3_range=(64, 192),
                 steps_range=(50, 500)) -> list:
    """Poisson arrivals at `rate` requests/s: half 2-D boxes with sides
    log-uniform in n2_range, half 3-D cubes with sides log-uniform in n3_range,
    each the periodic random-mode box with one p = 100 sphere (radius 0.1) at
    a random centre, gamma 5/3, CFL 0.3, steps uniform in steps_range."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        ndim = 2 if rng.random() < 0.5 else 3
        lo_, hi_ = n2_range if ndim == 2 else n3_range
        n = int(round(math.exp(rng.uniform(math.log(lo_), math.log(hi_)))))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        sd = int(rng.integers(0, 2 ** 31 - 1))
        centre = tuple(float(c) for c in rng.uniform(0.0, 1.0, size=3))
        out.append(Request(i, t, ndim, n, steps, sd, centre))
    return out
