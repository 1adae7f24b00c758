"""Exact solution of the Riemann problem for the 1-D Euler equations of an
ideal gas, written from the mathematics (Rankine-Hugoniot shock curves and
isentropic rarefaction curves joined at the star-region pressure, found by
Newton iteration on the pressure function; self-similar sampling in x/t).

Used only as a closed-form pin of the oracle: the shock-tube problems of the
paper's verification section (Table "Initial state of the shock tube
problem") and the seeded 1-D Riemann workload have this exact solution.
"""
from __future__ import annotations

import math

import numpy as np


def _pressure_fn(p, rho, pk, ck, g):
    """f_K(p) and its derivative: velocity change across the K wave."""
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        sq = math.sqrt(A / (p + B))
        f = (p - pk) * sq
        df = sq * (1.0 - 0.5 * (p - pk) / (B + p))
    else:  # rarefaction
        pr = p / pk
        f = 2.0 * ck / (g - 1.0) * (pr ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rho * ck) * pr ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(left, right, g):
    """Star pressure and velocity for states (rho, u, p)."""
    rL, uL, pL = left
    rR, uR, pR = right
    cL = math.sqrt(g * pL / rL)
    cR = math.sqrt(g * pR / rR)
    du = uR - uL
    if 2.0 * (cL + cR) / (g - 1.0) <= du:
        raise ValueError("initial data generate vacuum")
    # initial guess: linearised (acoustic) solution, floored
    p = 0.5 * (pL + pR) - 0.125 * du * (rL + rR) * (cL + cR)
    p = max(p, 1e-8 * min(pL, pR))
    for _ in range(200):
        fL, dL = _pressure_fn(p, rL, pL, cL, g)
        fR, dR = _pressure_fn(p, rR, pR, cR, g)
        f = fL + fR + du
        dp = f / (dL + dR)
        pn = p - dp
        if pn <= 0.0:
            pn = 0.5 * p
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fL, _ = _pressure_fn(p, rL, pL, cL, g)
    fR, _ = _pressure_fn(p, rR, pR, cR, g)
    u = 0.5 * (uL + uR) + 0.5 * (fR - fL)
    return p, u


def sample(left, right, g, s, pstar=None, ustar=None):
    """(rho, u, p) at similarity coordinate s = (x - x0)/t."""
    rL, uL, pL = left
    rR, uR, pR = right
    if pstar is None:
        pstar, ustar = star_state(left, right, g)
    cL = math.sqrt(g * pL / rL)
    cR = math.sqrt(g * pR / rR)
    gm = (g - 1.0) / (g + 1.0)
    if s <= ustar:  # left of contact
        if pstar > pL:  # left shock
            SL = uL - cL * math.sqrt((g + 1.0) / (2.0 * g) * pstar / pL + (g - 1.0) / (2.0 * g))
            if s <= SL:
                return rL, uL, pL
            rho = rL * (pstar / pL + gm) / (gm * pstar / pL + 1.0)
            return rho, ustar, pstar
        cLs = cL * (pstar / pL) ** ((g - 1.0) / (2.0 * g))
        SHL, STL = uL - cL, ustar - cLs
        if s <= SHL:
            return rL, uL, pL
        if s >= STL:
            return rL * (pstar / pL) ** (1.0 / g), ustar, pstar
        u = 2.0 / (g + 1.0) * (cL + (g - 1.0) / 2.0 * uL + s)
        c = 2.0 / (g + 1.0) * (cL + (g - 1.0) / 2.0 * (uL - s))
        rho = rL * (c / cL) ** (2.0 / (g - 1.0))
        p = pL * (c / cL) ** (2.0 * g / (g - 1.0))
        return rho, u, p
    # right of contact
    if pstar > pR:
        SR = uR + cR * math.sqrt((g + 1.0) / (2.0 * g) * pstar / pR + (g - 1.0) / (2.0 * g))
        if s >= SR:
            return rR, uR, pR
        rho = rR * (pstar / pR + gm) / (gm * pstar / pR + 1.0)
        return rho, ustar, pstar
    cRs = cR * (pstar / pR) ** ((g - 1.0) / (2.0 * g))
    SHR, STR = uR + cR, ustar + cRs
    if s >= SHR:
        return rR, uR, pR
    if s <= STR:
        return rR * (pstar / pR) ** (1.0 / g), ustar, pstar
    u = 2.0 / (g + 1.0) * (-cR + (g - 1.0) / 2.0 * uR + s)
    c = 2.0 / (g + 1.0) * (cR - (g - 1.0) / 2.0 * (uR - s))
    rho = rR * (c / cR) ** (2.0 / (g - 1.0))
    p = pR * (c / cR) ** (2.0 * g / (g - 1.0))
    return rho, u, p


def cell_averages(left, right, g, x0, t, edges, sub=16):
    """Exact (rho, u, p) averaged over cells with the given edges (sub-sampled)."""
    pstar, ustar = star_state(left, right, g)
    n = len(edges) - 1
    out = np.zeros((3, n))
    for i in range(n):
        xs = edges[i] + (np.arange(sub) + 0.5) / sub * (edges[i + 1] - edges[i])
        acc = np.zeros(3)
        for x in xs:
            acc += sample(left, right, g, (x - x0) / t, pstar, ustar)
        out[:, i] = acc / sub
    return out


def max_wave_speed(left, right, g):
    """Largest |speed| of any wave front of the exact solution."""
    rL, uL, pL = left
    rR, uR, pR = right
    pstar, ustar = star_state(left, right, g)
    cL = math.sqrt(g * pL / rL)
    cR = math.sqrt(g * pR / rR)
    if pstar > pL:
        sl = uL - cL * math.sqrt((g + 1.0) / (2.0 * g) * pstar / pL + (g - 1.0) / (2.0 * g))
    else:
        sl = uL - cL
    if pstar > pR:
        sr = uR + cR * math.sqrt((g + 1.0) / (2.0 * g) * pstar / pR + (g - 1.0) / (2.0 * g))
    else:
        sr = uR + cR
    return max(abs(sl), abs(sr), abs(ustar))
