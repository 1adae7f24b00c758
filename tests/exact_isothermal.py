"""Exact solution of the Riemann problem for the 1-D isothermal Euler
equations (p = a^2 rho), written from the mathematics: across a shock the
Rankine-Hugoniot conditions give the mass flux a sqrt(rho_K rho*), hence a
velocity jump a (rho* - rho_K) / sqrt(rho* rho_K); across a rarefaction the
Riemann invariant u +- a ln(rho) is constant.  The star density solves
f_L(rho*) + f_R(rho*) + u_R - u_L = 0 (f increasing, so bisection in ln rho);
there is no density jump at the contact (the pressure is a^2 rho).

Used only as a closed-form pin of the oracle's isothermal variant.
"""
from __future__ import annotations

import math

import numpy as np


def _f(rho, rk, a):
    if rho > rk:
        return a * (rho - rk) / math.sqrt(rho * rk)
    return a * math.log(rho / rk)


def star_state(left, right, a):
    """(rho*, u*) for states (rho, u)."""
    rL, uL = left
    rR, uR = right
    lo, hi = math.log(min(rL, rR)) - 60.0, math.log(max(rL, rR)) + 60.0
    for _ in range(400):
        mid = 0.5 * (lo + hi)
        r = math.exp(mid)
        if _f(r, rL, a) + _f(r, rR, a) + (uR - uL) > 0.0:
            hi = mid
        else:
            lo = mid
    rs = math.exp(0.5 * (lo + hi))
    us = 0.5 * (uL + uR) + 0.5 * (_f(rs, rR, a) - _f(rs, rL, a))
    return rs, us


def sample(left, right, a, s, rs=None, us=None):
    """(rho, u) at similarity coordinate s = (x - x0) / t."""
    rL, uL = left
    rR, uR = right
    if rs is None:
        rs, us = star_state(left, right, a)
    if s <= us:
        if rs > rL:  # left shock
            return (rL, uL) if s <= uL - a * math.sqrt(rs / rL) else (rs, us)
        if s <= uL - a:  # left rarefaction: head, tail, fan
            return rL, uL
        if s >= us - a:
            return rs, us
        u = s + a
        return rL * math.exp((uL - u) / a), u
    if rs > rR:  # right shock
        return (rR, uR) if s >= uR + a * math.sqrt(rs / rR) else (rs, us)
    if s >= uR + a:
        return rR, uR
    if s <= us + a:
        return rs, us
    u = s - a
    return rR * math.exp((u - uR) / a), u


def cell_averages(left, right, a, x0, t, edges, sub=16):
    """Exact (rho, u) averaged over cells with the given edges (sub-sampled)."""
    rs, us = star_state(left, right, a)
    n = len(edges) - 1
    out = np.zeros((2, n))
    for i in range(n):
        xs = edges[i] + (np.arange(sub) + 0.5) / sub * (edges[i + 1] - edges[i])
        acc = np.zeros(2)
        for x in xs:
            acc += sample(left, right, a, (x - x0) / t, rs, us)
        out[:, i] = acc / sub
    return out
