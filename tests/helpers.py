"""Shared test helpers: build an oracle grid from a workload Problem, read
the golden fixtures."""
from __future__ import annotations

import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def make_oracle(prob, lib=None, first_order=False, cfl=None, vacuum_ratio=1e-5):
    o = oracle.Oracle(prob.ndim, prob.n, prob.lo, prob.hi, prob.gamma, prob.cfl if cfl is None else cfl,
                      bc=prob.bc, vacuum_ratio=vacuum_ratio, potential=prob.potential,
                      first_order=first_order, lib=lib, inflow=getattr(prob, "inflow", None),
                      self_gravity=getattr(prob, "self_gravity", None),
                      isothermal=getattr(prob, "isothermal", None))
    o.set_primitive(prob.rho, prob.vx, prob.vy, prob.vz, prob.p)
    return o


def shock_tubes():
    rows = []
    with open(os.path.join(GOLDEN, "shock_tubes.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                rows.append([float(v) for v in line.split()])
    return rows


def printed(key):
    with open(os.path.join(GOLDEN, "printed_numbers.txt")) as f:
        for line in f:
            s = line.split("#")[0].split()
            if len(s) >= 2 and s[0] == key:
                return float(s[1])
    raise KeyError(key)


def l1(a, b):
    return float(np.mean(np.abs(np.asarray(a) - np.asarray(b))))


def shock_width_cells(rho, lo_val, hi_val, frac=(0.1, 0.9)):
    """Number of cells whose density lies strictly between 10% and 90% of a jump."""
    a = lo_val + frac[0] * (hi_val - lo_val)
    b = lo_val + frac[1] * (hi_val - lo_val)
    lo_, hi_ = min(a, b), max(a, b)
    return int(np.sum((rho > lo_) & (rho < hi_)))
