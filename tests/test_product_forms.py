"""The product build's reformulations of the reconstruction (Appendix), checked
on the CPU against the paper's formulas written out directly, on random
values that include ties, zeros and jumps of opposite sign:

* the limited slope as two medians, med(q+ - q-, 4 med(d+, d-, 0), 0), is
  exactly twice the paper's slope in FP32 and FP64;
* the monotonised one-sided jumps as medians, med(dl, 2 dr, 0) and
  med(dr, 2 dl, 0), give the paper's monotonised edges;
* the strip means from the jumps, c + (1 - z)^2 dr + z (1 - z) dl next to the
  right edge and c - (1 - z)^2 dl - z (1 - z) dr next to the left edge, equal
  the paper's strip averages of the parabola;
* the upwind flux weights a = z (1 - z)^2, b = z^2 (1 - z) (swapped for an
  upwind cell on the right) give v times the upwind strip mean.
"""
from __future__ import annotations

import numpy as np
import pytest


def med0(a, b):
    return np.maximum(np.minimum(a, b), np.minimum(np.maximum(a, b), 0.0))


def paper_slope(qm, q0, qp):
    dq = 0.5 * (qp - qm)
    dp, dm = qp - q0, q0 - qm
    m = np.minimum(np.abs(dq), np.minimum(2.0 * np.abs(dp), 2.0 * np.abs(dm)))
    return np.where(dp * dm > 0, np.copysign(m, dq), 0.0)


def paper_monotonize(c, l, r):
    l, r = l.copy(), r.copy()
    flat = (r - c) * (c - l) <= 0
    d = r - l
    s6 = 6.0 * (c - 0.5 * (l + r))
    ds, dd = d * s6, d * d
    lo = ~flat & (ds > dd)
    hi = ~flat & ~(ds > dd) & (ds < -dd)
    l2 = np.where(lo, 3.0 * c - 2.0 * r, l)
    r2 = np.where(hi, 3.0 * c - 2.0 * l, r)
    L = np.where(flat, c, l2)
    R = np.where(flat, c, r2)
    return L, R, 6.0 * (c - 0.5 * (L + R))


def avg_left(L, R, Q6, z):   # mean over the strip of width z h next to the right edge
    return R - 0.5 * z * ((R - L) - Q6 * (1.0 - 2.0 * z / 3.0))


def avg_right(L, R, Q6, z):  # next to the left edge
    return L + 0.5 * z * ((R - L) + Q6 * (1.0 - 2.0 * z / 3.0))


def _values(rng, n, dtype):
    # a mix of smooth, monotone, extremal, flat and tied neighbourhoods
    base = rng.normal(size=(3, n))
    base[:, : n // 8] = np.round(base[:, : n // 8] * 2) / 2       # ties and zero differences
    base[1, n // 8: n // 4] = base[0, n // 8: n // 4]              # one-sided zero jumps
    return [b.astype(dtype) for b in base]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_median_slope_is_exactly_twice_the_paper_slope(dtype):
    rng = np.random.default_rng(11)
    qm, q0, qp = _values(rng, 200000, dtype)
    two = dtype(2)
    ours = med0(qp - qm, dtype(4) * med0(qp - q0, q0 - qm))
    ref = paper_slope(qm, q0, qp).astype(dtype)
    assert ours.dtype == dtype
    assert np.array_equal(ours, two * ref)


def test_median_jumps_give_the_monotonised_edges():
    rng = np.random.default_rng(12)
    c, l, r = _values(rng, 200000, np.float64)
    dl, dr = c - l, r - c
    jl, jr = med0(dl, 2.0 * dr), med0(dr, 2.0 * dl)
    L, R, _ = paper_monotonize(c, l, r)
    scale = np.abs(c) + np.abs(l) + np.abs(r) + 1e-300
    assert np.max(np.abs((c - jl) - L) / scale) < 1e-15
    assert np.max(np.abs((c + jr) - R) / scale) < 1e-15


def test_strip_means_and_flux_weights_from_the_jumps():
    rng = np.random.default_rng(13)
    c, l, r = _values(rng, 200000, np.float64)
    z = rng.uniform(0.0, 1.0, size=c.size)
    L, R, Q6 = paper_monotonize(c, l, r)
    dl, dr = c - L, R - c
    y = 1.0 - z
    right_edge = c + y * y * dr + z * y * dl
    left_edge = c - y * y * dl - z * y * dr
    scale = np.abs(c) + np.abs(L) + np.abs(R) + 1e-300
    assert np.max(np.abs(right_edge - avg_left(L, R, Q6, z)) / scale) < 1e-14
    assert np.max(np.abs(left_edge - avg_right(L, R, Q6, z)) / scale) < 1e-14
    # upwind flux times tau/h through a face, vs = v tau / h: the cell on the
    # left is upwind for vs >= 0 (mean next to its right edge), the cell on
    # the right for vs < 0 (mean next to its left edge)
    vs = rng.uniform(-1.0, 1.0, size=c.size)
    za = np.abs(vs)
    p, q = za * (1 - za) ** 2, za * za * (1 - za)
    left = vs >= 0
    a, b = np.where(left, p, q), np.where(left, q, p)
    flux = vs * c + a * dr + b * dl
    mean = np.where(left, avg_left(L, R, Q6, za), avg_right(L, R, Q6, za))
    assert np.max(np.abs(flux - vs * mean) / scale) < 1e-14
