"""Method-of-images solutions for a flat surface (pins of the time stepper).

Test infrastructure (see ``oracle/__init__.py``).

The paper's flat-surface limit: a free surface (p = 0) reflects with coefficient -1 and
a rigid one (zero normal velocity) with +1 (section "Application to the 2nd-Order
Acoustic Wave Equation" and the rigid-surface example).  For p_tt = c^2 lap p + s(t)
delta(x - x_s) the free-space responses are
  3D: p = s(t - r/c) / (4 pi c^2 r),
  2D: p = (1 / (2 pi c^2)) int_0^{acosh(ct/r)} s(t - (r/c) cosh u) du,
and a flat surface at depth z_s adds the mirrored source with sign -1 (free) or +1
(rigid).  Lateral periodicity adds copies shifted by the period.
"""
from __future__ import annotations

import numpy as np


def ricker(t, f0, t0=None):
    """Ricker wavelet (1 - 2 pi^2 f^2 tau^2) exp(-pi^2 f^2 tau^2), tau = t - t0."""
    if t0 is None:
        t0 = 1.5 / f0
    a = (np.pi * f0 * (np.asarray(t) - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def green_2d(r, t, c, s, nq=400):
    """2D response to source time function s at distance r (vectorised over t).

    Gauss-Legendre quadrature in u on [0, acosh(ct/r)]; the integrand is smooth."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    out = np.zeros_like(t)
    live = c * t > r
    if not live.any():
        return out
    xg, wg = _gauss(nq)
    umax = np.arccosh(c * t[live] / r)
    u = 0.5 * umax[:, None] * (xg[None, :] + 1.0)
    vals = s(t[live][:, None] - (r / c) * np.cosh(u))
    out[live] = 0.5 * umax * np.sum(wg[None, :] * vals, axis=1) / (2.0 * np.pi * c * c)
    return out


_GAUSS = {}


def _gauss(n):
    if n not in _GAUSS:
        _GAUSS[n] = np.polynomial.legendre.leggauss(n)
    return _GAUSS[n]


def green_3d(r, t, c, s):
    t = np.asarray(t, dtype=np.float64)
    return s(t - r / c) / (4.0 * np.pi * c * c * r)


def image_trace(src, rec, z_s, t, c, s, kind='free', period=None, nper=1):
    """Trace at ``rec`` from ``src`` (physical coordinates, (x, [y,] z)) with a flat
    surface at depth z_s.  ``period`` = lateral period(s) (tuple) for periodic images."""
    src = np.asarray(src, dtype=np.float64)
    rec = np.asarray(rec, dtype=np.float64)
    d = len(src)
    img = src.copy()
    img[-1] = 2.0 * z_s - src[-1]
    sign = -1.0 if kind == 'free' else 1.0
    shifts = [np.zeros(d)]
    if period is not None:
        shifts = []
        rng = range(-nper, nper + 1)
        if d == 2:
            for a in rng:
                shifts.append(np.array([a * period[0], 0.0]))
        else:
            for a in rng:
                for b in rng:
                    shifts.append(np.array([a * period[0], b * period[1], 0.0]))
    g = green_2d if d == 2 else green_3d
    out = np.zeros_like(np.asarray(t, dtype=np.float64))
    for sh in shifts:
        for p, sg in ((src, 1.0), (img, sign)):
            r = np.linalg.norm(rec - (p + sh))
            out += sg * g(r, t, c, s)
    return out
