"""Manufactured solutions for inhomogeneous boundary conditions (shared by the oracle pins
and the GPU tests; plain mathematics, no part of either implementation)."""
import math

import numpy as np


def undulating_surface(x, Lx):
    """Periodic 2D surface depth (m) around 200 m with 35 m of relief (the library keeps
    the surface at least 9.5 cells below the top of the box)."""
    return 200.0 + 25.0 * np.sin(2 * math.pi * x / Lx) + 10.0 * np.cos(6 * math.pi * x / Lx)


def standing_wave(nx, h, c):
    """p = cos(w t) cos(kx x) cos(kz (z - z0)) solves p_tt = c^2 lap p (no source) with
    w = c |k|; returns (p(x, z, t), free-surface condition values g_q(x_b), w)."""
    kx = 2 * math.pi * 2 / (nx * h)
    kz = 2 * math.pi / 300.0
    z0 = 37.0
    kk = kx * kx + kz * kz
    w = c * math.sqrt(kk)

    def p(x, z, t):
        return math.cos(w * t) * np.cos(kx * x) * np.cos(kz * (z - z0))

    def g(xb, q):
        return (-kk) ** q * np.cos(kx * xb[..., 0]) * np.cos(kz * (xb[..., -1] - z0))

    return p, g, w


def robin_coefficient(x, Lx):
    """Positive, laterally varying coefficient a (m) of the mixed surface p + a dp/dn = 0."""
    return 12.0 + 6.0 * np.sin(2 * math.pi * x / Lx + 0.4)


def robin_standing_wave(Lx, zs, a, c):
    """Standing wave below a flat surface z = zs satisfying p + a dp/dn = 0 there (n the
    outward normal, -z): p = cos(w t) cos(kx x) (a kz cos(kz (z - zs)) + sin(kz (z - zs))).
    Every member lap^q p + a dp/dn of the hierarchy then vanishes too (lap^q p is a multiple
    of p); a = 0 is the free-surface standing wave.  Returns (p(x, z, t), w)."""
    kx = 2 * math.pi * 2 / Lx
    kz = 2 * math.pi / 300.0
    w = c * math.sqrt(kx * kx + kz * kz)

    def p(x, z, t):
        return math.cos(w * t) * np.cos(kx * x) * (a * kz * np.cos(kz * (z - zs)) + np.sin(kz * (z - zs)))

    return p, w
