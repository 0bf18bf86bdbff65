"""Textbook finite-difference weights on regular grids (the interior discretisation).

Test infrastructure (see ``oracle/__init__.py``).

The paper's interior operator is the standard centred stencil obtained by inverting
the square Taylor system on M+1 equispaced points (section "Constructing
Finite-Difference Approximations": the rows of A^{-1} are stencils for every
derivative up to the basis order).  Here the same weights are produced by
Fornberg's recurrence (B. Fornberg, Math. Comp. 51, 1988), an independent route
whose results the tests pin against closed-form values.
"""
from __future__ import annotations

import numpy as np


def fornberg(z: float, x, m: int):
    """Weights c[k, j] of the k-th derivative (k <= m) at z from nodes x[j]."""
    x = np.asarray(x, dtype=float)
    n = len(x) - 1
    c = np.zeros((m + 1, n + 1))
    c1 = 1.0
    c4 = x[0] - z
    c[0, 0] = 1.0
    for i in range(1, n + 1):
        mn = min(i, m)
        c2 = 1.0
        c5 = c4
        c4 = x[i] - z
        for j in range(i):
            c3 = x[i] - x[j]
            c2 *= c3
            if j == i - 1:
                for k in range(mn, 0, -1):
                    c[k, i] = c1 * (k * c[k - 1, i - 1] - c5 * c[k, i - 1]) / c2
                c[0, i] = -c1 * c5 * c[0, i - 1] / c2
            for k in range(mn, 0, -1):
                c[k, j] = (c4 * c[k, j] - k * c[k - 1, j]) / c3
            c[0, j] = c4 * c[0, j] / c3
        c1 = c2
    return c


def second_derivative_weights(M: int):
    """Centred M-th order d^2/dx^2 weights at offsets -M/2..M/2 (grid units)."""
    offs = np.arange(-M // 2, M // 2 + 1, dtype=float)
    return fornberg(0.0, offs, 2)[2]


def staggered_first_derivative_weights(M: int):
    """M-th order staggered d/dx at 0 from nodes at +-1/2, +-3/2, ... (grid units).

    Returned for offsets -(M-1)/2 .. (M-1)/2 in steps of one (M values).
    """
    offs = np.arange(M, dtype=float) - (M - 1) / 2.0
    return fornberg(0.0, offs, 1)[1]


def nyquist_symbol(M: int) -> float:
    """max over wavenumbers of -(symbol of the centred 2nd-derivative stencil)."""
    w = second_derivative_weights(M)
    k = np.arange(-M // 2, M // 2 + 1)
    return float(-np.sum(w * np.cos(np.pi * k)))


def critical_dt(h: float, c_max: float, M: int, d: int) -> float:
    """Leapfrog stability limit of the interior scheme, 2 h / (c sqrt(d lambda_M))."""
    return 2.0 * h / (c_max * np.sqrt(d * nyquist_symbol(M)))
