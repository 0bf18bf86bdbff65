"""Truncated N-dimensional Taylor basis and the rows of the fitting matrix A.

Test infrastructure (see ``oracle/__init__.py``).

Paper: section "Constructing Finite-Difference Approximations" (the 1D expansion, its
N-D generalisation, the truncation M_x+M_y+M_z=M and the graded term order of the
vectors a and delta) and section "Approximating Boundary Conditions" (a linear
boundary condition sum alpha_mnl d^{m+n+l} f(x_b) = g(x_b) turns into the row obtained
by applying the same derivative operator to the basis vector a, evaluated at x_b-x_0).

All offsets are in grid units: the derivative vector delta is scaled by powers of the
grid increment, exactly as in the paper's scaled 2D delta vector.
"""
from __future__ import annotations

import functools
import math
from fractions import Fraction

import numpy as np


def _compositions(k: int, d: int):
    """All d-tuples of non-negative integers summing to k, first entry descending."""
    if d == 1:
        return [(k,)]
    out = []
    for a in range(k, -1, -1):
        for rest in _compositions(k - a, d - 1):
            out.append((a,) + rest)
    return out


_FACT = np.array([math.factorial(i) for i in range(32)], dtype=np.float64)


@functools.lru_cache(maxsize=None)
def _multi_indices_cached(M: int, d: int):
    out = []
    for k in range(M + 1):
        out.extend(_compositions(k, d))
    return tuple(out)


@functools.lru_cache(maxsize=None)
def _exponent_array(M: int, d: int):
    E = np.array(_multi_indices_cached(M, d), dtype=np.int64)
    E.setflags(write=False)
    return E


def multi_indices(M: int, d: int):
    """Exponents of the basis terms of total degree <= M in graded order.

    Degree 0, 1, ..., M; inside one degree the power of the first axis descends,
    then the second (1, x, y, x^2/2, xy, y^2/2, ... in 2D; x^2, xy, xz, y^2, yz, z^2
    in 3D), which is the order the paper lists a and delta in.
    """
    return list(_multi_indices_cached(M, d))


def n_terms(M: int, d: int) -> int:
    """Number of expansion terms = required rank (binomial(M+d, d))."""
    return len(multi_indices(M, d))


def taylor_row(delta, M: int):
    """Row a(x - x_0) of A for a data point at offset ``delta`` (length d).

    Entry for exponent e is prod_n delta_n^e_n / e_n!  (the N-D Taylor expansion).
    """
    delta = [float(v) for v in delta]
    d = len(delta)
    row = []
    for e in multi_indices(M, d):
        v = 1.0
        for n in range(d):
            v *= delta[n] ** e[n] / math.factorial(e[n])
        row.append(v)
    return np.array(row)


def derivative_row(delta, M: int, beta):
    """d^beta applied to the basis vector a, evaluated at offset ``delta``.

    d^beta (x^e / e!) = x^(e-beta) / (e-beta)! when e >= beta componentwise, else 0.
    """
    delta = np.asarray(delta, dtype=np.float64)
    d = len(delta)
    E = _exponent_array(M, d)
    P = E - np.asarray(beta, dtype=np.int64)[None, :]
    ok = np.all(P >= 0, axis=1)
    Pc = np.where(P >= 0, P, 0)
    fac = _FACT[Pc]
    vals = np.prod(delta[None, :] ** Pc / fac, axis=1)
    return np.where(ok, vals, 0.0)


# ---------------------------------------------------------------------------
# Linear differential operators, stored as {beta: coefficient}.
# ---------------------------------------------------------------------------

def op_identity(d: int):
    return {(0,) * d: 1.0}


def op_laplacian_power(q: int, d: int):
    """nabla^{2q} = (sum_n d_n^2)^q expanded by the multinomial theorem."""
    ops = {}
    for g in _compositions(q, d):
        coef = math.factorial(q)
        for gn in g:
            coef //= math.factorial(gn)
        beta = tuple(2 * gn for gn in g)
        ops[beta] = ops.get(beta, 0.0) + float(coef)
    return ops


def op_then_derivative(op, axis: int, weight: float = 1.0):
    """weight * d_axis composed with ``op``."""
    out = {}
    for beta, c in op.items():
        b = list(beta)
        b[axis] += 1
        b = tuple(b)
        out[b] = out.get(b, 0.0) + weight * c
    return out


def op_add(a, b):
    out = dict(a)
    for k, v in b.items():
        out[k] = out.get(k, 0.0) + v
    return out


def op_normal_derivative(op, normal):
    """n . grad composed with ``op``."""
    out = {}
    for axis, nv in enumerate(normal):
        if nv != 0.0:
            out = op_add(out, op_then_derivative(op, axis, float(nv)))
    return out


def op_order(op) -> int:
    return max(sum(b) for b in op)


def apply_op_row(op, delta, M: int):
    """Row of A for the boundary condition (op f)(x_b) = g with delta = x_b - x_0."""
    row = np.zeros(n_terms(M, len(delta)))
    for beta, c in op.items():
        if sum(beta) <= M:
            row += c * derivative_row(delta, M, beta)
    return row


def free_surface_ops(M: int, d: int):
    """Pressure free-surface hierarchy p = 0, nabla^2 p = 0, nabla^4 p = 0, ...

    Section "Application to the 2nd-Order Acoustic Wave Equation" and its
    "Free-Surface Boundary Constraints": conditions of order above M give 0 = 0 and
    are dropped, so q runs while 2q <= M.
    """
    return [op_laplacian_power(q, d) for q in range(M // 2 + 1)]


def rigid_surface_ops(M: int, d: int, normal):
    """Rigid surface for the pressure field: n.grad(nabla^{2q} p) = 0 while 2q+1 <= M.

    The paper defines the rigid surface as zero particle velocity (the 2D and 3D
    rigid-surface examples) but prints no rows; zero normal velocity gives
    n.grad p = 0 through the velocity equation, and differentiating twice in time
    through the wave equation gives the higher members.  (Reading recorded as G11.)
    """
    return [op_normal_derivative(op_laplacian_power(q, d), normal)
            for q in range((M - 1) // 2 + 1) if 2 * q + 1 <= M]


def robin_surface_ops(M: int, d: int, normal_out, a: float):
    """Mixed surface with a position-varying coefficient: lap^q p + a n.grad(lap^q p) = 0
    for 2q <= M, n the normal pointing out of the physical domain, a (grid units) the value
    at the boundary point.

    Section "Approximating Boundary Conditions" allows the coefficients of a condition to
    vary with the boundary point.  The zeroth member is p + a dp/dn = 0; differentiating
    it twice in time through the wave equation (c constant near the surface, as for the
    free-surface hierarchy) gives the higher members.  The paper drops the conditions that
    reduce to 0 = 0 on the basis; a member with 2q <= M never does (its lap^q part
    survives), so the members are those of the free surface, q = 0 .. M/2, and a = 0 gives
    the free surface exactly.  The normal-derivative part of the member with 2q = M has
    order M + 1 and vanishes on the basis.  (Dropping that member instead leaves the M = 4
    operator with growing modes on curved surfaces.)
    """
    return [op_add(op_laplacian_power(q, d), op_normal_derivative(op_laplacian_power(q, d), [a * v for v in normal_out]))
            for q in range(M // 2 + 1)]


# ---------------------------------------------------------------------------
# Exact rational helpers used by the worked-example pins.
# ---------------------------------------------------------------------------

def taylor_row_exact(delta, M: int):
    """taylor_row in exact rationals (for printed-matrix pins)."""
    d = len(delta)
    row = []
    for e in multi_indices(M, d):
        v = Fraction(1)
        for n in range(d):
            v *= Fraction(delta[n]) ** e[n] / math.factorial(e[n])
        row.append(v)
    return row
