"""Inhomogeneous boundary conditions of the second-order pressure form.

Test infrastructure (see ``oracle/__init__.py``).

Paper: section "Approximating Boundary Conditions" writes a boundary condition as a
linear combination of derivatives of the field at the boundary point set equal to a value
g(x_b); section "Reconciliation with the Interior Numerical Discretization" forms the
exterior values as B A^+ applied to the data and the condition values, and drops the
columns that multiply g only because g is zero in its examples.  Keeping those columns:

    free  surface:  nabla^{2q} p (x_b)             = g_q(x_b),  q = 0 .. M_b / 2
    rigid surface:  n . grad(nabla^{2q} p) (x_b)   = g_q(x_b),  2q + 1 <= M_b
    robin surface:  (1 + a n_out . grad) nabla^{2q} p (x_b) = g_q(x_b),  q = 0 .. M_b / 2

and the modified Laplacian of IB point i becomes, in grid units,

    (L p)_i = sum_j u_ij p_j + sum_{b,q} v_ibq h^{o_q} g_q(x_b),

v_ibq being the entries of y = (A^+)^T c on the condition rows of boundary point b and
o_q the derivative order of condition q (2q free, 2q + 1 rigid): the condition rows are
built in grid units, so a value in physical units is scaled by h^{o_q}.

Reading (silent passage): the paper's g carries no time argument; here each condition
of the hierarchy has its own time function, g_q(x_b, t_n) = g_q(x_b) s_q(t_n), which
covers a prescribed boundary pressure (its higher members are its time derivatives
through the wave equation).
"""
from __future__ import annotations

import numpy as np


def n_conditions(surface: str, M: int) -> int:
    """Members of the condition hierarchy at basis order M."""
    return (M - 1) // 2 + 1 if surface == "rigid" else M // 2 + 1


def order_of(surface: str, q: int) -> int:
    """Derivative order of condition q (the robin member lap^q p + a dp/dn counts as 2q: a
    carries the extra length)."""
    return 2 * q + 1 if surface == "rigid" else 2 * q


def forcing_row(sol):
    """[(boundary point index, condition q, weight v)] of one IB point (grid units)."""
    out = []
    for b, row in zip(sol["bc_points"], sol["bc_weights"]):
        for q, v in enumerate(row):
            out.append((int(b), q, float(v)))
    return out


def forcing_vectors(model, sols, g):
    """B[q] over all nodes (memory order): the grid-unit Laplacian's affine part per
    condition, sum_b v_ibq h^{o_q} g[b, q], nonzero at IB points only.

    g: [n_boundary_points][nq] condition values in physical units, indexed like the
    model's boundary points."""
    g = np.asarray(g, dtype=np.float64)
    nq = g.shape[1]
    N = int(np.prod(model.shape))
    h = model.geom.h
    B = np.zeros((nq, N))
    for i, sol in sols.items():
        r = _lin(i, model.shape)
        for b, q, v in forcing_row(sol):
            if q < nq:
                B[q, r] += v * h ** order_of(model.surface_kind, q) * g[b, q]
    return B


def _lin(g, shape):
    if len(shape) == 2:
        return int(g[1]) * shape[0] + int(g[0])
    return (int(g[2]) * shape[1] + int(g[1])) * shape[0] + int(g[0])
