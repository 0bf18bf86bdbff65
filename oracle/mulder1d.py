"""Per-axis 1D extrapolation: the alternative table of the modified Laplacian.

Test infrastructure (see ``oracle/__init__.py``).

Paper section "Reduction to 1D" (with the 1D example of "Approximating Boundary
Conditions"): choosing, for a stencil that the boundary truncates along one axis, the
boundary conditions at the point where that axis line crosses the surface plus the M/2
interior points of the line closest to it (farther than eta*dx from it) gives a square
system whose inverse continues the field along the line; this is the 1D scheme of the
paper's comparison.  Free surface: p = 0 and every even derivative up to order M vanish
at the crossing, so the square system has (M/2 + 1) boundary rows and M/2 interior rows
for the M + 1 Taylor coefficients of a degree-M polynomial.

Readings (silent passages): the crossing is the first surface crossing between the IB
point and the first exterior node of the truncated side, found on the same cubic surface
as the N-D scheme (column height for the depth axis, a root of the surface along lateral
lines); the interior points are the nearest interior nodes of the line on the IB point's
side of the crossing; each truncated side of each axis has its own fit; the rigid surface
has no 1D reduction in the paper (its condition involves the normal) and is not offered.
"""
from __future__ import annotations

import math

import numpy as np

from . import fd


def crossing(model, g, axis, sgn, k):
    """Distance t_b in (k-1, k] along the line g + sgn * t * e_axis at which it meets the
    surface, node k being the first exterior node on that side."""
    geom = model.geom
    d = model.d
    g = np.asarray(g, dtype=np.float64)
    if axis == d - 1:                                   # depth axis: the column height
        H = float(geom.column_height(np.array([g[:-1].astype(np.int64)]))[0])
        return sgn * (H - g[-1])

    def f(t):
        q = g[:-1].copy()
        q[axis] += sgn * t
        H = float(geom.surface.eval(q[None, :])[0][0])
        return geom.sign * (g[-1] - H)                   # > 0 on the physical side

    a, b = float(k - 1), float(k)
    fa, fb = f(a), f(b)
    assert fa > 0.0 >= fb
    for _ in range(200):                                # bisection to the last bit
        m = 0.5 * (a + b)
        if m <= a or m >= b:
            break
        fm = f(m)
        if fm > 0.0:
            a = m
        else:
            b = m
    return 0.5 * (a + b)


def side_fit(model, g, axis, sgn):
    """Exterior nodes of one side of one axis stencil and their extrapolation weights:
    ([(offset e, {interior offset j: weight})], t_b) or None when the side is whole."""
    M, half = model.M, model.M // 2
    g = np.asarray(g, dtype=np.int64)

    def node(t):
        q = g.copy()
        q[axis] += sgn * t
        return q

    k = next((t for t in range(1, half + 1) if model.exterior(node(t))), None)
    if k is None:
        return None
    tb = crossing(model, g, axis, sgn, k)
    # the M/2 interior nodes of the line nearest the crossing, farther than eta from it
    data = []
    t = k - 1
    while len(data) < half:
        q = node(t)
        if not model.interior(q):
            raise RuntimeError(f"node {tuple(g)} axis {axis}: line leaves the interior before {half} points")
        if tb - t > model.eta:
            data.append(t)
        t -= 1
    # square system for the Taylor coefficients about the IB point (t = 0): data rows,
    # then p^(2q)(t_b) = 0 for 2q <= M
    n = M + 1
    A = np.zeros((n, n))
    for r, tj in enumerate(data):
        A[r] = [tj ** m / math.factorial(m) for m in range(n)]
    for q in range(half + 1):
        A[half + q] = [tb ** (m - 2 * q) / math.factorial(m - 2 * q) if m >= 2 * q else 0.0 for m in range(n)]
    Ainv = np.linalg.inv(A)
    out = []
    for e in range(k, half + 1):
        if not model.exterior(node(e)):
            continue                                     # interior again: its own value is used
        a_e = np.array([e ** m / math.factorial(m) for m in range(n)])
        wts = a_e @ Ainv[:, :half]                       # boundary rows carry zero forcing
        out.append((e, {int(sgn * tj): float(w) for tj, w in zip(data, wts)}))
    return out, tb


def extrapolation_row_1d(model, g):
    """The part of IB point g's modified Laplacian row that the 1D extrapolations add:
    {node tuple: weight} (the interior cross stencil is the rest of the row)."""
    if model.surface_kind != "free":
        raise ValueError("the 1D reduction is defined for the free surface")
    half = model.M // 2
    w2 = fd.second_derivative_weights(model.M)
    g = np.asarray(g, dtype=np.int64)
    row = {}
    for axis in range(model.d):
        for sgn in (1, -1):
            res = side_fit(model, g, axis, sgn)
            if res is None:
                continue
            for e, wts in res[0]:
                for off, w in wts.items():
                    q = g.copy()
                    q[axis] += off
                    key = model.geom.wrap(q)
                    row[key] = row.get(key, 0.0) + w2[sgn * e + half] * w
    return row


def laplacian_row_1d(model, g):
    """Full modified Laplacian row (grid units) of IB point g: {node tuple: weight}."""
    half = model.M // 2
    w2 = fd.second_derivative_weights(model.M)
    g = np.asarray(g, dtype=np.int64)
    row = extrapolation_row_1d(model, g)
    for axis in range(model.d):
        for k in range(-half, half + 1):
            q = g.copy()
            q[axis] += k
            if q[-1] < 0 or q[-1] >= model.shape[-1] or not model.interior(q):
                continue
            key = model.geom.wrap(q)
            row[key] = row.get(key, 0.0) + w2[k + half]
    return row


def assemble_laplacian_1d(model, rows=None):
    """Sparse L with the 1D-extrapolation rows at the IB points; ``rows`` maps IB point
    tuples to extrapolation rows (computed here when absent)."""
    import scipy.sparse as sp

    from . import stepper
    L = stepper.assemble_laplacian(model, {})
    shape = model.shape
    r_, c_, v_ = [], [], []
    for g in model.ib_points():
        key = tuple(int(v) for v in g)
        ext = rows[key] if rows is not None else extrapolation_row_1d(model, g)
        for q, w in ext.items():
            r_.append(_lin(g, shape))
            c_.append(_lin(q, shape))
            v_.append(w)
    N = int(np.prod(shape))
    return (L + sp.csr_matrix((v_, (r_, c_)), shape=(N, N))).tocsr()


def _lin(g, shape):
    if len(shape) == 2:
        return int(g[1]) * shape[0] + int(g[0])
    return (int(g[2]) * shape[1] + int(g[1])) * shape[0] + int(g[0])
