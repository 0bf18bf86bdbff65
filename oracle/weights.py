"""Immersed-boundary points and their modified stencils (pressure, second-order form).

Test infrastructure (see ``oracle/__init__.py``).

Paper sections followed, in order:
  * "Approximating Boundary Conditions": the system A delta = [f(X); g_1(X_b); ...]
    with one Taylor row per interior data point and one row per boundary condition per
    boundary point; hyperspherical support of initial radius (M+1)/2 grown until
    rank(A) equals the number of expansion terms; basis-order reduction as the
    fallback.
  * "Reconciliation with the Interior Numerical Discretization": the exterior values
    the interior stencil needs are the projection B delta with delta = A^+ [...]; the
    modified stencil is w_i . f(X_i) + w_e . B A^+ [f(X); g].  With g = 0 the forcing
    columns drop out, so the data weights are y = (A^+)^T c with c = B^T w_e
    = sum_e w_e a(x_e - x_0); the entries of the same y on the boundary-condition rows
    are the weights of the values g (kept for inhomogeneous conditions).
  * "Application to the 2nd-Order Acoustic Wave Equation": one modified second
    derivative per axis; they share the one extrapolant of their stencil centre, so
    the modified Laplacian row is the standard cross stencil plus sum_j y_j f(x_j)
    with c summed over the exterior points of all axes.

Readings (silent or ambiguous passages): radius grows by one cell, up to
``max_radius_steps`` times, then the basis order drops by one and the radius restarts
at (M_b+1)/2; a boundary point is inside the support by its position; numerical rank
is numpy's default (tolerance sigma_max * max(m, n) * eps); an interior point is an
IB point when any node of its axis stencils (+-1..M/2) is exterior.
"""
from __future__ import annotations

import math

import numpy as np

from . import basis, fd
from .geometry import Geometry


def ball_offsets(r: float, d: int):
    """Integer offsets o with |o|_2 <= r, in memory order (z slowest, x fastest).

    Returned with axis order (x, [y,] z)."""
    R = int(math.floor(r))
    out = []
    if d == 2:
        for dz in range(-R, R + 1):
            for dx in range(-R, R + 1):
                if dx * dx + dz * dz <= r * r:
                    out.append((dx, dz))
    else:
        for dz in range(-R, R + 1):
            for dy in range(-R, R + 1):
                for dx in range(-R, R + 1):
                    if dx * dx + dy * dy + dz * dz <= r * r:
                        out.append((dx, dy, dz))
    return np.array(out, dtype=np.int64)


def taylor_rows(deltas, M: int):
    """Vectorised basis.taylor_row for many offsets (P, d) -> (P, n_terms)."""
    deltas = np.atleast_2d(np.asarray(deltas, dtype=np.float64))
    E = np.array(basis.multi_indices(M, deltas.shape[1]))
    fac = np.array([[math.factorial(v) for v in e] for e in E], dtype=np.float64)
    return np.prod(deltas[:, None, :] ** E[None, :, :] / fac[None, :, :], axis=2)


class IBModel:
    """Classification + modified stencils of the second-order pressure form."""

    def __init__(self, heights, h, shape, M=8, surface='free', physical_below=True,
                 eta=0.5, max_radius_steps=3, min_basis_order=None, columns=None, robin=None):
        """surface: 'free', 'rigid' or 'robin' (p + a dp/dn = 0 with the outward normal and
        a(x_b) in metres, linear (2D) or bilinear (3D) periodic interpolation of the
        per-column samples ``robin``, shaped like ``heights``)."""
        self.geom = Geometry(heights, h, shape, physical_below)
        self.d = self.geom.d
        self.shape = self.geom.shape
        self.M = int(M)
        self.surface_kind = surface
        self.eta = float(eta)
        self.K = int(max_radius_steps)
        self.min_order = int(min_basis_order) if min_basis_order is not None else max(2, self.M // 2)
        self.w2 = fd.second_derivative_weights(self.M)
        bp = self.geom.boundary_points(columns)
        self.bp_host = bp['host']
        self.bp_xb = bp['xb']
        self.bp_normal = bp['normal']
        if surface == 'robin':
            if robin is None:
                raise ValueError("the robin surface needs its coefficient samples")
            self.bp_robin = _periodic_lerp(np.asarray(robin, dtype=np.float64), self.bp_xb[:, :-1]) / float(h)
        self.excluded = self.geom.excluded_nodes(self.bp_xb, self.eta)
        # grid-shaped views (memory order [z, (y,) x]) of the two node classes
        self.inter_grid = self.geom.interior_grid()
        self.excl_grid = np.zeros_like(self.inter_grid)
        for g in self.excluded:
            self.excl_grid[tuple(reversed(g))] = True

    # --- node classes -------------------------------------------------------
    def interior(self, g):
        g = self.geom.wrap(g)
        if g[-1] < 0 or g[-1] >= self.shape[-1]:
            return False
        return bool(self.geom.interior(np.array([g]))[0])

    def is_data(self, g):
        g = self.geom.wrap(g)
        return self.interior(g) and g not in self.excluded

    def exterior(self, g):
        g = self.geom.wrap(g)
        if g[-1] < 0 or g[-1] >= self.shape[-1]:
            return False          # outside the box: zero padding, not extrapolated
        return not self.interior(g)

    def ib_points(self):
        """All IB points (P, d) sorted in memory order."""
        inter = self.geom.interior_grid()                 # [z, (y,) x]
        ext = ~inter
        ib = np.zeros_like(inter)
        half = self.M // 2
        nzax = 0                                          # z is array axis 0
        for k in range(1, half + 1):
            for sgn in (1, -1):
                # depth axis: no wrap; outside the box is not exterior
                sh = np.zeros_like(ext)
                if sgn > 0:
                    sh[:-k] = ext[k:]
                else:
                    sh[k:] = ext[:-k]
                ib |= sh
                for ax in range(1, self.d):               # lateral array axes wrap
                    ib |= np.roll(ext, -sgn * k, axis=ax)
        ib &= inter
        idx = np.argwhere(ib)                             # rows (z, [y,] x) in memory order
        return idx[:, ::-1].copy()

    # --- boundary points near a point --------------------------------------
    def boundary_points_within(self, i, r):
        """Indices of boundary points with |x_b - i|_2 <= r (lateral minimum image)."""
        rel = self.bp_xb - np.asarray(i, dtype=np.float64)[None, :]
        for n in range(self.d - 1):
            L = self.shape[n]
            rel[:, n] = rel[:, n] - L * np.round(rel[:, n] / L)
        dist2 = np.sum(rel * rel, axis=1)
        sel = np.nonzero(dist2 <= r * r)[0]
        return sel, rel[sel]

    def bc_ops(self, Mb, k):
        """Condition operators at boundary point k (grid units)."""
        if self.surface_kind == 'free':
            return basis.free_surface_ops(Mb, self.d)
        if self.surface_kind == 'robin':
            n_out = -self.geom.sign * np.asarray(self.bp_normal[k])
            return basis.robin_surface_ops(Mb, self.d, n_out, float(self.bp_robin[k]))
        return basis.rigid_surface_ops(Mb, self.d, self.bp_normal[k])

    # --- per-point system -------------------------------------------------
    def system(self, i, Mb, r):
        """(A, data offsets) for IB point i at basis order Mb and radius r."""
        offs = ball_offsets(r, self.d)
        g = np.asarray(i, dtype=np.int64)[None, :] + offs
        for n in range(self.d - 1):
            g[:, n] %= self.shape[n]
        inside = (g[:, -1] >= 0) & (g[:, -1] < self.shape[-1])
        gz = np.clip(g[:, -1], 0, self.shape[-1] - 1)
        idx = (gz,) + tuple(g[:, n] for n in range(self.d - 2, -1, -1))
        is_data = inside & self.inter_grid[idx] & ~self.excl_grid[idx]
        data = offs[is_data]
        rows = [taylor_rows(data, Mb)] if len(data) else []
        sel, rel = self.boundary_points_within(i, r)
        for k, rb in zip(sel, rel):
            for op in self.bc_ops(Mb, k):
                rows.append(basis.apply_op_row(op, rb, Mb)[None, :])
        A = np.concatenate(rows, axis=0) if rows else np.zeros((0, basis.n_terms(Mb, self.d)))
        return A, data

    def extrapolation_target(self, i, Mb):
        """c = sum over exterior cross-stencil nodes e of w_e a(e - i)."""
        c = np.zeros(basis.n_terms(Mb, self.d))
        half = self.M // 2
        for n in range(self.d):
            for k in range(-half, half + 1):
                if k == 0:
                    continue
                e = np.array(i, dtype=np.int64)
                e[n] += k
                if self.exterior(tuple(e)):
                    off = np.zeros(self.d)
                    off[n] = k
                    c += self.w2[k + half] * taylor_rows(off[None, :], Mb)[0]
        return c

    def solve_point(self, i):
        """Modified stencil of IB point i.

        Returns dict(radius_step, order, radius, offsets (data, memory order),
        weights y (data rows), rank, cond, m)."""
        for Mb in range(self.M, self.min_order - 1, -1):
            nt = basis.n_terms(Mb, self.d)
            for k in range(self.K + 1):
                r = (Mb + 1) / 2.0 + k
                A, data = self.system(i, Mb, r)
                if A.shape[0] < nt:
                    continue
                s = np.linalg.svd(A, compute_uv=False)
                tol = s.max() * max(A.shape) * np.finfo(np.float64).eps
                rank = int(np.sum(s > tol))
                if rank == nt:
                    c = self.extrapolation_target(i, Mb)
                    y = np.linalg.pinv(A).T @ c
                    # entries of y on the boundary-condition rows: the forcing columns
                    # of B A^+ (they multiply the condition values g, zero in the
                    # homogeneous case), one row per (boundary point, condition)
                    sel, _ = self.boundary_points_within(i, r)
                    nbc = A.shape[0] - len(data)
                    nops = nbc // len(sel) if len(sel) else 0
                    return dict(radius_step=k, order=Mb, radius=r, offsets=data,
                                weights=y[:len(data)], rank=rank, cond=s.max() / s.min(),
                                m=A.shape[0], sigma_ratio=s.min() / s.max(), tol_ratio=tol / s.max(),
                                bc_points=sel, bc_weights=y[len(data):].reshape(len(sel), nops))
        raise RuntimeError(f"IB point {tuple(i)} unconstrained after radius growth and order reduction")

    def laplacian_row(self, i, sol=None):
        """Full modified Laplacian row (grid units) of IB point i: {node: weight}."""
        if sol is None:
            sol = self.solve_point(i)
        row = {}
        half = self.M // 2
        i = np.asarray(i, dtype=np.int64)
        for n in range(self.d):
            for k in range(-half, half + 1):
                e = i.copy()
                e[n] += k
                e = self.geom.wrap(e)
                if e[-1] < 0 or e[-1] >= self.shape[-1] or not self.interior(e):
                    continue
                row[e] = row.get(e, 0.0) + self.w2[k + half]
        for o, w in zip(sol['offsets'], sol['weights']):
            g = self.geom.wrap(i + o)
            row[g] = row.get(g, 0.0) + w
        return row


def _periodic_lerp(samples, lat):
    """Linear (2D: samples [nx]) or bilinear (3D: samples [ny][nx]) periodic interpolation of
    per-column samples at lateral positions ``lat`` (grid units, (P, d-1))."""
    out = np.zeros(len(lat))
    if samples.ndim == 1:
        nx = samples.shape[0]
        for k, (x,) in enumerate(lat):
            i = math.floor(x)
            f = x - i
            out[k] = (1 - f) * samples[i % nx] + f * samples[(i + 1) % nx]
        return out
    ny, nx = samples.shape
    for k, (x, y) in enumerate(lat):
        i, j = math.floor(x), math.floor(y)
        fx, fy = x - i, y - j
        out[k] = ((1 - fx) * (1 - fy) * samples[j % ny, i % nx] + fx * (1 - fy) * samples[j % ny, (i + 1) % nx]
                  + (1 - fx) * fy * samples[(j + 1) % ny, i % nx] + fx * fy * samples[(j + 1) % ny, (i + 1) % nx])
    return out
