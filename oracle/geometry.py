"""Surface geometry: signed distance, boundary points, interior and exclusion masks.

Test infrastructure (see ``oracle/__init__.py``).

Paper: section "Approximating Boundary Conditions" - boundary points are where the
boundary normal through a grid node meets the boundary, kept when that intersection
lies inside the node-centred box of one grid increment per side; an interior node is
excluded from the extrapolation data when a boundary point lies inside its node-centred
box of half-width eta*dx_n.  Section "Implementation" / "Examples": the surface is
given as a signed distance function on the grid (zero isosurface = surface).

Readings where the paper is silent (each is listed in the design notes):
  * the surface is a heightfield z = H(x[, y]) (depth positive downward) given by
    samples at the node columns and interpolated by the periodic Catmull-Rom
    (tensor-product) cubic; the signed distance of a node is +-|x - x_b| with x_b the
    closest surface point, positive on the physical side;
  * node g is interior iff it is strictly on the physical side (for a heightfield the
    sign of the distance is the sign of z - H at the node's own column);
  * the closest point is found by a coarse search over lateral offsets -1..1 step 1/8
    followed by Newton's method on |(xi, H(xi)) - g|^2, halving steps longer than 1e-6
    that would increase it (a node can only host a boundary point within sqrt(d)/2 of
    it, which the window covers);
  * hosting uses the half-open box -1/2 <= (x_b - g)_n < 1/2; exclusion the strict
    |x_b - g|_n < eta for every axis;
  * lateral axes are periodic.
All positions are in grid units with axis order (x, [y,] z); grid arrays are indexed
[z, [y,] x].
"""
from __future__ import annotations

import math

import numpy as np

COARSE_STEPS = 8          # coarse search spacing 1/8 of a cell
COARSE_HALF = 1.0         # lateral search window half-width (cells)
NEWTON_ITERS = 20
NEWTON_TOL = 1e-13
BACKTRACK_MIN = 1e-6


def _cr_weights(t):
    """Periodic Catmull-Rom cubic weights for samples k-1, k, k+1, k+2 and derivatives."""
    t2 = t * t
    t3 = t2 * t
    w = np.stack([0.5 * (-t + 2 * t2 - t3), 0.5 * (2 - 5 * t2 + 3 * t3),
                  0.5 * (t + 4 * t2 - 3 * t3), 0.5 * (-t2 + t3)], axis=-1)
    dw = np.stack([0.5 * (-1 + 4 * t - 3 * t2), 0.5 * (-10 * t + 9 * t2),
                   0.5 * (1 + 8 * t - 9 * t2), 0.5 * (-2 * t + 3 * t2)], axis=-1)
    ddw = np.stack([0.5 * (4 - 6 * t), 0.5 * (-10 + 18 * t),
                    0.5 * (8 - 18 * t), 0.5 * (-2 + 6 * t)], axis=-1)
    return w, dw, ddw


class Surface:
    """Heightfield z = H(x[, y]) in grid units from samples ``heights`` (metres).

    ``heights`` has shape (nx,) in 2D or (ny, nx) in 3D.
    """

    def __init__(self, heights, h: float):
        self.Hs = np.asarray(heights, dtype=np.float64) / float(h)
        self.lateral = self.Hs.ndim

    def eval(self, xi):
        """H, grad H (P, L) and Hessian (P, L, L) at lateral points xi (P, L)."""
        xi = np.atleast_2d(np.asarray(xi, dtype=np.float64))
        if self.lateral == 1:
            nx = self.Hs.shape[0]
            k = np.floor(xi[:, 0])
            t = xi[:, 0] - k
            k = k.astype(np.int64)
            w, dw, ddw = _cr_weights(t)
            idx = (k[:, None] + np.arange(-1, 3)[None, :]) % nx
            P = self.Hs[idx]
            H = np.sum(w * P, axis=1)
            g = np.sum(dw * P, axis=1)[:, None]
            hh = np.sum(ddw * P, axis=1)[:, None, None]
            return H, g, hh
        ny, nx = self.Hs.shape
        kx = np.floor(xi[:, 0])
        ky = np.floor(xi[:, 1])
        tx = xi[:, 0] - kx
        ty = xi[:, 1] - ky
        kx = kx.astype(np.int64)
        ky = ky.astype(np.int64)
        wx, dwx, ddwx = _cr_weights(tx)
        wy, dwy, ddwy = _cr_weights(ty)
        ix = (kx[:, None] + np.arange(-1, 3)[None, :]) % nx
        iy = (ky[:, None] + np.arange(-1, 3)[None, :]) % ny
        P = self.Hs[iy[:, :, None], ix[:, None, :]]          # (P, 4y, 4x)
        H = np.einsum('pb,pa,pba->p', wy, wx, P)
        gx = np.einsum('pb,pa,pba->p', wy, dwx, P)
        gy = np.einsum('pb,pa,pba->p', dwy, wx, P)
        hxx = np.einsum('pb,pa,pba->p', wy, ddwx, P)
        hyy = np.einsum('pb,pa,pba->p', ddwy, wx, P)
        hxy = np.einsum('pb,pa,pba->p', dwy, dwx, P)
        g = np.stack([gx, gy], axis=1)
        hh = np.stack([np.stack([hxx, hxy], 1), np.stack([hxy, hyy], 1)], 1)
        return H, g, hh

    def normal(self, xi):
        """Unit normal (x, [y,] z) at the surface point above/below xi, pointing to +z."""
        _, g, _ = self.eval(xi)
        n = np.concatenate([-g, np.ones((g.shape[0], 1))], axis=1)
        return n / np.linalg.norm(n, axis=1, keepdims=True)


def coarse_offsets(lateral: int):
    u = -COARSE_HALF + np.arange(2 * COARSE_STEPS + 1) / COARSE_STEPS
    if lateral == 1:
        return u[:, None]
    a, b = np.meshgrid(u, u, indexing='ij')      # x offset outer, y offset inner
    return np.stack([a.ravel(), b.ravel()], axis=1)


def _objective(surface, xi, xp, z):
    H, _, _ = surface.eval(xi)
    return np.sum((xi - xp) ** 2, axis=1) + (H - z) ** 2


def foot_points(surface: Surface, nodes):
    """Closest surface point of each node (P, d) -> positions (P, d), grid units.

    Coarse search over the lateral window, then Newton on
    F(xi) = |xi - x_perp|^2 + (H(xi) - z)^2 with step halving when F would increase.
    """
    nodes = np.atleast_2d(np.asarray(nodes, dtype=np.float64))
    L = surface.lateral
    P = nodes.shape[0]
    xp = nodes[:, :L]
    z = nodes[:, L]
    offs = coarse_offsets(L)                                     # (C, L)
    best = np.full(P, np.inf)
    xi = np.zeros((P, L))
    for c in range(offs.shape[0]):                               # first minimum wins
        cand = xp + offs[c][None, :]
        F = _objective(surface, cand, xp, z)
        better = F < best
        best = np.where(better, F, best)
        xi = np.where(better[:, None], cand, xi)
    active = np.ones(P, dtype=bool)
    for _ in range(NEWTON_ITERS):
        if not active.any():
            break
        ids = np.nonzero(active)[0]
        x = xi[ids]
        H, g, hh = surface.eval(x)
        r = H - z[ids]
        grad = 2.0 * (x - xp[ids]) + 2.0 * r[:, None] * g
        hess = 2.0 * np.eye(L)[None] + 2.0 * g[:, :, None] * g[:, None, :] + 2.0 * r[:, None, None] * hh
        step = -0.5 * grad
        if L == 1:
            ok = hess[:, 0, 0] > 0
            step = np.where(ok[:, None], -grad / np.where(ok, hess[:, 0, 0], 1.0)[:, None], step)
        else:
            a, b, d_ = hess[:, 0, 0], hess[:, 0, 1], hess[:, 1, 1]
            det = a * d_ - b * b
            ok = (a > 0) & (det > 0)
            sdet = np.where(ok, det, 1.0)
            sx = -(d_ * grad[:, 0] - b * grad[:, 1]) / sdet
            sy = -(-b * grad[:, 0] + a * grad[:, 1]) / sdet
            step = np.where(ok[:, None], np.stack([sx, sy], 1), step)
        # step halving only for large steps: below 1e-6 the objective changes by less
        # than its rounding error and Newton's quadratic convergence takes over
        F0 = _objective(surface, x, xp[ids], z[ids])
        for _h in range(30):
            F1 = _objective(surface, x + step, xp[ids], z[ids])
            worse = (F1 > F0) & (np.max(np.abs(step), axis=1) > BACKTRACK_MIN)
            if not worse.any():
                break
            step = np.where(worse[:, None], 0.5 * step, step)
        xi[ids] = x + step
        done = np.max(np.abs(step), axis=1) < NEWTON_TOL
        active[ids[done]] = False
    H, _, _ = surface.eval(xi)
    return np.concatenate([xi, H[:, None]], axis=1)


class Geometry:
    """Classification of the nodes of a grid against a heightfield surface.

    shape = (nx, nz) in 2D or (nx, ny, nz) in 3D (axis order x, [y,] z).
    """

    def __init__(self, heights, h: float, shape, physical_below: bool = True):
        self.surface = Surface(heights, h)
        self.shape = tuple(int(v) for v in shape)
        self.d = len(self.shape)
        self.h = float(h)
        self.sign = 1.0 if physical_below else -1.0
        assert self.surface.lateral == self.d - 1
        lat_shape = self.shape[:-1]
        assert tuple(self.surface.Hs.shape[::-1]) == lat_shape, "heights must be [y][x]"

    # --- interior ---------------------------------------------------------
    def column_height(self, lateral_idx):
        """Sample height (grid units) at integer lateral indices (P, L)."""
        lat = np.atleast_2d(lateral_idx)
        if self.d == 2:
            return self.surface.Hs[lat[:, 0] % self.shape[0]]
        return self.surface.Hs[lat[:, 1] % self.shape[1], lat[:, 0] % self.shape[0]]

    def interior(self, nodes):
        """Node strictly on the physical side of the surface (signed distance > 0)."""
        nodes = np.atleast_2d(np.asarray(nodes))
        H = self.column_height(nodes[:, :-1])
        return self.sign * (nodes[:, -1] - H) > 0

    def interior_grid(self):
        """Boolean interior mask indexed [z, [y,] x]."""
        if self.d == 2:
            nx, nz = self.shape
            z = np.arange(nz)[:, None]
            return self.sign * (z - self.surface.Hs[None, :]) > 0
        nx, ny, nz = self.shape
        z = np.arange(nz)[:, None, None]
        return self.sign * (z - self.surface.Hs[None, :, :]) > 0

    # --- boundary points ---------------------------------------------------
    def candidate_nodes(self, columns=None):
        """Nodes that may host a boundary point: per column, depths within 1.5 cells of
        the surface's range over the coarse lateral window."""
        L = self.d - 1
        if columns is None:
            if L == 1:
                columns = np.arange(self.shape[0])[:, None]
            else:
                jx, jy = np.meshgrid(np.arange(self.shape[0]), np.arange(self.shape[1]), indexing='xy')
                columns = np.stack([jx.ravel(), jy.ravel()], axis=1)
        columns = np.atleast_2d(columns)
        offs = coarse_offsets(L)
        Hmin = np.full(columns.shape[0], np.inf)
        Hmax = np.full(columns.shape[0], -np.inf)
        for c in range(offs.shape[0]):
            H, _, _ = self.surface.eval(columns + offs[c][None, :])
            Hmin = np.minimum(Hmin, H)
            Hmax = np.maximum(Hmax, H)
        k0 = np.maximum(np.ceil(Hmin - 1.5), 0).astype(np.int64)
        k1 = np.minimum(np.floor(Hmax + 1.5), self.shape[-1] - 1).astype(np.int64)
        nodes = []
        for col, a, b in zip(columns, k0, k1):
            for k in range(a, b + 1):
                nodes.append(list(col) + [k])
        return np.array(nodes, dtype=np.int64).reshape(-1, self.d)

    def boundary_points(self, columns=None):
        """Hosted boundary points: dict(host (P, d) int, xb (P, d), normal (P, d)).

        Sorted by host node in memory order (z, then y, then x)."""
        nodes = self.candidate_nodes(columns)
        if nodes.shape[0] == 0:
            return dict(host=nodes, xb=np.zeros((0, self.d)), normal=np.zeros((0, self.d)))
        xb = foot_points(self.surface, nodes.astype(np.float64))
        rel = xb - nodes
        hosted = np.all((rel >= -0.5) & (rel < 0.5), axis=1)
        host = nodes[hosted]
        xb = xb[hosted]
        normal = self.surface.normal(xb[:, :-1])
        order = np.lexsort(tuple(host[:, a] for a in range(self.d)))   # last key = z primary
        return dict(host=host[order], xb=xb[order], normal=normal[order])

    # --- eta exclusion -----------------------------------------------------
    def excluded_nodes(self, xb, eta: float):
        """Set of node tuples (wrapped laterally) excluded by the boundary points."""
        out = set()
        if eta <= 0.0:
            return out
        for p in xb:
            ranges = []
            for n in range(self.d):
                lo = math.floor(p[n] - eta) + 1
                hi = math.ceil(p[n] + eta) - 1
                ranges.append([g for g in range(lo, hi + 1) if abs(p[n] - g) < eta])
            for g in _product(ranges):
                out.add(self.wrap(g))
        return out

    def wrap(self, g):
        g = list(int(v) for v in g)
        for n in range(self.d - 1):
            g[n] %= self.shape[n]
        return tuple(g)


def _product(ranges):
    if not ranges:
        yield ()
        return
    for a in ranges[0]:
        for rest in _product(ranges[1:]):
            yield (a,) + rest
