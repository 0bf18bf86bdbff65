"""First-order pressure-velocity form on a staggered grid, with its immersed boundary.

Test infrastructure (see ``oracle/__init__.py``).

Paper sections followed:
  * "Extension to Multiple Fields and the 1st-Order Acoustic Wave Equation": the system
    p_t = rho c^2 div v + f, v_t = grad p / rho (signs as printed), so a free surface
    (p = 0) also imposes div v = 0 and its higher members lap^q div v = 0;
  * "Boundary Conditions Spanning Multiple Fields": one Taylor basis per field, the
    block-diagonal system, and boundary rows that span every field they involve, merging
    the blocks into one system solved together;
  * "The Particle Velocity Free-Surface": the characteristic divergence row, the same
    boundary points for every field, eta = 0 for the velocity fields, the staggered grid
    with a backward-staggered base stencil.

Readings (silent passages): p sits on the nodes, v_n at node + dx_n/2; the modified
operators are d/dx_n p at v_n nodes (pressure extrapolated about the v_n node, free-surface
pressure hierarchy, eta_p) and div v at p nodes (all velocity components extrapolated
jointly about the p node, divergence hierarchy); the rigid surface uses n.grad lap^q p = 0
for the pressure and n.v = 0, n.grad lap^(q-1) div v = 0 for the velocity; rho = 1; the
leapfrog is v^{n+1/2} = [(1 - s) v^{n-1/2} + dt D+ p^n]/(1 + s),
p^{n+1} = [(1 - s) p^n + dt c^2 D- . v^{n+1/2} + dt f^n]/(1 + s) with the damping of the
node index; sources spread multilinearly over p nodes with weight / h^d.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import basis, fd
from .geometry import Geometry
from .stepper import damping_profile, multilinear
from .weights import taylor_rows


def shifted_ball(r, d, shift):
    """Integer offsets o with |o + shift| <= r, memory order (z slowest); axis order
    (x, [y,] z)."""
    R = int(math.floor(r)) + 1
    out = []
    sh = np.asarray(shift, dtype=float)
    rng = range(-R, R + 1)
    if d == 2:
        for dz in rng:
            for dx in rng:
                if (dx + sh[0]) ** 2 + (dz + sh[1]) ** 2 <= r * r:
                    out.append((dx, dz))
    else:
        for dz in rng:
            for dy in rng:
                for dx in rng:
                    if (dx + sh[0]) ** 2 + (dy + sh[1]) ** 2 + (dz + sh[2]) ** 2 <= r * r:
                        out.append((dx, dy, dz))
    return np.array(out, dtype=np.int64).reshape(-1, d)


class StaggeredModel:
    """Node classes and modified operators of the staggered p-v form."""

    def __init__(self, heights, h, shape, M=8, surface="free", physical_below=True, eta_p=0.5, eta_v=0.0,
                 max_radius_steps=3, min_basis_order=None):
        self.geom = Geometry(heights, h, shape, physical_below)
        self.d = self.geom.d
        self.shape = self.geom.shape
        self.M = int(M)
        self.kind = surface
        self.K = int(max_radius_steps)
        self.min_order = int(min_basis_order) if min_basis_order is not None else max(2, self.M // 2)
        self.ws = fd.staggered_first_derivative_weights(self.M)     # offsets -(M-1)/2 .. (M-1)/2
        bp = self.geom.boundary_points()
        self.bp_xb, self.bp_normal = bp["xb"], bp["normal"]
        self.inter = {"p": self.geom.interior_grid()}
        for n in range(self.d):
            self.inter[n] = self._interior_shifted(n)
        self.excl = {"p": self._excluded(np.zeros(self.d), eta_p)}
        for n in range(self.d):
            off = np.zeros(self.d)
            off[n] = 0.5
            self.excl[n] = self._excluded(off, eta_v)

    # --- classes ------------------------------------------------------------
    def offset(self, field):
        off = np.zeros(self.d)
        if field != "p":
            off[field] = 0.5
        return off

    def _interior_shifted(self, n):
        """Interior mask [z, (y,) x] of the v_n nodes (position node + e_n / 2)."""
        d = self.d
        sgn = self.geom.sign
        if n == d - 1:                                  # depth component: column samples
            Hs = self.geom.surface.Hs
            nz = self.shape[-1]
            z = (np.arange(nz) + 0.5).reshape((nz,) + (1,) * (d - 1))
            return sgn * (z - Hs[None]) > 0
        lat = self.shape[:-1]
        if d == 2:
            xi = (np.arange(lat[0]) + 0.5)[:, None]
            H, _, _ = self.geom.surface.eval(xi)
            Hg = H[None, :]
        else:
            X, Y = np.meshgrid(np.arange(lat[0]) + (0.5 if n == 0 else 0.0),
                               np.arange(lat[1]) + (0.5 if n == 1 else 0.0), indexing="xy")
            H, _, _ = self.geom.surface.eval(np.stack([X.ravel(), Y.ravel()], 1))
            Hg = H.reshape(lat[1], lat[0])[None]
        nz = self.shape[-1]
        z = np.arange(nz).reshape((nz,) + (1,) * (d - 1))
        return sgn * (z - Hg) > 0

    def _excluded(self, off, eta):
        """Nodes of a field (positions node + off) with a boundary point strictly inside
        their half-width-eta box."""
        ex = np.zeros(self.inter["p"].shape, dtype=bool)
        if eta <= 0:
            return ex
        for p in self.bp_xb:
            q = p - off
            ranges = []
            for n in range(self.d):
                lo = math.floor(q[n] - eta) + 1
                hi = math.ceil(q[n] + eta) - 1
                ranges.append([g for g in range(lo, hi + 1) if abs(q[n] - g) < eta])
            for g in _product(ranges):
                g = list(g)
                for n in range(self.d - 1):
                    g[n] %= self.shape[n]
                if 0 <= g[-1] < self.shape[-1]:
                    ex[tuple(reversed(g))] = True
        return ex

    def _get(self, mask, g):
        g = list(int(v) for v in g)
        if not (0 <= g[-1] < self.shape[-1]):
            return None
        for n in range(self.d - 1):
            g[n] %= self.shape[n]
        return bool(mask[tuple(reversed(g))])

    def interior(self, field, g):
        v = self._get(self.inter[field], g)
        return bool(v)

    def exterior(self, field, g):
        v = self._get(self.inter[field], g)
        return v is not None and not v

    def is_data(self, field, g):
        v = self._get(self.inter[field], g)
        return bool(v) and not self._get(self.excl[field], g)

    # --- IB sets ---------------------------------------------------------------
    def _nodes(self, mask):
        return np.argwhere(mask)[:, ::-1]

    def ib_v(self, n):
        """Interior v_n nodes whose D+ stencil reaches an exterior p node (memory order)."""
        out = []
        half = self.M // 2
        for g in self._nodes(self.inter[n]):
            for m in range(-half + 1, half + 1):
                e = g.copy()
                e[n] += m
                if self.exterior("p", e):
                    out.append(g)
                    break
        return np.array(out, dtype=np.int64).reshape(-1, self.d)

    def ib_p(self):
        """Interior p nodes whose D- . v stencils reach an exterior v node (memory order)."""
        out = []
        half = self.M // 2
        for g in self._nodes(self.inter["p"]):
            hit = False
            for n in range(self.d):
                for m in range(-half, half):
                    e = g.copy()
                    e[n] += m
                    if self.exterior(n, e):
                        hit = True
                        break
                if hit:
                    break
            if hit:
                out.append(g)
        return np.array(out, dtype=np.int64).reshape(-1, self.d)

    # --- boundary rows -------------------------------------------------------
    def bpoints_within(self, x0, r):
        rel = self.bp_xb - np.asarray(x0, dtype=float)[None, :]
        for n in range(self.d - 1):
            L = self.shape[n]
            rel[:, n] -= L * np.round(rel[:, n] / L)
        sel = np.nonzero(np.sum(rel * rel, axis=1) <= r * r)[0]
        return sel, rel[sel]

    def p_ops(self, Mb, normal):
        if self.kind == "free":
            return basis.free_surface_ops(Mb, self.d)
        return basis.rigid_surface_ops(Mb, self.d, normal)

    def v_ops(self, Mb, normal):
        """Boundary rows of the velocity fields: list of per-block operator lists."""
        d = self.d
        rows = []
        if self.kind == "free":
            for q in range(Mb + 1):
                if 2 * q + 1 > Mb:
                    break
                lap = basis.op_laplacian_power(q, d)
                rows.append([basis.op_then_derivative(lap, m) for m in range(d)])
        else:
            rows.append([{(0,) * d: float(normal[m])} for m in range(d)])
            for q in range(1, Mb // 2 + 1):
                lap = basis.op_laplacian_power(q - 1, d)
                rows.append([basis.op_normal_derivative(basis.op_then_derivative(lap, m), normal)
                             for m in range(d)])
        return rows

    # --- per-point systems -----------------------------------------------------
    def solve_v_point(self, n, g):
        """Modified D+_n p at v_n node g: dict(weights on p nodes, offsets, order, radius)."""
        d = self.d
        x0 = np.asarray(g, dtype=float) + self.offset(n)
        half = self.M // 2
        for Mb in range(self.M, self.min_order - 1, -1):
            nt = basis.n_terms(Mb, d)
            for k in range(self.K + 1):
                r = (Mb + 1) / 2.0 + k
                offs = shifted_ball(r, d, -self.offset(n))        # p nodes o: |o - off| <= r
                data = [o for o in offs if self.is_data("p", np.asarray(g) + o)]
                data = np.array(data, dtype=np.int64).reshape(-1, d)
                rows = [taylor_rows(data - self.offset(n), Mb)] if len(data) else []
                sel, rel = self.bpoints_within(x0, r)
                for j, rb in zip(sel, rel):
                    for op in self.p_ops(Mb, self.bp_normal[j]):
                        rows.append(basis.apply_op_row(op, rb, Mb)[None, :])
                A = np.concatenate(rows, 0) if rows else np.zeros((0, nt))
                if A.shape[0] < nt:
                    continue
                s = np.linalg.svd(A, compute_uv=False)
                if int(np.sum(s > s.max() * max(A.shape) * np.finfo(float).eps)) != nt:
                    continue
                c = np.zeros(nt)
                for m in range(-half + 1, half + 1):
                    e = np.asarray(g).copy()
                    e[n] += m
                    if self.exterior("p", e):
                        c += self.ws[m + half - 1] * taylor_rows((e - x0)[None, :], Mb)[0]
                y = np.linalg.pinv(A).T @ c
                return dict(offsets=data, weights=y[:len(data)], order=Mb, radius_step=k, radius=r,
                            cond=s.max() / s.min())
        raise RuntimeError(f"v_{n} node {tuple(g)} unconstrained")

    def solve_p_point(self, g):
        """Modified D- . v at p node g: per-field data offsets and weights."""
        d = self.d
        x0 = np.asarray(g, dtype=float)
        half = self.M // 2
        for Mb in range(self.M, self.min_order - 1, -1):
            nt = basis.n_terms(Mb, d)
            for k in range(self.K + 1):
                r = (Mb + 1) / 2.0 + k
                blocks, datas = [], []
                for n in range(d):
                    offs = shifted_ball(r, d, self.offset(n))      # v_n nodes: |o + off| <= r
                    data = [o for o in offs if self.is_data(n, np.asarray(g) + o)]
                    data = np.array(data, dtype=np.int64).reshape(-1, d)
                    datas.append(data)
                    blk = np.zeros((len(data), d * nt))
                    if len(data):
                        blk[:, n * nt:(n + 1) * nt] = taylor_rows(data + self.offset(n), Mb)
                    blocks.append(blk)
                rows = blocks[:]
                sel, rel = self.bpoints_within(x0, r)
                for j, rb in zip(sel, rel):
                    for row_ops in self.v_ops(Mb, self.bp_normal[j]):
                        row = np.concatenate([basis.apply_op_row(op, rb, Mb) for op in row_ops])
                        rows.append(row[None, :])
                A = np.concatenate(rows, 0)
                if A.shape[0] < d * nt:
                    continue
                s = np.linalg.svd(A, compute_uv=False)
                if int(np.sum(s > s.max() * max(A.shape) * np.finfo(float).eps)) != d * nt:
                    continue
                c = np.zeros(d * nt)
                for n in range(d):
                    for m in range(-half, half):
                        e = np.asarray(g).copy()
                        e[n] += m
                        if self.exterior(n, e):
                            pos = e + self.offset(n) - x0
                            c[n * nt:(n + 1) * nt] += self.ws[m + half] * taylor_rows(pos[None, :], Mb)[0]
                y = np.linalg.pinv(A).T @ c
                out, k0 = [], 0
                for n in range(d):
                    out.append((datas[n], y[k0:k0 + len(datas[n])]))
                    k0 += len(datas[n])
                return dict(fields=out, order=Mb, radius_step=k, radius=r, cond=s.max() / s.min())
        raise RuntimeError(f"p node {tuple(g)} unconstrained")


def _product(ranges):
    if not ranges:
        yield ()
        return
    for a in ranges[0]:
        for rest in _product(ranges[1:]):
            yield (a,) + rest


def _lin(g, shape):
    if len(shape) == 2:
        return g[1] * shape[0] + g[0]
    return (g[2] * shape[1] + g[1]) * shape[0] + g[0]


def _wrap(g, shape):
    g = [int(v) for v in g]
    for n in range(len(shape) - 1):
        g[n] %= shape[n]
    return g


def assemble(model, vsol=None, psol=None):
    """Sparse D+_n (v_n rows, p columns) for each n and D- (p rows, [v_1..v_d] columns)."""
    shape, d = model.shape, model.d
    N = int(np.prod(shape))
    half = model.M // 2
    ws = model.ws
    G = []
    for n in range(d):
        rows, cols, vals = [], [], []
        vs = vsol[n] if vsol is not None else {}
        for g in model._nodes(model.inter[n]):
            r = _lin(g, shape)
            key = tuple(int(v) for v in g)
            for m in range(-half + 1, half + 1):
                e = g.copy()
                e[n] += m
                if model.interior("p", e):
                    rows.append(r)
                    cols.append(_lin(_wrap(e, shape), shape))
                    vals.append(ws[m + half - 1])
            if key in vs:
                for o, wv in zip(vs[key]["offsets"], vs[key]["weights"]):
                    rows.append(r)
                    cols.append(_lin(_wrap(g + o, shape), shape))
                    vals.append(wv)
        Gn = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
        Gn.sum_duplicates()
        G.append(Gn)
    rows, cols, vals = [], [], []
    ps = psol if psol is not None else {}
    for g in model._nodes(model.inter["p"]):
        r = _lin(g, shape)
        key = tuple(int(v) for v in g)
        for n in range(d):
            for m in range(-half, half):
                e = g.copy()
                e[n] += m
                if model.interior(n, e):
                    rows.append(r)
                    cols.append(n * N + _lin(_wrap(e, shape), shape))
                    vals.append(ws[m + half])
        if key in ps:
            for n, (offs, wts) in enumerate(ps[key]["fields"]):
                for o, wv in zip(offs, wts):
                    rows.append(r)
                    cols.append(n * N + _lin(_wrap(g + o, shape), shape))
                    vals.append(wv)
    D = sp.csr_matrix((vals, (rows, cols)), shape=(N, d * N))
    D.sum_duplicates()
    return G, D


def solve_all(model):
    vsol = [{tuple(int(v) for v in g): model.solve_v_point(n, g) for g in model.ib_v(n)} for n in range(model.d)]
    psol = {tuple(int(v) for v in g): model.solve_p_point(g) for g in model.ib_p()}
    return vsol, psol


class StaggeredSimulation:
    """FP64 stepping of one shot of the staggered p-v form (rho = 1)."""

    def __init__(self, model, G, D, vel, dt, src_pos, rec_pos, damp_width=0, damp_R=1e-3):
        self.m = model
        self.shape = model.shape
        self.d = model.d
        self.N = int(np.prod(self.shape))
        self.h = model.geom.h
        self.dt = float(dt)
        self.G, self.D = G, D
        vel = np.asarray(vel, dtype=np.float64).ravel()
        self.mask_p = model.inter["p"].ravel()
        self.mask_v = [model.inter[n].ravel() for n in range(self.d)]
        self.c2 = np.where(self.mask_p, vel ** 2, 0.0)
        self.s = damping_profile(self.shape, self.h, dt, float(vel.max()), damp_width, damp_R, form="pv1")
        self.src = [multilinear(np.asarray(q, float) / self.h, self.shape) for q in src_pos]
        self.rec = [multilinear(np.asarray(q, float) / self.h, self.shape) for q in rec_pos]
        self.p = np.zeros(self.N)
        self.v = [np.zeros(self.N) for _ in range(self.d)]

    def step(self, amps):
        dt, h, s = self.dt, self.h, self.s
        for n in range(self.d):
            nv = ((1 - s) * self.v[n] + dt / h * (self.G[n] @ self.p)) / (1 + s)
            self.v[n] = np.where(self.mask_v[n], nv, 0.0)
        f = np.zeros(self.N)
        for ws_, a in zip(self.src, amps):
            for j, w in ws_:
                f[j] += a * w / h ** self.d
        div = self.D @ np.concatenate(self.v)
        np_ = ((1 - s) * self.p + dt * self.c2 * div / h + dt * f) / (1 + s)
        self.p = np.where(self.mask_p, np_, 0.0)
        return np.array([sum(w * self.p[j] for j, w in r) for r in self.rec])

    def run(self, wavelet, nt):
        wavelet = np.atleast_2d(wavelet)
        return np.stack([self.step(wavelet[:, n]) for n in range(nt)])
