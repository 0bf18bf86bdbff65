"""Second-order pressure form: modified Laplacian and the damped leapfrog stepper.

Test infrastructure (see ``oracle/__init__.py``).

Paper: section "Application to the 2nd-Order Acoustic Wave Equation": p_tt =
c^2 lap p + f, discretised by the centred second difference in time,
p^{t+1} = 2p^t - p^{t-1} + dt^2 c^2 lap p + f dt^2, with the modified second-derivative
operators near the surface.  The damping layer (the paper only says one would use
one on the outer edges) is the damped leapfrog of p_tt + d(x) p_t = c^2 lap p + f:

    p^{n+1} = [2 p^n - (1 - s) p^{n-1} + K (L p^n) + dt^2 f^n] / (1 + s),
    s = d dt / 2,  K = (c dt / h)^2 at interior nodes and 0 elsewhere,

where L is the grid-unit modified Laplacian.  The profile is
d = d_max sum_axes (l_axis / W)^2 over the lateral faces and the bottom, l the depth
into the layer in cells (``damping_profile``).
Sources: multilinear spreading of a point source, f = wavelet * w_l / h^d.
Receivers: multilinear interpolation of p^{n+1}.  Lateral axes periodic; the box is
zero-padded above and below.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import fd


def _lin(g, shape):
    """Linear index of node (x, [y,] z) in [z][y][x] memory order."""
    if len(shape) == 2:
        return g[1] * shape[0] + g[0]
    return (g[2] * shape[1] + g[1]) * shape[0] + g[0]


def assemble_laplacian(model, ib_solutions=None):
    """Sparse CSR modified Laplacian (grid units) over all nodes, memory order.

    Interior rows: standard centred cross stencil restricted to interior nodes (exterior
    values are identically zero) plus, at IB points, the extrapolation weights.
    Exterior rows are empty."""
    shape = model.shape
    d = model.d
    N = int(np.prod(shape))
    inter = model.geom.interior_grid().ravel()          # memory order
    w2 = model.w2
    half = model.M // 2
    rows, cols, vals = [], [], []
    idx = np.nonzero(inter)[0]
    # decode memory index -> (x, [y,] z)
    if d == 2:
        gz, gx = np.divmod(idx, shape[0])
        coords = [gx, gz]
    else:
        gzy, gx = np.divmod(idx, shape[0])
        gz, gy = np.divmod(gzy, shape[1])
        coords = [gx, gy, gz]
    for n in range(d):
        for k in range(-half, half + 1):
            c = [a.copy() for a in coords]
            c[n] = c[n] + k
            if n < d - 1:
                c[n] %= shape[n]
                ok = np.ones(len(idx), dtype=bool)
            else:
                ok = (c[n] >= 0) & (c[n] < shape[-1])
            cz = np.clip(c[-1], 0, shape[-1] - 1)
            if d == 2:
                j = cz * shape[0] + c[0]
            else:
                j = (cz * shape[1] + c[1]) * shape[0] + c[0]
            ok &= inter[j]
            rows.append(idx[ok])
            cols.append(j[ok])
            vals.append(np.full(int(ok.sum()), w2[k + half]))
    if ib_solutions is not None:
        for i, sol in ib_solutions.items():
            r = _lin(i, shape)
            for o, w in zip(sol['offsets'], sol['weights']):
                g = model.geom.wrap(np.asarray(i) + o)
                rows.append(np.array([r]))
                cols.append(np.array([_lin(g, shape)]))
                vals.append(np.array([w]))
    L = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    L.sum_duplicates()
    return L


def solve_all(model, points=None):
    """{tuple(i): solution} for every IB point (or the given ones)."""
    pts = model.ib_points() if points is None else points
    return {tuple(int(v) for v in p): model.solve_point(p) for p in pts}


def damping_profile(shape, h, dt, c_max, width, R, form="p2"):
    """s = d dt / 2 at every node (memory order), lateral faces + bottom.

    d = d_max (l / W)^2 summed over the faces, l the depth into the layer in cells.  The
    constant makes the WKB amplitude of a wave crossing the layer, reflected by the outer
    edge and crossing back equal to R: the damping term d p_t of the second-order form
    attenuates the amplitude at the rate d / 2, the terms of the first-order form (one on
    each field) at the rate d, and the integral of (l / W)^2 over the layer is W h / 3, so
    d_max = 3 c_max ln(1/R) / (W h) for ``form`` "p2" and half of it for "pv1"."""
    d = len(shape)
    if width <= 0:
        return np.zeros(int(np.prod(shape)))
    if form not in ("p2", "pv1"):
        raise ValueError("form must be 'p2' or 'pv1'")
    dmax = 3.0 * c_max * math.log(1.0 / R) / (width * h)
    if form == "pv1":
        dmax *= 0.5

    def axis_prof(n, both):
        i = np.arange(n, dtype=np.float64)
        l = np.zeros(n)
        if both:
            l = np.maximum(l, width - i)
        l = np.maximum(l, i - (n - 1 - width))
        l = np.clip(l, 0.0, None)
        return dmax * (l / width) ** 2

    profs = [axis_prof(shape[n], True) for n in range(d - 1)] + [axis_prof(shape[-1], False)]
    if d == 2:
        D = profs[1][:, None] + profs[0][None, :]
    else:
        D = profs[2][:, None, None] + profs[1][None, :, None] + profs[0][None, None, :]
    return (D * dt / 2.0).ravel()


def multilinear(pos, shape):
    """[(memory index, weight)] of the 2^d nodes around ``pos`` (grid units)."""
    d = len(shape)
    base = [int(math.floor(p)) for p in pos]
    frac = [p - b for p, b in zip(pos, base)]
    out = []
    for corner in range(1 << d):
        w = 1.0
        g = []
        for n in range(d):
            bit = (corner >> n) & 1
            w *= frac[n] if bit else 1.0 - frac[n]
            v = base[n] + bit
            if n < d - 1:
                v %= shape[n]
            g.append(v)
        if w != 0.0:
            if not (0 <= g[-1] < shape[-1]):
                raise ValueError("point outside the grid")
            out.append((_lin(g, shape), w))
    return out


class Simulation:
    """FP64 stepping of one shot of the second-order form."""

    def __init__(self, model, L, vel, dt, src_pos, rec_pos, damp_width=0, damp_R=1e-3, forcing=None):
        """forcing: optional (B, s) of inhomogeneous boundary conditions, B[q] the affine
        part of the grid-unit Laplacian per condition (``forcing.forcing_vectors``) and
        s[q][n] its time function; step n adds K * sum_q B[q] s[q][n] to K (L p^n)."""
        self.model = model
        self.forcing = forcing
        self.n = 0
        self.shape = model.shape
        self.d = model.d
        self.N = int(np.prod(self.shape))
        self.h = model.geom.h
        self.dt = float(dt)
        self.L = L
        inter = model.geom.interior_grid().ravel()
        vel = np.asarray(vel, dtype=np.float64).ravel()
        self.K = np.where(inter, (vel * dt / self.h) ** 2, 0.0)
        self.s = damping_profile(self.shape, self.h, dt, float(vel.max()), damp_width, damp_R)
        self.src = [multilinear(np.asarray(p, dtype=float) / self.h, self.shape) for p in src_pos]
        self.rec = [multilinear(np.asarray(p, dtype=float) / self.h, self.shape) for p in rec_pos]
        self.u = np.zeros(self.N)
        self.um = np.zeros(self.N)

    def step(self, wavelets_n):
        """Advance one step; wavelets_n[s] is the source amplitude of source s at t_n."""
        f = np.zeros(self.N)
        for ws, a in zip(self.src, wavelets_n):
            for j, w in ws:
                f[j] += a * w / self.h ** self.d
        Lu = self.L @ self.u
        if self.forcing is not None:
            B, sq = self.forcing
            Lu = Lu + np.asarray(B).T @ np.asarray(sq)[:, self.n]
        new = (2.0 * self.u - (1.0 - self.s) * self.um + self.K * Lu
               + self.dt ** 2 * f) / (1.0 + self.s)
        self.n += 1
        self.um = self.u
        self.u = new
        return np.array([sum(w * new[j] for j, w in r) for r in self.rec])

    def run(self, wavelet, nt):
        """wavelet: (nsrc, nt) amplitudes; returns traces (nt, nrec) of p^{n+1}."""
        wavelet = np.atleast_2d(wavelet)
        return np.stack([self.step(wavelet[:, n]) for n in range(nt)])
