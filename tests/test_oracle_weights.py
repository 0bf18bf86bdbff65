"""Pins of the oracle's modified stencils: polynomial reproduction (forced and
homogeneous), the explicit-extrapolation definition, counts, and far-field reduction."""
import math

import numpy as np
import pytest
from numpy.polynomial import polynomial as P

from oracle import basis, fd
from oracle.weights import IBModel, ball_offsets, taylor_rows


def _poly_eval(coef, pts):
    pts = np.asarray(pts, dtype=float)
    if coef.ndim == 2:
        return P.polyval2d(pts[:, 0], pts[:, 1], coef)
    return P.polyval3d(pts[:, 0], pts[:, 1], pts[:, 2], coef)


def _poly_deriv(coef, beta):
    c = coef
    for axis, k in enumerate(beta):
        if k:
            c = P.polyder(c, m=k, axis=axis)
    return c


def _random_poly(rng, deg, d):
    c = np.zeros((deg + 1,) * d)
    for e in np.ndindex(*c.shape):
        if sum(e) <= deg:
            c[e] = rng.normal()
    return c


def _apply_op_poly(op, coef, pts):
    out = np.zeros(len(pts))
    for beta, w in op.items():
        out += w * _poly_eval(_poly_deriv(coef, beta), pts)
    return out


def _sin_surface_2d(nx):
    x = np.arange(nx)
    return 12.0 + 2.2 * np.sin(2 * np.pi * x / nx * 2) + 0.4 * np.cos(2 * np.pi * x / nx * 5)


@pytest.mark.parametrize("kind", ["free", "rigid"])
@pytest.mark.parametrize("M", [4, 8])
def test_forced_polynomial_reproduction_2d(kind, M):
    # Any polynomial q of degree <= M is reproduced exactly at the exterior points when
    # the boundary rows carry the forcing g_j = (BC_j q)(x_b) (the projection
    # B A^+ [f(X); g] of the reconciliation section).  Derivatives of q come from
    # numpy.polynomial, independently of the oracle's Taylor-row algebra.
    nx, nz = 40, 30
    m = IBModel(_sin_surface_2d(nx), 1.0, (nx, nz), M=M, surface=kind)
    rng = np.random.default_rng(11)
    pts = m.ib_points()
    for i in pts[rng.choice(len(pts), 6, replace=False)]:
        sol = m.solve_point(i)
        Mb, r = sol["order"], sol["radius"]
        A, data = m.system(i, Mb, r)
        q = _random_poly(rng, Mb, 2)
        rhs = [_poly_eval(q, i + data)]
        sel, rel = m.boundary_points_within(i, r)
        for k, rb in zip(sel, rel):
            xb = (np.asarray(i, float) + rb)[None, :]
            for op in m.bc_ops(Mb, k):
                rhs.append(_apply_op_poly(op, q, xb))
        rhs = np.concatenate(rhs)
        delta = np.linalg.pinv(A) @ rhs
        for n in range(2):
            for k in range(1, M // 2 + 1):
                for s in (1, -1):
                    e = np.array(i)
                    e[n] += s * k
                    if m.exterior(tuple(e)):
                        off = (e - i).astype(float)
                        got = taylor_rows(off[None, :], Mb)[0] @ delta
                        want = _poly_eval(q, e[None, :])[0]
                        assert abs(got - want) <= 1e-9 * max(1.0, abs(want))


@pytest.mark.parametrize("kind,M,d", [("free", 4, 2), ("free", 8, 2), ("rigid", 8, 2), ("free", 8, 3), ("rigid", 8, 3)])
def test_flat_surface_laplacian_exact_on_admissible_polynomials(kind, M, d):
    # A flat surface z = z_s: q odd in (z - z_s) satisfies every free-surface condition,
    # q even satisfies every rigid one.  For deg q <= M the modified Laplacian (standard
    # cross stencil + extrapolation weights) equals lap q at the IB point exactly.
    zs = 6.3
    if d == 2:
        nx, nz = 24, 24
        H = np.full(nx, zs)
        shape = (nx, nz)
    else:
        nx, ny, nz = 12, 12, 20
        H = np.full((ny, nx), zs)
        shape = (nx, ny, nz)
    m = IBModel(H, 1.0, shape, M=M, surface=kind)
    rng = np.random.default_rng(3)
    # q = (z - zs)^p * s(x[,y], (z - zs)^2), p = 1 (free) or 0 (rigid), built in monomials
    zpoly = np.zeros(M + 1)
    def shifted(k):       # coefficients of (z - zs)^k in z
        return P.polypow([-zs, 1.0], k)
    q = np.zeros((M + 1,) * d)
    p0 = 1 if kind == "free" else 0
    for _ in range(6):
        lat = rng.integers(0, 3, size=d - 1)
        k = p0 + 2 * rng.integers(0, 3)
        if sum(lat) + k > M:
            continue
        zc = shifted(k) * rng.normal()
        for j, v in enumerate(zc):
            idx = tuple(lat) + (j,)
            q[idx] += v
    lapq = np.zeros_like(q)
    for a in range(d):
        dq = P.polyder(q, m=2, axis=a)
        sl = tuple(slice(0, n) for n in dq.shape)
        lapq[sl] += dq
    pts = m.ib_points()
    for i in pts[rng.choice(len(pts), 4, replace=False)]:
        row = m.laplacian_row(i)
        nodes = np.array(list(row.keys()), dtype=float)
        # undo the lateral wrap so nodes sit next to i
        for a in range(d - 1):
            L = shape[a]
            nodes[:, a] = nodes[:, a] + L * np.round((i[a] - nodes[:, a]) / L)
        w = np.array(list(row.values()))
        got = w @ _poly_eval(q, nodes)
        want = _poly_eval(lapq, np.asarray(i, float)[None, :])[0]
        scale = max(1.0, np.abs(_poly_eval(q, nodes)).max())
        assert abs(got - want) <= 1e-9 * scale


def test_explicit_extrapolation_definition_2d():
    # Brute force of the reconciliation step: extrapolate the exterior values with
    # B A^+ f(X) and apply the standard cross stencil; compare with the baked weights.
    nx, nz = 30, 26
    m = IBModel(_sin_surface_2d(nx), 1.0, (nx, nz), M=8, surface="free")
    rng = np.random.default_rng(9)
    field = rng.normal(size=(nz, nx))
    pts = m.ib_points()
    w2 = fd.second_derivative_weights(8)
    for i in pts[rng.choice(len(pts), 5, replace=False)]:
        sol = m.solve_point(i)
        A, data = m.system(i, sol["order"], sol["radius"])
        fX = np.array([field[g[1], g[0] % nx] for g in (i + data)])
        rhs = np.concatenate([fX, np.zeros(A.shape[0] - len(data))])
        delta = np.linalg.pinv(A) @ rhs
        total = 0.0
        for n in range(2):
            for k in range(-4, 5):
                e = np.array(i)
                e[n] += k
                if m.exterior(tuple(e)):
                    total += w2[k + 4] * (taylor_rows((e - i)[None, :].astype(float), sol["order"])[0] @ delta)
                else:
                    total += w2[k + 4] * field[e[1], e[0] % nx]
        row = m.laplacian_row(i, sol)
        baked = sum(w * field[g[1], g[0]] for g, w in row.items())
        assert abs(total - baked) < 1e-10 * max(1.0, abs(total))


def test_flat_counts_and_arc_radius():
    # M=8 flat surface: IB points are the first M/2 wet rows; initial radius (M+1)/2.
    nx, nz = 20, 24
    m = IBModel(np.full(nx, 6.3), 1.0, (nx, nz), M=8)
    pts = m.ib_points()
    assert sorted(set(pts[:, 1].tolist())) == [7, 8, 9, 10]
    assert len(pts) == 4 * nx
    sol = m.solve_point(pts[0])
    assert sol["radius"] == 4.5 and sol["order"] == 8
    m4 = IBModel(np.full(nx, 6.3), 1.0, (nx, nz), M=4)
    assert sorted(set(m4.ib_points()[:, 1].tolist())) == [7, 8]
    assert m4.solve_point(m4.ib_points()[0])["radius"] == 2.5


def test_lattice_ball_counts_brute_force():
    for r, n2, n3 in [(1.5, 9, 19), (2.5, 21, 81), (3.5, 37, 179), (4.5, 69, 389), (5.5, 97, 739)]:
        R = int(r) + 1
        b2 = sum(1 for x in range(-R, R + 1) for z in range(-R, R + 1) if x * x + z * z <= r * r)
        b3 = sum(1 for x in range(-R, R + 1) for y in range(-R, R + 1) for z in range(-R, R + 1)
                 if x * x + y * y + z * z <= r * r)
        assert len(ball_offsets(r, 2)) == b2 == n2
        assert len(ball_offsets(r, 3)) == b3 == n3


def _odd_null_poly(zs, zd, M, lateral=True):
    """Coefficients (numpy 2D, axes x, z) of q = (1 + x) (z - zs)((z - zs)^2 - (zd - zs)^2)
    (without the (1 + x) factor when ``lateral`` is False): odd in z - zs, so every
    free-surface condition lap^q p = 0 holds on the flat surface z = zs, and zero on the
    node row z = zd (and its mirror)."""
    zpoly = P.polymul([-zs, 1.0], P.polysub(P.polypow([-zs, 1.0], 2), [(zd - zs) ** 2]))
    xpoly = [1.0, 1.0] if lateral else [1.0]
    c = np.zeros((M + 1, M + 1))
    for a, xa in enumerate(xpoly):
        for b, zb in enumerate(zpoly):
            c[a, b] += xa * zb
    return c


def _taylor_vector(coef, i, Mb):
    """Scaled derivatives d^e q(i) in the oracle's term order (grid units), so that
    A @ delta lists q at the data nodes and the conditions at the boundary points."""
    out = []
    for e in basis.multi_indices(Mb, 2):
        out.append(_poly_eval(_poly_deriv(coef, e), np.asarray(i, float)[None, :])[0])
    return np.array(out)


def test_basis_order_reduction_pinned_by_null_polynomials():
    # A domain one node row thick (2D, M = 4, free surface 0.75 cells above the bottom
    # row, eta = 0.5 excludes nothing): all data of any support lie on that row, so the
    # odd polynomials (c + e x)(z - zs)((z - zs)^2 - 0.75^2) (degree 4) and
    # (z - zs)((z - zs)^2 - 0.75^2) (degree 3) satisfy every row of A at every radius:
    # orders 4 and 3 stay rank deficient whatever the growth.  At order 2 no odd
    # polynomial vanishes on the row, and the radius restarts at (2 + 1) / 2 = 1.5, where
    # 3 data nodes and 3 boundary points already fix all 6 terms.
    nx, nz = 16, 10
    zs = nz - 1 - 0.75
    m = IBModel(np.full(nx, zs), 1.0, (nx, nz), M=4, surface="free", eta=0.5)
    pts = m.ib_points()
    assert sorted(set(pts[:, 1].tolist())) == [nz - 1] and len(pts) == nx
    for i in pts[[0, 7]]:
        for Mb, lateral in ((4, True), (4, False), (3, False)):
            q = _odd_null_poly(zs, nz - 1, 4, lateral)
            delta = _taylor_vector(q, i, Mb)
            for k in range(4):
                A, _ = m.system(i, Mb, (Mb + 1) / 2 + k)
                assert np.abs(A @ delta).max() <= 1e-11 * np.abs(A).max() * np.abs(delta).max()
        sol = m.solve_point(i)
        assert (sol["order"], sol["radius_step"], sol["radius"]) == (2, 0, 1.5)
        assert sol["sigma_ratio"] > 1e-3
        assert len(sol["offsets"]) == 3 and set(sol["offsets"][:, 1].tolist()) == {0}


def test_radius_grows_by_one_cell_pinned_by_null_polynomial():
    # Flat free surface 0.75 cells above node row 5 of a deep domain, M = 4, eta = 2: rows
    # 5 and 6 lie within 2 cells of the surface and are excluded, so the first data row is
    # 7.  For an IB point of row 5 the initial ball (r = 2.5) holds data on row 7 only, and
    # (1 + x)(z - zs)((z - zs)^2 - 2.75^2) satisfies every row of A: rank deficient.  One
    # growth of one cell (r = 3.5) brings row 8 (offsets (+-1, 3), |o|^2 = 10 > 3^2) and
    # full rank; the accepted support holds them.
    nx, nz = 16, 20
    zs = 5 - 0.75
    m = IBModel(np.full(nx, zs), 1.0, (nx, nz), M=4, surface="free", eta=2.0)
    pts = m.ib_points()
    assert sorted(set(pts[:, 1].tolist())) == [5, 6]
    for i in pts[pts[:, 1] == 5][[0, 9]]:
        A, data = m.system(i, 4, 2.5)
        assert set(data[:, 1].tolist()) == {2}
        delta = _taylor_vector(_odd_null_poly(zs, 7, 4), i, 4)
        assert np.abs(A @ delta).max() <= 1e-11 * np.abs(A).max() * np.abs(delta).max()
        sol = m.solve_point(i)
        assert (sol["order"], sol["radius_step"], sol["radius"]) == (4, 1, 3.5)
        assert sol["sigma_ratio"] > 1e-3
        d2 = (sol["offsets"] ** 2).sum(axis=1)
        assert d2.max() == 10 and 3 in sol["offsets"][:, 1]
