"""Pins of the oracle geometry: closed-form foot points, brute-force closest points,
hosting and eta-exclusion rules."""
import numpy as np
import pytest

from oracle.geometry import Geometry, Surface, foot_points


def test_flat_surface_foot_points_and_hosts():
    nx, nz, h = 30, 20, 5.0
    zs = 7.3
    g = Geometry(np.full(nx, zs * h), h, (nx, nz))
    bp = g.boundary_points()
    # one boundary point per column, hosted by the node whose cell contains z_s
    assert len(bp["host"]) == nx
    np.testing.assert_array_equal(bp["host"][:, 1], 7)
    np.testing.assert_allclose(bp["xb"][:, 1], zs, atol=1e-14)
    np.testing.assert_allclose(bp["xb"][:, 0], bp["host"][:, 0], atol=1e-14)
    # half-open hosting: a surface exactly half-way belongs to the node above
    g2 = Geometry(np.full(nx, 7.5 * h), h, (nx, nz))
    np.testing.assert_array_equal(g2.boundary_points()["host"][:, 1], 8)
    # interior strictly below
    inter = g.interior_grid()
    assert not inter[7].any() and inter[8].all()


def test_tilted_plane_closed_form_3d():
    # Catmull-Rom reproduces linear data exactly away from the periodic seam, so the
    # closest point is the orthogonal projection onto the plane z = a + b x + c y.
    nx, ny, nz = 40, 40, 40
    a, b, c = 12.2, 0.31, -0.17
    x = np.arange(nx)
    y = np.arange(ny)
    X, Y = np.meshgrid(x, y, indexing="xy")
    H = a + b * X + c * Y
    s = Surface(H, 1.0)
    rng = np.random.default_rng(5)
    nodes = np.stack([rng.integers(10, 30, 50), rng.integers(10, 30, 50), np.zeros(50)], axis=1).astype(float)
    nodes[:, 2] = a + b * nodes[:, 0] + c * nodes[:, 1] + rng.uniform(-0.9, 0.9, 50)
    nodes[:, 2] = np.round(nodes[:, 2])
    xb = foot_points(s, nodes)
    n = np.array([-b, -c, 1.0])
    dist = (nodes @ n - a) / (n @ n)
    proj = nodes - dist[:, None] * n[None, :]
    np.testing.assert_allclose(xb, proj, atol=1e-11)


def test_sinusoid_closest_point_brute_force_2d():
    nx, h = 64, 1.0
    x = np.arange(nx)
    H = 20 + 3.0 * np.sin(2 * np.pi * x / 32) + 0.7 * np.cos(2 * np.pi * x / 9)
    s = Surface(H, h)
    nodes = np.array([[i, k] for i in range(8, 56, 3) for k in range(14, 26)], dtype=float)
    xb = foot_points(s, nodes)
    fine = np.linspace(0, nx, 64 * 4000, endpoint=False)
    Hf, _, _ = s.eval(fine[:, None])
    for p, q in zip(nodes, xb):
        near = np.abs(fine - p[0]) <= 1.0
        d2 = (fine[near] - p[0]) ** 2 + (Hf[near] - p[1]) ** 2
        dq = np.sum((q - p) ** 2)
        assert dq <= d2.min() + 1e-9
        if np.sqrt(dq) < 0.87:          # only points that can be hosted matter
            j = np.argmin(d2)
            assert abs(fine[near][j] - q[0]) < 2e-3


def test_sinusoid_closest_point_brute_force_3d():
    nx = ny = 24
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    H = 10 + 2.0 * np.sin(2 * np.pi * X / 12) * np.cos(2 * np.pi * Y / 8)
    s = Surface(H, 1.0)
    g = Geometry(H, 1.0, (nx, ny, 20))
    bp = g.boundary_points()
    u = np.linspace(-1, 1, 401)
    A, B = np.meshgrid(u, u, indexing="ij")
    for host, q in list(zip(bp["host"], bp["xb"]))[::37]:
        lat = np.stack([host[0] + A.ravel(), host[1] + B.ravel()], 1)
        Hf, _, _ = s.eval(lat)
        d2 = np.sum((lat - host[:2]) ** 2, 1) + (Hf - host[2]) ** 2
        assert np.sum((q - host) ** 2) <= d2.min() + 1e-9
        rel = q - host
        assert np.all(rel >= -0.5) and np.all(rel < 0.5)


def test_eta_exclusion_rule():
    nx, nz = 12, 12
    g = Geometry(np.full(nx, 4.3), 1.0, (nx, nz))
    xb = np.array([[3.0, 4.3]])
    # eta = 0: strict inequality excludes nothing
    assert g.excluded_nodes(xb, 0.0) == set()
    # eta = 0.5: only the node whose open half-cell box holds x_b
    assert g.excluded_nodes(xb, 0.5) == {(3, 4)}
    # eta = 1: x within (2, 4) -> 3 only (2 and 4 are at distance exactly 1); z within (3.3, 5.3)
    assert g.excluded_nodes(xb, 1.0) == {(3, 4), (3, 5)}


def test_physical_side_flip():
    nx, nz = 10, 12
    gb = Geometry(np.full(nx, 5.5), 1.0, (nx, nz), physical_below=True)
    ga = Geometry(np.full(nx, 5.5), 1.0, (nx, nz), physical_below=False)
    assert np.array_equal(gb.interior_grid(), ~ga.interior_grid())
