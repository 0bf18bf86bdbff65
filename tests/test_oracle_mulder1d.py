"""Pins of the oracle's per-axis 1D extrapolation (the paper's reduction to 1D)."""
import numpy as np
import pytest

from oracle import analytic, fd, mulder1d, stepper
from oracle.weights import IBModel
from paper_2309_03600_amd import workloads as W


def _truncated_sides(model, limit=60):
    out = []
    for g in model.ib_points():
        for axis in range(model.d):
            for sgn in (1, -1):
                r = mulder1d.side_fit(model, g, axis, sgn)
                if r is not None:
                    out.append((g, axis, sgn, r))
        if len(out) >= limit:
            break
    return out


@pytest.mark.parametrize("M", [2, 4, 8])
def test_odd_polynomials_about_the_crossing_are_continued_exactly(M):
    # the free-surface conditions make every odd polynomial in (t - t_b) of degree <= M - 1
    # admissible; the square 1D system continues each of them exactly
    wl = W.small2d(M=M, nt=10, hill=60.0)
    m = IBModel(wl.heights, wl.h, wl.shape, M=M, surface="free")
    sides = _truncated_sides(m)
    axes = {a for _, a, _, _ in sides}
    assert axes == {0, 1}                               # lateral and depth crossings both occur
    for g, axis, sgn, (ext, tb) in sides:
        for deg in range(1, M, 2):
            for e, wts in ext:
                got = sum(w * (sgn * off - tb) ** deg for off, w in wts.items())
                want = (e - tb) ** deg
                assert abs(got - want) <= 1e-9 * max(1.0, abs(want)), (g, axis, deg, got, want)


def test_second_order_reduces_to_the_linear_odd_extension():
    # M = 2: one interior point and p(t_b) = p''(t_b) = 0, i.e. the line through the
    # crossing and the interior point (the square case of the paper's 1D example)
    m = IBModel(np.full(24, 4.3 * 10.0), 10.0, (24, 24), M=2, surface="free")
    for g, axis, sgn, (ext, tb) in _truncated_sides(m):
        (e, wts), = ext
        (off, w), = wts.items()
        t1 = sgn * off
        assert abs(w - (e - tb) / (t1 - tb)) < 1e-14


def test_crossings_lie_on_the_surface():
    wl = W.small2d(M=8, nt=10, hill=60.0)
    m = IBModel(wl.heights, wl.h, wl.shape, M=8, surface="free")
    for g, axis, sgn, (ext, tb) in _truncated_sides(m):
        p = np.asarray(g, dtype=float)
        p[axis] += sgn * tb
        H = m.geom.surface.eval(p[None, :-1])[0][0]
        assert abs(p[-1] - H) < 1e-12


@pytest.mark.parametrize("M", [4, 8])
def test_flat_surface_rows_exact_on_admissible_polynomials(M):
    zs = 9.37
    m = IBModel(np.full(40, zs), 1.0, (40, 30), M=M, surface="free")
    for g in m.ib_points():
        row = mulder1d.laplacian_row_1d(m, g)
        for k in range(M // 2):
            deg = 2 * k + 1
            got = sum(w * (q[1] - zs) ** deg for q, w in row.items())
            want = deg * (deg - 1) * (g[1] - zs) ** (deg - 2) if deg >= 2 else 0.0
            assert abs(got - want) < 1e-8 * max(1.0, abs(want)), (g, deg, got, want)


def _images_error_1d(h, M=4, c=1500.0, f0=15.0, T=0.45):
    Lx, zs = 1000.0, 107.0
    nx, nz = int(round(Lx / h)), int(round(900.0 / h))
    m = IBModel(np.full(nx, zs), h, (nx, nz), M=M, surface="free")
    L = mulder1d.assemble_laplacian_1d(m)
    dt = 0.1 * fd.critical_dt(h, c, M, 2)
    nt = int(T / dt)
    src = (500.0, 210.0)
    recs = [(500.0 + dx, z) for dx in (0.0, 200.0) for z in (110.0, 160.0)]
    sim = stepper.Simulation(m, L, np.full((nz, nx), c), dt, [src], recs)
    tr = sim.run(analytic.ricker(np.arange(nt) * dt, f0)[None, :], nt)
    tt = (np.arange(nt) + 1) * dt
    s = lambda tau: analytic.ricker(tau, f0)
    return np.array([np.linalg.norm(tr[:, k] - analytic.image_trace(src, r, zs, tt, c, s, "free", (Lx,), 2))
                     / np.linalg.norm(analytic.image_trace(src, r, zs, tt, c, s, "free", (Lx,), 2))
                     for k, r in enumerate(recs)])


def test_method_of_images_convergence_1d():
    e1 = _images_error_1d(10.0)
    e2 = _images_error_1d(5.0)
    order = np.log2(e1 / e2)
    assert np.all(e2 < 0.01), e2
    assert np.all(order > 3.0), (e1, e2, order)


def test_flat_surface_spectrum_real_nonpositive_1d():
    m = IBModel(np.full(24, 4.3), 1.0, (24, 22), M=8, surface="free")
    L = mulder1d.assemble_laplacian_1d(m).toarray()
    inter = m.geom.interior_grid().ravel()
    ev = np.linalg.eigvals(L[np.ix_(inter, inter)])
    assert np.max(np.abs(ev.imag)) < 1e-8
    assert ev.real.max() < 1e-10


def test_rigid_surface_has_no_1d_reduction():
    m = IBModel(np.full(24, 4.3), 1.0, (24, 22), M=4, surface="rigid")
    with pytest.raises(ValueError):
        mulder1d.extrapolation_row_1d(m, m.ib_points()[0])
