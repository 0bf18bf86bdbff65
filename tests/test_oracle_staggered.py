"""Pins of the staggered pressure-velocity oracle: coupled polynomial reproduction,
exactness on admissible polynomials at a flat surface, and the method of images with
the convergence the paper reports for the first-order form (close to fourth order)."""
import numpy as np
import pytest
from numpy.polynomial import polynomial as P

from oracle import analytic, basis, fd
from oracle.staggered import StaggeredModel, StaggeredSimulation, assemble, shifted_ball, solve_all
from oracle.weights import taylor_rows


def _ev(c, pts):
    pts = np.asarray(pts, float)
    return P.polyval2d(pts[:, 0], pts[:, 1], c)


def _der(c, beta):
    for ax, k in enumerate(beta):
        if k:
            c = P.polyder(c, m=k, axis=ax)
    return c


def _op(op, c, pts):
    return sum(w * _ev(_der(c, b), pts) for b, w in op.items())


def _hill(nx):
    x = np.arange(nx)
    return 14.0 + 2.5 * np.sin(2 * np.pi * x / nx * 2) + 0.5 * np.cos(2 * np.pi * x / nx * 3)


@pytest.mark.parametrize("kind", ["free", "rigid"])
def test_coupled_velocity_extrapolation_reproduces_polynomials(kind):
    # a vector polynomial v (degree <= M_b per component) with the boundary rows forced
    # by its own boundary values is reproduced at the exterior velocity nodes
    nx, nz, M = 40, 32, 4
    m = StaggeredModel(_hill(nx), 1.0, (nx, nz), M=M, surface=kind)
    rng = np.random.default_rng(8)
    pts = m.ib_p()
    for g in pts[rng.choice(len(pts), 5, replace=False)]:
        sol = m.solve_p_point(g)
        Mb, r = sol["order"], sol["radius"]
        nt = basis.n_terms(Mb, 2)
        comps = []
        for _ in range(2):
            c = np.zeros((Mb + 1, Mb + 1))
            for e in np.ndindex(*c.shape):
                if sum(e) <= Mb:
                    c[e] = rng.normal()
            comps.append(c)
        rows, rhs = [], []
        for n in range(2):
            offs = shifted_ball(r, 2, m.offset(n))
            data = np.array([o for o in offs if m.is_data(n, g + o)]).reshape(-1, 2)
            blk = np.zeros((len(data), 2 * nt))
            blk[:, n * nt:(n + 1) * nt] = taylor_rows(data + m.offset(n), Mb)
            rows.append(blk)
            rhs.append(_ev(comps[n], g + data + m.offset(n)))
        sel, rel = m.bpoints_within(g, r)
        for j, rb in zip(sel, rel):
            xb = (np.asarray(g, float) + rb)[None, :]
            for row_ops in m.v_ops(Mb, m.bp_normal[j]):
                rows.append(np.concatenate([basis.apply_op_row(op, rb, Mb) for op in row_ops])[None, :])
                rhs.append(np.array([sum(_op(op, comps[n], xb)[0] for n, op in enumerate(row_ops))]))
        A = np.concatenate(rows)
        delta = np.linalg.pinv(A) @ np.concatenate(rhs)
        for n in range(2):
            for k in range(-M // 2, M // 2):
                e = np.array(g)
                e[n] += k
                if m.exterior(n, e):
                    pos = e + m.offset(n)
                    got = taylor_rows((pos - g)[None, :], Mb)[0] @ delta[n * nt:(n + 1) * nt]
                    want = _ev(comps[n], pos[None, :])[0]
                    assert abs(got - want) < 1e-9 * max(1.0, abs(want))


@pytest.mark.parametrize("kind", ["free", "rigid"])
def test_flat_surface_operators_exact_on_admissible_fields(kind):
    # flat surface z = zs: p odd (free) / even (rigid) in z - zs satisfies the pressure
    # hierarchy; v = grad phi with phi odd (free) / even (rigid) satisfies the velocity
    # one.  The modified staggered operators are then exact for polynomial fields.
    nx, nz, M, zs = 24, 26, 8, 6.3
    m = StaggeredModel(np.full(nx, zs), 1.0, (nx, nz), M=M, surface=kind)
    vs, ps = solve_all(m)
    G, D = assemble(m, vs, ps)
    rng = np.random.default_rng(2)
    par = 1 if kind == "free" else 0

    def admissible(deg):
        c = np.zeros((deg + 1, deg + 1))
        for _ in range(5):
            a = rng.integers(0, 3)
            k = par + 2 * rng.integers(0, 3)
            if a + k > deg:
                continue
            zc = P.polypow([-zs, 1.0], k) * rng.normal()
            for j, v in enumerate(zc):
                c[a, j] += v
        return c

    shape = (nx, nz)
    X, Z = np.meshgrid(np.arange(nx, dtype=float), np.arange(nz, dtype=float), indexing="xy")
    # D+ p at IB v nodes
    pc = admissible(M)
    pfield = _ev(pc, np.stack([X.ravel(), Z.ravel()], 1))
    for n in range(2):
        dp = _der(pc, (1, 0) if n == 0 else (0, 1))
        got = G[n] @ pfield
        for g in m.ib_v(n):
            idx = g[1] * nx + g[0]
            if g[0] < 6 or g[0] > nx - 7:
                continue                              # keep clear of the periodic seam
            pos = (g + m.offset(n))[None, :]
            assert abs(got[idx] - _ev(dp, pos)[0]) < 1e-8 * max(1.0, np.abs(pfield).max())
    # D- . v at IB p nodes, v = grad phi.  The velocity system drops its basis order
    # where the divergence rows cannot fix the rotational part (e.g. prod(z - z_k) over
    # the data rows of a flat surface has zero divergence): exact up to that order.
    mb = min(sol["order"] for sol in ps.values())
    assert mb >= M // 2
    phc = admissible(mb + 1)
    vfs = []
    for n in range(2):
        dn = _der(phc, (1, 0) if n == 0 else (0, 1))
        off = m.offset(n)
        vfs.append(_ev(dn, np.stack([X.ravel() + off[0], Z.ravel() + off[1]], 1)))
    lap = _der(phc, (2, 0))
    lz = _der(phc, (0, 2))
    got = D @ np.concatenate(vfs)
    for g in m.ib_p():
        if g[0] < 9 or g[0] > nx - 10:
            continue                                  # supports up to radius 7.5 clear the seam
        want = _ev(lap, g[None, :])[0] + _ev(lz, g[None, :])[0]
        assert abs(got[g[1] * nx + g[0]] - want) < 1e-8 * max(1.0, np.abs(vfs[0]).max())


def _images_error(h, kind, M=4, c=1500.0, f0=15.0, T=0.45, dtfac=0.1):
    Lx = 1000.0
    nx = int(round(Lx / h))
    zs = 107.0
    nz = int(round(900.0 / h))
    m = StaggeredModel(np.full(nx, zs), h, (nx, nz), M=M, surface=kind)
    vs, ps = solve_all(m)
    G, D = assemble(m, vs, ps)
    crit = 2 * h / (c * np.sqrt(2) * np.abs(fd.staggered_first_derivative_weights(M)).sum())
    dt = dtfac * crit
    nt = int(T / dt)
    src = (500.0, 210.0)
    recs = [(500.0 + dx, z) for dx in (0.0, 200.0) for z in (110.0, 160.0)]
    sim = StaggeredSimulation(m, G, D, np.full((nz, nx), c), dt, [src], recs)
    tr = sim.run(analytic.ricker(np.arange(nt) * dt, f0)[None, :], nt)
    tt = (np.arange(nt) + 1) * dt
    t0 = 1.5 / f0

    def sdot(tau):
        # p_tt = c^2 lap p + f_t: the pressure answers the time derivative of the source,
        # applied half a step later by the staggered update
        tau = tau - dt / 2 - t0
        a = (np.pi * f0 * tau) ** 2
        return -2 * np.pi ** 2 * f0 ** 2 * tau * (3 - 2 * a) * np.exp(-a)

    return np.array([np.linalg.norm(tr[:, k] - analytic.image_trace(src, r, zs, tt, c, sdot, kind, (Lx,), 2))
                     / np.linalg.norm(analytic.image_trace(src, r, zs, tt, c, sdot, kind, (Lx,), 2))
                     for k, r in enumerate(recs)])


@pytest.mark.parametrize("kind", ["free", "rigid"])
def test_first_order_form_method_of_images_convergence(kind):
    e1 = _images_error(10.0, kind)
    e2 = _images_error(5.0, kind)
    order = np.log2(e1 / e2)
    assert np.all(e2 < 0.015), e2
    assert np.all(order > 3.5), order
