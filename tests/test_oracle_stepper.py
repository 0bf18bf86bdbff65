"""Pins of the oracle time stepper: method of images for flat free / rigid surfaces
(with the convergence order the paper reports for M=4), spectra of the modified
operator, non-growth without damping and decay with it."""
import numpy as np
import pytest

from oracle import analytic, fd, stepper
from oracle.weights import IBModel


def _images_error(h, kind, M=4, c=1500.0, f0=15.0, T=0.45, dtfac=0.1):
    # flat surface at 107 m (off-grid for h = 10 and 5 m), source on a node 103 m below
    # it, receivers on nodes 3 m and 53 m below the surface at offsets 0 and 200 m;
    # lateral period 1000 m (images +-2, which arrive after the window anyway)
    Lx = 1000.0
    nx = int(round(Lx / h))
    zs = 107.0
    nz = int(round(900.0 / h))
    m = IBModel(np.full(nx, zs), h, (nx, nz), M=M, surface=kind)
    sols = stepper.solve_all(m)
    L = stepper.assemble_laplacian(m, sols)
    dt = dtfac * fd.critical_dt(h, c, M, 2)
    nt = int(T / dt)
    src = (500.0, 210.0)
    recs = [(500.0 + dx, z) for dx in (0.0, 200.0) for z in (110.0, 160.0)]
    sim = stepper.Simulation(m, L, np.full((nz, nx), c), dt, [src], recs)
    w = analytic.ricker(np.arange(nt) * dt, f0)[None, :]
    tr = sim.run(w, nt)
    tt = (np.arange(nt) + 1) * dt
    s = lambda tau: analytic.ricker(tau, f0)
    errs = []
    for k, r in enumerate(recs):
        a = analytic.image_trace(src, r, zs, tt, c, s, kind, period=(Lx,), nper=2)
        errs.append(np.linalg.norm(tr[:, k] - a) / np.linalg.norm(a))
    return np.array(errs)


@pytest.mark.parametrize("kind", ["free", "rigid"])
def test_method_of_images_convergence_m4(kind):
    # The paper reports close to fourth-order convergence for M=4 (convergence-testing
    # section, second-order form); halving h must cut the error by 2^3.5 or more.
    e1 = _images_error(10.0, kind)
    e2 = _images_error(5.0, kind)
    order = np.log2(e1 / e2)
    assert np.all(e2 < 0.01), e2
    assert np.all(order > 3.0), (e1, e2, order)
    assert np.median(order) > 3.5, order


def _dense_operator(model):
    sols = stepper.solve_all(model)
    L = stepper.assemble_laplacian(model, sols).toarray()
    inter = model.geom.interior_grid().ravel()
    return L[np.ix_(inter, inter)]


@pytest.mark.parametrize("kind,M", [("free", 4), ("free", 8), ("rigid", 4), ("rigid", 8)])
def test_flat_surface_spectrum_real_nonpositive(kind, M):
    nx, nz = 24, 22
    m = IBModel(np.full(nx, 4.3), 1.0, (nx, nz), M=M, surface=kind)
    ev = np.linalg.eigvals(_dense_operator(m))
    assert np.max(np.abs(ev.imag)) < 1e-8
    assert ev.real.max() < 1e-10
    # leapfrog with dt = 0.5 dt_crit is stable iff K*mu lies in [-4, 0]
    K = (0.5 * 2.0 / np.sqrt(2 * fd.nyquist_symbol(M))) ** 2
    assert (K * ev.real).min() > -4.0


def test_flat_surface_no_growth_and_damping_decay():
    nx, nz = 32, 30
    m = IBModel(np.full(nx, 5.3), 1.0, (nx, nz), M=8)
    sols = stepper.solve_all(m)
    L = stepper.assemble_laplacian(m, sols)
    rng = np.random.default_rng(1)
    inter = m.geom.interior_grid().ravel()
    dt = 0.5 * fd.critical_dt(1.0, 1.0, 8, 2)
    for width, check in ((0, "bounded"), (8, "decay")):
        sim = stepper.Simulation(m, L, np.ones((nz, nx)), dt, [], [], damp_width=width)
        sim.u = np.where(inter, rng.normal(size=sim.N), 0.0)
        sim.um = sim.u.copy()
        start = np.abs(sim.u).max()
        peak = 0.0
        for n in range(1500):
            sim.step([])
            peak = max(peak, np.abs(sim.u).max())
        if check == "bounded":
            assert peak < 20 * start
        else:
            assert np.abs(sim.u).max() < 0.5 * start


def test_source_receiver_multilinear_weights():
    shape = (10, 8)
    w = stepper.multilinear((3.25, 4.5), shape)
    assert abs(sum(v for _, v in w) - 1.0) < 1e-15
    assert dict(w) == {4 * 10 + 3: 0.75 * 0.5, 4 * 10 + 4: 0.25 * 0.5, 5 * 10 + 3: 0.375, 5 * 10 + 4: 0.125}
    # on a node: a single weight
    assert stepper.multilinear((2.0, 3.0), shape) == [(32, 1.0)]
