"""Pins of the oracle adjoint: central finite differences of the misfit and the
dot-product identity of the linearised recurrence."""
import numpy as np

from oracle import stepper
from oracle.adjoint import forward_fields, gradient_c
from oracle.weights import IBModel
from paper_2309_03600_amd import workloads as W


def _setup(surface):
    wl = W.small2d(nx=48, nz=44, M=8, surface=surface, nt=140, hill=30.0, cfg=96)
    m = IBModel(wl.heights, wl.h, wl.shape, M=wl.M, surface=wl.surface, eta=wl.eta)
    sols = stepper.solve_all(m)
    L = stepper.assemble_laplacian(m, sols)
    return wl, m, L


def _misfit(wl, m, L, vel, dobs):
    sim = stepper.Simulation(m, L, vel, wl.dt, wl.src, wl.rec, damp_width=0)
    tr, us = forward_fields(sim, wl.wavelets(np.float64), wl.nt)
    return 0.5 * np.sum((tr - dobs) ** 2), tr, us, sim


def test_gradient_matches_central_differences():
    for surface in ("free", "rigid"):
        wl, m, L = _setup(surface)
        rng = np.random.default_rng(4)
        v0 = wl.vel.copy()
        # observed data from a smooth +3 % anomaly
        zz, xx = np.meshgrid(np.arange(wl.shape[1]), np.arange(wl.shape[0]), indexing="ij")
        blob = np.exp(-((xx - 24) ** 2 + (zz - 30) ** 2) / (2 * 5.0 ** 2))
        _, dobs, _, _ = _misfit(wl, m, L, v0 * (1 + 0.03 * blob), 0.0)
        J0, tr, us, sim = _misfit(wl, m, L, v0, dobs)
        g = gradient_c(sim, v0, us, tr - dobs)
        dv = np.exp(-((xx - 20) ** 2 + (zz - 33) ** 2) / (2 * 4.0 ** 2)) * (1 + 0.2 * rng.standard_normal(xx.shape))
        dv *= 10.0
        eps = 1e-3
        Jp, *_ = _misfit(wl, m, L, v0 + eps * dv, dobs)
        Jm, *_ = _misfit(wl, m, L, v0 - eps * dv, dobs)
        fd = (Jp - Jm) / (2 * eps)
        an = float(np.sum(g * dv.ravel()))
        assert abs(fd - an) <= 1e-6 * abs(fd), (surface, fd, an)


def test_linearised_dot_product():
    # <L x, y> = <x, L^T y> for the assembled modified operator (sanity of the sparse
    # transpose used by the adjoint), including the IB rows
    wl, m, L = _setup("free")
    rng = np.random.default_rng(5)
    x = rng.standard_normal(L.shape[0])
    y = rng.standard_normal(L.shape[0])
    assert abs((L @ x) @ y - x @ (L.T @ y)) < 1e-10 * np.linalg.norm(L @ x) * np.linalg.norm(y)
