"""Discrete adjoint of the second-order stepper and the velocity gradient.

Test infrastructure (see ``oracle/__init__.py``).

Not a result of the paper (full-waveform inversion is only its motivation, in the
introduction); it differentiates the oracle's own recurrence exactly.  With
D = 1/(1+s) and P = D (2 + K L), Q = D (1 - s), the forward recurrence is
u^{n+1} = P u^n - Q u^{n-1} + D dt^2 f^n and the traces are d^n = R u^{n+1}.
For J with dJ/dd^n = res^n, mu^m = dJ/du^m obeys
    mu^m = R^T res^{m-1} + P^T mu^{m+1} - Q mu^{m+2},
so lambda = D mu follows the same damped leapfrog with L^T K in place of K L:
    lambda^m = D [2 lambda^{m+1} - (1 - s) lambda^{m+2} + L^T (K lambda^{m+1}) + R^T res^{m-1}],
and dJ/dK_i = sum_m lambda^m_i (L u^{m-1})_i, dJ/dc_i = dJ/dK_i * 2 c_i dt^2 / h^2 at
interior nodes (K is identically zero outside).  The damping profile is held fixed.
"""
from __future__ import annotations

import numpy as np


def forward_fields(sim, wavelet, nt):
    """Run ``sim`` from rest, returning traces (nt, nrec) and [u^0, ..., u^nt]."""
    wavelet = np.atleast_2d(wavelet)
    us = [sim.u.copy()]
    tr = []
    for n in range(nt):
        tr.append(sim.step(wavelet[:, n]))
        us.append(sim.u.copy())
    return np.array(tr), us


def receiver_transpose(sim, res_n):
    out = np.zeros(sim.N)
    for r, a in zip(sim.rec, res_n):
        for j, w in r:
            out[j] += w * a
    return out


def gradient_K(sim, us, residual):
    """dJ/dK for residual[n, r] = dJ/dd^n_r, given the forward fields us."""
    nt = residual.shape[0]
    LT = sim.L.T.tocsr()
    lam1 = np.zeros(sim.N)       # lambda^{m+1}
    lam2 = np.zeros(sim.N)       # lambda^{m+2}
    g = np.zeros(sim.N)
    for m in range(nt, 0, -1):
        lam = (2.0 * lam1 - (1.0 - sim.s) * lam2 + LT @ (sim.K * lam1)
               + receiver_transpose(sim, residual[m - 1])) / (1.0 + sim.s)
        g += lam * (sim.L @ us[m - 1])
        lam2, lam1 = lam1, lam
    return g


def gradient_c(sim, vel, us, residual):
    vel = np.asarray(vel, dtype=np.float64).ravel()
    gK = gradient_K(sim, us, residual)
    return np.where(sim.K != 0.0, gK * 2.0 * vel * sim.dt ** 2 / sim.h ** 2, 0.0)
