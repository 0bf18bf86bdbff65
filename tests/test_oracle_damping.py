"""Pins of the oracle's damping layer: the profile's values at chosen nodes (faces,
power, constant), and the amplitude a plane wave keeps after crossing the layer, being
reflected at the outer edge and crossing back, in both forms (1D leapfrogs written here
with the oracle's profile)."""
import math

import numpy as np
import pytest

from oracle import fd
from oracle.stepper import damping_profile


def test_profile_closed_form_values():
    # 2D (nx = 100, nz = 60), W = 10, h = 5 m, c_max = 2000 m/s, R = 1e-3: the lateral axis
    # is damped on both faces, depth only at the bottom; d = d_max (l / W)^2 per axis,
    # summed, with l the cells into the layer.
    nx, nz, W, h, c, dt, R = 100, 60, 10, 5.0, 2000.0, 1e-3, 1e-3
    dmax_p2 = 3.0 * c * math.log(1000.0) / (W * h)
    for form, dmax in (("p2", dmax_p2), ("pv1", dmax_p2 / 2)):
        s = damping_profile((nx, nz), h, dt, c, W, R, form=form).reshape(nz, nx)
        at = lambda x, z: s[z, x] / (dt / 2.0)          # back to d
        assert at(50, 0) == 0.0                           # top face: no layer
        assert at(50, 30) == 0.0                          # inside
        assert abs(at(0, 30) - dmax) < 1e-12 * dmax       # left edge, l = W
        assert abs(at(99, 30) - dmax) < 1e-12 * dmax      # right edge, l = W
        assert abs(at(5, 30) - dmax * 0.25) < 1e-12 * dmax   # l = W / 2 -> (1/2)^2
        assert abs(at(50, 59) - dmax) < 1e-12 * dmax      # bottom edge
        assert abs(at(50, 49 + 3) - dmax * 0.09) < 1e-12 * dmax   # l = 3 -> (3/10)^2
        assert at(50, 49) == 0.0                          # first node outside the bottom layer
        assert abs(at(0, 59) - 2 * dmax) < 1e-12 * dmax   # corner: the faces add
    # 3D: both lateral axes on both faces
    s3 = damping_profile((30, 30, 30), h, dt, c, W, R).reshape(30, 30, 30)
    assert abs(s3[0, 0, 0] / (dt / 2) - 2 * dmax_p2) < 1e-12 * dmax_p2     # top face undamped in z
    assert abs(s3[29, 15, 15] / (dt / 2) - dmax_p2) < 1e-12 * dmax_p2
    with pytest.raises(ValueError):
        damping_profile((8, 8), h, dt, c, 2, R, form="p3")


def _ricker(x, lam):
    a = (math.pi * x / lam) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def _layer(n, W, form, R=1e-3):
    """s of a depth axis of n nodes with the bottom layer of the oracle's profile, grid
    units (h = 1, c = 1), taken from a lateral column outside the lateral layers."""
    M = 8
    if form == "p2":
        dt = 0.5 * fd.critical_dt(1.0, 1.0, M, 1)
    else:
        ws = fd.staggered_first_derivative_weights(M)
        dt = 0.5 * 2.0 / np.sum(np.abs(ws))
    nx = 2 * W + 3
    s = damping_profile((nx, n), 1.0, dt, 1.0, W, R, form=form).reshape(n, nx)[:, nx // 2]
    return s, dt


def _reflection_p2(W, lam, n=700, z0=150.0, zr=250):
    s, dt = _layer(n, W, "p2")
    w2 = fd.second_derivative_weights(8)
    z = np.arange(n, dtype=float)
    p, pm = _ricker(z - z0, lam), _ricker(z - z0 + dt, lam)     # travelling down
    rec = []
    for _ in range(int(2.2 * (n - z0) / dt)):
        pad = np.concatenate([np.zeros(4), p, np.zeros(4)])
        lap = sum(w2[k] * pad[k:k + n] for k in range(9))
        p, pm = (2 * p - (1 - s) * pm + dt * dt * lap) / (1 + s), p
        rec.append(p[zr])
    rec = np.array(rec)
    t = (np.arange(len(rec)) + 1) * dt
    inc = np.abs(rec[t < (zr - z0) + 4 * lam]).max()
    ref = np.abs(rec[t > 2 * (n - 1 - W - zr)]).max()
    return ref / inc


def _reflection_pv1(W, lam, n=700, z0=150.0, zr=250):
    # p on nodes, v at node + 1/2, p_t = c^2 v_z, v_t = p_z (the signs of the first-order
    # system as printed), both damped with the profile of the node index
    s, dt = _layer(n, W, "pv1")
    ws = fd.staggered_first_derivative_weights(8)
    z = np.arange(n, dtype=float)
    p = _ricker(z - z0, lam)
    v = -_ricker(z + 0.5 - z0 + dt / 2, lam)                    # the down-going wave's v
    rec = []
    for _ in range(int(2.2 * (n - z0) / dt)):
        pp = np.concatenate([np.zeros(3), p, np.zeros(4)])
        v = ((1 - s) * v + dt * sum(ws[k] * pp[k:k + n] for k in range(8))) / (1 + s)
        vv = np.concatenate([np.zeros(4), v, np.zeros(3)])
        p = ((1 - s) * p + dt * sum(ws[k] * vv[k:k + n] for k in range(8))) / (1 + s)
        rec.append(p[zr])
    rec = np.array(rec)
    t = (np.arange(len(rec)) + 1) * dt
    inc = np.abs(rec[t < (zr - z0) + 4 * lam]).max()
    ref = np.abs(rec[t > 2 * (n - 1 - W - zr)]).max()
    return ref / inc


def test_layer_reflection_second_order_form():
    # a Ricker pulse of wavelength W / 5 comes back from a 40-cell layer with about R = 1e-3
    # of its amplitude (the WKB round trip; the layer's own gradient adds a little).  Half
    # the constant would give about R^(1/2), a linear profile several times R.
    r = _reflection_p2(40, 8.0)
    assert 1e-3 / 3 < r < 2e-3, r


def test_layer_reflection_first_order_form():
    # damping both fields keeps the impedance: about R also for a wavelength of W / 2
    r = _reflection_pv1(40, 20.0)
    assert 1e-3 / 3 < r < 2e-3, r
