"""Pins of the oracle's Taylor basis and boundary rows against what the paper prints."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import basis, fd

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_rows(X, Y):
    rows = {}
    for line in open(os.path.join(GOLDEN, "paper_rows_2d_m4.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, *exprs = line.split()
        rows[name] = np.array([eval(e, {"X": X, "Y": Y}) for e in exprs], dtype=float)
    return rows


def test_term_order_matches_scaled_delta_listing():
    # Section "Constructing Finite-Difference Approximations": the 2D fourth-order
    # scaled derivative vector lists 1, d/dx, d/dy, d2/dx2, d2/dxdy, d2/dy2, d3/dx3, ...
    expect = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 0), (2, 1), (1, 2), (0, 3),
              (4, 0), (3, 1), (2, 2), (1, 3), (0, 4)]
    assert basis.multi_indices(4, 2) == expect
    # 3D second degree: x^2, xy, xz, y^2, yz, z^2 (the 3D a vector).
    assert basis.multi_indices(2, 3)[4:] == [(2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2)]


@pytest.mark.parametrize("M", range(0, 11))
def test_required_rank_formulas(M):
    # Rank rule: M+1 (1D), (M+1)(M+2)/2 (2D), (M+1)(M+2)(M+3)/6 (3D).
    assert basis.n_terms(M, 1) == M + 1
    assert basis.n_terms(M, 2) == (M + 1) * (M + 2) // 2
    assert basis.n_terms(M, 3) == (M + 1) * (M + 2) * (M + 3) // 6


def test_m2_system_and_inverse_exact():
    # The regular-grid M=2 system and its printed inverse.
    A = [basis.taylor_row_exact((o,), 2) for o in (-1, 0, 1)]
    assert A == [[1, -1, Fraction(1, 2)], [1, 0, 0], [1, 1, Fraction(1, 2)]]
    printed_inv = np.array([[0, 1, 0], [-0.5, 0, 0.5], [1, -2, 1]])
    Af = np.array([[float(v) for v in r] for r in A])
    assert np.array_equal(np.linalg.inv(Af) @ Af, np.eye(3)) or np.allclose(np.linalg.inv(Af) @ Af, np.eye(3))
    np.testing.assert_allclose(np.linalg.inv(Af), printed_inv, atol=1e-15)
    # the float row builder agrees with the exact one
    for o, r in zip((-1, 0, 1), Af):
        np.testing.assert_array_equal(basis.taylor_row((o,), 2), r)


@pytest.mark.parametrize("X,Y", [(0.3, -0.7), (-1.25, 0.5), (0.0, 0.0)])
def test_printed_free_surface_rows(X, Y):
    g = _golden_rows(X, Y)
    d = (X, Y)
    ops = basis.free_surface_ops(4, 2)
    assert len(ops) == 3          # three rows per boundary point at M=4
    np.testing.assert_allclose(basis.apply_op_row(ops[0], d, 4), g["p0"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(basis.apply_op_row(ops[1], d, 4), g["lap"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(basis.apply_op_row(ops[2], d, 4), g["bih"], rtol=0, atol=1e-15)


def test_printed_velocity_divergence_row():
    X, Y = 0.4, -0.15
    g = _golden_rows(X, Y)["divv"]
    bx = basis.apply_op_row({(1, 0): 1.0}, (X, Y), 2)
    by = basis.apply_op_row({(0, 1): 1.0}, (X, Y), 2)
    np.testing.assert_allclose(np.concatenate([bx, by]), g, atol=1e-15)


def test_higher_order_conditions_drop_out():
    # conditions of order above M give 0 = 0: the operator row is identically zero
    op = basis.op_laplacian_power(3, 2)       # order 6
    assert not np.any(basis.apply_op_row(op, (0.2, 0.9), 4))
    assert len(basis.free_surface_ops(8, 3)) == 5
    assert len(basis.rigid_surface_ops(8, 3, (0.0, 0.0, 1.0))) == 4


def test_one_dimensional_worked_example():
    # Section "Approximating Boundary Conditions": two interior points, one boundary
    # point with f = 0 and f'' = 0; extrapolating f = alpha (x - x_b) must be exact.
    x0, x1, x2, xb = 0.0, 1.0, 2.0, -0.4
    A = np.array([basis.taylor_row((x1 - x0,), 2), basis.taylor_row((x2 - x0,), 2),
                  basis.apply_op_row(basis.op_identity(1), (xb - x0,), 2),
                  basis.apply_op_row(basis.op_laplacian_power(1, 1), (xb - x0,), 2)])
    printed = np.array([[1, x1 - x0, (x1 - x0) ** 2 / 2], [1, x2 - x0, (x2 - x0) ** 2 / 2],
                        [1, xb - x0, (xb - x0) ** 2 / 2], [0, 0, 1]])
    np.testing.assert_array_equal(A, printed)
    alpha = 1.7
    rhs = np.array([alpha * (x1 - xb), alpha * (x2 - xb), 0.0, 0.0])
    delta = np.linalg.pinv(A) @ rhs
    np.testing.assert_allclose(delta, [alpha * (x0 - xb), alpha, 0.0], atol=1e-13)
    for x3 in (-1.0, -2.0):
        B = basis.taylor_row((x3 - x0,), 2)
        assert abs(B @ delta - alpha * (x3 - xb)) < 1e-13


def test_fornberg_closed_forms():
    np.testing.assert_allclose(fd.second_derivative_weights(4), [-1 / 12, 4 / 3, -5 / 2, 4 / 3, -1 / 12], atol=1e-15)
    np.testing.assert_allclose(fd.second_derivative_weights(8),
                               [-1 / 560, 8 / 315, -1 / 5, 8 / 5, -205 / 72, 8 / 5, -1 / 5, 8 / 315, -1 / 560], atol=1e-14)
    np.testing.assert_allclose(fd.staggered_first_derivative_weights(8),
                               [5 / 7168, -49 / 5120, 245 / 3072, -1225 / 1024, 1225 / 1024, -245 / 3072, 49 / 5120, -5 / 7168],
                               atol=1e-15)
    # the M=2 second-derivative row of the printed inverse is [1, -2, 1]
    np.testing.assert_allclose(fd.second_derivative_weights(2), [1, -2, 1], atol=1e-15)
    assert abs(fd.nyquist_symbol(4) - 16 / 3) < 1e-13
    # M=8: sum of |w_k| over the even/odd alternation = 2(8/5+1/5+8/315+1/560)+205/72
    assert abs(fd.nyquist_symbol(8) - (2 * (8 / 5 + 1 / 5 + 8 / 315 + 1 / 560) + 205 / 72)) < 1e-13


def test_critical_timestep_config1():
    # 2D, M=4, h=10 m, c=1500 m/s: dt_crit = 2h / (c sqrt(2 * 16/3))
    dt = fd.critical_dt(10.0, 1500.0, 4, 2)
    assert abs(dt - 2 * 10 / (1500 * math.sqrt(32 / 3))) < 1e-15
    assert abs(0.5 * dt - 2.0412414523e-3) < 1e-12
