"""Pins for oracle.lsop: the discretised operator, its FFT route and the RHS.

Pins: exact symmetry of V, entries against mpmath's independent Hankel function,
the FFT convolution against the dense definition (two routes, same sum), q = 0
giving the identity, and the physics of the sign choice against the Mie series.
"""
import math

import mpmath
import numpy as np
import pytest

from oracle import lsop, mie, special
from paper_2204_00326_amd import inputs


def test_dense_V_symmetric_exactly():
    V = lsop.dense_V(16, 1.0, 10.0)
    assert np.array_equal(V, V.T)


def test_dense_V_entries_mpmath():
    n, L, kappa = 16, 1.0, 10.0
    h = 2 * L / n
    V = lsop.dense_V(n, L, kappa)
    x = lsop.grid_coords(n, L)
    rng = np.random.default_rng(3)
    for _ in range(12):
        i, j = rng.integers(0, n * n, size=2)
        if i == j:
            continue
        r = math.hypot(*(x[i] - x[j]))
        ref = h * h * 0.25j * complex(mpmath.hankel1(0, kappa * r))
        assert abs(V[i, j] - ref) <= 1e-14 * abs(ref)
    assert V[5, 5] == special.self_cell(h, kappa)


def test_grid_coordinates_match_inputs_convention():
    p = inputs.grid_points(8, 1.0)
    assert np.array_equal(p, lsop.grid_coords(8, 1.0))
    # a indexes the first coordinate: i = a*n + b
    assert p[1, 0] == p[0, 0] and p[1, 1] > p[0, 1]
    assert p[8, 0] > p[0, 0]


@pytest.mark.parametrize("n,kappa", [(16, 10.0), (24, 40.0)])
def test_fft_equals_dense(n, kappa):
    L = 1.0
    V = lsop.dense_V(n, L, kappa)
    x = inputs.random_vector(n * n, seed=1)
    y_dense = V @ x
    y_fft = lsop.FFTApplyV(n, L, kappa)(x)
    assert np.linalg.norm(y_fft - y_dense) <= 1e-13 * np.linalg.norm(y_dense)


def test_sampled_rows_match_dense():
    n, L, kappa = 20, 1.0, 15.0
    V = lsop.dense_V(n, L, kappa)
    x = inputs.random_vector(n * n, seed=2)
    rows = np.array([0, 7, 199, 399])
    got = lsop.sampled_rows_Vx(n, L, kappa, x, rows)
    assert np.allclose(got, (V @ x)[rows], rtol=1e-13, atol=0)


def test_zero_contrast_is_identity():
    n = 8
    A = lsop.dense_A(n, 1.0, 10.0, np.zeros(n * n))
    assert np.array_equal(A, np.eye(n * n))


def test_rhs_physical_sign():
    n, L, kappa = 8, 1.0, 10.0
    q = np.linspace(0, 1, n * n)
    f = lsop.rhs_planewave(n, L, kappa, q, 0.3, sign=-1)
    x = lsop.grid_coords(n, L)
    ref = kappa ** 2 * q * np.exp(1j * kappa * (math.cos(0.3) * x[:, 0] + math.sin(0.3) * x[:, 1]))
    assert np.allclose(f, ref, rtol=1e-15, atol=0)


def _disc_error(n, sign):
    kappa, R, q0, L = 10.0, 0.6, 1.0, 1.0
    pts = lsop.grid_coords(n, L)
    q = inputs.contrast_disc(pts, R, q0)
    A = lsop.dense_A(n, L, kappa, q, sign)
    f = lsop.rhs_planewave(n, L, kappa, q, 0.0, sign)
    psi = np.linalg.solve(A, f)
    inside = q > 0
    u = mie.total_field(pts[inside], kappa, R, q0)
    ref = kappa ** 2 * q0 * u
    return np.linalg.norm(psi[inside] - ref) / np.linalg.norm(ref)


def test_sign_against_mie_series():
    # The physical sign s = -1 reproduces the Mie solution to discretisation accuracy;
    # the printed sign of Eq. (eq:6) (s = +1) does not.
    e_minus = _disc_error(32, -1)
    e_plus = _disc_error(32, +1)
    assert e_minus < 0.15
    assert e_plus > 1.0


def test_discretisation_error_decreases():
    e32 = _disc_error(32, -1)
    e64 = _disc_error(64, -1)
    assert e64 < 0.5 * e32
