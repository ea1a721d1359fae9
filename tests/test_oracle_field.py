"""Pins of the off-grid field / error-function oracle (Section 6, Eq. (eq:error)).

* the cell integral at its own centre is the exact self-cell term W0 (closed form, and the
  value printed for (h, kappa) = (1/16, 10));
* for a distant cell it follows the midpoint rule with its second-order correction,
  h^2 G(d) (1 - (kappa h)^2 / 24), since Delta G = -kappa^2 G away from the source;
* the scattered field of the q = 1 disc evaluated off the grid (outside the square) approaches
  the Bessel-series (Mie) field;
* E(x) at a cell centre of an exact discrete solution reduces to |q_i sum_j (I_ij - V_ij) psi_j|
  (the discrete equation holds exactly there), and vanishes where q = 0 outside the grid.
"""
import math

import numpy as np
import pytest

from oracle import field as ofield
from oracle import lsop, mie
from oracle.special import green, self_cell


def test_cell_integral_at_own_centre_is_self_cell():
    h, kappa = 1.0 / 16.0, 10.0
    I = ofield.cell_integral((0.0, 0.0), 0, 0, 0.0, 0.0, h, kappa)
    ref = 1.000152508662452e-3 + 9.607582031344723e-4j
    assert abs(I - ref) < 1e-11 * abs(ref)
    assert abs(I - self_cell(h, kappa)) < 1e-11 * abs(ref)
    # off-centre inside the cell the integral changes, continuously
    I2 = ofield.cell_integral((0.2 * h, -0.1 * h), 0, 0, 0.0, 0.0, h, kappa)
    assert 1e-6 < abs(I2 - I) / abs(I) < 0.2


def test_distant_cell_follows_second_order_midpoint_rule():
    h, kappa = 0.05, 10.0          # kappa h = 0.5
    x = (0.0, 0.0)
    a, b = 10, 0                     # centre at distance 10 h
    I = ofield.cell_integral(x, a, b, 0.0, 0.0, h, kappa)
    mid = h * h * green(10 * h, kappa)
    corr = mid * (1.0 - (kappa * h) ** 2 / 24.0)
    assert abs(I - corr) < 2e-4 * abs(mid)
    assert abs(I - mid) > 5e-3 * abs(mid)      # the correction is really there


def test_scattered_field_off_grid_approaches_mie():
    # first-order convergence (staircased disc): 11% at n = 16, 5.5% at n = 32
    L, kappa, R, q0 = 1.0, 10.0, 0.6, 1.0
    targets = np.array([[1.5 * math.cos(t), 1.5 * math.sin(t)] for t in (0.0, 1.0, 2.5, 4.0)])
    ref = mie.total_field(targets, kappa, R, q0) - np.exp(1j * kappa * targets[:, 0])
    errs = []
    for n in (16, 32):
        h = 2 * L / n
        x = lsop.grid_coords(n, L)
        q = (np.hypot(x[:, 0], x[:, 1]) < R).astype(float) * q0
        psi = np.linalg.solve(lsop.dense_A(n, L, kappa, q), lsop.rhs_planewave(n, L, kappa, q, 0.0))
        u = ofield.field(targets, n, -L + 0.5 * h, -L + 0.5 * h, h, kappa, psi)
        errs.append(np.linalg.norm(u - ref) / np.linalg.norm(ref))
    assert errs[1] < 0.08 and errs[1] < 0.7 * errs[0], errs


def test_error_function_at_cell_centres_of_an_exact_discrete_solution():
    n, L, kappa = 6, 1.0, 4.0
    h = 2 * L / n
    x = lsop.grid_coords(n, L)
    rng = np.random.default_rng(3)
    q = rng.uniform(0.2, 1.0, n * n)
    A = lsop.dense_A(n, L, kappa, q)
    theta = 0.7
    f = lsop.rhs_planewave(n, L, kappa, q, theta)
    psi = np.linalg.solve(A, f)
    V = lsop.dense_V(n, L, kappa)
    x0 = -L + 0.5 * h
    for i in (0, 14, 35):
        ai, bi = divmod(i, n)
        I = np.array([ofield.cell_integral(x[i], a, b, x0, x0, h, kappa) for a in range(n) for b in range(n)])
        expect = abs(q[i] * np.dot(I - V[i], psi))
        E = ofield.error_function(x[i:i + 1], q[i:i + 1], theta, n, x0, x0, h, kappa, psi)[0]
        assert abs(E - expect) <= 1e-9 * max(expect, 1e-12) + 1e-14, (i, E, expect)
        assert E < 0.25 * abs(psi[i]) / kappa ** 2   # a fraction of the terms it balances
    # outside the grid and the contrast: nothing to miss
    E = ofield.error_function(np.array([[3.0, 0.5]]), np.array([0.0]), theta, n, x0, x0, h, kappa, psi)[0]
    assert E == 0.0
