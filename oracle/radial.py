"""Scattering by a radially symmetric contrast q(r), by separation of variables (oracle).

Test infrastructure: only tests/ use this module.

Paper, Section 1, Eq. (eq:1): Delta u + kappa^2 (1 + q) u = 0, u = u_inc + u_s with the radiation
condition (eq:4), u_inc = exp(i kappa x1) = sum_m i^m J_m(kappa r) e^{i m theta}.  For q = q(r)
supported in r <= R every angular mode separates: u = sum_m u_m(r) e^{i m theta}, and since the
modes m and -m carry the same coefficient, u = u_0 + 2 sum_{m >= 1} u_m(r) cos(m theta).

Inside, u_m = alpha_m v_m(r) with v_m the solution regular at 0 of
    v'' + v'/r + (kappa^2 (1 + q(r)) - m^2 / r^2) v = 0,
written as v = r^m z(r) (no underflow at large m):
    z'' + (2m + 1)/r z' + kappa^2 (1 + q(r)) z = 0,   z(0) = 1, z'(0) = 0,
integrated from r0 = 1e-8 R (z'(r0) from the series) with an explicit 8th-order Runge-Kutta
method to relative tolerance 1e-12.  Outside, u_m = i^m J_m(kappa r) + b_m H_m(kappa r); continuity of
u_m and u_m' at r = R fixes alpha_m and b_m.  A constant contrast reproduces the Bessel series
of the disc (tested against mie.py); for a smooth q the field is the reference that the high-order
panel discretisation (panels.py) converges to.  The volume density of the paper's formulation is
psi = kappa^2 q u.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate
from scipy.special import h1vp, hankel1, jv, jvp


def _mode(m: int, kappa: float, q_r, R: float):
    """(alpha_m, b_m, z-interpolant) for mode m >= 0; inside u_m(r) = alpha_m (r/R)^m z(r)."""
    r0 = 1e-8 * R
    k2 = kappa * kappa

    def rhs(r, y):
        z, dz = y
        return [dz, -(2 * m + 1) / r * dz - k2 * (1.0 + q_r(r)) * z]

    dz0 = -k2 * (1.0 + q_r(0.0)) * r0 / (2 * m + 2)
    sol = integrate.solve_ivp(rhs, (r0, R), [1.0, dz0], method="DOP853", rtol=1e-12, atol=1e-300,
                              dense_output=True)
    if not sol.success:
        raise RuntimeError(sol.message)
    zR, dzR = sol.y[0, -1], sol.y[1, -1]
    # with v scaled by R^m: V = z(R), V' = z'(R) + (m / R) z(R)
    V, Vp = zR, dzR + (m / R) * zR
    kR = kappa * R
    M = np.array([[V, -hankel1(m, kR)], [Vp, -kappa * h1vp(m, kR)]], dtype=complex)
    rhs_v = np.array([(1j ** m) * jv(m, kR), (1j ** m) * kappa * jvp(m, kR)], dtype=complex)
    alpha, b = np.linalg.solve(M, rhs_v)
    return alpha, b, sol.sol


def total_field(points: np.ndarray, kappa: float, q_r, R: float, qmax: float, mmax: int | None = None) -> np.ndarray:
    """u at points (m x 2) for the contrast q_r(r) supported in r <= R (qmax >= max q)."""
    points = np.atleast_2d(points)
    r = np.hypot(points[:, 0], points[:, 1])
    th = np.arctan2(points[:, 1], points[:, 0])
    if mmax is None:
        mmax = int(kappa * max(R, float(r.max())) * math.sqrt(1.0 + qmax)) + 30
    out = np.zeros(len(points), dtype=complex)
    inside = r < R
    for m in range(mmax + 1):
        alpha, b, zs = _mode(m, kappa, q_r, R)
        eps = 1.0 if m == 0 else 2.0
        c = eps * np.cos(m * th)
        if inside.any():
            ri = np.maximum(r[inside], 1e-8 * R)
            out[inside] += c[inside] * alpha * (ri / R) ** m * zs(ri)[0]
        if (~inside).any():
            out[~inside] += c[~inside] * b * hankel1(m, kappa * r[~inside])
    out[~inside] += np.exp(1j * kappa * points[~inside, 0])
    return out
