"""Bessel-series (Mie) solution for a constant-contrast disc (oracle).

Paper, Section 1, Eq. (eq:1): Delta u + kappa^2 (1 + q) u = 0 with u = u_inc + u_s and
the radiation condition (eq:4).  For q = q0 inside |x| < R and 0 outside and
u_inc = exp(i kappa x1) = sum_n i^n J_n(kappa r) e^{i n theta}, separation of variables
gives, with kappa1 = kappa sqrt(1 + q0),

    inside:  u = sum_n a_n J_n(kappa1 r) e^{i n theta}
    outside: u = u_inc + sum_n b_n H_n^(1)(kappa r) e^{i n theta}

and continuity of u and du/dr at r = R fixes
    a_n = i^n (2i / (pi R)) / [kappa J_n(kappa1 R) H_n'(kappa R) - kappa1 J_n'(kappa1 R) H_n(kappa R)],
    b_n = (a_n J_n(kappa1 R) - i^n J_n(kappa R)) / H_n(kappa R).
The volume density of the paper's formulation is psi = kappa^2 q u.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import h1vp, hankel1, jv, jvp


def coefficients(kappa: float, R: float, q0: float, nmax: int | None = None):
    k1 = kappa * math.sqrt(1.0 + q0)
    if nmax is None:
        nmax = int(k1 * R + 40)
    n = np.arange(-nmax, nmax + 1)
    den = kappa * jv(n, k1 * R) * h1vp(n, kappa * R) - k1 * jvp(n, k1 * R) * hankel1(n, kappa * R)
    a = (1j ** n) * (2j / (math.pi * R)) / den
    b = (a * jv(n, k1 * R) - (1j ** n) * jv(n, kappa * R)) / hankel1(n, kappa * R)
    return n, a, b, k1


def total_field(points: np.ndarray, kappa: float, R: float, q0: float) -> np.ndarray:
    n, a, b, k1 = coefficients(kappa, R, q0)
    r = np.hypot(points[:, 0], points[:, 1])
    th = np.arctan2(points[:, 1], points[:, 0])
    out = np.zeros(len(points), dtype=complex)
    inside = r < R
    ph = np.exp(1j * np.outer(th, n))
    ri, ro = r[inside], r[~inside]
    out[inside] = (jv(n[None, :], k1 * ri[:, None]) * a[None, :] * ph[inside]).sum(axis=1)
    uinc = np.exp(1j * kappa * points[~inside, 0])
    out[~inside] = uinc + (hankel1(n[None, :], kappa * ro[:, None]) * b[None, :] * ph[~inside]).sum(axis=1)
    return out


def interior_series_at(r: float, th: float, kappa: float, R: float, q0: float) -> complex:
    n, a, _, k1 = coefficients(kappa, R, q0)
    return complex((a * jv(n, k1 * r) * np.exp(1j * n * th)).sum())


def exterior_series_at(r: float, th: float, kappa: float, R: float, q0: float) -> complex:
    n, _, b, _ = coefficients(kappa, R, q0)
    uinc = np.exp(1j * kappa * r * math.cos(th))
    return complex(uinc + (b * hankel1(n, kappa * r) * np.exp(1j * n * th)).sum())
