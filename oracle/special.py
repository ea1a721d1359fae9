"""Green's function and the singular self-cell integral (oracle).

Paper, Section 1: the 2D Helmholtz Green's function is G(x, y) = (i/4) H0^(1)(kappa |x - y|).
Paper, Section 2.2, Eq. (eq:13): matrix entries are integrals of G against the
leaf basis; with one Chebyshev node per cell (p = 1) the only basis function is
the constant 1, so V_ij is the integral of G(x_i, y) over cell j.  For the
diagonal (i = j) this integral is weakly singular and is evaluated exactly:

    W0 = int_{[-h/2,h/2]^2} (i/4) H0(kappa |y|) dy
       = 8 int_0^{pi/4} (i/4) [ R H1(kappa R)/kappa + 2i/(pi kappa^2) ] dtheta,
    R(theta) = h / (2 cos theta),

using d/dr [r H1(kappa r)] = kappa r H0(kappa r) and r H1(kappa r)/kappa -> -2i/(pi kappa^2)
as r -> 0.  The theta integral is smooth and is done with Gauss-Legendre.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import hankel1


def green(r, kappa: float):
    """G = (i/4) H0^(1)(kappa r) (Section 1)."""
    return 0.25j * hankel1(0, kappa * np.asarray(r, dtype=float))


def self_cell(h: float, kappa: float, nquad: int = 64) -> complex:
    """Exact integral of G over a square cell of side h centred at the target."""
    x, w = np.polynomial.legendre.leggauss(nquad)
    half = math.pi / 8.0
    theta = (x + 1.0) * half          # [-1, 1] -> [0, pi/4]
    weight = w * half
    R = (0.5 * h) / np.cos(theta)
    radial = R * hankel1(1, kappa * R) / kappa + 2j / (math.pi * kappa * kappa)
    return complex(8.0 * np.sum(weight * 0.25j * radial))
