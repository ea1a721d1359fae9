"""Off-grid evaluation of the volume potential and the error function E(x) (oracle).

Test infrastructure: only tests/ and the bench's CPU leg use this module.

Paper, Section 6 (the paragraph before Section 6.1): the scattered field is u_scat = V[psi],
computed from the discrete density on the same grid; Section 6.2, Eq. (eq:error): the error
function E(x) is the residual of the continuous equation at any x in the domain, with the
density interpolated by the leaf basis (Eq. (eq:7)).  At p = 1 that basis is the constant 1 on
each cell, so for any point x

    (V psi)(x) = sum_j psi_j int_{cell j} G(|x - y|) dy,        G(r) = (i/4) H0^(1)(kappa r),

and, with the sign s of A = I + s kappa^2 q V (reading R1) and f(x) = -s kappa^2 q(x) u_inc(x),

    E(x) = | psi(x) + s kappa^2 q(x) (V psi)(x) - f(x) | / kappa^2,

psi(x) being the value of the cell that contains x (zero outside the grid) and q(x) the contrast
at x itself, so that f(x) does not depend on the grid.

The cell integrals are done with scipy's adaptive two-dimensional quadrature wherever the
integrand is singular or nearly so (cells within two cells of x; a cell that contains x is split
at x into rectangles having the singular point as a corner) and with a 12 x 12 tensor
Gauss-Legendre rule (numpy's nodes) on cells farther away, where the integrand is smooth.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate
from scipy.special import hankel1


def _g_re(y1, y0, x, kappa):
    r = math.hypot(y0 - x[0], y1 - x[1])
    return -0.25 * float(hankel1(0, kappa * r).imag) if r > 0 else 0.0


def _g_im(y1, y0, x, kappa):
    r = math.hypot(y0 - x[0], y1 - x[1])
    return 0.25 * float(hankel1(0, kappa * r).real) if r > 0 else 0.0


def rect_integral_adaptive(x, a0, a1, b0, b1, kappa) -> complex:
    """int over [a0,a1] x [b0,b1] of G(|x - y|) dy by adaptive quadrature; the rectangle is split
    at x where x lies inside it, so that the log singularity sits at a corner."""
    xs = [a0] + ([x[0]] if a0 < x[0] < a1 else []) + [a1]
    ys = [b0] + ([x[1]] if b0 < x[1] < b1 else []) + [b1]
    tot = 0j
    for i in range(len(xs) - 1):
        for j in range(len(ys) - 1):
            opts = dict(epsabs=1e-14, epsrel=1e-12)
            re, _ = integrate.dblquad(_g_re, xs[i], xs[i + 1], ys[j], ys[j + 1], args=(x, kappa), **opts)
            im, _ = integrate.dblquad(_g_im, xs[i], xs[i + 1], ys[j], ys[j + 1], args=(x, kappa), **opts)
            tot += re + 1j * im
    return tot


def rect_integral_gauss(x, a0, a1, b0, b1, kappa, npts: int = 12) -> complex:
    """Tensor Gauss-Legendre rule for a rectangle away from x (smooth integrand)."""
    t, w = np.polynomial.legendre.leggauss(npts)
    ya = 0.5 * (a1 - a0) * t + 0.5 * (a1 + a0)
    yb = 0.5 * (b1 - b0) * t + 0.5 * (b1 + b0)
    wa = 0.5 * (a1 - a0) * w
    wb = 0.5 * (b1 - b0) * w
    Y0, Y1 = np.meshgrid(ya, yb, indexing="ij")
    r = np.hypot(Y0 - x[0], Y1 - x[1])
    return complex(np.sum(np.outer(wa, wb) * 0.25j * hankel1(0, kappa * r)))


def cell_bounds(a, b, x0, y0, h):
    """cell (a, b) of the grid with cell centres (x0 + a h, y0 + b h)"""
    return x0 + (a - 0.5) * h, x0 + (a + 0.5) * h, y0 + (b - 0.5) * h, y0 + (b + 0.5) * h


def cell_integral(x, a, b, x0, y0, h, kappa) -> complex:
    """int_{cell (a, b)} G(|x - y|) dy for any point x"""
    a0, a1, b0, b1 = cell_bounds(a, b, x0, y0, h)
    # distance from x to the cell, in units of h
    dx = max(a0 - x[0], 0.0, x[0] - a1)
    dy = max(b0 - x[1], 0.0, x[1] - b1)
    if math.hypot(dx, dy) < 2.0 * h:
        return rect_integral_adaptive(x, a0, a1, b0, b1, kappa)
    return rect_integral_gauss(x, a0, a1, b0, b1, kappa)


def field(targets, n, x0, y0, h, kappa, psi_grid) -> np.ndarray:
    """(V psi)(x_t) for every target; psi_grid[a*n + b] is the density of cell (a, b)."""
    out = np.zeros(len(targets), dtype=complex)
    for t, x in enumerate(np.asarray(targets, dtype=float)):
        acc = 0j
        for a in range(n):
            for b in range(n):
                if psi_grid[a * n + b] != 0:   # cells without density contribute nothing
                    acc += cell_integral(x, a, b, x0, y0, h, kappa) * psi_grid[a * n + b]
        out[t] = acc
    return out


def containing_cell(x, n, x0, y0, h):
    a = math.floor((x[0] - x0) / h + 0.5)
    b = math.floor((x[1] - y0) / h + 0.5)
    return (a, b) if 0 <= a < n and 0 <= b < n else None


def error_function(targets, q_t, theta, n, x0, y0, h, kappa, psi_grid, sign: int = -1) -> np.ndarray:
    """E(x_t) of Eq. (eq:error) at p = 1 (see the module docstring)."""
    u = field(targets, n, x0, y0, h, kappa, psi_grid)
    out = np.zeros(len(targets))
    for t, x in enumerate(np.asarray(targets, dtype=float)):
        c = containing_cell(x, n, x0, y0, h)
        psi_x = psi_grid[c[0] * n + c[1]] if c is not None else 0.0
        uinc = np.exp(1j * kappa * (math.cos(theta) * x[0] + math.sin(theta) * x[1]))
        f = -sign * kappa * kappa * q_t[t] * uinc
        out[t] = abs(psi_x + sign * kappa * kappa * q_t[t] * u[t] - f) / (kappa * kappa)
    return out
