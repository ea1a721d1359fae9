"""The discretised Lippmann-Schwinger operator (oracle).

Paper, Section 1, Eqs. (eq:3), (eq:5), (eq:6) and Section 2.2, Eqs. (eq:12a), (eq:13),
at p = 1 on a uniform cell-centred grid (one node per cell, Q = Q^+ = [1]):

    V_ij = h^2 G(|x_i - x_j|)          (i != j, one-point rule for the cell integral)
    V_ii = W0(h, kappa)                (exact singular self-cell integral)
    A    = I + s kappa^2 diag(q) V,     f = -s kappa^2 q * u_inc,   u_inc = exp(i kappa d.x)

with s = -1.  The paper prints Eq. (eq:6) with a plus sign and f = -kappa^2 q u_inc;
with G = (i/4) H0^(1), which solves (Delta + kappa^2) G = -delta, Eqs. (eq:3) and (eq:5)
give psi = kappa^2 q u and psi - kappa^2 q V[psi] = kappa^2 q u_inc, i.e. s = -1.
``sign=+1`` reproduces Eq. (eq:6) literally.

Vectors are in grid order (flat index i = a*n + b, a along the first coordinate).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import fft as sfft

from .special import green, self_cell


def grid_coords(n: int, L: float) -> np.ndarray:
    """Cell centres x_ab = (-L + (a+1/2)h, -L + (b+1/2)h), flat index a*n + b."""
    h = 2.0 * L / n
    c = -L + (np.arange(n) + 0.5) * h
    a, b = np.meshgrid(c, c, indexing="ij")
    return np.stack([a.ravel(), b.ravel()], axis=1)


def dense_V(n: int, L: float, kappa: float) -> np.ndarray:
    """V by its definition: h^2 G(|x_i - x_j|) off the diagonal, W0 on it (N <= ~4096)."""
    h = 2.0 * L / n
    x = grid_coords(n, L)
    d = np.sqrt((x[:, None, 0] - x[None, :, 0]) ** 2 + (x[:, None, 1] - x[None, :, 1]) ** 2)
    np.fill_diagonal(d, 1.0)   # placeholder, overwritten below
    V = (h * h) * green(d, kappa)
    np.fill_diagonal(V, self_cell(h, kappa))
    return V


def dense_A(n: int, L: float, kappa: float, q: np.ndarray, sign: int = -1) -> np.ndarray:
    """A = I + s kappa^2 diag(q) V (Eq. (eq:13) at p = 1)."""
    V = dense_V(n, L, kappa)
    return np.eye(n * n, dtype=complex) + sign * kappa * kappa * q[:, None] * V


def offset_table(n: int, L: float, kappa: float) -> np.ndarray:
    """W[da + n-1, db + n-1] = V entry for a grid offset (da, db); W at (0,0) is W0."""
    h = 2.0 * L / n
    k = np.arange(-(n - 1), n)
    da, db = np.meshgrid(k, k, indexing="ij")
    r = h * np.sqrt(da * da + db * db).astype(float)
    r[n - 1, n - 1] = 1.0
    W = (h * h) * green(r, kappa)
    W[n - 1, n - 1] = self_cell(h, kappa)
    return W


class FFTApplyV:
    """y = V x as a 2-D discrete convolution with the offset table, zero-padded to (2n)^2.

    V is block-Toeplitz with Toeplitz blocks (V_ij depends only on a_i - a_j, b_i - b_j),
    so the product equals the dense sum up to rounding by the discrete convolution theorem.
    """

    def __init__(self, n: int, L: float, kappa: float, workers: int = -1):
        self.n = n
        self.workers = workers
        W = offset_table(n, L, kappa)
        m = 2 * n
        ker = np.zeros((m, m), dtype=complex)
        # place offset (da, db) at index (da mod m, db mod m)
        k = np.arange(-(n - 1), n) % m
        ker[np.ix_(k, k)] = W
        self.khat = sfft.fft2(ker, workers=workers)

    def __call__(self, x: np.ndarray) -> np.ndarray:
        n, m = self.n, 2 * self.n
        X = np.zeros((m, m), dtype=complex)
        X[:n, :n] = x.reshape(n, n)
        Y = sfft.ifft2(sfft.fft2(X, workers=self.workers) * self.khat, workers=self.workers)
        return Y[:n, :n].reshape(-1)


def apply_A(Vx_fn, x: np.ndarray, q: np.ndarray, kappa: float, sign: int = -1) -> np.ndarray:
    """y = x + s kappa^2 q * (V x)."""
    return x + sign * kappa * kappa * q * Vx_fn(x)


def sampled_rows_Vx(n: int, L: float, kappa: float, x: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """(V x)_i for selected rows i, each summed directly from the definition."""
    h = 2.0 * L / n
    pts = grid_coords(n, L)
    w0 = self_cell(h, kappa)
    out = np.empty(len(rows), dtype=complex)
    for t, i in enumerate(rows):
        d = np.sqrt(((pts - pts[i]) ** 2).sum(axis=1))
        d[i] = 1.0
        g = (h * h) * green(d, kappa)
        g[i] = w0
        out[t] = np.dot(g, x)
    return out


def rhs_planewave(n: int, L: float, kappa: float, q: np.ndarray, theta: float = 0.0,
                  sign: int = -1) -> np.ndarray:
    """f = -s kappa^2 q u_inc with u_inc = exp(i kappa (cos(theta) x1 + sin(theta) x2))."""
    x = grid_coords(n, L)
    uinc = np.exp(1j * kappa * (math.cos(theta) * x[:, 0] + math.sin(theta) * x[:, 1]))
    return -sign * kappa * kappa * q * uinc


def incident(n: int, L: float, kappa: float, theta: float = 0.0) -> np.ndarray:
    x = grid_coords(n, L)
    return np.exp(1j * kappa * (math.cos(theta) * x[:, 0] + math.sin(theta) * x[:, 1]))
