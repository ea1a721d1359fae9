"""Seeded synthetic problem generators.

This module only *describes problems*: grid coordinates, contrast functions,
incidence angles and random test vectors.  It holds none of the solver's
arithmetic (no kernel entries, no right-hand side, no operator), so both the
HIP path and the independent CPU oracle can be fed from it.

Grid convention (uniform, cell-centred, one collocation point per cell):
    Omega = [-L, L]^2, n x n cells, h = 2L/n,
    x_ab = (-L + (a + 1/2) h, -L + (b + 1/2) h),  flat index i = a*n + b,
so ``a`` indexes the first coordinate and ``b`` the second.

The contrast families follow the paper's experiments (Gaussian contrast of
Experiment 2, multiple Gaussians of Experiment 7) and the constant-contrast
disc used for the Mie-series check.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def grid_points(n: int, L: float = 1.0) -> np.ndarray:
    """Cell centres of the uniform n x n grid on [-L, L]^2, shape (n*n, 2)."""
    h = 2.0 * L / n
    c = -L + (np.arange(n) + 0.5) * h
    a, b = np.meshgrid(c, c, indexing="ij")
    return np.stack([a.ravel(), b.ravel()], axis=1)


def contrast_gaussian(points: np.ndarray, amp: float = 1.5, alpha: float = 40.0) -> np.ndarray:
    """q(x) = amp * exp(-alpha |x|^2) (the paper's Gaussian contrast family)."""
    r2 = points[:, 0] ** 2 + points[:, 1] ** 2
    return amp * np.exp(-alpha * r2)


@dataclass
class Bump:
    amp: float
    sigma: float
    cx: float
    cy: float


def draw_bumps(rng: np.random.Generator, count: int | None = None) -> list[Bump]:
    """Draw Gaussian bumps: count (1..8 when not given), then per bump
    A ~ U[0.5, 2], sigma ~ U[0.05, 0.2], c ~ U[-0.7, 0.7]^2, in that order."""
    if count is None:
        count = int(rng.integers(1, 9))
    out = []
    for _ in range(count):
        amp = float(rng.uniform(0.5, 2.0))
        sigma = float(rng.uniform(0.05, 0.2))
        cx = float(rng.uniform(-0.7, 0.7))
        cy = float(rng.uniform(-0.7, 0.7))
        out.append(Bump(amp, sigma, cx, cy))
    return out


def contrast_bumps(points: np.ndarray, bumps: list[Bump]) -> np.ndarray:
    """q(x) = sum_b A_b exp(-|x - c_b|^2 / (2 sigma_b^2))."""
    q = np.zeros(points.shape[0])
    for bp in bumps:
        d2 = (points[:, 0] - bp.cx) ** 2 + (points[:, 1] - bp.cy) ** 2
        q += bp.amp * np.exp(-d2 / (2.0 * bp.sigma ** 2))
    return q


def contrast_disc(points: np.ndarray, radius: float = 0.6, q0: float = 1.0) -> np.ndarray:
    """q = q0 strictly inside the disc |x| < radius (point value at the cell centre), else 0."""
    r2 = points[:, 0] ** 2 + points[:, 1] ** 2
    return np.where(r2 < radius * radius, q0, 0.0)


def random_vector(N: int, nrhs: int = 1, seed: int = 0) -> np.ndarray:
    """Complex128 Gaussian test vector(s), shape (N,) or (N, nrhs) column-major semantics."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((N, nrhs)) + 1j * rng.standard_normal((N, nrhs))
    return v[:, 0].copy() if nrhs == 1 else np.asfortranarray(v)


@dataclass
class Problem:
    """A synthetic Lippmann-Schwinger problem on a uniform grid."""
    name: str
    n: int
    L: float
    kappa: float
    q: np.ndarray
    thetas: np.ndarray = field(default_factory=lambda: np.zeros(1))

    @property
    def N(self) -> int:
        return self.n * self.n

    @property
    def h(self) -> float:
        return 2.0 * self.L / self.n

    def points(self) -> np.ndarray:
        return grid_points(self.n, self.L)


def problem_gaussian_small() -> Problem:
    """32 x 32 grid on [-1,1]^2, kappa = 10, q = 1.5 exp(-40|x|^2), theta = 0."""
    n, L = 32, 1.0
    p = grid_points(n, L)
    return Problem("gauss32_k10", n, L, 10.0, contrast_gaussian(p, 1.5, 40.0))


def problem_bumps(n: int, kappa: float, seed: int, count: int | None = None,
                  nangles: int = 1, L: float = 1.0) -> Problem:
    """Gaussian-bump contrast on an n x n grid; nangles incidence angles 2*pi*j/nangles."""
    rng = np.random.default_rng(seed)
    bumps = draw_bumps(rng, count)
    p = grid_points(n, L)
    thetas = 2.0 * math.pi * np.arange(nangles) / nangles
    return Problem(f"bumps{n}_k{kappa:g}_s{seed}", n, L, float(kappa), contrast_bumps(p, bumps), thetas)


def problem_disc(n: int, kappa: float, radius: float = 0.6, q0: float = 1.0, L: float = 1.0) -> Problem:
    """Constant-contrast disc (Mie-series checkable)."""
    p = grid_points(n, L)
    return Problem(f"disc{n}_k{kappa:g}", n, L, float(kappa), contrast_disc(p, radius, q0))


def problem_queue(seed: int = 2, count: int = 16) -> list[Problem]:
    """Queue of independent problems: n uniform from {64, 96, 128, 192, 256},
    kappa uniform integer in [10, 60], 1..8 Gaussian bumps, one angle each."""
    rng = np.random.default_rng(seed)
    sizes = [64, 96, 128, 192, 256]
    out = []
    for j in range(count):
        n = int(sizes[int(rng.integers(0, len(sizes)))])
        kappa = float(rng.integers(10, 61))
        bumps = draw_bumps(rng)
        p = grid_points(n, 1.0)
        out.append(Problem(f"queue{j}_n{n}_k{kappa:g}", n, 1.0, kappa, contrast_bumps(p, bumps)))
    return out


def problem_learned(seed: int, n: int = 128, angles: int = 1, L: float = 1.0) -> Problem:
    """Warm-start training/evaluation problem: kappa ~ U[20, 60], 1..8 Gaussian bumps, then
    `angles` incidence angles ~ U[0, 2 pi), all drawn from default_rng(seed) in that order."""
    rng = np.random.default_rng(seed)
    kappa = float(rng.uniform(20.0, 60.0))
    bumps = draw_bumps(rng)
    thetas = rng.uniform(0.0, 2.0 * math.pi, size=angles)
    p = grid_points(n, L)
    return Problem(f"learned{n}_s{seed}", n, L, kappa, contrast_bumps(p, bumps), np.asarray(thetas))
