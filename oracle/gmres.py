"""Restarted GMRES (oracle).

Paper, Section 6 ("GMRES solver" and the Hybrid solver, Eq. (eq:hybrid)): GMRES
(Saad & Schultz) with every product computed by the operator, stopped on the
relative residual ||A psi - f|| / ||f|| <= eps_GMRES.

Plain textbook form: Arnoldi with modified Gram-Schmidt, Givens rotations on the
Hessenberg matrix, restart length m, x0 = 0 unless given.  With a preconditioner
M^{-1} the iteration is right-preconditioned (A M^{-1} y = f, x = M^{-1} y), so the
monitored quantity is the true residual of the original system; the stop is
relative to ||f||.  At every restart (and at exit) the residual is recomputed
explicitly as f - A x.
"""
from __future__ import annotations

import numpy as np


def _givens(a: complex, b: complex):
    """Rotation [c, s; -conj(s), c] mapping (a, b) to (r, 0), c real."""
    if b == 0:
        return 1.0, 0.0 + 0.0j
    if a == 0:
        return 0.0, np.conj(b) / abs(b)
    t = np.hypot(abs(a), abs(b))
    c = abs(a) / t
    s = (a / abs(a)) * np.conj(b) / t
    return c, s


def gmres(matvec, f: np.ndarray, tol: float, restart: int = 200, maxit: int = 5000,
          x0: np.ndarray | None = None, precond=None):
    """Solve A x = f.  Returns (x, iterations, history of relative residual estimates)."""
    nf = np.linalg.norm(f)
    x = np.zeros_like(f) if x0 is None else x0.astype(complex).copy()
    hist = []
    its = 0
    if nf == 0:
        return np.zeros_like(f), 0, [0.0]
    while True:
        r = f - matvec(x)
        beta = np.linalg.norm(r)
        hist.append(beta / nf)
        if beta / nf <= tol or its >= maxit:
            break
        m = restart
        Q = [r / beta]
        H = np.zeros((m + 1, m), dtype=complex)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=complex)
        g = np.zeros(m + 1, dtype=complex)
        g[0] = beta
        k = 0
        for j in range(m):
            z = precond(Q[j]) if precond is not None else Q[j]
            w = matvec(z)
            for i in range(j + 1):                     # modified Gram-Schmidt
                H[i, j] = np.vdot(Q[i], w)
                w = w - H[i, j] * Q[i]
            H[j + 1, j] = np.linalg.norm(w)
            for i in range(j):                         # previous rotations
                hi, hi1 = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * hi + sn[i] * hi1
                H[i + 1, j] = -np.conj(sn[i]) * hi + cs[i] * hi1
            c, s = _givens(H[j, j], H[j + 1, j])
            cs[j], sn[j] = c, s
            H[j, j] = c * H[j, j] + s * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(s) * g[j]
            g[j] = c * g[j]
            its += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / nf)
            hnext = np.linalg.norm(w)
            if abs(g[j + 1]) / nf <= tol or its >= maxit or hnext == 0:
                break
            Q.append(w / hnext)
        y = np.zeros(k, dtype=complex)                 # back substitution
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
        dx = np.zeros_like(f)
        for i in range(k):
            dx = dx + y[i] * Q[i]
        x = x + (precond(dx) if precond is not None else dx)
    return x, its, hist
