"""Neural-operator warm start: reference forward and backward in FP64 (oracle).

Not part of the paper: the learned GMRES warm start is an extension.  This module is
the plain definition the GPU kernels are checked against; every operation is written
out with numpy (no autograd), and its gradients are pinned by central finite differences
in the tests.

Network (FNO-style, all maps on an n x n image, channels first):

    V0   = P X + p                                   lift, X has 6 input channels
    Z_l  = SC_l(V_{l-1}) + W_l V_{l-1} + b_l         l = 1..L
    V_l  = gelu(Z_l) for l < L,  V_L = Z_L
    O    = Q V_L + q                                 2 output channels (Re, Im)

Spectral convolution with M modes per axis (kh in {0..M-1} U {n-M..n-1}, kw in {0..M-1}):

    A1[c,h,kw] = sum_w V[c,h,w] e^{-2 pi i kw w / n}
    A2[c,j,kw] = sum_h A1[c,h,kw] e^{-2 pi i f(j) h / n},     f(j) = j (j < M) else n - 2M + j
    S [o,j,kw] = sum_c A2[c,j,kw] R[c,o,j,kw]
    B1[o,h,kw] = sum_j S[o,j,kw] e^{+2 pi i f(j) h / n}
    Y [o,h,w]  = (1/n^2) sum_kw c_kw Re(B1[o,h,kw] e^{+2 pi i kw w / n}),  c_0 = 1, c_kw = 2

Warm start (demodulated by a straight-ray WKB phase, so that the network only predicts a
complex envelope):  psi0 = b (1 + Oc),  Oc = O_re + i O_im,  b = f exp(i phi),

    phi(x) = kappa h sum_{k=0}^{2n-1} g(x - (k + 1/2) h d),   g = sqrt(max(1 + q, 0)) - 1,

the midpoint rule along the incoming ray of the phase the local wavenumber kappa sqrt(1 + q)
adds to the incident wave, with g bilinearly interpolated between cell centres and zero
outside them.  Loss per sample (relative error of psi0 against psi):
L = |w*Oc - t|^2 / |s|^2 with w = b/kappa^2, t = (psi - b)/kappa^2, s = psi/kappa^2, averaged over
the batch.  gelu(x) = x Phi(x) (exact, erf form).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def twiddles(n: int, M: int):
    w = np.arange(n)
    kw = np.arange(M)
    tw_w = np.exp(-2j * np.pi * np.outer(w, kw) / n)          # [w, kw]
    f = np.concatenate([np.arange(M), n - M + np.arange(M)])
    tw_h = np.exp(-2j * np.pi * np.outer(w, f) / n)           # [h, j]
    return tw_w, tw_h


def init_params(n_in: int, width: int, modes: int, layers: int, n_out: int = 2, seed: int = 0) -> dict:
    rng = np.random.default_rng(seed)
    p = {"P": rng.standard_normal((width, n_in)) / math.sqrt(n_in), "p": np.zeros(width)}
    for l in range(layers):
        s = 1.0 / (width * width)
        p[f"R{l}"] = s * (rng.random((width, width, 2 * modes, modes)) + 1j * rng.random((width, width, 2 * modes, modes)))
        p[f"W{l}"] = rng.standard_normal((width, width)) / math.sqrt(width)
        p[f"b{l}"] = np.zeros(width)
    p["Q"] = rng.standard_normal((n_out, width)) / math.sqrt(width) * 0.1
    p["q"] = np.zeros(n_out)
    return p


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def spectral(V, R, tw_w, tw_h, n):
    """V: [B, C, n, n] real -> Y [B, O, n, n]; also returns intermediates for the adjoint."""
    M = tw_w.shape[1]
    A1 = np.einsum("bchw,wk->bchk", V, tw_w)
    A2 = np.einsum("bchk,hj->bcjk", A1, tw_h)
    S = np.einsum("bcjk,cojk->bojk", A2, R)
    B1 = np.einsum("bojk,hj->bohk", S, np.conj(tw_h))
    ck = np.full(M, 2.0)
    ck[0] = 1.0
    Y = np.einsum("bohk,wk,k->bohw", B1, np.conj(tw_w), ck).real / (n * n)
    return Y, A2


def spectral_adjoint(dY, A2, R, tw_w, tw_h, n):
    """Gradients of sum(dY * Y) w.r.t. V (real) and R (as d/dRe + i d/dIm)."""
    M = tw_w.shape[1]
    ck = np.full(M, 2.0)
    ck[0] = 1.0
    gB1 = np.einsum("bohw,wk,k->bohk", dY, tw_w, ck) / (n * n)
    gS = np.einsum("bohk,hj->bojk", gB1, tw_h)
    gA2 = np.einsum("bojk,cojk->bcjk", gS, np.conj(R))
    gR = np.einsum("bcjk,bojk->cojk", np.conj(A2), gS)
    gA1 = np.einsum("bcjk,hj->bchk", gA2, np.conj(tw_h))
    dV = np.einsum("bchk,wk->bchw", gA1, np.conj(tw_w)).real
    return dV, gR


def pointwise(W, b, V):
    return np.einsum("oc,bchw->bohw", W, V) + b[None, :, None, None]


def forward(params: dict, X: np.ndarray, layers: int, modes: int):
    n = X.shape[-1]
    tw_w, tw_h = twiddles(n, modes)
    cache = {"X": X}
    V = pointwise(params["P"], params["p"], X)
    cache["V0"] = V
    for l in range(layers):
        Y, A2 = spectral(V, params[f"R{l}"], tw_w, tw_h, n)
        Z = Y + pointwise(params[f"W{l}"], params[f"b{l}"], V)
        cache[f"A2_{l}"] = A2
        cache[f"Z{l}"] = Z
        V = gelu(Z) if l < layers - 1 else Z
        cache[f"V{l + 1}"] = V
    O = pointwise(params["Q"], params["q"], V)
    return O, cache


def loss(O, w, t, s):
    """O: [B, 2, n, n]; w, t, s: [B, n, n] complex (w may be real)."""
    Oc = O[:, 0] + 1j * O[:, 1]
    r = w * Oc - t
    den = np.sum(np.abs(s) ** 2, axis=(1, 2))
    L = np.mean(np.sum(np.abs(r) ** 2, axis=(1, 2)) / den)
    B = O.shape[0]
    g = 2.0 * np.conj(w) * r / den[:, None, None] / B     # dL/dRe(Oc) + i dL/dIm(Oc)
    dO = np.stack([g.real, g.imag], axis=1)
    return L, dO


def backward(params: dict, cache: dict, dO: np.ndarray, layers: int, modes: int) -> dict:
    X = cache["X"]
    n = X.shape[-1]
    tw_w, tw_h = twiddles(n, modes)
    g = {}
    V = cache[f"V{layers}"]
    g["Q"] = np.einsum("bkhw,bchw->kc", dO, V)
    g["q"] = dO.sum(axis=(0, 2, 3))
    dV = np.einsum("kc,bkhw->bchw", params["Q"], dO)
    for l in range(layers - 1, -1, -1):
        Z = cache[f"Z{l}"]
        dZ = dV * gelu_grad(Z) if l < layers - 1 else dV
        Vin = cache[f"V{l}"]
        g[f"W{l}"] = np.einsum("bohw,bchw->oc", dZ, Vin)
        g[f"b{l}"] = dZ.sum(axis=(0, 2, 3))
        dVs, gR = spectral_adjoint(dZ, cache[f"A2_{l}"], params[f"R{l}"], tw_w, tw_h, n)
        g[f"R{l}"] = gR
        dV = np.einsum("oc,bohw->bchw", params[f"W{l}"], dZ) + dVs
    g["P"] = np.einsum("bohw,bihw->oi", dV, X)
    g["p"] = dV.sum(axis=(0, 2, 3))
    return g


def bilinear_zero(grid: np.ndarray, u: float, v: float) -> float:
    """Bilinear interpolation at fractional index (u, v) of an n x n grid, zero outside it."""
    n = grid.shape[0]
    i0, j0 = math.floor(u), math.floor(v)
    fu, fv = u - i0, v - j0
    val = 0.0
    for di, wi in ((0, 1.0 - fu), (1, fu)):
        for dj, wj in ((0, 1.0 - fv), (1, fv)):
            i, j = i0 + di, j0 + dj
            if 0 <= i < n and 0 <= j < n:
                val += wi * wj * grid[i, j]
    return val


def ray_phase(n: int, L: float, q: np.ndarray, kappa: float, theta: float) -> np.ndarray:
    """phi at every cell centre (grid order), by the midpoint sum written above (slow: small n)."""
    h = 2.0 * L / n
    g = np.sqrt(np.maximum(1.0 + q.reshape(n, n), 0.0)) - 1.0
    d = (math.cos(theta), math.sin(theta))
    phi = np.zeros((n, n))
    for a in range(n):
        for b in range(n):
            x1, x2 = -L + (a + 0.5) * h, -L + (b + 0.5) * h
            acc = 0.0
            for k in range(2 * n):
                t = (k + 0.5) * h
                acc += bilinear_zero(g, (x1 - t * d[0] + L) / h - 0.5, (x2 - t * d[1] + L) / h - 0.5)
            phi[a, b] = kappa * h * acc
    return phi.ravel()


def features(n: int, L: float, q: np.ndarray, kappa: float, theta: float, phi: np.ndarray | None = None) -> np.ndarray:
    """Input channels: q, cos and sin of the WKB phase kappa d.x + phi, kappa/60, x1, x2
    (grid order, image [a][b])."""
    h = 2.0 * L / n
    c = -L + (np.arange(n) + 0.5) * h
    x1, x2 = np.meshgrid(c, c, indexing="ij")
    if phi is None:
        phi = ray_phase(n, L, q, kappa, theta)
    ph = kappa * (math.cos(theta) * x1 + math.sin(theta) * x2) + phi.reshape(n, n)
    return np.stack([q.reshape(n, n), np.cos(ph), np.sin(ph), np.full((n, n), kappa / 60.0), x1, x2])


def warm_start(f: np.ndarray, phi: np.ndarray, O: np.ndarray) -> np.ndarray:
    """psi0 = f exp(i phi) (1 + O_re + i O_im) for one sample, O: [2, n, n]."""
    return f * np.exp(1j * phi) * (1.0 + O[0].ravel() + 1j * O[1].ravel())
