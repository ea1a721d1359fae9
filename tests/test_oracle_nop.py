"""Pins for oracle.nop: analytic gradients against central finite differences, the spectral
convolution against numpy's real FFT, and the loss at its minimum."""
import numpy as np
import pytest

from oracle import nop


def tiny():
    n, width, modes, layers = 8, 3, 2, 2
    rng = np.random.default_rng(7)
    params = nop.init_params(6, width, modes, layers, seed=3)
    for k in params:   # non-zero biases and a non-trivial spectral part
        if params[k].dtype == complex:
            params[k] = params[k] * 30 + 0.2j * rng.standard_normal(params[k].shape)
        elif k in ("p", "q") or k.startswith("b"):
            params[k] = 0.1 * rng.standard_normal(params[k].shape)
    X = rng.standard_normal((2, 6, n, n))
    q = rng.random((2, n, n))
    t = rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n))
    s = t + 0.5
    return params, X, q, t, s, layers, modes


def total_loss(params, X, q, t, s, layers, modes):
    O, _ = nop.forward(params, X, layers, modes)
    return nop.loss(O, q, t, s)[0]


def test_gradients_match_finite_differences():
    params, X, q, t, s, layers, modes = tiny()
    O, cache = nop.forward(params, X, layers, modes)
    L0, dO = nop.loss(O, q, t, s)
    g = nop.backward(params, cache, dO, layers, modes)
    rng = np.random.default_rng(0)
    eps = 1e-6
    for key, val in params.items():
        flat = val.reshape(-1)
        for idx in rng.choice(flat.size, size=min(4, flat.size), replace=False):
            for part in ((1.0,) if val.dtype != complex else (1.0, 1j)):
                old = flat[idx]
                flat[idx] = old + eps * part
                Lp = total_loss(params, X, q, t, s, layers, modes)
                flat[idx] = old - eps * part
                Lm = total_loss(params, X, q, t, s, layers, modes)
                flat[idx] = old
                fd = (Lp - Lm) / (2 * eps)
                an = g[key].reshape(-1)[idx]
                an = an.real if part == 1.0 else an.imag
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (key, idx, part, fd, an)


def test_spectral_identity_is_truncated_rfft():
    n, M, C = 16, 5, 2
    rng = np.random.default_rng(1)
    V = rng.standard_normal((1, C, n, n))
    R = np.zeros((C, C, 2 * M, M), dtype=complex)
    for c in range(C):
        R[c, c] = 1.0
    tw_w, tw_h = nop.twiddles(n, M)
    Y, _ = nop.spectral(V, R, tw_w, tw_h, n)
    F = np.fft.rfft2(V, axes=(2, 3))
    mask = np.zeros_like(F)
    rows = np.r_[0:M, n - M:n]
    mask[:, :, rows, :M] = 1
    ref = np.fft.irfft2(F * mask, s=(n, n), axes=(2, 3))
    assert np.max(np.abs(Y - ref)) < 1e-12


def test_loss_zero_at_exact_prediction():
    n = 8
    rng = np.random.default_rng(2)
    q = rng.random((1, n, n)) + 0.1
    Oc = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    t = q * Oc
    O = np.stack([Oc.real, Oc.imag])[None]
    L, dO = nop.loss(O, q, t, t + 1.0)
    assert L == 0.0 and np.all(dO == 0.0)


def _bump_g(n, L, A, sig, c=(0.0, 0.0)):
    h = 2.0 * L / n
    x = -L + (np.arange(n) + 0.5) * h
    x1, x2 = np.meshgrid(x, x, indexing="ij")
    return A * np.exp(-((x1 - c[0]) ** 2 + (x2 - c[1]) ** 2) / (2 * sig * sig)), x1, x2


def test_ray_phase_matches_line_integral_second_order():
    # g = sqrt(1+q) - 1 a Gaussian: the phase along d = (1, 0) is
    # kappa * A exp(-x2^2/2s^2) * s sqrt(pi/2) * (1 + erf(x1 / (s sqrt 2)))
    from scipy.special import erf
    L, kappa, A, sig = 1.0, 30.0, 0.4, 0.15
    errs = []
    for n in (32, 64):
        g, x1, x2 = _bump_g(n, L, A, sig)
        q = (1.0 + g) ** 2 - 1.0
        phi = nop.ray_phase(n, L, q.ravel(), kappa, 0.0).reshape(n, n)
        exact = kappa * A * np.exp(-x2 ** 2 / (2 * sig * sig)) * sig * np.sqrt(np.pi / 2) * (1 + erf(x1 / (sig * np.sqrt(2))))
        errs.append(np.max(np.abs(phi - exact)) / np.max(np.abs(exact)))
    assert errs[0] < 2e-2 and errs[1] < errs[0] / 3.0, errs


def test_ray_phase_symmetries_and_zero_contrast():
    n, L, kappa = 16, 1.0, 20.0
    g, _, _ = _bump_g(n, L, 0.5, 0.2, c=(0.2, -0.3))
    q = ((1.0 + g) ** 2 - 1.0)
    p0 = nop.ray_phase(n, L, q.ravel(), kappa, 0.0).reshape(n, n)
    # rotating the incidence by pi/2 is the transpose problem; by pi, the mirrored one
    p90 = nop.ray_phase(n, L, q.T.ravel(), kappa, np.pi / 2).reshape(n, n)
    p180 = nop.ray_phase(n, L, q[::-1].ravel(), kappa, np.pi).reshape(n, n)
    assert np.allclose(p90.T, p0, atol=1e-10) and np.allclose(p180[::-1], p0, atol=1e-10)
    # the phase is accumulated downstream of the bump only
    a_up, a_dn = 2, n - 3
    b = int((-0.3 + 1.0) / (2.0 / n))
    assert abs(p0[a_up, b]) < 1e-3 * abs(p0[a_dn, b])
    assert np.all(nop.ray_phase(n, L, np.zeros(n * n), kappa, 0.7) == 0.0)
    X = nop.features(n, L, np.zeros(n * n), kappa, 0.7)
    ui = np.exp(1j * kappa * (np.cos(0.7) * X[4] + np.sin(0.7) * X[5]))
    assert np.allclose(X[1] + 1j * X[2], ui, atol=1e-12)
