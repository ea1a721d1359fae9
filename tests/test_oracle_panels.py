"""Pins of the high-order panel oracle (oracle/panels.py, Section 2 at p > 1) and of the radial
reference it is checked against (oracle/radial.py).

* Q and its pseudo-inverse: Qdag Q = I and exact recovery of any polynomial of total degree
  below p from its node values (Eqs. (eq:9)-(eq:10)); the basis has N_p = p(p+1)/2 members.
* Moments: the constant moment of a box at its own centre equals the closed-form cell integral
  (special.self_cell, a one-dimensional radial formula); a polynomial-weighted moment at an
  interior point and at a point just outside the box equals scipy's adaptive two-dimensional
  quadrature of the same integrand (split at the singular point); the near (Duffy) and far
  (Gauss-Legendre) rules agree where the library switches between them.
* The radial separation-of-variables solver equals the Bessel series of the disc (mie.py).
* The whole discretisation: for a smooth radial contrast the panel solution converges to the
  radial reference as p grows (high order: each step of p gains a factor), on a uniform tree.
* The adaptive tree: leaves tile the domain, neighbours differ by at most one level, every leaf
  resolves q to eps_grid and no leaf is in the high-frequency regime.
"""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import hankel1

from oracle import mie, panels, radial, special


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6])
def test_interpolation_recovers_polynomials_below_degree_p(p):
    assert len(panels.basis(p)) == p * (p + 1) // 2
    Q, Qd = panels.interp_matrix(p), panels.interp_pinv(p)
    assert Q.shape == (p * p, p * (p + 1) // 2)
    assert np.abs(Qd @ Q - np.eye(Q.shape[1])).max() < 1e-13
    # a polynomial of total degree < p written in monomials, not in the basis
    rng = np.random.default_rng(p)
    nd = panels.ref_nodes(p)
    coef = {(a, b): rng.standard_normal() for a in range(p) for b in range(p - a)}
    poly = lambda u, v: sum(c * u ** a * v ** b for (a, b), c in coef.items())
    c = Qd @ poly(nd[:, 0], nd[:, 1])
    pts = rng.uniform(-1, 1, (50, 2))
    assert np.allclose(panels.basis_values(p, pts[:, 0], pts[:, 1]) @ c, poly(pts[:, 0], pts[:, 1]),
                       rtol=0, atol=1e-12)


def test_cheb_is_chebyshev():
    x = np.linspace(-1, 1, 41)
    for n in range(7):
        assert np.allclose(panels.cheb(n, x), np.cos(n * np.arccos(x)), atol=1e-13)


@pytest.mark.parametrize("kappa", [10.0, 40.0])
def test_constant_self_moment_is_the_cell_integral(kappa):
    box = panels.Box(0.3, -0.2, 0.125, 3)
    m = panels.moments(np.array([[0.3, -0.2]]), box, 3, kappa)[0]
    ref = special.self_cell(0.25, kappa)
    assert abs(m[0] - ref) < 1e-11 * abs(ref)


def _dblquad_moment(x, box, a, b, kappa):
    """int_box G(|x - y|) T_a(u) T_b(v) dy by scipy's adaptive quadrature, split at x."""
    def f(y1, y0, part):
        r = math.hypot(y0 - x[0], y1 - x[1])
        if r == 0:
            return 0.0
        g = 0.25j * hankel1(0, kappa * r)
        w = np.cos(a * np.arccos(np.clip((y0 - box.cx) / box.beta, -1, 1))) * \
            np.cos(b * np.arccos(np.clip((y1 - box.cy) / box.beta, -1, 1)))
        v = g * w
        return v.real if part == 0 else v.imag
    xs = [box.cx - box.beta] + ([x[0]] if abs(x[0] - box.cx) < box.beta else []) + [box.cx + box.beta]
    ys = [box.cy - box.beta] + ([x[1]] if abs(x[1] - box.cy) < box.beta else []) + [box.cy + box.beta]
    tot = 0j
    for i in range(len(xs) - 1):
        for j in range(len(ys) - 1):
            for part in (0, 1):
                v, _ = integrate.dblquad(f, xs[i], xs[i + 1], ys[j], ys[j + 1], args=(part,), epsabs=1e-13,
                                         epsrel=1e-11)
                tot += v if part == 0 else 1j * v
    return tot


@pytest.mark.parametrize("x", [(0.05, -0.04), (0.13, 0.02)])
def test_weighted_moment_matches_adaptive_quadrature(x):
    # one target inside the box (off centre), one just outside its right edge
    box = panels.Box(0.0, 0.0, 0.125, 3)
    p, kappa = 4, 12.0
    m = panels.moments(np.array([x]), box, p, kappa)[0]
    for l in (2, 7):
        a, b = panels.basis(p)[l]
        ref = _dblquad_moment(x, box, a, b, kappa)
        assert abs(m[l] - ref) < 1e-9 * max(abs(ref), 1e-3 * abs(m[0])), (l, m[l], ref)


def test_near_and_far_rules_agree_at_the_switch():
    box = panels.Box(0.0, 0.0, 0.125, 3)
    x = np.array([[0.25, 0.03]])          # a half-width from the box
    for kappa in (10.0, 40.0):
        far = panels._far_moments(x, box, 4, kappa)[0]
        near = panels._near_moments(x[0], box, 4, kappa)
        assert np.abs(far - near).max() < 1e-8 * np.abs(near).max()


def test_radial_solver_is_the_disc_bessel_series():
    rng = np.random.default_rng(1)
    pts = rng.uniform(-1, 1, (120, 2))
    kappa, R, q0 = 6.0, 0.5, 2.0
    u = radial.total_field(pts, kappa, lambda r: q0, R, q0)
    ref = mie.total_field(pts, kappa, R, q0)
    assert np.linalg.norm(u - ref) / np.linalg.norm(ref) < 1e-10


def _bump(q0, R):
    def q_r(r):
        x = np.clip(np.asarray(r, dtype=float) / R, 0, 1)
        with np.errstate(divide="ignore", over="ignore"):
            return np.where(x < 1, q0 * np.exp(1.0 - 1.0 / np.maximum(1.0 - x * x, 1e-300)), 0.0)
    return q_r


def test_panel_solution_converges_to_the_radial_reference():
    kappa, R, q0 = 6.0, 0.8, 1.0
    q_r = _bump(q0, R)
    q_fn = lambda x, y: q_r(np.hypot(x, y))
    boxes = panels.uniform_tree(4)
    errs = []
    for p in (2, 4, 6):
        A = panels.dense_A(boxes, p, kappa, q_fn)
        f = panels.rhs_planewave(boxes, p, kappa, q_fn)
        psi = np.linalg.solve(A, f)
        X = panels.all_nodes(boxes, p)
        q = q_fn(X[:, 0], X[:, 1])
        m = q > 1e-12
        ref = kappa ** 2 * q[m] * radial.total_field(X[m], kappa, lambda r: float(q_r(r)), R, q0)
        errs.append(np.linalg.norm(psi[m] - ref) / np.linalg.norm(ref))
    print("relative errors p = 2, 4, 6:", errs)
    assert errs[0] > 5 * errs[1] > 5 * 5 * errs[2]
    assert errs[2] < 5e-3


def test_adaptive_tree_is_level_restricted_and_resolves_the_contrast():
    kappa = 12.0
    q_fn = lambda x, y: 1.5 * np.exp(-60.0 * ((x - 0.3) ** 2 + (y + 0.2) ** 2))
    u_fn = lambda x, y: np.exp(1j * kappa * x)
    p, eps = 4, 1e-3
    leaves = panels.build_tree(q_fn, u_fn, p, eps, kappa, T=16.0, max_level=6)
    area = sum((2 * b.beta) ** 2 for b in leaves)
    assert abs(area - 4.0) < 1e-12
    levels = {b.level for b in leaves}
    assert len(levels) > 1                         # adaptive: refined around the bump
    for a in leaves:
        assert (kappa * a.beta) ** 2 <= 16.0
        assert a.level == 6 or panels._resolved(q_fn, a, p, eps)
        for b in leaves:
            if panels.neighbours(a, b):
                assert abs(a.level - b.level) <= 1


def test_hodlr_order_halves_the_boxes_into_rectangles():
    # the HODLR order of a uniform tree: whole boxes per leaf, and every node of the binary tree
    # (a half of its parent's index range) holds the boxes of one axis-aligned rectangle
    nside, p = 8, 2
    perm = panels.hodlr_order(nside, p)
    n2, N = p * p, nside * nside * p * p
    assert sorted(perm.tolist()) == list(range(N))
    box = perm.reshape(-1, n2) // n2
    assert (box == box[:, :1]).all()                     # a box's nodes stay together
    order = box[:, 0]
    lp = panels.hodlr_leaf(nside, p)
    assert lp == 64 and lp % n2 == 0
    size = len(order)
    while size >= 1:
        for lo in range(0, len(order), size):
            ix, iy = order[lo:lo + size] // nside, order[lo:lo + size] % nside
            area = (ix.max() - ix.min() + 1) * (iy.max() - iy.min() + 1)
            assert area == size, (size, lo)
        size //= 2 if size > 1 else 2
    assert [panels.hodlr_leaf(8, q) for q in (1, 3, 4, 5, 8)] == [64, 36, 64, 25, 64]


def test_panel_hodlr_at_full_rank_is_the_inverse():
    # the fixed-rank HODLR of the panel matrix (HODLR order, leaves of hodlr_leaf unknowns):
    # at a rank no off-diagonal block exceeds, A~ = A and its solve is the dense solve; below
    # it the approximation error falls as the rank grows
    from oracle.hodlr import HODLR
    nside, p, kappa = 8, 2, 10.0
    boxes = panels.uniform_tree(nside)
    q_fn = lambda x, y: 1.5 * np.exp(-8.0 * (x * x + (y - 0.1) ** 2))
    A = panels.dense_A(boxes, p, kappa, q_fn)
    perm = panels.hodlr_order(nside, p)
    Ah = A[np.ix_(perm, perm)]
    lp = panels.hodlr_leaf(nside, p)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(len(A)) + 1j * rng.standard_normal(len(A))
    H = HODLR(Ah, lp, rank=len(A) // 2)
    assert np.abs(H.dense() - Ah).max() <= 1e-12 * np.abs(Ah).max()
    ref = np.linalg.solve(Ah, b)
    assert np.linalg.norm(H.solve(b) - ref) <= 1e-10 * np.linalg.norm(ref)
    errs = [np.linalg.norm(HODLR(Ah, lp, rank=k).dense() - Ah) / np.linalg.norm(Ah) for k in (4, 8, 16, 32)]
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-5, errs


def test_leaf_order_of_a_uniform_tree_is_the_uniform_order():
    # on the leaves of a uniform tree the general HODLR order is the uniform one (same Morton
    # order of boxes, no padding at p = 4); on an adaptive tree every position holds a distinct
    # unknown or padding, padding only at the end, whole boxes in every leaf
    p = 4
    perm, lp = panels.hodlr_order_leaves(panels.uniform_tree(8), p)
    assert lp == panels.hodlr_leaf(8, p) == 64
    assert (perm == panels.hodlr_order(8, p)).all()
    q_fn = lambda x, y: 1.5 * np.exp(-60.0 * ((x - 0.3) ** 2 + (y + 0.2) ** 2))
    leaves = panels.build_tree(q_fn, lambda x, y: np.exp(12j * x), 3, 1e-3, 12.0, T=16.0, max_level=5)
    perm, lp = panels.hodlr_order_leaves(leaves, 3)
    N = len(leaves) * 9
    assert lp == 63 and len(perm) % lp == 0 and (len(perm) // lp) & (len(perm) // lp - 1) == 0
    assert sorted(perm[:N].tolist()) == list(range(N)) and (perm[N:] == -1).all() and len(perm) - N < len(perm) / 2
    assert all(perm[t] // 9 == perm[t - t % 9] // 9 for t in range(N))
    A = np.arange(16.0).reshape(4, 4)
    P = panels.padded(A, np.array([2, -1, 0, 3, 1, -1]))
    assert P[0, 0] == A[2, 2] and P[0, 2] == A[2, 0] and P[1, 1] == 1 and P[1, 0] == 0 and P[5, 5] == 1
