"""High-order leaf panels (oracle): the discretisation of Section 2 at p > 1.

Test infrastructure: only tests/ use this module.

Section 2.2, Eqs. (eq:7)-(eq:13).  On each leaf box B (centre alpha, half-width beta) the density
is represented by the N_p = p(p+1)/2 Chebyshev polynomials of total degree below p,
b_l(u, v) = T_a(u) T_b(v) with a + b < p, on the box scaled to [-1, 1]^2 (Eq. (eq:7)).  The
unknowns are the values at the p x p tensor Chebyshev nodes of every leaf; the coefficients
follow from them through the pseudo-inverse of the interpolation matrix Q (Eqs. (eq:9)-(eq:10)),
and the entries of the discrete operator are (Eq. (eq:13), with the sign s of reading R1)

    A_ij = delta_ij + s kappa^2 q(x_i) sum_l Qdag[l, j'] M_l(x_i, B(j)),
    M_l(x, B) = int_B G(|x - y|) b_l((y - alpha) / beta) dy,    G(r) = (i/4) H0^(1)(kappa r).

Readings (where Section 2 leaves the choice open): the nodes are Chebyshev points of the first
kind (interior, so neighbouring leaves share no node); the node of index i * p + j has the
coordinates (alpha_1 + beta x_i, alpha_2 + beta x_j) with x ascending; the basis is ordered by
total degree, then by the first index.

The moments M_l are computed directly (Section 2.3 tabulates the same numbers): boxes at least a
half-width away from the target by a tensor Gauss-Legendre rule (the integrand is smooth there);
nearer boxes, the box containing the target included, by splitting the box into the signed
triangles with apex at the target and mapping each to the unit square (Duffy: the logarithmic
singularity at the apex becomes a smooth integrand), with a fixed Gauss rule along the ray and
scipy's adaptive vector quadrature across it.  Moments are cached by the target's position
relative to the box (rounded to 1e-12 of the half-width), the half-width and kappa: on a uniform
or level-restricted tree the same few configurations recur, as Section 2.3 observes.

The adaptive tree of Section 2.1: a box is split while q or the incident field is not resolved
(the p-th order Chebyshev interpolant on the box, evaluated at the nodes of its four children,
differs from the function there by more than eps_grid relative to the largest value), or while
it lies in the high-frequency regime ((kappa w)^2 > T, Section 3, w the half-width); then boxes
are split until neighbours (boxes sharing a boundary segment) differ by at most one level.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate
from scipy.special import hankel1


# ---------------------------------------------------------------------------------------------
# Chebyshev basis, interpolation matrix (Eqs. (eq:7), (eq:9), (eq:9b), (eq:10))
# ---------------------------------------------------------------------------------------------
def cheb_nodes(p: int) -> np.ndarray:
    """First-kind Chebyshev points on [-1, 1], ascending."""
    k = np.arange(p)
    return np.sort(np.cos((2 * k + 1) * math.pi / (2 * p)))


def basis(p: int) -> list[tuple[int, int]]:
    """Index pairs (a, b), a + b < p: the N_p = p(p+1)/2 polynomials T_a(u) T_b(v)."""
    return [(a, d - a) for d in range(p) for a in range(d + 1)]


def cheb(n: int, x: np.ndarray) -> np.ndarray:
    """T_n(x) by the three-term recurrence (any real x)."""
    x = np.asarray(x, dtype=float)
    t0, t1 = np.ones_like(x), x
    if n == 0:
        return t0
    for _ in range(n - 1):
        t0, t1 = t1, 2 * x * t1 - t0
    return t1


def basis_values(p: int, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """b_l(u, v) for every l: array (len(u), N_p)."""
    u = np.asarray(u, dtype=float)
    v = np.asarray(v, dtype=float)
    Tu = [cheb(a, u) for a in range(p)]
    Tv = [cheb(b, v) for b in range(p)]
    return np.stack([Tu[a] * Tv[b] for a, b in basis(p)], axis=-1)


def ref_nodes(p: int) -> np.ndarray:
    """The p^2 tensor nodes on [-1, 1]^2, node i * p + j = (x_i, x_j)."""
    x = cheb_nodes(p)
    U, V = np.meshgrid(x, x, indexing="ij")
    return np.stack([U.ravel(), V.ravel()], axis=1)


def interp_matrix(p: int) -> np.ndarray:
    """Q (p^2 x N_p): Q[i, l] = b_l(node i) (Eq. (eq:9b))."""
    nd = ref_nodes(p)
    return basis_values(p, nd[:, 0], nd[:, 1])


def interp_pinv(p: int) -> np.ndarray:
    """Qdag = pseudo-inverse of Q (Eq. (eq:10))."""
    return np.linalg.pinv(interp_matrix(p))


# ---------------------------------------------------------------------------------------------
# Boxes and trees (Section 2.1)
# ---------------------------------------------------------------------------------------------
class Box:
    """A square box: centre (cx, cy), half-width beta, tree level."""

    __slots__ = ("cx", "cy", "beta", "level")

    def __init__(self, cx: float, cy: float, beta: float, level: int):
        self.cx, self.cy, self.beta, self.level = float(cx), float(cy), float(beta), int(level)

    def children(self) -> list["Box"]:
        h = self.beta / 2
        return [Box(self.cx + sx * h, self.cy + sy * h, h, self.level + 1) for sx in (-1, 1) for sy in (-1, 1)]

    def nodes(self, p: int) -> np.ndarray:
        return np.array([self.cx, self.cy]) + self.beta * ref_nodes(p)

    def __repr__(self):
        return f"Box({self.cx}, {self.cy}, {self.beta}, {self.level})"


def uniform_tree(nside: int, L: float = 1.0) -> list[Box]:
    """The nside x nside leaves of [-L, L]^2 (row-major in the first coordinate)."""
    lvl = int(round(math.log2(nside)))
    b = L / nside
    c = -L + (2 * np.arange(nside) + 1) * b
    return [Box(x, y, b, lvl) for x in c for y in c]


def _resolved(fn, box: Box, p: int, eps: float) -> bool:
    """The p-th order interpolant of fn on box, evaluated at the nodes of the four children,
    agrees with fn there to eps relative to the largest value (Section 2.1)."""
    nd = box.nodes(p)
    vals = fn(nd[:, 0], nd[:, 1])
    coef = interp_pinv(p) @ vals
    pts = np.concatenate([ch.nodes(p) for ch in box.children()])
    u = (pts[:, 0] - box.cx) / box.beta
    v = (pts[:, 1] - box.cy) / box.beta
    approx = basis_values(p, u, v) @ coef
    exact = fn(pts[:, 0], pts[:, 1])
    scale = max(np.max(np.abs(exact)), np.max(np.abs(vals)), 1e-300)
    return float(np.max(np.abs(approx - exact))) <= eps * scale


def neighbours(a: Box, b: Box) -> bool:
    """a and b share a boundary segment of positive length."""
    dx = abs(a.cx - b.cx)
    dy = abs(a.cy - b.cy)
    s = a.beta + b.beta
    tol = 1e-12 * s
    touch_x = abs(dx - s) <= tol and dy < s - tol
    touch_y = abs(dy - s) <= tol and dx < s - tol
    return touch_x or touch_y


def build_tree(q_fn, uinc_fn, p: int, eps_grid: float, kappa: float, T: float = 16.0, L: float = 1.0,
               max_level: int = 6, min_level: int = 1) -> list[Box]:
    """Adaptive, level-restricted quadtree on [-L, L]^2 (Section 2.1).  q_fn, uinc_fn take
    coordinate arrays (x, y) and return values."""
    root = Box(0.0, 0.0, L, 0)
    leaves = []
    stack = [root]
    while stack:
        b = stack.pop()
        split = b.level < min_level
        if not split and b.level < max_level:
            hf = (kappa * b.beta) ** 2 > T
            split = hf or not _resolved(q_fn, b, p, eps_grid) or not _resolved(uinc_fn, b, p, eps_grid)
        if split and b.level < max_level:
            stack.extend(b.children())
        else:
            leaves.append(b)
    # level restriction: split any leaf with a neighbour more than one level finer
    changed = True
    while changed:
        changed = False
        out = []
        for b in leaves:
            if any(neighbours(b, o) and o.level > b.level + 1 for o in leaves):
                out.extend(b.children())
                changed = True
            else:
                out.append(b)
        leaves = out
    return leaves


# ---------------------------------------------------------------------------------------------
# Moments M_l(x, B) (Section 2.3)
# ---------------------------------------------------------------------------------------------
def green(r, kappa: float):
    return 0.25j * hankel1(0, kappa * np.asarray(r))


_GL_RAY = 48
_cache: dict = {}


def _gauss01(n: int):
    t, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (t + 1), 0.5 * w


def _far_moments(x: np.ndarray, box: Box, p: int, kappa: float) -> np.ndarray:
    """Tensor Gauss-Legendre rule, for targets x (m x 2) at least a half-width from the box."""
    n = max(16, int(math.ceil(2.0 * kappa * box.beta)) + 12)
    t, w = np.polynomial.legendre.leggauss(n)
    U, V = np.meshgrid(t, t, indexing="ij")
    W = np.outer(w, w).ravel() * box.beta ** 2
    Bv = basis_values(p, U.ravel(), V.ravel()) * W[:, None]          # (n^2, N_p)
    y = np.stack([box.cx + box.beta * U.ravel(), box.cy + box.beta * V.ravel()], axis=1)
    r = np.hypot(x[:, None, 0] - y[None, :, 0], x[:, None, 1] - y[None, :, 1])
    return green(r, kappa) @ Bv                                         # (m, N_p)


def _triangle_moments(x: np.ndarray, a: np.ndarray, b: np.ndarray, box: Box, p: int, kappa: float) -> np.ndarray:
    """int over the triangle (x, a, b), with its orientation sign, of G(|x - y|) b_l(y^): the
    point y = x + s (a + t (b - a) - x), dy = s |J| ds dt with J = cross(a - x, b - a); s = u^2."""
    J = (a[0] - x[0]) * (b[1] - a[1]) - (a[1] - x[1]) * (b[0] - a[0])
    if abs(J) <= 1e-15 * box.beta ** 2:
        return np.zeros(len(basis(p)), dtype=complex)
    u, w = _gauss01(_GL_RAY)
    s = u * u
    ws = 2.0 * u * u * u * w           # s ds = 2 u^3 du
    Np = len(basis(p))

    def f(t):
        e = a + t * (b - a) - x
        y0 = x[0] + s * e[0]
        y1 = x[1] + s * e[1]
        r = s * math.hypot(e[0], e[1])
        g = green(r, kappa) * ws
        Bv = basis_values(p, (y0 - box.cx) / box.beta, (y1 - box.cy) / box.beta)
        val = g @ Bv
        return np.concatenate([val.real, val.imag])

    # the foot of the perpendicular from x on the edge line, where the integrand varies fastest
    d = b - a
    t0 = float(np.dot(x - a, d) / np.dot(d, d))
    pts = [t0] if 0.0 < t0 < 1.0 else None
    res, _ = integrate.quad_vec(f, 0.0, 1.0, epsabs=1e-14, epsrel=1e-12, points=pts)
    return J * (res[:Np] + 1j * res[Np:])


def _near_moments(x: np.ndarray, box: Box, p: int, kappa: float) -> np.ndarray:
    c = [np.array([box.cx - box.beta, box.cy - box.beta]), np.array([box.cx + box.beta, box.cy - box.beta]),
         np.array([box.cx + box.beta, box.cy + box.beta]), np.array([box.cx - box.beta, box.cy + box.beta])]
    return sum(_triangle_moments(x, c[k], c[(k + 1) % 4], box, p, kappa) for k in range(4))


def box_distance(x: np.ndarray, box: Box) -> np.ndarray:
    """Distance from the points x (m x 2) to the box (0 inside)."""
    dx = np.maximum(np.abs(x[:, 0] - box.cx) - box.beta, 0.0)
    dy = np.maximum(np.abs(x[:, 1] - box.cy) - box.beta, 0.0)
    return np.hypot(dx, dy)


def moments(x: np.ndarray, box: Box, p: int, kappa: float) -> np.ndarray:
    """M_l(x_i, box) for the targets x (m x 2): array (m, N_p)."""
    x = np.atleast_2d(np.asarray(x, dtype=float))
    out = np.empty((len(x), len(basis(p))), dtype=complex)
    far = box_distance(x, box) >= box.beta
    if far.any():
        out[far] = _far_moments(x[far], box, p, kappa)
    for i in np.nonzero(~far)[0]:
        rel = (x[i] - np.array([box.cx, box.cy])) / box.beta
        key = (p, round(float(kappa), 12), round(box.beta, 14), round(rel[0], 12), round(rel[1], 12))
        if key not in _cache:
            _cache[key] = _near_moments(x[i], box, p, kappa)
        out[i] = _cache[key]
    return out


# ---------------------------------------------------------------------------------------------
# The discrete operator (Eqs. (eq:11c), (eq:12a), (eq:13)) and right-hand side
# ---------------------------------------------------------------------------------------------
def all_nodes(boxes: list[Box], p: int) -> np.ndarray:
    """Every unknown's point, box by box (node index i * p + j inside a box)."""
    return np.concatenate([b.nodes(p) for b in boxes])


def dense_V(boxes: list[Box], p: int, kappa: float) -> np.ndarray:
    """V_ij = sum_l Qdag[l, j'] M_l(x_i, B(j)): (V psi)(x_i) for the panel density."""
    X = all_nodes(boxes, p)
    Qd = interp_pinv(p)            # (N_p, p^2)
    n2 = p * p
    V = np.empty((len(X), len(boxes) * n2), dtype=complex)
    for k, b in enumerate(boxes):
        V[:, k * n2:(k + 1) * n2] = moments(X, b, p, kappa) @ Qd
    return V


def dense_A(boxes: list[Box], p: int, kappa: float, q_fn, sign: int = -1) -> np.ndarray:
    X = all_nodes(boxes, p)
    q = q_fn(X[:, 0], X[:, 1])
    return np.eye(len(X)) + sign * kappa ** 2 * q[:, None] * dense_V(boxes, p, kappa)


def rhs_planewave(boxes: list[Box], p: int, kappa: float, q_fn, theta: float = 0.0, sign: int = -1) -> np.ndarray:
    """f = -s kappa^2 q u_inc at every node, u_inc = exp(i kappa (cos theta, sin theta) . x)."""
    X = all_nodes(boxes, p)
    q = q_fn(X[:, 0], X[:, 1])
    u = np.exp(1j * kappa * (math.cos(theta) * X[:, 0] + math.sin(theta) * X[:, 1]))
    return -sign * kappa ** 2 * q * u


def interpolate(boxes: list[Box], p: int, psi: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """psi^B(x) (Eq. (eq:11)) at points pts (m x 2), each in the first leaf that contains it."""
    pts = np.atleast_2d(pts)
    Qd = interp_pinv(p)
    out = np.zeros(len(pts), dtype=complex)
    done = np.zeros(len(pts), dtype=bool)
    n2 = p * p
    for k, b in enumerate(boxes):
        inside = (np.abs(pts[:, 0] - b.cx) <= b.beta) & (np.abs(pts[:, 1] - b.cy) <= b.beta) & ~done
        done |= inside
        if inside.any():
            c = Qd @ psi[k * n2:(k + 1) * n2]
            Bv = basis_values(p, (pts[inside, 0] - b.cx) / b.beta, (pts[inside, 1] - b.cy) / b.beta)
            out[inside] = Bv @ c
    return out


# ---------------------------------------------------------------------------------------------
# HODLR order of a uniform tree's unknowns (Section 6 applied to the panel system)
# ---------------------------------------------------------------------------------------------
def hodlr_order(nside: int, p: int) -> np.ndarray:
    """perm[t] = box-major index of the unknown at HODLR position t: boxes in Morton order (as
    the cell-centred grid's leaves), the p^2 nodes of a box in their own order."""
    from .hodlr import morton_permutation
    order = morton_permutation(nside, 1)
    n2 = p * p
    return (order[:, None] * n2 + np.arange(n2)[None, :]).ravel()


def hodlr_leaf(nside: int, p: int) -> int:
    """Leaf size of the panel HODLR: 4^j whole boxes, the largest such group of at most 64
    unknowns (a reading: leaves of about the cell-centred grid's size)."""
    n2 = p * p
    lb = 1
    while lb * 4 * n2 <= 64 and lb * 4 <= nside * nside:
        lb *= 4
    return lb * n2



def hodlr_order_leaves(boxes: list[Box], p: int):
    """HODLR order of the unknowns on the leaves of any tree: boxes sorted (stably) by the Morton
    code of their lower-left corner on the grid of the smallest box width (y bits at even, x bits
    at odd positions), nodes inside a box in their own order, leaves of floor(64 / p^2) whole
    boxes, and padding positions (-1: an identity row and column) after the last box up to a
    power-of-two number of leaves.  Returns (perm, lp): perm[t] = index of the unknown at position
    t in the given box order, or -1."""
    n2 = p * p
    xmin = min(b.cx - b.beta for b in boxes)
    ymin = min(b.cy - b.beta for b in boxes)
    hmin = min(b.beta for b in boxes)

    def code(b):
        ix = int(math.floor((b.cx - b.beta - xmin) / (2 * hmin) + 0.5))
        iy = int(math.floor((b.cy - b.beta - ymin) / (2 * hmin) + 0.5))
        c = 0
        for bit in range(31):
            c |= ((iy >> bit) & 1) << (2 * bit)
            c |= ((ix >> bit) & 1) << (2 * bit + 1)
        return c

    order = sorted(range(len(boxes)), key=lambda k: code(boxes[k]))
    lp = max(1, 64 // n2) * n2
    nleaves = 1
    while nleaves * lp < len(boxes) * n2:
        nleaves *= 2
    perm = -np.ones(nleaves * lp, dtype=np.int64)
    for t, k in enumerate(order):
        perm[t * n2:(t + 1) * n2] = k * n2 + np.arange(n2)
    return perm, lp


def padded(A: np.ndarray, perm: np.ndarray) -> np.ndarray:
    """A in the order perm, with identity rows and columns at the padding positions (-1)."""
    M = len(perm)
    out = np.eye(M, dtype=complex)
    real = np.nonzero(perm >= 0)[0]
    out[np.ix_(real, real)] = A[np.ix_(perm[real], perm[real])]
    return out
