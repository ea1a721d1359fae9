"""Fixed-rank HODLR approximation of A and its inverse (oracle).

Paper, Section 6 (Hybrid solver, Eq. (eq:hybrid)) and Section 6.1: the HODLR
preconditioner A~ is built by fixing a priori the rank r of its off-diagonal
blocks; GMRES then solves A~^{-1} A psi = A~^{-1} f.  The paper does not spell the
construction out.  The reading used here:

* Index order: quadtree leaves in Morton (Z) order, points row-major inside a
  leaf; a binary tree halves the index range down to single quadtree leaves.
* Each off-diagonal block A[I1, I2] and A[I2, I1] of a node is compressed with
  partially pivoted ACA (``aca``) stopped at rank r.
* Leaves keep the exact diagonal block of A.
* A~_node = blockdiag(A~_1, A~_2) + U W^T with U = blockdiag(P, R) and
  W = [[0, S], [Q, 0]] where A[I1,I2] ~ P Q^T and A[I2,I1] ~ R S^T, so that by
  Sherman-Morrison-Woodbury
      A~_node^{-1} b = z - Y (I + W^T Y)^{-1} W^T z,  z = blockdiag(A~_1, A~_2)^{-1} b,
  Y = blockdiag(A~_1^{-1} P, A~_2^{-1} R).

ACA (partial pivoting, as referenced by the paper for its pivot search and for
HODLR): start at the first row; the column pivot is the largest residual entry of
the pivot row over unused columns, the next row pivot the largest entry of the new
column over unused rows; an exactly zero residual row is skipped in favour of the
next unused row; entries within a relative 1e-9 of the maximum count as ties and
the lowest index wins; stop at ``max_rank``, at min(m, n), when no nonzero row
remains, or when ||u_k|| ||v_k|| <= eps ||S_k||_F.
"""
from __future__ import annotations

import numpy as np

TIE_REL = 1e-9


def _tie_argmax(vals: np.ndarray, allowed: np.ndarray) -> int:
    """Lowest allowed index whose |value| is within TIE_REL of the allowed maximum; -1 if all zero."""
    a = np.abs(vals)
    a = np.where(allowed, a, -1.0)
    m = a.max() if a.size else -1.0
    if m <= 0.0:
        return -1
    return int(np.nonzero(a >= (1.0 - TIE_REL) * m)[0][0])


def aca(M: np.ndarray, max_rank: int, eps: float = 0.0):
    """Partially pivoted ACA of a dense block M ~ U V^T.  Returns (U, V, row pivots, col pivots)."""
    m, n = M.shape
    us, vs, rows, cols = [], [], [], []
    row_used = np.zeros(m, dtype=bool)
    col_used = np.zeros(n, dtype=bool)
    normS2 = 0.0
    i = 0
    kmax = min(max_rank, m, n)
    while len(us) < kmax:
        # find a pivot row with a nonzero residual, starting at row i
        while True:
            r = M[i, :].copy()
            for u, v in zip(us, vs):
                r -= u[i] * v
            row_used[i] = True
            j = _tie_argmax(r, ~col_used)
            if j >= 0:
                break
            rest = np.nonzero(~row_used)[0]
            if rest.size == 0:
                return _pack(us, vs, rows, cols, m, n)
            i = int(rest[0])
        v = r / r[j]
        u = M[:, j].copy()
        for uu, vv in zip(us, vs):
            u -= vv[j] * uu
        col_used[j] = True
        rows.append(i)
        cols.append(j)
        # ||S_k||_F^2 update
        cross = 0.0
        for uu, vv in zip(us, vs):
            cross += 2.0 * np.real(np.vdot(uu, u) * np.vdot(v, vv))
        nu, nv = np.linalg.norm(u), np.linalg.norm(v)
        normS2 += cross + (nu * nv) ** 2
        us.append(u)
        vs.append(v)
        if eps > 0.0 and nu * nv <= eps * np.sqrt(max(normS2, 0.0)):
            break
        if len(us) >= kmax:
            break
        inext = _tie_argmax(u, ~row_used)
        if inext < 0:
            rest = np.nonzero(~row_used)[0]
            if rest.size == 0:
                break
            inext = int(rest[0])
        i = inext
    return _pack(us, vs, rows, cols, m, n)


def _pack(us, vs, rows, cols, m, n):
    k = len(us)
    U = np.zeros((m, k), dtype=complex)
    V = np.zeros((n, k), dtype=complex)
    for t in range(k):
        U[:, t] = us[t]
        V[:, t] = vs[t]
    return U, V, rows, cols


def morton_permutation(n: int, side: int) -> np.ndarray:
    """perm[t] = grid index of the t-th point in HODLR order (Morton leaves, row-major inside)."""
    nl = n // side

    def code(la, lb):
        c = 0
        for bit in range(16):
            c |= ((lb >> bit) & 1) << (2 * bit)
            c |= ((la >> bit) & 1) << (2 * bit + 1)
        return c

    leaves = sorted(((code(la, lb), la, lb) for la in range(nl) for lb in range(nl)))
    perm = []
    for _, la, lb in leaves:
        for a in range(side):
            for b in range(side):
                perm.append((la * side + a) * n + (lb * side + b))
    return np.array(perm, dtype=np.int64)


class HODLR:
    """A~ for a dense matrix A given in HODLR (Morton) order, leaves of ``leaf`` indices.

    ``rank`` is the off-diagonal rank of every node, as in the paper.  ``level_ranks``, if
    given, overrides it per depth of the binary tree (root = depth 0): the blocks of a node at
    depth d are compressed at rank level_ranks[d].
    """

    def __init__(self, A: np.ndarray, leaf: int, rank: int, level_ranks=None):
        self.A = A
        self.leaf = leaf
        self.rank = rank
        self.level_ranks = None if level_ranks is None else [int(k) for k in level_ranks]
        self.root = self._build(0, A.shape[0], 0)

    def rank_at(self, depth: int) -> int:
        if self.level_ranks is None:
            return self.rank
        return self.level_ranks[depth]

    def _build(self, lo, hi, depth):
        node = {"lo": lo, "hi": hi, "depth": depth}
        if hi - lo <= self.leaf:
            node["leaf"] = True
            node["D"] = self.A[lo:hi, lo:hi].copy()
            return node
        mid = (lo + hi) // 2
        node["leaf"] = False
        node["c1"] = self._build(lo, mid, depth + 1)
        node["c2"] = self._build(mid, hi, depth + 1)
        k = self.rank_at(depth)
        P, Q, _, _ = aca(self.A[lo:mid, mid:hi], k)
        R, S, _, _ = aca(self.A[mid:hi, lo:mid], k)
        node["P"], node["Q"], node["R"], node["S"] = P, Q, R, S
        # Y = blockdiag(A~1^{-1} P, A~2^{-1} R);  core = I + W^T Y
        Y1 = self._solve(node["c1"], P) if P.shape[1] else P
        Y2 = self._solve(node["c2"], R) if R.shape[1] else R
        node["Y1"], node["Y2"] = Y1, Y2
        kp, kr = P.shape[1], R.shape[1]
        core = np.eye(kp + kr, dtype=complex)
        # W^T z = [Q^T z2 ; S^T z1]; W^T Y = [[0, Q^T Y2], [S^T Y1, 0]]
        core[:kp, kp:] += Q.T @ Y2
        core[kp:, :kp] += S.T @ Y1
        node["core"] = core
        return node

    def _solve(self, node, b):
        if node["leaf"]:
            return np.linalg.solve(node["D"], b)
        lo, mid = node["lo"], node["c1"]["hi"]
        z1 = self._solve(node["c1"], b[: mid - lo])
        z2 = self._solve(node["c2"], b[mid - lo:])
        kp = node["P"].shape[1]
        t = np.concatenate([node["Q"].T @ z2, node["S"].T @ z1], axis=0)
        s = np.linalg.solve(node["core"], t)
        z1 = z1 - node["Y1"] @ s[:kp]
        z2 = z2 - node["Y2"] @ s[kp:]
        return np.concatenate([z1, z2], axis=0)

    def solve(self, b: np.ndarray) -> np.ndarray:
        """A~^{-1} b for b in HODLR order."""
        return self._solve(self.root, b)

    def dense(self) -> np.ndarray:
        """Assemble A~ densely (for checks)."""
        N = self.A.shape[0]
        out = np.zeros((N, N), dtype=complex)

        def fill(node):
            lo, hi = node["lo"], node["hi"]
            if node["leaf"]:
                out[lo:hi, lo:hi] = node["D"]
                return
            mid = node["c1"]["hi"]
            out[lo:mid, mid:hi] = node["P"] @ node["Q"].T
            out[mid:hi, lo:mid] = node["R"] @ node["S"].T
            fill(node["c1"])
            fill(node["c2"])

        fill(self.root)
        return out
