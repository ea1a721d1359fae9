"""Pins for oracle.gmres, oracle.hodlr and oracle.mie.

GMRES is pinned to numpy.linalg.solve (LAPACK), to finite termination on small
systems, to the monotone residual of unrestarted GMRES and to one-step convergence
with an exact preconditioner.  ACA is pinned to exactly low-rank matrices; the
HODLR inverse to the densely assembled approximation it represents and, at full
rank, to the exact inverse.  The Mie series is pinned by the interface conditions.
"""
import math

import numpy as np
import pytest
from scipy.special import jv

from oracle import gmres, hodlr, lsop, mie
from paper_2204_00326_amd import inputs


def _c1():
    p = inputs.problem_gaussian_small()
    A = lsop.dense_A(p.n, p.L, p.kappa, p.q, -1)
    f = lsop.rhs_planewave(p.n, p.L, p.kappa, p.q, 0.0, -1)
    return p, A, f


def test_gmres_matches_direct_solve_gaussian32():
    p, A, f = _c1()
    x, its, hist = gmres.gmres(lambda v: A @ v, f, 1e-10, restart=200)
    xs = np.linalg.solve(A, f)
    assert np.linalg.norm(A @ x - f) <= 1e-10 * np.linalg.norm(f) * 1.0001
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    assert 5 <= its <= 20


def test_gmres_monotone_unrestarted():
    p, A, f = _c1()
    _, _, hist = gmres.gmres(lambda v: A @ v, f, 1e-12, restart=500)
    h = np.array(hist[1:-1])
    assert np.all(np.diff(h) <= 1e-14)


def test_gmres_finite_termination():
    rng = np.random.default_rng(0)
    n = 20
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 4 * np.eye(n)
    b = rng.standard_normal(n) + 0j
    x, its, _ = gmres.gmres(lambda v: A @ v, b, 1e-12, restart=50)
    assert its <= n + 1
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-12)


def test_gmres_restarted_and_preconditioned():
    p, A, f = _c1()
    x, its, _ = gmres.gmres(lambda v: A @ v, f, 1e-9, restart=4)
    assert np.linalg.norm(A @ x - f) <= 1e-9 * np.linalg.norm(f) * 1.0001
    Ainv = np.linalg.inv(A)
    x2, its2, _ = gmres.gmres(lambda v: A @ v, f, 1e-10, precond=lambda v: Ainv @ v)
    assert its2 == 1
    assert np.linalg.norm(x2 - np.linalg.solve(A, f)) <= 1e-9 * np.linalg.norm(x2)


def test_gmres_warm_start_exact():
    p, A, f = _c1()
    xs = np.linalg.solve(A, f)
    x, its, _ = gmres.gmres(lambda v: A @ v, f, 1e-8, x0=xs)
    assert its == 0


def test_aca_exact_low_rank():
    rng = np.random.default_rng(1)
    U = rng.standard_normal((60, 5)) + 1j * rng.standard_normal((60, 5))
    V = rng.standard_normal((45, 5)) + 1j * rng.standard_normal((45, 5))
    M = U @ V.T
    Ua, Va, rows, cols = hodlr.aca(M, 20, eps=1e-12)
    assert Ua.shape[1] in (5, 6)
    assert np.linalg.norm(Ua @ Va.T - M) <= 1e-10 * np.linalg.norm(M)
    # cross structure: v_k equals 1 at its column pivot, pivots are distinct
    for k, j in enumerate(cols):
        assert abs(Va[j, k] - 1) < 1e-14
    assert len(set(rows)) == len(rows) and len(set(cols)) == len(cols)


def test_aca_skips_zero_rows_and_ties_lowest_index():
    M = np.zeros((6, 4), dtype=complex)
    M[3] = [1, 2, 2, 1]
    M[5] = [2, 4, 4, 2]
    Ua, Va, rows, cols = hodlr.aca(M, 3)
    assert rows[0] == 3          # rows 0..2 are zero: next nonzero row
    assert cols[0] == 1          # tie between columns 1 and 2: lowest index
    assert np.allclose(Ua @ Va.T, M)


def test_morton_permutation():
    perm = hodlr.morton_permutation(16, 4)
    assert sorted(perm.tolist()) == list(range(256))
    first = perm[:16]
    a, b = first // 16, first % 16
    assert a.max() == 3 and b.max() == 3
    second = perm[16:32]            # leaf (la, lb) = (0, 1)
    assert (second // 16).max() == 3 and (second % 16).min() == 4


@pytest.mark.parametrize("rank", [3, 10])
def test_hodlr_smw_inverse_of_assembled(rank):
    p, A, f = _c1()
    perm = hodlr.morton_permutation(p.n, 8)
    Ah = A[np.ix_(perm, perm)]
    H = hodlr.HODLR(Ah, 64, rank)
    b = inputs.random_vector(p.N, seed=4)
    z = H.solve(b)
    assert np.linalg.norm(H.dense() @ z - b) <= 1e-10 * np.linalg.norm(b)


def test_hodlr_full_rank_is_exact():
    p, A, f = _c1()
    perm = hodlr.morton_permutation(p.n, 8)
    Ah = A[np.ix_(perm, perm)]
    H = hodlr.HODLR(Ah, 64, 1024)
    assert np.linalg.norm(H.dense() - Ah) <= 1e-11 * np.linalg.norm(Ah)
    b = inputs.random_vector(p.N, seed=5)
    assert np.linalg.norm(H.solve(b) - np.linalg.solve(Ah, b)) <= 1e-10 * np.linalg.norm(np.linalg.solve(Ah, b))


def _offdiag_blocks(H):
    """(depth, upper block, lower block) of every non-leaf node of the assembled A~."""
    D = H.dense()
    out = []

    def walk(node):
        if node["leaf"]:
            return
        lo, hi, mid = node["lo"], node["hi"], node["c1"]["hi"]
        out.append((node["depth"], D[lo:mid, mid:hi], D[mid:hi, lo:mid]))
        walk(node["c1"])
        walk(node["c2"])

    walk(H.root)
    return out


def test_hodlr_level_ranks_full_rank_is_exact():
    # full rank at every depth (the child block size): A~ = A and A~^{-1} b = A^{-1} b
    p, A, f = _c1()
    perm = hodlr.morton_permutation(p.n, 8)
    Ah = A[np.ix_(perm, perm)]
    full = [p.N >> (d + 1) for d in range(4)]
    H = hodlr.HODLR(Ah, 64, 1, level_ranks=full)
    assert np.linalg.norm(H.dense() - Ah) <= 1e-11 * np.linalg.norm(Ah)
    b = inputs.random_vector(p.N, seed=6)
    x = np.linalg.solve(Ah, b)
    assert np.linalg.norm(H.solve(b) - x) <= 1e-10 * np.linalg.norm(x)


def test_hodlr_level_ranks_set_each_depth():
    # every off-diagonal block at depth d has numerical rank exactly level_ranks[d] (the C1
    # blocks have higher rank, so a rank taken from the wrong depth shows), and a constant list
    # reproduces the single-rank construction
    p, A, f = _c1()
    perm = hodlr.morton_permutation(p.n, 8)
    Ah = A[np.ix_(perm, perm)]
    ranks = [7, 3, 5, 2]
    H = hodlr.HODLR(Ah, 64, 99, level_ranks=ranks)
    blocks = _offdiag_blocks(H)
    assert sorted({d for d, _, _ in blocks}) == [0, 1, 2, 3]
    for d, U, L in blocks:
        for B in (U, L):
            sv = np.linalg.svd(B, compute_uv=False)
            k = ranks[d]
            assert sv[k - 1] > 1e-6 * sv[0] and sv[k] <= 1e-10 * sv[0], (d, k, sv[: k + 2])
    H1 = hodlr.HODLR(Ah, 64, 4)
    H2 = hodlr.HODLR(Ah, 64, 99, level_ranks=[4, 4, 4, 4])
    assert np.array_equal(H1.dense(), H2.dense())


def test_hodlr_preconditioner_reduces_iterations():
    p = inputs.problem_disc(32, 20.0)
    A = lsop.dense_A(p.n, p.L, p.kappa, p.q, -1)
    f = lsop.rhs_planewave(p.n, p.L, p.kappa, p.q, 0.0, -1)
    perm = hodlr.morton_permutation(p.n, 8)
    inv = np.argsort(perm)
    H = hodlr.HODLR(A[np.ix_(perm, perm)], 64, 10)
    M = lambda v: H.solve(v[perm])[inv]
    _, it0, _ = gmres.gmres(lambda v: A @ v, f, 1e-8)
    _, it1, _ = gmres.gmres(lambda v: A @ v, f, 1e-8, precond=M)
    assert it1 < it0


def test_mie_interface_continuity():
    kappa, R, q0 = 10.0, 0.6, 1.0
    for th in (0.0, 0.7, 2.5):
        ui = mie.interior_series_at(R, th, kappa, R, q0)
        uo = mie.exterior_series_at(R, th, kappa, R, q0)
        assert abs(ui - uo) <= 1e-10 * abs(ui)
        dr = 1e-5
        gi = (mie.interior_series_at(R, th, kappa, R, q0) - mie.interior_series_at(R - dr, th, kappa, R, q0)) / dr
        go = (mie.exterior_series_at(R + dr, th, kappa, R, q0) - mie.exterior_series_at(R, th, kappa, R, q0)) / dr
        assert abs(gi - go) <= 1e-3 * abs(gi)


def test_mie_vanishing_contrast_is_incident():
    kappa, R = 10.0, 0.6
    pts = np.array([[0.1, 0.2], [-0.3, 0.05], [0.9, -0.2]])
    u = mie.total_field(pts, kappa, R, 1e-12)
    assert np.allclose(u, np.exp(1j * kappa * pts[:, 0]), atol=1e-9)
