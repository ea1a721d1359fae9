"""HODLR direct solver (ls_direct_solve; Section 6, the factorisation used as the solver) with
tolerance-controlled off-diagonal ranks (hodlr_tol) and FP64 iterative refinement, against the
dense solve of the oracle operator."""
import sys

import numpy as np
import pytest

from oracle import lsop
from paper_2204_00326_amd import inputs, ls

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ls.lib()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gauss32():
    pb = inputs.problem_gaussian_small()
    A = lsop.dense_A(pb.n, pb.L, pb.kappa, pb.q)
    return pb, A


def test_tight_tolerance_factorisation_is_a_direct_solver():
    pb, A = gauss32()
    P = ls.Problem(pb.points(), pb.q, pb.kappa, 1e-12, ls.Options(hodlr_rank=128, hodlr_tol=1e-12))
    f = P.rhs_planewave([0.0, 1.3])
    F = f.cpu().numpy()
    psi, info = P.direct_solve(f, tol=0.0, max_refine=0)
    st = P.stats()
    say("ranks used", st["hodlr_rank_used_max"], st["hodlr_rank_used_sum"] / st["hodlr_blocks"], info)
    X = psi.cpu().numpy()
    for c in range(2):
        ref = np.linalg.solve(A, F[c])
        assert rel(X[c], ref) < 1e-8, c
        assert info[c]["iters"] == 0 and info[c]["relres"] < 1e-8
    assert st["hodlr_rank_used_max"] < 128       # the tolerance, not the cap, stopped the ACA


def test_loose_tolerance_with_refinement_reaches_the_residual():
    pb, A = gauss32()
    Pt = ls.Problem(pb.points(), pb.q, pb.kappa, 1e-12, ls.Options(hodlr_rank=128, hodlr_tol=1e-12))
    Pl = ls.Problem(pb.points(), pb.q, pb.kappa, 1e-12, ls.Options(hodlr_rank=128, hodlr_tol=1e-3))
    assert Pl.stats()["hodlr_rank_used_sum"] < Pt.stats()["hodlr_rank_used_sum"]
    f = Pl.rhs_planewave([0.4])
    psi0, i0 = Pl.direct_solve(f, tol=0.0, max_refine=0)
    psi, info = Pl.direct_solve(f, tol=1e-10, max_refine=20)
    say("loose: no refinement", i0, "refined", info)
    ref = np.linalg.solve(A, f.cpu().numpy())
    assert 1e-9 < i0[0]["relres"] < 1e-1              # the loose factorisation alone is inexact
    assert info[0]["status"] == "CONVERGED" and info[0]["relres"] <= 1e-10 and info[0]["iters"] <= 10
    assert rel(psi.cpu().numpy(), ref) < 1e-8


def test_block_of_right_hand_sides_equals_single_columns():
    pb, A = gauss32()
    P = ls.Problem(pb.points(), pb.q, pb.kappa, 1e-12, ls.Options(hodlr_rank=64, hodlr_tol=1e-6))
    angles = [0.0, 0.9, 2.2, 4.0]
    F = P.rhs_planewave(angles)
    X, infos = P.direct_solve(F, tol=1e-10, max_refine=20)
    for c, th in enumerate(angles):
        x1, i1 = P.direct_solve(P.rhs_planewave([th]), tol=1e-10, max_refine=20)
        assert infos[c]["relres"] <= 1e-10
        assert rel(X[c].cpu().numpy(), x1.cpu().numpy()[0] if x1.dim() > 1 else x1.cpu().numpy()) < 1e-10


def test_device_aca_matches_host_aca():
    # the batched device ACA (fixed rank) and the host routine (a tolerance too small to stop
    # it, so it also runs to the rank cap) choose the same pivots: the preconditioners agree
    n, kappa = 64, 25.0
    pb = inputs.problem_bumps(n, kappa, seed=6, count=5)
    Pd = ls.Problem(pb.points(), pb.q, kappa, 1e-10, ls.Options(hodlr_rank=12))
    Ph = ls.Problem(pb.points(), pb.q, kappa, 1e-10, ls.Options(hodlr_rank=12, hodlr_tol=1e-300))
    assert Pd.stats()["hodlr_rank_used_sum"] == Ph.stats()["hodlr_rank_used_sum"]
    b = torch.from_numpy(inputs.random_vector(n * n, seed=3)).cuda()
    zd = Pd.precond_apply(b).cpu().numpy()
    zh = Ph.precond_apply(b).cpu().numpy()
    say("device vs host ACA", rel(zd, zh))
    assert rel(zd, zh) < 1e-10


def test_direct_solve_needs_a_factorisation():
    pb, A = gauss32()
    P = ls.Problem(pb.points(), pb.q, pb.kappa, 1e-12, ls.Options(hodlr_rank=0))
    f = P.rhs_planewave([0.0])
    with pytest.raises(ls.LsError):
        P.direct_solve(f)


def test_hodlr_needs_leaves_of_at_most_64_points():
    pb = inputs.problem_bumps(64, 10.0, seed=1, count=2)
    with pytest.raises(ls.LsError) as e:
        ls.Problem(pb.points(), pb.q, 10.0, 1e-8, ls.Options(hodlr_rank=8, leaf_max=256))
    assert e.value.code == ls.LS_ENOTSUP
