"""More parity of the HIP path against the oracle: the per-level HODLR rank cap, the literal
sign of Eq. (eq:6), the NCA tolerance sweep of Experiment 1 (Section 6.2), the vector-ALU form
of the DAFMM passes, grids whose leaves hold an odd number of points, several right-hand
sides on one-sided contrasts, and the solver statuses forced from the host.

Tolerances as in the other parity modules: HODLR applies built by the same ACA rules agree
with the oracle's to 1e-9 (complex128 factors), 1e-5 (complex64) and 2e-2 (complex bfloat16,
8-bit mantissa); DAFMM products at NCA tolerance 1e-10 to 1e-8 of the dense product.
"""
import math
import sys

import numpy as np
import pytest

from oracle import hodlr as ohodlr
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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_hodlr(n, kappa, q, side, rank, level_ranks=None, sign=-1):
    A = lsop.dense_A(n, 1.0, kappa, q, sign)
    perm = ohodlr.morton_permutation(n, side)
    H = ohodlr.HODLR(A[np.ix_(perm, perm)], side * side, rank, level_ranks=level_ranks)
    return A, perm, H


def oracle_apply(H, perm, b):
    z = np.empty_like(b)
    z[perm] = H.solve(b[perm])
    return z


def capped_ranks(N, levels, rank, div):
    # hodlr_rank_div = d: the blocks of a node at depth l (children of N >> (l + 1) points) get
    # rank min(hodlr_rank, child size / d), at least 1
    return [max(1, min(rank, (N >> (l + 1)) // div)) for l in range(levels)]


# ---------------------------------------------------------------------------------------
# per-level rank cap (the bench's hodlr_rank_div = 4) against the oracle HODLR with the same
# per-level ranks: dense contrast (fused and wide updates), a small disc (listed updates) and
# contrast in one quadrant (W^T z chunks and K^-1 products skipped where they meet a zero Y)
CONTRASTS = {
    "disc06": lambda x: (np.hypot(x[:, 0], x[:, 1]) < 0.6).astype(float),
    "disc03": lambda x: (np.hypot(x[:, 0], x[:, 1]) < 0.3).astype(float),
    "quadrant": lambda x: (np.hypot(x[:, 0] - 0.5, x[:, 1] - 0.5) < 0.3).astype(float),
}


@pytest.mark.parametrize("kind", list(CONTRASTS))
def test_precond_rank_cap_matches_oracle(kind):
    n, kappa, rank, div = 64, 30.0, 64, 4
    q = CONTRASTS[kind](inputs.grid_points(n))
    P = ls.Problem(inputs.grid_points(n), q, kappa, 1e-10, ls.Options(hodlr_rank=rank, hodlr_rank_div=div))
    st = P.stats()
    lb, side, N = st["hodlr_levels"], st["leaf_side"], n * n
    ranks = capped_ranks(N, lb, rank, div)
    assert ranks[-1] < rank and ranks[0] == rank      # the cap binds on the deep levels only
    A, perm, H = oracle_hodlr(n, kappa, q, side, rank, level_ranks=ranks)
    say(kind, "level ranks", ranks, "rows active", st["hodlr_rows_active"], "core nodes", st["hodlr_core_nodes"][:lb])
    for seed in (41, 42):
        b = inputs.random_vector(N, seed=seed)
        zref = oracle_apply(H, perm, b)
        z64 = host(P.precond_apply(dev(b), prec=ls.LS_FP64))
        z32 = host(P.precond_apply(dev(b), prec=ls.LS_FP32))
        z16 = host(P.precond_apply(dev(b), prec=ls.LS_MIXED))
        say(kind, seed, rel(z64, zref), rel(z32, zref), rel(z16, zref))
        assert rel(z64, zref) < 1e-9
        assert rel(z32, zref) < 1e-5
        assert rel(z16, zref) < 2e-2
    P.close()


def test_odd_leaf_side_sparse_contrast_applies_match_oracle():
    # n = 80: 25-point leaves (5 x 5 cells), so HODLR node halves hold 25 * 2^k rows, which a
    # kernel taking 4 (bfloat16) or 2 (complex64) consecutive rows per lane with one s cannot
    # split; a small disc leaves most 256-row blocks without contrast
    n, kappa, rank = 80, 20.0, 12
    x = inputs.grid_points(n)
    q = (np.hypot(x[:, 0], x[:, 1]) < 0.3).astype(float)
    P = ls.Problem(x, q, kappa, 1e-10, ls.Options(hodlr_rank=rank))
    st = P.stats()
    side = st["leaf_side"]
    assert side == 5 and st["hodlr_rows_active"] * 4 < 3 * n * n
    A, perm, H = oracle_hodlr(n, kappa, q, side, rank)
    b = inputs.random_vector(n * n, seed=43)
    zref = oracle_apply(H, perm, b)
    z64 = host(P.precond_apply(dev(b), prec=ls.LS_FP64))
    z32 = host(P.precond_apply(dev(b), prec=ls.LS_FP32))
    z16 = host(P.precond_apply(dev(b), prec=ls.LS_MIXED))
    say("n=80 small disc", rel(z64, zref), rel(z32, zref), rel(z16, zref))
    assert rel(z64, zref) < 1e-9
    assert rel(z32, zref) < 1e-5
    assert rel(z16, zref) < 2e-2
    f = P.rhs_planewave([0.2])
    xm, im = P.solve(f, tol=1e-8, prec=ls.LS_MIXED)
    assert im[0]["relres"] <= 1e-8
    assert rel(host(xm), np.linalg.solve(A, host(f))) < 1e-6
    P.close()


@pytest.mark.parametrize("nrhs", [3, 8])
def test_precond_multi_rhs_one_sided_contrast_equals_single_columns(nrhs):
    # several right-hand sides on a one-sided contrast take the masked multi-column launch
    # shapes (the child-list W^T z with right-hand sides fastest, the 8-column core products with
    # the activity mask); every column equals its single-column apply to rounding
    n, kappa, rank = 64, 20.0, 12
    x = inputs.grid_points(n)
    q = CONTRASTS["quadrant"](x)
    P = ls.Problem(x, q, kappa, 1e-10, ls.Options(hodlr_rank=rank))
    B = torch.stack([dev(inputs.random_vector(n * n, seed=60 + j)) for j in range(nrhs)])
    for prec in (ls.LS_FP64, ls.LS_FP32, ls.LS_MIXED):
        Z = host(P.precond_apply(B, prec=prec))
        for j in range(nrhs):
            z1 = host(P.precond_apply(B[j].contiguous(), prec=prec))
            assert np.max(np.abs(Z[j] - z1)) <= 1e-12 * np.max(np.abs(z1)), (prec, j)
    P.close()


# ---------------------------------------------------------------------------------------
def test_sign_plus_one_matches_oracle():
    # sign = +1 reproduces Eq. (eq:6) as printed: A = I + kappa^2 diag(q) V, f = -kappa^2 q u_inc
    pb = inputs.problem_gaussian_small()
    n, kappa, q = pb.n, pb.kappa, pb.q
    P = ls.Problem(pb.points(), q, kappa, 1e-10, ls.Options(hodlr_rank=5, sign=1))
    A = lsop.dense_A(n, 1.0, kappa, q, +1)
    X = inputs.random_vector(n * n, nrhs=2, seed=44)
    Y = host(P.matvec(dev(np.ascontiguousarray(X.T))))
    for j in range(2):
        assert rel(Y[j], A @ X[:, j]) < 1e-8
    f = host(P.rhs_planewave([0.0]))
    fo = lsop.rhs_planewave(n, 1.0, kappa, q, 0.0, sign=+1)
    assert np.allclose(f, fo, rtol=1e-14, atol=1e-14)
    psi, info = P.solve(dev(fo), tol=1e-10, prec=ls.LS_FP64)
    xs = np.linalg.solve(A, fo)
    say("sign +1", info, rel(host(psi), xs))
    assert info[0]["status"] == "CONVERGED" and rel(host(psi), xs) < 1e-8
    # the two signs give different operators (the test is not vacuous)
    Am = lsop.dense_A(n, 1.0, kappa, q, -1)
    assert rel(Y[0], Am @ X[:, 0]) > 1e-2
    P.close()


def test_nca_tolerance_sweep_error_decreases():
    # Experiment 1's design (Section 6.2): the DAFMM product against the exact product as the
    # NCA tolerance tightens, on a grid with high-frequency levels (n = 64, kappa = 40); the error
    # falls with the tolerance and stays below ten times it
    n, kappa = 64, 40.0
    pb = inputs.problem_bumps(n, kappa, seed=3)
    Vop = lsop.FFTApplyV(n, 1.0, kappa)
    x = inputs.random_vector(n * n, seed=45)
    Vx = Vop(x)
    errs = []
    for tol in (1e-4, 1e-6, 1e-8, 1e-10):
        P = ls.Problem(pb.points(), pb.q, kappa, tol, ls.Options(hodlr_rank=0, build_fp32=0))
        st = P.stats()
        assert st["nlevels_hf"] >= 1
        e = rel(host(P.apply_V(dev(x))), Vx)
        say(f"eps_NCA {tol:g}: rank max {st['rank_max64']}, far entries {st['entries_far64']}, error {e:.3e}")
        errs.append((tol, e, st["entries_far64"]))
        P.close()
    for (t0, e0, f0), (t1, e1, f1) in zip(errs, errs[1:]):
        assert e1 < e0 and f1 > f0
    for tol, e, _ in errs:
        assert e < 10 * tol


def test_full_rank_pivots_are_exact():
    # NCA at a tolerance below rounding keeps every pivot the cross approximation can find:
    # each far-field block is then reproduced to rounding and the product equals the dense one
    pb = inputs.problem_gaussian_small()
    P = ls.Problem(pb.points(), pb.q, pb.kappa, 1e-15, ls.Options(hodlr_rank=0, build_fp32=0))
    V = lsop.dense_V(pb.n, 1.0, pb.kappa)
    x = inputs.random_vector(pb.n * pb.n, seed=46)
    e = rel(host(P.apply_V(dev(x))), V @ x)
    say("eps_NCA 1e-15: rank max", P.stats()["rank_max64"], "error", e)
    assert e < 1e-12
    P.close()


@pytest.mark.parametrize("n,kappa,seed", [(64, 40.0, 3), (128, 80.0, 4)])
def test_valu_stencil_matches_oracle(n, kappa, seed):
    # stencil_mfma = 0: the same DAFMM sums on the vector ALUs
    pb = inputs.problem_bumps(n, kappa, seed)
    P = ls.Problem(pb.points(), pb.q, kappa, 1e-10, ls.Options(hodlr_rank=0, stencil_mfma=0))
    x = inputs.random_vector(n * n, seed=seed + 200)
    Vx = lsop.FFTApplyV(n, 1.0, kappa)(x)
    ref = x - kappa * kappa * pb.q * Vx
    y = host(P.matvec(dev(x)))
    y32 = host(P.matvec(dev(x), prec=ls.LS_FP32))
    say("valu stencil", n, rel(y, ref), rel(y32, ref))
    assert rel(y, ref) < 1e-8
    assert rel(y32, ref) < 2e-5
    P.close()


# ---------------------------------------------------------------------------------------
# solver statuses forced from the host (every kernel still runs to its normal end)
def test_status_maxit():
    pb = inputs.problem_gaussian_small()
    for gi in (0, 1):
        P = ls.Problem(pb.points(), pb.q, pb.kappa, 1e-10, ls.Options(hodlr_rank=0, maxit=3, restart=3, graph_iters=gi))
        f = P.rhs_planewave([0.0])
        psi, info = P.solve(f, tol=1e-12)
        say("maxit", gi, info)
        assert info[0]["status"] == "MAXIT" and info[0]["iters"] == 3
        assert 1e-12 < info[0]["relres"] < 1.0 and bool(torch.isfinite(psi).all())
        P.close()


def test_status_nan():
    pb = inputs.problem_gaussian_small()
    P = ls.Problem(pb.points(), pb.q, pb.kappa, 1e-10, ls.Options(hodlr_rank=5))
    f = P.rhs_planewave([0.0])
    f[17] = complex(float("nan"), 0.0)
    for prec in (ls.LS_FP64, ls.LS_MIXED):
        psi, info = P.solve(f, tol=1e-8, prec=prec)
        say("nan", prec, info)
        assert info[0]["status"] == "NAN"
    # the handle stays usable
    g = P.rhs_planewave([0.0])
    psi, info = P.solve(g, tol=1e-8)
    assert info[0]["status"] == "CONVERGED"
    P.close()


def test_status_refine_stagnated_after_max_refine_cycles():
    # mixed solve with short cycles and a refinement budget of one cycle: the second cycle
    # starts with FP64 products, the column converges and reports REFINE_STAGNATED
    n, kappa = 64, 30.0
    pb = inputs.problem_bumps(n, kappa, seed=9)
    P = ls.Problem(pb.points(), pb.q, kappa, 1e-10, ls.Options(hodlr_rank=4, restart=5, max_refine=1,
                                                               inner_tol=1e-2, maxit=3000))
    Q = ls.Problem(pb.points(), pb.q, kappa, 1e-10, ls.Options(hodlr_rank=4, restart=5, inner_tol=1e-2, maxit=3000))
    f = P.rhs_planewave([0.3])
    x64, i64 = P.solve(f, tol=1e-9, prec=ls.LS_FP64)
    xs, isg = P.solve(f, tol=1e-9, prec=ls.LS_MIXED)
    xq, iq = Q.solve(f, tol=1e-9, prec=ls.LS_MIXED)
    say("max_refine 1", isg, "default", iq, "fp64", i64)
    assert isg[0]["status"] == "REFINE_STAGNATED" and isg[0]["relres"] <= 1e-9
    assert isg[0]["n_refine"] > 1
    assert iq[0]["status"] in ("CONVERGED", "REFINE_STAGNATED") and iq[0]["relres"] <= 1e-9
    assert rel(host(xs), host(x64)) < 1e-6
    P.close()
    Q.close()


def test_queue_failed_problem_leaves_the_others():
    # a right-hand side with a NaN inside a queue: that problem reports NAN, the others converge
    # to their single-problem solutions
    probs = inputs.problem_queue(2, 4)
    Ps, fs = [], []
    for pb in probs:
        P = ls.Problem(pb.points(), pb.q, pb.kappa, 1e-10, ls.Options(hodlr_rank=15, restart=300))
        Ps.append(P)
        fs.append(P.rhs_planewave([0.0]))
    refs = [host(P.solve(f, tol=1e-8, prec=ls.LS_FP64)[0]) for P, f in zip(Ps, fs)]
    bad = 1
    fs[bad][5] = complex(float("nan"), float("nan"))
    for gi in (0, 4):
        psis, infos = ls.solve_queue(Ps, fs, tol=1e-8, prec=ls.LS_FP64, nworkers=2, graph_iters=gi)
        say("queue with a NaN problem", gi, [(i["iters"], i["status"]) for i in infos])
        assert infos[bad]["status"] == "NAN"
        for p in range(len(Ps)):
            if p == bad:
                continue
            assert infos[p]["status"] == "CONVERGED" and infos[p]["relres"] <= 1e-8
            assert rel(host(psis[p]), refs[p]) < 1e-6
    for P in Ps:
        P.close()


@pytest.mark.parametrize("n,kappa,leaf_max", [(8, 6.0, 4), (64, 40.0, 64), (128, 80.0, 64)])
def test_fused_dafmm_launch_equals_per_pass_launches(n, kappa, leaf_max):
    # fmm_fused = 1: every pass in one persistent launch (blocks taken from a queue in dependency
    # order, per-stage completion counts) against one launch per pass (whose long tasks split K
    # over workgroups, so the sums differ in order only): products of A and V agree to rounding,
    # for both precisions and several right-hand sides, and each path repeats bit for bit
    pb = inputs.problem_bumps(n, kappa, seed=5, count=4)
    opt = dict(hodlr_rank=0, leaf_max=leaf_max)
    Pf = ls.Problem(pb.points(), pb.q, kappa, 1e-10, ls.Options(fmm_fused=1, **opt))
    Pu = ls.Problem(pb.points(), pb.q, kappa, 1e-10, ls.Options(fmm_fused=0, **opt))
    X = torch.stack([dev(inputs.random_vector(n * n, seed=300 + j)) for j in range(3)])
    for prec, tol in ((ls.LS_FP64, 1e-13), (ls.LS_FP32, 2e-6)):
        yf0, yu0 = Pf.matvec(X, prec=prec), Pu.matvec(X, prec=prec)
        for rep in range(3):
            yf, yu = Pf.matvec(X, prec=prec), Pu.matvec(X, prec=prec)
            vf, vu = Pf.apply_V(X[0].contiguous(), prec=prec), Pu.apply_V(X[0].contiguous(), prec=prec)
            torch.cuda.synchronize()
            assert torch.equal(yf, yf0) and torch.equal(yu, yu0), (prec, rep)
            assert rel(host(yf), host(yu)) < tol and rel(host(vf), host(vu)) < tol, (prec, rep)
    ref = X[1].cpu().numpy() - kappa * kappa * pb.q * lsop.FFTApplyV(n, 1.0, kappa)(X[1].cpu().numpy())
    assert rel(host(Pf.matvec(X[1].contiguous())), ref) < 1e-8
    Pf.close()
    Pu.close()
