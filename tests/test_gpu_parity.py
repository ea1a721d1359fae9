"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Tolerances: the FP64 DAFMM product at NCA tolerance 1e-10 must be within 1e-8 (relative
L2) of the oracle's dense / FFT product; solutions within 1e-6 of the oracle's; the
HODLR apply, which both sides build with the same ACA rules, within 1e-9; the kernel
table within 1e-13 relative per entry.  FP32 products are checked at 2e-5 (complex64
accumulation over a few thousand terms).
"""
import math
import sys

import numpy as np
import pytest

from oracle import gmres as ogmres
from oracle import hodlr as ohodlr
from oracle import lsop, special
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


_cache = {}


def problem(name, n, kappa, q, tol=1e-10, **opt):
    key = (name, n, kappa, tol, tuple(sorted(opt.items())))
    if key not in _cache:
        say(f"setup {name} n={n} kappa={kappa} tol={tol} {opt}")
        _cache[key] = ls.Problem(inputs.grid_points(n), q, kappa, tol, ls.Options(**opt))
    return _cache[key]


def gauss32():
    p = inputs.problem_gaussian_small()
    return p.n, p.kappa, p.q


# ---------------------------------------------------------------------------------------
def test_green_table_matches_scipy():
    from scipy.special import hankel1
    for n, kappa in [(512, 80.0), (32, 10.0), (96, 3.0)]:
        h = 2.0 / n
        say(f"green table n={n} kappa={kappa}")
        W = host(ls.green_table(n, h, kappa))
        ref = lsop.offset_table(n, 1.0, kappa)
        err = np.abs(W - ref) / np.abs(ref)
        assert err.max() < 1e-13, (n, kappa, err.max())
        assert abs(W[n - 1, n - 1] - special.self_cell(h, kappa)) < 1e-13 * abs(W[n - 1, n - 1])
    # branch boundaries of the evaluator (z = 4 and z = 20) and the far end of the range
    n, h = 300, 1.0
    for kappa in (4.0 / 3.0, 20.0 / 7.0, 226.0 / 299.0):
        W = host(ls.green_table(n, h * 0.01, kappa * 100.0))
        ref = lsop.offset_table(n, n * h * 0.01 / 2, kappa * 100.0)
        assert (np.abs(W - ref) / np.abs(ref)).max() < 1e-13


def test_matvec_dense_gaussian32():
    n, kappa, q = gauss32()
    P = problem("gauss32", n, kappa, q)
    A = lsop.dense_A(n, 1.0, kappa, q, -1)
    X = inputs.random_vector(n * n, nrhs=3, seed=11)
    Y = host(P.matvec(dev(np.ascontiguousarray(X.T))))
    for j in range(3):
        assert rel(Y[j], A @ X[:, j]) < 1e-8
    Y32 = host(P.matvec(dev(np.ascontiguousarray(X.T)), prec=ls.LS_FP32))
    assert rel(Y32[0], A @ X[:, 0]) < 2e-5


@pytest.mark.parametrize("n,kappa,seed", [(32, 20.0, 5), (128, 80.0, 6)])
def test_matvec_wide_block(n, kappa, seed):
    # blocks of 8 or more columns run the passes in their wide layout (longer chains, four row
    # tiles per block, separate gather and epilogue): every column against the oracle, and
    # column 0 against the same column applied alone (narrow layout)
    pb = inputs.problem_bumps(n, kappa, seed)
    P = problem(pb.name, n, kappa, pb.q)
    nrhs = 9
    X = inputs.random_vector(n * n, nrhs=nrhs, seed=seed + 200)
    Vx = lsop.FFTApplyV(n, 1.0, kappa)
    say(f"wide block n={n} nrhs={nrhs}")
    Y = host(P.matvec(dev(np.ascontiguousarray(X.T))))
    Y32 = host(P.matvec(dev(np.ascontiguousarray(X.T)), prec=ls.LS_FP32))
    for j in range(nrhs):
        ref = X[:, j] - kappa * kappa * pb.q * Vx(X[:, j])
        assert rel(Y[j], ref) < 1e-8, j
        assert rel(Y32[j], ref) < 2e-5, j
    y0 = host(P.matvec(dev(np.ascontiguousarray(X[:, 0]))))
    assert rel(Y[0], y0) < 1e-12


@pytest.mark.parametrize("n,kappa,seed", [(64, 40.0, 3), (128, 80.0, 4), (256, 40.0, 0)])
def test_matvec_fft(n, kappa, seed):
    pb = inputs.problem_bumps(n, kappa, seed, count=8 if seed == 0 else None)
    P = problem(pb.name, n, kappa, pb.q)
    x = inputs.random_vector(n * n, seed=seed + 100)
    say(f"matvec n={n}")
    y = host(P.matvec(dev(x)))
    Vx = lsop.FFTApplyV(n, 1.0, kappa)(x)
    ref = x - kappa * kappa * pb.q * Vx
    assert rel(y, ref) < 1e-8
    v = host(P.apply_V(dev(x)))
    assert rel(v, Vx) < 1e-8
    y32 = host(P.matvec(dev(x), prec=ls.LS_FP32))
    assert rel(y32, ref) < 2e-5


def test_matvec_disc512_full_size():
    pb = inputs.problem_disc(512, 80.0)
    P = problem(pb.name, 512, 80.0, pb.q)
    x = inputs.random_vector(512 * 512, seed=7)
    say("matvec n=512 kappa=80")
    v = host(P.apply_V(dev(x)))
    Vx = lsop.FFTApplyV(512, 1.0, 80.0)(x)
    assert rel(v, Vx) < 1e-8
    rows = np.array([0, 511, 1000, 131072 + 256, 200000, 262143])
    direct = lsop.sampled_rows_Vx(512, 1.0, 80.0, x, rows)
    assert np.max(np.abs(v[rows] - direct)) < 1e-8 * np.linalg.norm(Vx) / math.sqrt(len(x))
    st = P.stats()
    say("stats", st)
    assert st["m2l_pairs"] == 1616 + 34988 + 66236 + 105276


def test_rhs_planewave():
    n, kappa, q = gauss32()
    P = problem("gauss32", n, kappa, q)
    f = host(P.rhs_planewave([0.0, 1.3]))
    assert np.allclose(f[0], lsop.rhs_planewave(n, 1.0, kappa, q, 0.0), rtol=1e-14, atol=1e-14)
    assert np.allclose(f[1], lsop.rhs_planewave(n, 1.0, kappa, q, 1.3), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("n,kappa,rank,kind", [(32, 10.0, 5, "gauss"), (32, 10.0, 15, "gauss"),
                                               (64, 40.0, 10, "disc"), (64, 40.0, 160, "disc")])
def test_precond_matches_oracle_hodlr(n, kappa, rank, kind):
    if kind == "gauss":
        _, _, q = gauss32()
    else:
        q = inputs.problem_disc(n, kappa).q
    P = problem(f"{kind}{n}", n, kappa, q, hodlr_rank=rank)
    side = P.stats()["leaf_side"]
    A = lsop.dense_A(n, 1.0, kappa, q, -1)
    perm = ohodlr.morton_permutation(n, side)
    H = ohodlr.HODLR(A[np.ix_(perm, perm)], side * side, rank)
    b = inputs.random_vector(n * n, seed=21)
    say(f"precond n={n} r={rank}")
    z = host(P.precond_apply(dev(b)))
    zref = np.empty_like(b)
    zref[perm] = H.solve(b[perm])
    assert rel(z, zref) < 1e-9
    z32 = host(P.precond_apply(dev(b), prec=ls.LS_FP32))
    assert rel(z32, zref) < 1e-4


def test_sparse_contrast_updates_match_oracle():
    # a disc of radius 0.3 leaves three quarters of the 256-row blocks without contrast: the level
    # updates then run over the listed blocks only (complex64 and bfloat16 factors); the rows of Y
    # they skip are zero, so the applies still match the oracle HODLR and the solve the FP64 one
    n, kappa, rank = 64, 20.0, 12
    x = inputs.grid_points(n)
    q = (np.hypot(x[:, 0], x[:, 1]) < 0.3).astype(float)
    P = problem("smalldisc64", n, kappa, q, hodlr_rank=rank)
    st = P.stats()
    assert st["hodlr_rows_active"] * 4 < 3 * n * n
    side = st["leaf_side"]
    A = lsop.dense_A(n, 1.0, kappa, q, -1)
    perm = ohodlr.morton_permutation(n, side)
    H = ohodlr.HODLR(A[np.ix_(perm, perm)], side * side, rank)
    b = inputs.random_vector(n * n, seed=23)
    zref = np.empty_like(b)
    zref[perm] = H.solve(b[perm])
    z64 = host(P.precond_apply(dev(b)))
    z32 = host(P.precond_apply(dev(b), prec=ls.LS_FP32))
    zm = host(P.precond_apply(dev(b), prec=ls.LS_MIXED))
    say("sparse contrast: rows active", st["hodlr_rows_active"], rel(z64, zref), rel(z32, zref), rel(zm, zref))
    assert rel(z64, zref) < 1e-9
    assert rel(z32, zref) < 1e-5
    assert rel(zm, zref) < 2e-2
    f = P.rhs_planewave([0.7])
    x64, i64 = P.solve(f, tol=1e-10, prec=ls.LS_FP64)
    xm, im = P.solve(f, tol=1e-8, prec=ls.LS_MIXED)
    assert i64[0]["status"] == "CONVERGED" and im[0]["relres"] <= 1e-8
    assert rel(host(xm), host(x64)) < 1e-6
    assert rel(host(x64), np.linalg.solve(A, host(f)[0] if host(f).ndim > 1 else host(f))) < 1e-6


def test_one_sided_nodes_skip_dot_and_core_and_match_oracle():
    # contrast in one quadrant only: from the root down, many nodes have one child without
    # contrast (its Y is zero, so the sibling's W^T z chunks feed nothing and K^-1 is the
    # identity on the half of s the other child uses) and many have none; the masked applies
    # skip that work and still match the oracle HODLR, and the solves the dense solve
    n, kappa, rank = 64, 20.0, 12
    x = inputs.grid_points(n)
    q = (np.hypot(x[:, 0] - 0.5, x[:, 1] - 0.5) < 0.3).astype(float)
    P = problem("quadrantdisc64", n, kappa, q, hodlr_rank=rank)
    st = P.stats()
    N, lb = n * n, st["hodlr_levels"]
    say("dot rows", st["hodlr_dot_rows"][:lb], "core nodes", st["hodlr_core_nodes"][:lb])
    assert st["hodlr_core_nodes"][0] == 0 and st["hodlr_dot_rows"][0] == N // 2
    assert all(0 <= st["hodlr_core_nodes"][l] < (1 << l) for l in range(lb))
    assert all(0 < st["hodlr_dot_rows"][l] <= N for l in range(lb))
    side = st["leaf_side"]
    A = lsop.dense_A(n, 1.0, kappa, q, -1)
    perm = ohodlr.morton_permutation(n, side)
    H = ohodlr.HODLR(A[np.ix_(perm, perm)], side * side, rank)
    for seed in (29, 31):
        b = inputs.random_vector(n * n, seed=seed)
        zref = np.empty_like(b)
        zref[perm] = H.solve(b[perm])
        z64 = host(P.precond_apply(dev(b)))
        z32 = host(P.precond_apply(dev(b), prec=ls.LS_FP32))
        zm = host(P.precond_apply(dev(b), prec=ls.LS_MIXED))
        say("one-sided nodes: seed", seed, rel(z64, zref), rel(z32, zref), rel(zm, zref))
        assert rel(z64, zref) < 1e-9
        assert rel(z32, zref) < 1e-5
        assert rel(zm, zref) < 2e-2
    f = P.rhs_planewave([0.4])
    x64, i64 = P.solve(f, tol=1e-10, prec=ls.LS_FP64)
    xm, im = P.solve(f, tol=1e-8, prec=ls.LS_MIXED)
    assert i64[0]["status"] == "CONVERGED" and im[0]["relres"] <= 1e-8
    assert rel(host(xm), host(x64)) < 1e-6
    assert rel(host(x64), np.linalg.solve(A, host(f)[0] if host(f).ndim > 1 else host(f))) < 1e-6


def test_precond_full_rank_is_inverse():
    n, kappa = 8, 6.0
    q = inputs.contrast_gaussian(inputs.grid_points(n), 1.5, 10.0)
    P = problem("tiny8", n, kappa, q, hodlr_rank=32, leaf_max=4)
    A = lsop.dense_A(n, 1.0, kappa, q, -1)
    b = inputs.random_vector(n * n, seed=5)
    z = host(P.precond_apply(dev(b)))
    assert rel(z, np.linalg.solve(A, b)) < 1e-11


def test_precond_bf16_factors_close_to_fp64():
    # complex bfloat16 off-diagonal factors (8-bit mantissa): the apply stays within 1e-2 of
    # the complex128 one; complex64 factors within 1e-5
    n, kappa = 128, 40.0
    pb = inputs.problem_bumps(n, kappa, seed=2, count=5)
    P = problem("bumps128-bf16", n, kappa, pb.q, hodlr_rank=15)
    b = dev(inputs.random_vector(n * n, seed=8))
    z64 = host(P.precond_apply(b, prec=ls.LS_FP64))
    z32 = host(P.precond_apply(b, prec=ls.LS_FP32))
    z16 = host(P.precond_apply(b, prec=ls.LS_MIXED))
    say("precond bf16 vs fp64", rel(z16, z64), "fp32", rel(z32, z64))
    assert rel(z32, z64) < 1e-5
    assert 1e-6 < rel(z16, z64) < 1e-2


def test_precond_low_precision_leaf_and_core_solves():
    # pc_lowp_solves = 1 keeps the leaf and SMW core inverses in the factors' precision too: the
    # mixed apply moves away from the complex128 one but stays within bfloat16 accuracy, and the
    # default (complex128 leaf and core solves) is closer
    n, kappa = 128, 40.0
    pb = inputs.problem_bumps(n, kappa, seed=2, count=5)
    P = problem("bumps128-bf16", n, kappa, pb.q, hodlr_rank=15)
    L = problem("bumps128-lowp", n, kappa, pb.q, hodlr_rank=15, pc_lowp_solves=1)
    b = dev(inputs.random_vector(n * n, seed=8))
    z64 = host(P.precond_apply(b, prec=ls.LS_FP64))
    z16 = host(P.precond_apply(b, prec=ls.LS_MIXED))
    l16 = host(L.precond_apply(b, prec=ls.LS_MIXED))
    l32 = host(L.precond_apply(b, prec=ls.LS_FP32))
    say("lowp solves: bf16", rel(l16, z64), "c64", rel(l32, z64), "default bf16", rel(z16, z64))
    assert rel(l16, z64) < 2e-2 and rel(l32, z64) < 1e-5
    assert rel(z16, z64) < rel(l16, z64)


def test_precond_multi_rhs_equals_single_columns():
    # several right-hand sides take the right-hand-side-fastest launch shapes; each column must
    # equal its single-column apply exactly (the same sums in the same order)
    n, kappa = 128, 40.0
    pb = inputs.problem_bumps(n, kappa, seed=2, count=5)
    P = problem("bumps128-bf16", n, kappa, pb.q, hodlr_rank=15)
    B = torch.stack([dev(inputs.random_vector(n * n, seed=20 + j)) for j in range(3)])
    for prec in (ls.LS_FP64, ls.LS_FP32, ls.LS_MIXED):
        Z = host(P.precond_apply(B, prec=prec))
        for j in range(3):
            z1 = host(P.precond_apply(B[j].contiguous(), prec=prec))
            assert np.max(np.abs(Z[j] - z1)) <= 1e-14 * np.max(np.abs(z1)), (prec, j)


def test_solve_gaussian32_unpreconditioned():
    n, kappa, q = gauss32()
    P = problem("gauss32-noprec", n, kappa, q, hodlr_rank=0)
    A = lsop.dense_A(n, 1.0, kappa, q, -1)
    f = lsop.rhs_planewave(n, 1.0, kappa, q, 0.0)
    psi, info = P.solve(dev(f), tol=1e-10)
    psi = host(psi)
    xs = np.linalg.solve(A, f)
    _, its, _ = ogmres.gmres(lambda v: A @ v, f, 1e-10)
    say("gauss32", info, "oracle its", its)
    assert info[0]["status"] == "CONVERGED"
    assert rel(psi, xs) < 1e-8
    assert abs(info[0]["iters"] - its) <= 2
    assert np.linalg.norm(A @ psi - f) / np.linalg.norm(f) < 1.01e-10


@pytest.mark.parametrize("prec", [ls.LS_FP64, ls.LS_MIXED])
def test_solve_disc64_hybrid(prec):
    n, kappa = 64, 40.0
    q = inputs.problem_disc(n, kappa).q
    P = problem("disc64-" + str(prec), n, kappa, q, hodlr_rank=15, prec=prec)
    f = lsop.rhs_planewave(n, 1.0, kappa, q, 0.0)
    say(f"solve disc64 prec={prec}")
    psi, info = P.solve(dev(f), tol=1e-8)
    psi = host(psi)
    Vop = lsop.FFTApplyV(n, 1.0, kappa)
    Aop = lambda v: lsop.apply_A(Vop, v, q, kappa)
    res = np.linalg.norm(Aop(psi) - f) / np.linalg.norm(f)
    say(info, "oracle residual", res)
    assert info[0]["status"] == "CONVERGED"
    assert res < 1.2e-8
    xo, its, _ = ogmres.gmres(Aop, f, 1e-10, restart=200)
    assert rel(psi, xo) < 1e-6


def test_solve_batched_matches_single():
    n, kappa = 64, 30.0
    pb = inputs.problem_bumps(n, kappa, seed=9)
    P = problem(pb.name, n, kappa, pb.q, hodlr_rank=10)
    angles = [0.0, 0.5, 2.0, 4.0]
    F = P.rhs_planewave(angles)
    psiB, infoB = P.solve(F, tol=1e-9)
    psiB = host(psiB)
    for j, th in enumerate(angles):
        psi1, info1 = P.solve(P.rhs_planewave([th]), tol=1e-9)
        assert rel(psiB[j], host(psi1)) < 1e-7
        assert infoB[j]["status"] == "CONVERGED"
        assert abs(infoB[j]["iters"] - info1[0]["iters"]) <= 1


def test_solve_zero_rhs_and_warm_start():
    n, kappa, q = gauss32()
    P = problem("gauss32", n, kappa, q)
    z = torch.zeros(n * n, dtype=torch.complex128, device="cuda")
    psi, info = P.solve(z, tol=1e-8)
    assert info[0]["status"] == "CONVERGED" and float(psi.abs().max()) == 0.0
    f = P.rhs_planewave([0.0])
    psi, info = P.solve(f, tol=1e-10)
    psi2, info2 = P.solve(f, psi=psi.clone(), tol=1e-8, x0=True)
    assert info2[0]["iters"] == 0 and info2[0]["status"] == "CONVERGED"
    assert info2[0]["relres0"] < 1e-9
    # a poor guess is scaled by xi = (A g)^H f / ||A g||^2 (checked with an independent product)
    g = torch.full_like(f, 1e6)
    Ag = P.matvec(g)
    xi = torch.vdot(Ag, f) / torch.vdot(Ag, Ag).real
    expect = float(torch.linalg.vector_norm(f - xi * Ag) / torch.linalg.vector_norm(f))
    psi3, info3 = P.solve(f, psi=g.clone(), tol=1e-8, x0=True)
    assert info3[0]["status"] == "CONVERGED"
    assert abs(info3[0]["relres0"] - expect) < 1e-6 * expect and expect < 1.0
    assert rel(host(psi3), host(psi)) < 1e-6
    # a guess that cannot lower the residual is replaced by zero
    psi4, info4 = P.solve(f, psi=torch.full_like(f, float("nan")), tol=1e-8, x0=True)
    assert info4[0]["status"] == "WARMSTART_REJECTED" and info4[0]["relres0"] == 1.0
    assert rel(host(psi4), host(psi)) < 1e-6
    psi5, info5 = P.solve(f, psi=torch.zeros_like(f), tol=1e-8, x0=True)
    assert info5[0]["status"] == "WARMSTART_REJECTED"


def test_solve_bumps256_full_size():
    n, kappa = 256, 40.0
    pb = inputs.problem_bumps(n, kappa, seed=0, count=8)
    P = problem(pb.name + "-solve", n, kappa, pb.q, hodlr_rank=15)
    say("solve bumps256 full size", P.stats())
    f = P.rhs_planewave([0.0])
    psi, info = P.solve(f, tol=1e-8)
    say(info)
    Vop = lsop.FFTApplyV(n, 1.0, kappa)
    fh = host(f)
    res = np.linalg.norm(lsop.apply_A(Vop, host(psi), pb.q, kappa) - fh) / np.linalg.norm(fh)
    assert info[0]["status"] == "CONVERGED"
    assert res < 1.2e-8
