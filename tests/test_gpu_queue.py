"""Graph-captured GMRES driver and the multi-problem queue, through the C ABI.

The device-driven driver (Arnoldi index, Givens rotations and stop test on the device,
graph_iters steps per HIP graph; delayed CGS2 by default, CGS2 on request) runs the same
method as the host-driven one (CGS2): it must take the same number of iterations (within
one, for rounding in the rotations and the orthogonalisation) and give the same solution to
1e-9, across restarts that end in the middle of a graph, for several right-hand sides that
stop at different iterations, and in mixed precision.  Every solution of the
queue must equal the single-problem FP64 solve to 1e-6 and reach the tolerance; the
FP64 oracle pins the small case.
"""
import sys

import numpy as np
import pytest

from oracle import gmres as ogmres
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


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def pair(n, kappa, q, **opt):
    """the same problem twice: host-driven and graph-driven GMRES"""
    pts = inputs.grid_points(n)
    gi = opt.pop("graph_iters_b", 4)
    A = ls.Problem(pts, q, kappa, 1e-10, ls.Options(**opt))
    B = ls.Problem(pts, q, kappa, 1e-10, ls.Options(graph_iters=gi, **opt))
    return A, B


def test_graph_driver_matches_host_driver_and_oracle():
    pb = inputs.problem_gaussian_small()
    say("gauss32 graph vs host, unpreconditioned")
    A, B = pair(pb.n, pb.kappa, pb.q, hodlr_rank=0, restart=200)
    f = A.rhs_planewave([0.0])
    xa, ia = A.solve(f, tol=1e-10, prec=ls.LS_FP64)
    xb, ib = B.solve(f, tol=1e-10, prec=ls.LS_FP64)
    say(ia, ib)
    assert ib[0]["status"] == "CONVERGED" and ib[0]["relres"] <= 1e-10
    assert abs(ia[0]["iters"] - ib[0]["iters"]) <= 1
    assert rel(host(xb), host(xa)) < 1e-9
    Ad = lsop.dense_A(pb.n, pb.L, pb.kappa, pb.q)
    ref = np.linalg.solve(Ad, host(f))
    assert rel(host(xb), ref) < 1e-6


def test_graph_driver_restarts_inside_a_graph_and_multiple_rhs():
    n, kappa = 64, 30.0
    pb = inputs.problem_bumps(n, kappa, seed=3, count=4)
    # restart 7 with 3 steps per graph: cycles end in the middle of a replay
    A, B = pair(n, kappa, pb.q, hodlr_rank=4, restart=7, maxit=3000, graph_iters_b=3)
    F = A.rhs_planewave([0.0, 1.0, 2.5])
    xa, ia = A.solve(F, tol=1e-9, prec=ls.LS_FP64)
    xb, ib = B.solve(F, tol=1e-9, prec=ls.LS_FP64)
    say([i["iters"] for i in ia], [i["iters"] for i in ib])
    for c in range(3):
        assert ib[c]["status"] == "CONVERGED" and ib[c]["relres"] <= 1e-9
        assert abs(ia[c]["iters"] - ib[c]["iters"]) <= 2
        assert rel(host(xb)[c], host(xa)[c]) < 1e-7
    # the same columns one at a time take the same iterations (columns do not interact)
    for c, th in enumerate([0.0, 1.0, 2.5]):
        x1, i1 = B.solve(B.rhs_planewave([th]), tol=1e-9, prec=ls.LS_FP64)
        assert abs(i1[0]["iters"] - ib[c]["iters"]) <= 1


def test_graph_driver_mixed_precision():
    n, kappa = 128, 40.0
    pb = inputs.problem_bumps(n, kappa, seed=5, count=6)
    A, B = pair(n, kappa, pb.q, hodlr_rank=15, restart=300, graph_iters_b=8)
    f = A.rhs_planewave([0.3])
    x64, i64 = A.solve(f, tol=1e-8, prec=ls.LS_FP64)
    xm, im = B.solve(f, tol=1e-8, prec=ls.LS_MIXED)
    xh, ih = A.solve(f, tol=1e-8, prec=ls.LS_MIXED)
    say("fp64", i64, "mixed graph", im, "mixed host", ih)
    assert im[0]["status"] in ("CONVERGED", "REFINE_STAGNATED") and im[0]["relres"] <= 1e-8
    assert rel(host(xm), host(x64)) < 1e-6
    assert abs(im[0]["iters"] - ih[0]["iters"]) <= 3


def test_one_step_graphs_cgs2_high_rank_mixed():
    # the bench's driver (device-driven CGS2, one Arnoldi step per captured graph) with a HODLR
    # rank above 128 (SMW cores above 256 x 256): the mixed solve reaches the tolerance, equals the
    # FP64 host-driven solve to 1e-6 and takes its iterations within one
    n, kappa = 256, 80.0
    pb = inputs.problem_bumps(n, kappa, seed=5, count=6)
    A, B = pair(n, kappa, pb.q, hodlr_rank=160, hodlr_rank_div=4, restart=300, graph_iters_b=1, dcgs2=0)
    f = A.rhs_planewave([0.3])
    x64, i64 = A.solve(f, tol=1e-8, prec=ls.LS_FP64)
    xm, im = B.solve(f, tol=1e-8, prec=ls.LS_MIXED)
    xd, idd = B.solve(f, tol=1e-8, prec=ls.LS_FP64)
    say("fp64 host", i64, "mixed one-step graphs", im, "fp64 one-step graphs", idd)
    assert im[0]["status"] in ("CONVERGED", "REFINE_STAGNATED") and im[0]["relres"] <= 1e-8
    assert rel(host(xm), host(x64)) < 1e-6
    assert abs(idd[0]["iters"] - i64[0]["iters"]) <= 1 and rel(host(xd), host(x64)) < 1e-9


@pytest.mark.parametrize("prec", [ls.LS_FP64, ls.LS_MIXED])
def test_delayed_cgs2_matches_cgs2(prec):
    # delayed CGS2 (one reduction and one update pass per step) against two-pass CGS2 in the
    # same device-driven driver: same iteration count within one, same solution, and the
    # basis stays orthonormal enough that the Arnoldi estimate matches the true residual
    n, kappa = 128, 40.0
    pb = inputs.problem_bumps(n, kappa, seed=5, count=6)
    pts = inputs.grid_points(n)
    opt = dict(hodlr_rank=15, restart=300, graph_iters=8, inner_tol=1e-4)
    A = ls.Problem(pts, pb.q, kappa, 1e-10, ls.Options(dcgs2=0, **opt))
    B = ls.Problem(pts, pb.q, kappa, 1e-10, ls.Options(dcgs2=1, **opt))
    F = A.rhs_planewave([0.3, 2.0])
    xa, ia = A.solve(F, tol=1e-9, prec=prec)
    xb, ib = B.solve(F, tol=1e-9, prec=prec)
    say(prec, [(i["iters"], i["relres"]) for i in ia], [(i["iters"], i["relres"]) for i in ib])
    for c in range(2):
        assert ib[c]["status"] in ("CONVERGED", "REFINE_STAGNATED") and ib[c]["relres"] <= 1e-9
        assert abs(ia[c]["iters"] - ib[c]["iters"]) <= 1
        assert rel(host(xb)[c], host(xa)[c]) < 1e-7


def test_autotune_choices_and_solution_unchanged():
    n, kappa = 96, 35.0
    pb = inputs.problem_bumps(n, kappa, seed=7, count=3)
    P = ls.Problem(inputs.grid_points(n), pb.q, kappa, 1e-10, ls.Options(hodlr_rank=15, graph_iters=8))
    f = P.rhs_planewave([0.0])
    x0, i0 = P.solve(f, tol=1e-8, prec=ls.LS_FP64)
    t = P.autotune()
    say("autotune", t)
    assert t["gs_rows"] in (256, 512, 1024, 2048, 4096) and t["hodlr_rows"] in (128, 256, 512, 1024, 2048)
    assert all(v > 0 for v in t["gs_us"]) and all(v > 0 for v in t["pc_us"])
    x1, i1 = P.solve(f, tol=1e-8, prec=ls.LS_FP64)
    assert abs(i1[0]["iters"] - i0[0]["iters"]) <= 1 and rel(host(x1), host(x0)) < 1e-8


def test_queue_of_uneven_problems_matches_single_solves():
    probs = inputs.problem_queue(2, 16)
    Ps, fs = [], []
    for pb in probs:
        P = ls.Problem(pb.points(), pb.q, pb.kappa, 1e-10, ls.Options(hodlr_rank=15, restart=300, maxit=2000))
        Ps.append(P)
        fs.append(P.rhs_planewave([0.0]))
    say("queue of", len(Ps), [(pb.n, pb.kappa) for pb in probs])
    refs = [P.solve(f, tol=1e-8, prec=ls.LS_FP64)[0] for P, f in zip(Ps, fs)]
    for prec in (ls.LS_MIXED, ls.LS_FP64):
        psis, infos = ls.solve_queue(Ps, fs, tol=1e-8, prec=prec, nworkers=4, graph_iters=8)
        say(prec, [(i["iters"], i["status"]) for i in infos])
        for p in range(len(Ps)):
            assert infos[p]["relres"] <= 1e-8, (p, infos[p])
            assert infos[p]["status"] in ("CONVERGED", "REFINE_STAGNATED"), (p, infos[p])
            assert rel(host(psis[p]), host(refs[p])) < 1e-6, p
    # the oracle pins the smallest problem of the queue
    k = min(range(len(probs)), key=lambda i: probs[i].n * 1000 + probs[i].kappa)
    pb = probs[k]
    V = lsop.FFTApplyV(pb.n, pb.L, pb.kappa)
    fo = lsop.rhs_planewave(pb.n, pb.L, pb.kappa, pb.q, 0.0)
    xo, _, _ = ogmres.gmres(lambda x: lsop.apply_A(V, x, pb.q, pb.kappa), fo, 1e-10, restart=300)
    assert rel(host(psis[k]), xo) < 1e-6


def test_queue_rejects_bad_arguments():
    pb = inputs.problem_gaussian_small()
    P = ls.Problem(inputs.grid_points(pb.n), pb.q, pb.kappa, 1e-10, ls.Options(hodlr_rank=0))
    f = P.rhs_planewave([0.0])
    with pytest.raises(ls.LsError):
        ls.solve_queue([P, P], [f, f])
    with pytest.raises(ls.LsError):
        ls.solve_queue([P], [f], nworkers=17)
