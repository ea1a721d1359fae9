"""Kernel timing classes (ls_profile_enable / ls_profile_read) and the setup phase timers.

A mixed-precision solve with a bfloat16 HODLR preconditioner runs every class the bench
reports: the near-field + M2L launches of both operators, the leaf solves, the fused and
unfused HODLR level launches and the SMW core products.  Sampling every launch must time all
of them (timed == all launches), sampling every 3rd a third of them, and the timers must not
change the solution.  The setup timers must be parts of the HODLR setup time.
"""
import sys

import numpy as np
import pytest

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


def problem():
    n, kappa = 128, 30.0
    pb = inputs.problem_bumps(n, kappa, seed=3, count=4)
    opt = ls.Options(hodlr_rank=32, prec=ls.LS_MIXED)
    return ls.Problem(pb.points(), pb.q, kappa, 1e-10, opt)


def test_every_class_is_timed_and_timers_do_not_change_the_solve():
    P = problem()
    f = P.rhs_planewave([0.3])
    psi0, i0 = P.solve(f, tol=1e-8)
    for every in (1, 3):
        for c in ls.PROFILE_CLASSES:
            P.profile_enable(c, every)
        psi, info = P.solve(f, tol=1e-8)
        got = {c: P.profile_read(c) for c in ls.PROFILE_CLASSES}
        for c in ls.PROFILE_CLASSES:
            P.profile_enable(c, 0)
        say(every, {c: (round(v[0], 3), v[1], v[2]) for c, v in got.items()})
        assert info[0]["iters"] == i0[0]["iters"]
        assert torch.equal(psi, psi0)
        # single-column applies run the leaf solves with the deepest levels in one launch
        leaf = "hodlr_subtree" if P.stats()["hodlr_subtree_level"] >= 0 else "leaf_solve"
        for c in ("near_m2l64", "near_m2l32", leaf, "hodlr_upd_dot", "hodlr_core"):
            ms, timed, launches = got[c]
            assert launches > 0, c
            assert timed == (launches + every - 1) // every, (c, timed, launches)
            assert ms > 0.0, c


def test_setup_timers_are_parts_of_the_hodlr_setup():
    P = problem()
    st = P.stats()
    parts = st["t_hodlr_aca_ms"] + st["t_hodlr_apply_ms"] + st["t_hodlr_cores_ms"]
    say({k: round(st[k], 2) for k in ("t_plan_ms", "t_nca_ms", "t_hodlr_ms", "t_hodlr_aca_ms", "t_hodlr_apply_ms",
                                      "t_hodlr_cores_ms", "t_setup_ms")})
    assert all(st[k] > 0.0 for k in ("t_hodlr_aca_ms", "t_hodlr_apply_ms", "t_hodlr_cores_ms"))
    assert parts <= st["t_hodlr_ms"] <= st["t_setup_ms"]


def test_pass_spans_of_the_product_cover_every_pass_once():
    # one span per pass group and product; the spans lie inside the product, so their sum is
    # at most the time of the whole product between two events around it
    P = problem()
    x = torch.from_numpy(inputs.random_vector(P.N, seed=5)).cuda()
    y0 = P.matvec(x, prec=ls.LS_FP64)
    for b, prec in (("64", ls.LS_FP64), ("32", ls.LS_FP32)):
        keys = [k for k in ls.PROFILE_SPANS if k.startswith(f"mv{b}_")]
        for k in keys:
            P.profile_enable(k, 1)
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(4):
            y = P.matvec(x, prec=prec)
        e1.record(s)
        torch.cuda.synchronize()
        got = {k: P.profile_read(k) for k in keys}
        for k in keys:
            P.profile_enable(k, 0)
        say(b, {k: (round(v[0], 4), v[1], v[2]) for k, v in got.items()}, "whole", e0.elapsed_time(e1))
        for k, (ms, timed, launches) in got.items():
            if k.endswith(("_gather", "_epilogue")) and launches == 0:
                continue  # folded into P2M and L2P: no launch, no span
            assert timed == launches == 4 and ms > 0.0, k
        assert sum(v[0] for v in got.values()) <= e0.elapsed_time(e1)
        if prec == ls.LS_FP64:
            assert torch.equal(y, y0)
