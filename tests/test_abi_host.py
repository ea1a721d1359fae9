"""Host-side tests of libls: the library loads and exports every declared symbol, the
quadtree/cone/list planner agrees with a brute force written from the paper's
definitions, and invalid inputs are rejected before any device use."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from paper_2204_00326_amd import inputs, ls

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "ls.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ls_[a-z_A-Z0-9]+)\s*\(", txt)))


def test_library_exports_every_header_symbol():
    L = ls.lib()
    names = header_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name


def brute_force_lists(n, kappa, L=1.0, T=16.0, leaf_max=64):
    """Per-level interaction-list pair counts from the definitions of Section 3 and the
    notation table: neighbours by centre distance (< 4w in LF, < kappa w^2 in HF), IL(B) =
    children of the parent's neighbours that are not neighbours of B."""
    h = 2 * L / n
    leaf = None
    for lvl in range(1, 20):
        if n % (1 << lvl):
            break
        side = n >> lvl
        w = 0.5 * side * h
        if side * side <= leaf_max and (kappa * w) ** 2 <= T:
            leaf = lvl
            break
    counts = {}
    for nu in range(1, leaf + 1):
        nb = 1 << nu
        w = L / nb
        wp = 2 * w
        hf = (kappa * w) ** 2 > T
        hfp = (kappa * wp) ** 2 > T
        c = -L + (np.arange(nb) + 0.5) * 2 * w
        X, Y = np.meshgrid(c, c, indexing="ij")
        X, Y = X.ravel(), Y.ravel()
        d = np.hypot(X[:, None] - X[None, :], Y[:, None] - Y[None, :])
        nbr = d < (kappa * w * w if hf else 4 * w)
        cp = -L + (np.arange(nb // 2) + 0.5) * 2 * wp
        par = (np.arange(nb)[:, None] // 2) * (nb // 2) + (np.arange(nb)[None, :] // 2)
        par = par.ravel()
        XP, YP = np.meshgrid(cp, cp, indexing="ij")
        XP, YP = XP.ravel(), YP.ravel()
        dp = np.hypot(XP[:, None] - XP[None, :], YP[:, None] - YP[None, :])
        nbrp = dp < (kappa * wp * wp if hfp else 4 * wp)
        il = nbrp[par[:, None], par[None, :]] & ~nbr
        counts[nu] = int(il.sum())
    lnb = 1 << leaf
    near = sum(1 for a in range(lnb) for b in range(lnb) for da in (-1, 0, 1) for db in (-1, 0, 1)
               if 0 <= a + da < lnb and 0 <= b + db < lnb)
    return leaf, counts, near


@pytest.mark.parametrize("n,kappa", [(32, 10.0), (64, 40.0), (128, 60.0), (128, 80.0), (256, 40.0), (512, 80.0)])
def test_plan_matches_brute_force(n, kappa):
    d = ls.plan_describe(n, 1.0, kappa)
    leaf, counts, near = brute_force_lists(n, kappa)
    assert d["levels"] == leaf
    assert d["near_pairs"] == near
    top = d["top_level"]
    for nu, cnt in counts.items():
        assert d["il_pairs"][nu] == (cnt if nu >= top else 0), (nu, d["il_pairs"][nu], cnt)
    for nu in range(1, top):
        assert counts.get(nu, 0) == 0
    assert d["coverage"] == (1, 1)
    # leaves are low-frequency; cone counts double going up through HF levels
    assert not d["hf"][leaf]
    for nu in range(leaf):
        if d["hf"][nu] and d["hf"][nu + 1]:
            assert d["ndir"][nu] == 2 * d["ndir"][nu + 1]
        if d["hf"][nu]:
            w = 1.0 / (1 << nu)
            assert math.pi / d["ndir"][nu] <= 1.0 / (kappa * w)   # cone half-angle within 1/(kappa w)


@pytest.mark.parametrize("n,kappa", [(96, 30.0), (192, 50.0), (64, 60.0)])
def test_plan_coverage_queue_sizes(n, kappa):
    d = ls.plan_describe(n, 1.0, kappa)
    assert d["coverage"] == (1, 1)
    assert d["leaf_side"] * d["leaf_side"] <= 64


def _setup_status(points, q, kappa=10.0, tol=1e-10):
    L = ls.lib()
    h = C.c_void_p()
    o = ls.Options()._c()
    pts = np.ascontiguousarray(points, dtype=np.float64)
    qq = np.ascontiguousarray(q, dtype=np.float64)
    code = L.ls_setup(pts.ctypes.data, pts.shape[0], qq.ctypes.data, kappa, tol, C.byref(o), C.byref(h))
    return code, L.ls_last_error().decode(), h.value


def test_setup_rejects_invalid_inputs():
    p = inputs.grid_points(8)
    q = np.ones(64)
    assert _setup_status(p, q, kappa=-1.0)[0] == ls.LS_EINVAL
    assert _setup_status(p, q, kappa=0.0)[0] == ls.LS_EINVAL
    assert _setup_status(p, q, tol=0.0)[0] == ls.LS_EINVAL
    assert _setup_status(p, q, tol=1.5)[0] == ls.LS_EINVAL
    qn = q.copy()
    qn[3] = np.nan
    assert _setup_status(p, qn)[0] == ls.LS_EINVAL
    pn = p.copy()
    pn[5, 0] = np.inf
    assert _setup_status(pn, q)[0] == ls.LS_EINVAL
    dup = p.copy()
    dup[1] = dup[0]
    code, msg, h = _setup_status(dup, q)
    assert code in (ls.LS_EINVAL, ls.LS_ENOTSUP) and h is None
    assert _setup_status(p[:63], q[:63])[0] == ls.LS_ENOTSUP          # not a square grid
    jitter = p.copy()
    jitter[10, 1] += 0.01
    assert _setup_status(jitter, q)[0] == ls.LS_ENOTSUP


def test_setup_rejects_null_and_empty():
    L = ls.lib()
    h = C.c_void_p()
    assert L.ls_setup(None, 0, None, 1.0, 1e-8, None, C.byref(h)) == ls.LS_EINVAL
    assert "NULL" in L.ls_last_error().decode() or "positive" in L.ls_last_error().decode()


def test_plan_rejects_bad_options():
    with pytest.raises(ls.LsError):
        ls.plan_describe(32, 1.0, 10.0, ls.Options(sign=2))
    with pytest.raises(ls.LsError):
        ls.plan_describe(31, 1.0, 10.0)       # odd side: no quadtree split
    with pytest.raises(ls.LsError):
        ls.plan_describe(32, 1.0, -3.0)


def test_profile_readers_reject_bad_arguments():
    L = ls.lib()
    n = C.c_int64()
    ms = C.c_double()
    assert L.ls_profile_read_each(None, 5, None, None, 0, C.byref(n)) == ls.LS_EINVAL
    assert L.ls_profile_read(None, 0, C.byref(ms), C.byref(n), None) == ls.LS_EINVAL
    assert L.ls_profile_enable(None, 0, 1) == ls.LS_EINVAL


def test_panels_reject_invalid_inputs():
    # argument checks of the high-order panel calls run before any device use
    L = ls.lib()
    h = C.c_void_p()
    q = np.zeros(16 * 9)
    for args in ((0, 1.0, 3, 10.0, 1), (4, 1.0, 0, 10.0, -1), (4, 1.0, 9, 10.0, -1), (4, -1.0, 3, 10.0, -1),
                 (4, 1.0, 3, 0.0, -1), (4, 1.0, 3, 10.0, 0), (2000, 1.0, 3, 10.0, -1)):
        nside, Lh, p, kappa, sign = args
        assert L.ls_panels_setup(nside, Lh, p, kappa, q.ctypes.data, sign, C.byref(h)) == ls.LS_EINVAL, args
        assert not h
    assert L.ls_panels_setup(4, 1.0, 3, 10.0, None, -1, C.byref(h)) == ls.LS_EINVAL
    bad = q.copy()
    bad[5] = np.nan
    assert L.ls_panels_setup(4, 1.0, 3, 10.0, bad.ctypes.data, -1, C.byref(h)) == ls.LS_EINVAL
    assert L.ls_panels_setup(4, 1.0, 3, 10.0, q.ctypes.data, -1, None) == ls.LS_EINVAL
    x = np.zeros(4)
    assert L.ls_panels_apply(None, x.ctypes.data, x.ctypes.data, 1, 144, 0, None) == ls.LS_EINVAL
    assert L.ls_panels_moments(None, 0, 0, x.ctypes.data) == ls.LS_EINVAL
    n, npb, nf = C.c_int64(), C.c_int(), C.c_int()
    assert L.ls_panels_info(None, C.byref(n), C.byref(npb), C.byref(nf)) == ls.LS_EINVAL
    assert L.ls_panels_precond_setup(None, 8) == ls.LS_EINVAL
    assert L.ls_panels_precond_apply(None, x.ctypes.data, x.ctypes.data, 1, 144, None) == ls.LS_EINVAL
    r, lf, lv, mx, mr, ms = C.c_int(), C.c_int(), C.c_int(), C.c_int(), C.c_double(), C.c_double()
    assert L.ls_panels_precond_info(None, C.byref(r), C.byref(lf), C.byref(lv), C.byref(mr), C.byref(mx),
                                    C.byref(ms)) == ls.LS_EINVAL


def test_panels_leaves_reject_invalid_inputs():
    L = ls.lib()
    h = C.c_void_p()
    q = np.zeros(2 * 9)
    good = np.array([[-0.5, 0.0, 0.5], [0.5, 0.0, 0.5]])
    bad = good.copy()
    bad[1, 2] = -0.5
    assert L.ls_panels_setup_leaves(0, good.ctypes.data, 3, 10.0, q.ctypes.data, -1, C.byref(h)) == ls.LS_EINVAL
    assert L.ls_panels_setup_leaves(2, bad.ctypes.data, 3, 10.0, q.ctypes.data, -1, C.byref(h)) == ls.LS_EINVAL
    assert L.ls_panels_setup_leaves(2, good.ctypes.data, 9, 10.0, q.ctypes.data, -1, C.byref(h)) == ls.LS_EINVAL
    assert L.ls_panels_setup_leaves(2, good.ctypes.data, 3, 10.0, None, -1, C.byref(h)) == ls.LS_EINVAL
    many = np.tile(good, (2000, 1))
    assert L.ls_panels_setup_leaves(4000, many.ctypes.data, 3, 10.0, np.zeros(36000).ctypes.data, -1,
                                    C.byref(h)) == ls.LS_ENOTSUP
    assert not h
