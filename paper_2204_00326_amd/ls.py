"""ctypes binding of libls (argument marshalling only; every step runs in the library).

Vectors are torch tensors on the GPU, complex128, shaped (N,) or (nrhs, N) (row j of a
2-D tensor is right-hand side j, i.e. column-major N x nrhs with ld = N), in the
caller's point order.  The library raises if it was not built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libls.so")

LS_OK, LS_EINVAL, LS_ENOMEM, LS_EDEVICE, LS_ENOTSUP = 0, -1, -2, -3, -4
LS_FP64, LS_FP32, LS_MIXED = 0, 1, 2
STATUS = {0: "CONVERGED", 1: "MAXIT", 2: "BREAKDOWN", 3: "NAN", 4: "REFINE_STAGNATED", 5: "WARMSTART_REJECTED"}
PROFILE_CLASSES = {"near_m2l64": 0, "hodlr_update": 1, "leaf_solve": 2, "gs_dot": 3, "near_m2l32": 4,
                   "hodlr_dot": 5, "hodlr_upd_dot": 6, "hodlr_core": 7, "dafmm64": 8, "dafmm32": 9,
                   "hodlr_subtree": 20}
# spans of the per-pass DAFMM product (every launch between two stream events)
PROFILE_SPANS = {f"mv{b}_{k}": o + i for b, o in (("64", 10), ("32", 15))
                 for i, k in enumerate(("gather", "up", "near_m2l", "down", "epilogue"))}


def _prof_index(cls: str) -> int:
    return PROFILE_CLASSES[cls] if cls in PROFILE_CLASSES else PROFILE_SPANS[cls]


class LsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libls error {code}: {msg}")
        self.code = code


class _Options(C.Structure):
    _fields_ = [("leaf_max", C.c_int), ("T", C.c_double), ("sign", C.c_int), ("hodlr_rank", C.c_int),
                ("eps_inner", C.c_double), ("restart", C.c_int), ("maxit", C.c_int), ("prec", C.c_int),
                ("inner_tol", C.c_double), ("max_refine", C.c_int), ("build_fp32", C.c_int),
                ("hodlr_rank_div", C.c_int), ("graph_iters", C.c_int),
                ("stencil_mfma", C.c_int), ("pc_bf16", C.c_int), ("dcgs2", C.c_int), ("pc_lowp_solves", C.c_int),
                ("hodlr_tol", C.c_double), ("fmm_fused", C.c_int), ("nca_device", C.c_int)]


class _Info(C.Structure):
    _fields_ = [("iters", C.c_int), ("relres", C.c_double), ("status", C.c_int), ("n_refine", C.c_int),
                ("t_solve_ms", C.c_double), ("relres0", C.c_double)]


class _Stats(C.Structure):
    _fields_ = [("N", C.c_int64), ("n", C.c_int), ("levels", C.c_int), ("leaf_side", C.c_int),
                ("top_level", C.c_int), ("nlevels_hf", C.c_int), ("rank_max64", C.c_int), ("rank_max32", C.c_int),
                ("entries_near", C.c_int64), ("entries_far64", C.c_int64), ("entries_far32", C.c_int64),
                ("entries_m2l64", C.c_int64), ("entries_m2l32", C.c_int64),
                ("m2l_pairs", C.c_int64), ("stored_bytes64", C.c_int64), ("stored_bytes32", C.c_int64),
                ("hodlr_bytes", C.c_int64), ("hodlr_levels", C.c_int), ("hodlr_rank_sum", C.c_int),
                ("hodlr_dense_leaves", C.c_int64), ("t_plan_ms", C.c_double), ("t_nca_ms", C.c_double),
                ("t_hodlr_ms", C.c_double), ("t_setup_ms", C.c_double),
                ("hodlr_rank_used_sum", C.c_int64), ("hodlr_blocks", C.c_int64), ("hodlr_rank_used_max", C.c_int),
                ("t_hodlr_aca_ms", C.c_double), ("t_hodlr_apply_ms", C.c_double), ("t_hodlr_cores_ms", C.c_double),
                ("hodlr_rows_active", C.c_int64), ("hodlr_dot_rows", C.c_int64 * 32),
                ("hodlr_core_nodes", C.c_int * 32), ("entries_mid64", C.c_int64), ("entries_mid32", C.c_int64),
                ("hodlr_subtree_level", C.c_int)]


class _PlanInfo(C.Structure):
    _fields_ = [("levels", C.c_int), ("leaf_side", C.c_int), ("top_level", C.c_int), ("hf", C.c_int * 32),
                ("ndir", C.c_int * 32), ("max_il", C.c_int * 32), ("il_pairs", C.c_int64 * 32),
                ("near_pairs", C.c_int64), ("coverage_min", C.c_int), ("coverage_max", C.c_int)]


class _TuneInfo(C.Structure):
    _fields_ = [("gs_rows", C.c_int), ("hodlr_rows", C.c_int), ("gs_us", C.c_double * 5), ("pc_us", C.c_double * 5)]


class _NopConfig(C.Structure):
    _fields_ = [("n", C.c_int), ("width", C.c_int), ("modes", C.c_int), ("layers", C.c_int),
                ("batch_max", C.c_int), ("seed", C.c_uint64), ("bf16", C.c_int)]


_lib = None


def lib():
    """Load libls.so (built in-tree by paper_2204_00326_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2204_00326_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i64, ci, cd = C.c_void_p, C.c_int64, C.c_int, C.c_double
    L.ls_default_options.argtypes = [C.POINTER(_Options)]
    L.ls_default_options.restype = None
    L.ls_last_error.restype = C.c_char_p
    L.ls_setup.argtypes = [vp, i64, vp, cd, cd, C.POINTER(_Options), C.POINTER(vp)]
    for name in ("ls_matvec", "ls_apply_V", "ls_precond_apply", "ls_precond_apply_noalloc"):
        getattr(L, name).argtypes = [vp, vp, vp, ci, i64, ci, vp]
    L.ls_rhs_planewave.argtypes = [vp, vp, ci, vp, i64, vp]
    L.ls_solve.argtypes = [vp, vp, vp, ci, i64, cd, ci, ci, C.POINTER(_Info), vp]
    L.ls_direct_solve.argtypes = [vp, vp, vp, ci, i64, cd, ci, C.POINTER(_Info), vp]
    L.ls_stats.argtypes = [vp, C.POINTER(_Stats)]
    L.ls_solve_queue.argtypes = [vp, ci, vp, vp, cd, ci, ci, ci, C.POINTER(_Info)]
    L.ls_autotune.argtypes = [vp, C.POINTER(_TuneInfo), vp]
    L.ls_destroy.argtypes = [vp]
    L.ls_destroy.restype = None
    L.ls_plan_describe.argtypes = [ci, cd, cd, C.POINTER(_Options), C.POINTER(_PlanInfo)]
    L.ls_green_table.argtypes = [ci, cd, cd, vp, vp]
    L.ls_field_eval.argtypes = [vp, vp, i64, vp, vp, vp]
    L.ls_error_eval.argtypes = [vp, vp, i64, vp, cd, vp, vp, vp]
    L.ls_profile_enable.argtypes = [vp, ci, ci]
    L.ls_profile_read.argtypes = [vp, ci, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.ls_profile_read_each.argtypes = [vp, ci, vp, vp, i64, C.POINTER(C.c_int64)]
    L.ls_nop_create.argtypes = [C.POINTER(_NopConfig), C.POINTER(vp)]
    L.ls_nop_param_count.argtypes = [vp]
    L.ls_nop_param_count.restype = C.c_int64
    for name in ("ls_nop_get_params", "ls_nop_set_params", "ls_nop_get_grads"):
        getattr(L, name).argtypes = [vp, vp, i64]
        getattr(L, name).restype = C.c_int
    L.ls_nop_forward.argtypes = [vp, vp, vp, ci, vp]
    L.ls_nop_backward.argtypes = [vp, vp, vp]
    L.ls_nop_loss.argtypes = [vp, vp, vp, vp, vp, ci, vp, vp, vp]
    L.ls_nop_adam_step.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float, vp]
    L.ls_nop_features.argtypes = [ci, cd, vp, cd, cd, vp, vp]
    L.ls_nop_warmstart.argtypes = [ci, cd, vp, cd, cd, vp, vp, vp, vp]
    L.ls_nop_destroy.argtypes = [vp]
    L.ls_nop_destroy.restype = None
    for name in ("ls_nop_create", "ls_nop_forward", "ls_nop_backward", "ls_nop_loss", "ls_nop_adam_step",
                 "ls_nop_features", "ls_nop_warmstart"):
        getattr(L, name).restype = C.c_int
    L.ls_panels_setup.argtypes = [ci, cd, ci, cd, vp, ci, C.POINTER(vp)]
    L.ls_panels_apply.argtypes = [vp, vp, vp, ci, i64, ci, vp]
    L.ls_panels_setup_leaves.argtypes = [ci, vp, ci, cd, vp, ci, C.POINTER(vp)]
    L.ls_panels_moments.argtypes = [vp, ci, ci, vp]
    L.ls_panels_solve.argtypes = [vp, vp, vp, cd, ci, ci, C.POINTER(_Info), vp]
    L.ls_panels_info.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.ls_panels_precond_setup.argtypes = [vp, ci]
    L.ls_panels_precond_apply.argtypes = [vp, vp, vp, ci, i64, vp]
    L.ls_panels_precond_info.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                         C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_double)]
    L.ls_panels_build_tree.argtypes = [cd, ci, cd, cd, cd, ci, ci, _POINT_FN, _POINT_FN, vp, ci, vp,
                                       C.POINTER(C.c_int)]
    L.ls_panels_destroy.argtypes = [vp]
    L.ls_panels_destroy.restype = None
    for name in ("ls_panels_setup", "ls_panels_apply", "ls_panels_moments", "ls_panels_info", "ls_panels_solve",
                 "ls_panels_setup_leaves", "ls_panels_precond_setup", "ls_panels_precond_apply",
                 "ls_panels_precond_info", "ls_panels_build_tree"):
        getattr(L, name).restype = C.c_int
    for name in ("ls_setup", "ls_matvec", "ls_apply_V", "ls_precond_apply", "ls_precond_apply_noalloc",
                 "ls_rhs_planewave", "ls_solve",
                 "ls_stats", "ls_plan_describe", "ls_profile_enable", "ls_profile_read", "ls_profile_read_each",
                 "ls_green_table",
                 "ls_solve_queue", "ls_autotune"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _targets(t):
    import torch
    if t.dtype != torch.float64 or t.dim() != 2 or t.shape[1] != 2 or not t.is_contiguous() or not t.is_cuda:
        raise ValueError("targets must be a contiguous device float64 tensor of shape [M, 2]")
    return t


def _check(code: int):
    if code != LS_OK:
        raise LsError(code, lib().ls_last_error().decode())


@dataclass
class Options:
    leaf_max: int = 64
    T: float = 16.0
    sign: int = -1
    hodlr_rank: int = 15
    eps_inner: float = 1e-7
    restart: int = 200
    maxit: int = 2000
    prec: int = LS_FP64
    inner_tol: float = 1e-5
    max_refine: int = 10
    build_fp32: int = 1
    hodlr_rank_div: int = 0
    graph_iters: int = 0
    stencil_mfma: int = 1
    pc_bf16: int = 1
    dcgs2: int = 1
    pc_lowp_solves: int = 0
    hodlr_tol: float = 0.0
    fmm_fused: int = 0
    nca_device: int = 1

    def _c(self) -> _Options:
        o = _Options()
        for f in fields(self):
            setattr(o, f.name, getattr(self, f.name))
        return o


def plan_describe(n: int, L: float, kappa: float, options: Options | None = None) -> dict:
    """Quadtree / cone / list summary and the coverage count (host only)."""
    info = _PlanInfo()
    o = (options or Options())._c()
    _check(lib().ls_plan_describe(n, L, kappa, C.byref(o), C.byref(info)))
    lv = info.levels
    return {
        "levels": lv, "leaf_side": info.leaf_side, "top_level": info.top_level,
        "hf": [bool(info.hf[i]) for i in range(lv + 1)], "ndir": [info.ndir[i] for i in range(lv + 1)],
        "il_pairs": [info.il_pairs[i] for i in range(lv + 1)], "max_il": [info.max_il[i] for i in range(lv + 1)],
        "near_pairs": info.near_pairs, "coverage": (info.coverage_min, info.coverage_max),
    }


def green_table(n: int, h: float, kappa: float, stream=None):
    """Device table of V entries for grid offsets, shape (2n-1, 2n-1) complex128 (index da+n-1, db+n-1)."""
    import torch
    out = torch.empty((2 * n - 1, 2 * n - 1), dtype=torch.complex128, device="cuda")
    _check(lib().ls_green_table(n, float(h), float(kappa), out.data_ptr(), _stream(stream)))
    return out


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(int(stream))


def _vec(t, N: int):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError("expected a complex128 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if t.dim() == 1:
        if t.shape[0] != N:
            raise ValueError(f"expected length {N}")
        return 1
    if t.dim() == 2 and t.shape[1] == N:
        return t.shape[0]
    raise ValueError(f"expected shape (N,) or (nrhs, N) with N = {N}")


class Problem:
    """Handle of an ls_setup()-built solver."""

    def __init__(self, points: np.ndarray, q: np.ndarray, kappa: float, tol: float = 1e-10,
                 options: Options | None = None):
        pts = np.ascontiguousarray(points, dtype=np.float64)
        qq = np.ascontiguousarray(q, dtype=np.float64)
        if pts.ndim != 2 or pts.shape[1] != 2 or qq.shape != (pts.shape[0],):
            raise ValueError("points must be (N, 2) and q (N,)")
        self.N = int(pts.shape[0])
        self.options = options or Options()
        o = self.options._c()
        h = C.c_void_p()
        _check(lib().ls_setup(pts.ctypes.data, self.N, qq.ctypes.data, float(kappa), float(tol), C.byref(o),
                              C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().ls_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _out(self, x, y):
        import torch
        return torch.empty_like(x) if y is None else y

    def matvec(self, x, y=None, prec: int = LS_FP64, stream=None):
        nrhs = _vec(x, self.N)
        y = self._out(x, y)
        _vec(y, self.N)
        _check(lib().ls_matvec(self._h, x.data_ptr(), y.data_ptr(), nrhs, self.N, prec, _stream(stream)))
        return y

    def apply_V(self, x, y=None, prec: int = LS_FP64, stream=None):
        nrhs = _vec(x, self.N)
        y = self._out(x, y)
        _check(lib().ls_apply_V(self._h, x.data_ptr(), y.data_ptr(), nrhs, self.N, prec, _stream(stream)))
        return y

    def precond_apply(self, r, z=None, prec: int = LS_FP64, stream=None):
        nrhs = _vec(r, self.N)
        z = self._out(r, z)
        _check(lib().ls_precond_apply(self._h, r.data_ptr(), z.data_ptr(), nrhs, self.N, prec, _stream(stream)))
        return z

    def precond_apply_noalloc(self, r, z, prec: int = LS_FP64, stream=None):
        """ls_precond_apply_noalloc: z must be given (the call allocates nothing)."""
        nrhs = _vec(r, self.N)
        if _vec(z, self.N) != nrhs:
            raise ValueError("z must have the shape of r")
        _check(lib().ls_precond_apply_noalloc(self._h, r.data_ptr(), z.data_ptr(), nrhs, self.N, prec,
                                              _stream(stream)))
        return z

    def field_eval(self, targets, psi, stream=None):
        """(V psi)(x_t) at arbitrary points: targets a device float64 tensor [M, 2], psi a device
        complex128 vector of N in the caller's point order; returns complex128 [M]."""
        import torch
        tg = _targets(targets)
        if _vec(psi, self.N) != 1:
            raise ValueError("psi must be one vector of length N")
        u = torch.empty(tg.shape[0], dtype=torch.complex128, device=tg.device)
        _check(lib().ls_field_eval(self._h, tg.data_ptr(), tg.shape[0], psi.data_ptr(), u.data_ptr(), _stream(stream)))
        return u

    def error_eval(self, targets, q_t, theta: float, psi, stream=None):
        """E(x_t) of Eq. (eq:error): q_t = q(x_t) (device float64 [M]); returns float64 [M]."""
        import torch
        tg = _targets(targets)
        if q_t.dtype != torch.float64 or not q_t.is_contiguous() or q_t.numel() != tg.shape[0] or not q_t.is_cuda:
            raise ValueError("q_t must be a contiguous device float64 tensor with one value per target")
        if _vec(psi, self.N) != 1:
            raise ValueError("psi must be one vector of length N")
        E = torch.empty(tg.shape[0], dtype=torch.float64, device=tg.device)
        _check(lib().ls_error_eval(self._h, tg.data_ptr(), tg.shape[0], q_t.data_ptr(), float(theta),
                                   psi.data_ptr(), E.data_ptr(), _stream(stream)))
        return E

    def rhs_planewave(self, angles, stream=None):
        import torch
        ang = np.ascontiguousarray(np.atleast_1d(np.asarray(angles, dtype=np.float64)))
        nrhs = ang.shape[0]
        f = torch.empty((nrhs, self.N) if nrhs > 1 else (self.N,), dtype=torch.complex128, device="cuda")
        _check(lib().ls_rhs_planewave(self._h, ang.ctypes.data, nrhs, f.data_ptr(), self.N, _stream(stream)))
        return f

    def solve(self, f, psi=None, tol: float = 1e-8, x0: bool = False, prec: int = -1, stream=None):
        import torch
        nrhs = _vec(f, self.N)
        if psi is None:
            psi = torch.zeros_like(f)
        infos = (_Info * nrhs)()
        _check(lib().ls_solve(self._h, f.data_ptr(), psi.data_ptr(), nrhs, self.N, float(tol), int(bool(x0)),
                              int(prec), infos, _stream(stream)))
        out = [{"iters": i.iters, "relres": i.relres, "status": STATUS.get(i.status, str(i.status)),
                "n_refine": i.n_refine, "t_solve_ms": i.t_solve_ms,
                "relres0": i.relres0} for i in infos]
        return psi, out

    def direct_solve(self, f, psi=None, tol: float = 1e-8, max_refine: int = 10, stream=None):
        """HODLR direct solve with FP64 iterative refinement (ls_direct_solve)."""
        import torch
        nrhs = _vec(f, self.N)
        if psi is None:
            psi = torch.zeros_like(f)
        infos = (_Info * nrhs)()
        _check(lib().ls_direct_solve(self._h, f.data_ptr(), psi.data_ptr(), nrhs, self.N, float(tol),
                                     int(max_refine), infos, _stream(stream)))
        out = [{"iters": i.iters, "relres": i.relres, "status": STATUS.get(i.status, str(i.status)),
                "n_refine": i.n_refine, "t_solve_ms": i.t_solve_ms} for i in infos]
        return psi, out

    def autotune(self, stream=None) -> dict:
        t = _TuneInfo()
        _check(lib().ls_autotune(self._h, C.byref(t), _stream(stream)))
        return {"gs_rows": t.gs_rows, "hodlr_rows": t.hodlr_rows, "gs_us": list(t.gs_us), "pc_us": list(t.pc_us)}

    def stats(self) -> dict:
        s = _Stats()
        _check(lib().ls_stats(self._h, C.byref(s)))
        return {f[0]: (list(getattr(s, f[0])) if isinstance(getattr(s, f[0]), C.Array) else getattr(s, f[0]))
                for f in _Stats._fields_}

    def profile_enable(self, cls: str, every: int = 1):
        """Time every `every`-th launch of a kernel class (0 or False: stop)."""
        _check(lib().ls_profile_enable(self._h, _prof_index(cls), int(every)))

    def profile_read_each(self, cls: str):
        """[(ms, tag)] of the timed launches of a class in launch order (tag: HODLR level or -1)"""
        n = C.c_int64()
        _check(lib().ls_profile_read_each(self._h, _prof_index(cls), None, None, 0, C.byref(n)))
        ms = (C.c_double * max(n.value, 1))()
        tg = (C.c_int * max(n.value, 1))()
        _check(lib().ls_profile_read_each(self._h, _prof_index(cls), ms, tg, n.value, C.byref(n)))
        return [(ms[i], tg[i]) for i in range(n.value)]

    def profile_read(self, cls: str):
        """(summed ms of the timed launches, timed launches, all launches since enabling)"""
        ms = C.c_double()
        n = C.c_int64()
        a = C.c_int64()
        _check(lib().ls_profile_read(self._h, _prof_index(cls), C.byref(ms), C.byref(n), C.byref(a)))
        return ms.value, n.value, a.value



class NeuralOperator:
    """Handle of the learned warm-start network (ls_nop_*).  Tensors are float32 CUDA tensors."""

    def __init__(self, n: int, width: int = 32, modes: int = 16, layers: int = 4, batch_max: int = 16,
                 seed: int = 0, bf16: bool = False):
        cfg = _NopConfig(n, width, modes, layers, batch_max, seed, int(bool(bf16)))
        h = C.c_void_p()
        _check(lib().ls_nop_create(C.byref(cfg), C.byref(h)))
        self._h = h
        self.n, self.width, self.modes, self.layers, self.batch_max = n, width, modes, layers, batch_max
        self.bf16 = bool(bf16)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().ls_nop_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nparams(self) -> int:
        return int(lib().ls_nop_param_count(self._h))

    def get_params(self) -> np.ndarray:
        out = np.empty(self.nparams, dtype=np.float32)
        _check(lib().ls_nop_get_params(self._h, out.ctypes.data, out.size))
        return out

    def set_params(self, flat: np.ndarray):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        _check(lib().ls_nop_set_params(self._h, a.ctypes.data, a.size))

    def get_grads(self) -> np.ndarray:
        out = np.empty(self.nparams, dtype=np.float32)
        _check(lib().ls_nop_get_grads(self._h, out.ctypes.data, out.size))
        return out

    def forward(self, X, O=None, stream=None):
        import torch
        B = X.shape[0]
        if O is None:
            O = torch.empty((B, 2, self.n, self.n), dtype=torch.float32, device=X.device)
        _check(lib().ls_nop_forward(self._h, X.data_ptr(), O.data_ptr(), B, _stream(stream)))
        return O

    def backward(self, dO, stream=None):
        _check(lib().ls_nop_backward(self._h, dO.data_ptr(), _stream(stream)))

    def loss(self, O, w, t, snorm2, stream=None):
        """w, t: complex64 [B, n, n] (w = f/kappa^2, t = (psi - f)/kappa^2); snorm2: float32 [B]."""
        import torch
        B = O.shape[0]
        dO = torch.empty_like(O)
        lb = torch.empty(B, dtype=torch.float32, device=O.device)
        _check(lib().ls_nop_loss(self._h, O.data_ptr(), w.data_ptr(), t.data_ptr(), snorm2.data_ptr(), B,
                                 dO.data_ptr(), lb.data_ptr(), _stream(stream)))
        return lb, dO

    def adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream=None):
        _check(lib().ls_nop_adam_step(self._h, lr, beta1, beta2, eps, _stream(stream)))


def nop_features(n: int, L: float, q_dev, kappa: float, theta: float, X=None, stream=None):
    """6-channel input image of one problem (q_dev: float64 CUDA tensor of n*n values, grid order)."""
    import torch
    if X is None:
        X = torch.empty((6, n, n), dtype=torch.float32, device=q_dev.device)
    _check(lib().ls_nop_features(n, float(L), q_dev.data_ptr(), float(kappa), float(theta), X.data_ptr(),
                                 _stream(stream)))
    return X


def nop_warmstart(n: int, L: float, q_dev, kappa: float, theta: float, O, f, psi0=None, stream=None):
    """psi0 = f exp(i phi) (1 + O_re + i O_im) for one problem (grid order); O=None gives the
    WKB start f exp(i phi) alone."""
    import torch
    if psi0 is None:
        psi0 = torch.empty_like(f)
    _check(lib().ls_nop_warmstart(n, float(L), q_dev.data_ptr(), float(kappa), float(theta),
                                  None if O is None else O.data_ptr(), f.data_ptr(), psi0.data_ptr(),
                                  _stream(stream)))
    return psi0


def _info_dict(i) -> dict:
    return {"iters": i.iters, "relres": i.relres, "status": STATUS.get(i.status, str(i.status)),
            "n_refine": i.n_refine, "t_solve_ms": i.t_solve_ms, "relres0": i.relres0}


def solve_queue(problems, fs, tol: float = 1e-8, prec: int = -1, nworkers: int = 0, graph_iters: int = 0):
    """ls_solve_queue: one right-hand side per problem (complex128 CUDA tensors of N_p entries);
    returns the solutions and one info dict per problem."""
    import torch
    n = len(problems)
    if len(fs) != n:
        raise ValueError("one right-hand side per problem")
    psis = [torch.zeros_like(f) for f in fs]
    for P, f in zip(problems, fs):
        if f.dtype != torch.complex128 or not f.is_cuda or f.numel() != P.N or not f.is_contiguous():
            raise ValueError("right-hand sides must be contiguous complex128 CUDA tensors of N entries")
    hs = (C.c_void_p * n)(*[P._h.value for P in problems])
    fp = (C.c_void_p * n)(*[f.data_ptr() for f in fs])
    pp = (C.c_void_p * n)(*[p.data_ptr() for p in psis])
    infos = (_Info * n)()
    _check(lib().ls_solve_queue(hs, n, fp, pp, float(tol), int(prec), int(nworkers), int(graph_iters), infos))
    return psis, [_info_dict(i) for i in infos]


_POINT_FN = C.CFUNCTYPE(None, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                       C.POINTER(C.c_double), C.c_void_p)


def build_tree(q_fn, uinc_fn, p: int, eps_grid: float, kappa: float, T: float = 16.0, L: float = 1.0,
               max_level: int = 6, min_level: int = 1) -> np.ndarray:
    """ls_panels_build_tree: the adaptive, level-restricted quadtree's leaves, array (nboxes, 4) of
    (centre x, centre y, half-width, level).  q_fn, uinc_fn take coordinate arrays (x, y) and
    return values (an exception becomes NaN values, which the library rejects)."""
    def wrap(fn):
        def cb(n, x, y, re, im, ctx):
            try:
                xs = np.ctypeslib.as_array(x, shape=(n,)).copy()
                ys = np.ctypeslib.as_array(y, shape=(n,)).copy()
                v = np.broadcast_to(np.asarray(fn(xs, ys), dtype=np.complex128), (n,))
                np.ctypeslib.as_array(re, shape=(n,))[:] = v.real
                np.ctypeslib.as_array(im, shape=(n,))[:] = v.imag
            except Exception:
                np.ctypeslib.as_array(re, shape=(n,))[:] = np.nan
        return _POINT_FN(cb)

    cq, cu = wrap(q_fn), wrap(uinc_fn)
    cap = 4096
    while True:
        out = np.empty((cap, 4))
        n = C.c_int(0)
        code = lib().ls_panels_build_tree(float(L), int(p), float(kappa), float(eps_grid), float(T), int(min_level),
                                          int(max_level), cq, cu, None, cap, out.ctypes.data, C.byref(n))
        if code == LS_EINVAL and n.value > cap:
            cap = n.value
            continue
        _check(code)
        return out[:n.value].copy()


class Panels:
    """Handle of an ls_panels_setup()-built high-order panel operator on a uniform tree (nside x
    nside boxes of [-L, L]^2, p x p Chebyshev nodes per box; unknowns box-major, node-minor)."""

    def __init__(self, nside: int, L: float, p: int, kappa: float, q: np.ndarray, sign: int = -1, boxes=None):
        """boxes (optional, array nboxes x 3 of centre x, centre y, half-width): the leaves of any
        tree (ls_panels_setup_leaves); nside and L are then ignored"""
        q = np.ascontiguousarray(q, dtype=np.float64)
        nb = nside * nside if boxes is None else len(boxes)
        if q.shape != (nb * p * p,):
            raise ValueError("q must hold one value per node")
        self._h = C.c_void_p()
        if boxes is None:
            _check(lib().ls_panels_setup(int(nside), float(L), int(p), float(kappa), q.ctypes.data, int(sign),
                                         C.byref(self._h)))
        else:
            bx = np.ascontiguousarray(boxes, dtype=np.float64).reshape(-1, 3)
            _check(lib().ls_panels_setup_leaves(len(bx), bx.ctypes.data, int(p), float(kappa), q.ctypes.data,
                                                int(sign), C.byref(self._h)))
        n, npb, nf = C.c_int64(), C.c_int(), C.c_int()
        _check(lib().ls_panels_info(self._h, C.byref(n), C.byref(npb), C.byref(nf)))
        self.N, self.np, self.nfar = n.value, npb.value, nf.value
        self.nside, self.p = nside, p

    def apply(self, x, y=None, op: int = 0, stream=None):
        """op 0: y = A x; op 1: y = V x (complex128 CUDA tensors, shape (N,) or (nrhs, N))"""
        import torch
        nrhs = _vec(x, self.N)
        y = torch.empty_like(x) if y is None else y
        _check(lib().ls_panels_apply(self._h, x.data_ptr(), y.data_ptr(), nrhs, self.N, int(op), _stream(stream)))
        return y

    def solve(self, f, tol: float = 1e-10, restart: int = 200, maxit: int = 2000, stream=None):
        """ls_panels_solve: psi = A^-1 f (complex128 CUDA tensor of N entries) and the info dict"""
        import torch
        if _vec(f, self.N) != 1:
            raise ValueError("one right-hand side")
        psi = torch.empty_like(f)
        info = _Info()
        _check(lib().ls_panels_solve(self._h, f.data_ptr(), psi.data_ptr(), float(tol), int(restart), int(maxit),
                                     C.byref(info), _stream(stream)))
        return psi, _info_dict(info)

    def precondition(self, rank: int) -> dict:
        """ls_panels_precond_setup (rank <= 0 drops the factors); returns ls_panels_precond_info"""
        _check(lib().ls_panels_precond_setup(self._h, int(rank)))
        return self.precond_info()

    def precond_info(self) -> dict:
        r, lf, lv, mx = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        mr, ms = C.c_double(), C.c_double()
        _check(lib().ls_panels_precond_info(self._h, C.byref(r), C.byref(lf), C.byref(lv), C.byref(mr), C.byref(mx),
                                            C.byref(ms)))
        return {"rank": r.value, "leaf": lf.value, "levels": lv.value, "mean_rank": mr.value,
                "max_rank": mx.value, "setup_ms": ms.value}

    def precond_apply(self, r, z=None, stream=None):
        """z = A~^-1 r (complex128 CUDA tensors, shape (N,) or (nrhs, N), box-major order)"""
        import torch
        nrhs = _vec(r, self.N)
        z = torch.empty_like(r) if z is None else z
        _check(lib().ls_panels_precond_apply(self._h, r.data_ptr(), z.data_ptr(), nrhs, self.N, _stream(stream)))
        return z

    def moments(self, dx: int, dy: int) -> np.ndarray:
        """M_l(node a of the target box, source box) for box offset (dx, dy): array (p^2, N_p)"""
        out = np.empty((self.p * self.p, self.np), dtype=np.complex128)
        _check(lib().ls_panels_moments(self._h, int(dx), int(dy), out.ctypes.data))
        return out

    def close(self):
        if self._h:
            lib().ls_panels_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
