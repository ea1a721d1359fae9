// C ABI of libls: vector entry points (products, preconditioner, solves, right-hand sides,
// field evaluation) and the launch timers; the other entry points live in api_setup.cpp and
// api_queue.cpp.
#include "api_internal.h"

namespace ls {
void set_last_error(const std::string& msg) { lsi::g_last_error = msg; }
}  // namespace ls

namespace lsi {

thread_local std::string g_last_error;

// ---------------------------------------------------------------------------------------
// Device scratch of the allocation-free preconditioner apply: a fixed array in the code object
// (one copy per GPU, allocated when the library's code is loaded there, kept until the process
// ends).  Host code never passes the array's name to a kernel: its device address is looked up
// once per device with hipGetSymbolAddress and only that address is used.
// ---------------------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(64) << 20;


}  // namespace lsi

static __device__ __align__(256) unsigned char scratch[lsi::kScratchBytes];

namespace lsi {

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_dev;  // per device ordinal: device address of `scratch`, or null

// device address of the scratch array on the current device (looked up once per device)
void* scratch_address(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_dev.size() <= device) g_scratch_dev.resize(device + 1, nullptr);
  if (!g_scratch_dev[device]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      throw LsError(LS_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[device] = ptr;
  }
  return g_scratch_dev[device];
}

inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }


static void check_vec_args(ls_problem* P, const void* x, const void* y, int nrhs, int64_t ld) {
  if (!P) throw LsError(LS_EINVAL, "problem is NULL");
  if (!x || !y) throw LsError(LS_EINVAL, "vector pointer is NULL");
  if (nrhs <= 0) throw LsError(LS_EINVAL, "nrhs must be positive");
  if (ld < P->N) throw LsError(LS_EINVAL, "ld must be >= N");
}


static void ensure_ws(ls_problem* P, int nrhs) {
  if (P->ws_cap >= nrhs) return;
  P->w_x.alloc((size_t)P->N * nrhs * 16);
  P->w_y.alloc((size_t)P->N * nrhs * 16);
  P->w_t.alloc((size_t)P->N * nrhs * 16);
  P->ws_cap = nrhs;
}


// ls_solve's body; graph_iters > 0 selects the graph-captured GMRES driver
void solve_impl(ls_problem* P, const void* f, void* psi, int nrhs, int64_t ld, double tol, int x0_given,
                       int prec_override, ls_solve_info* info, hipStream_t stream, int graph_iters) {
  {
    double t0 = now_ms();
    check_vec_args(P, f, psi, nrhs, ld);
    if (!(tol > 0 && tol < 1)) throw LsError(LS_EINVAL, "tol must be in (0, 1)");
    hipStream_t s = (hipStream_t)stream;
    const long long N = P->N;
    if (prec_override < -1 || prec_override > 2) throw LsError(LS_EINVAL, "prec must be -1, LS_FP64, LS_FP32 or LS_MIXED");
    const int prec = prec_override >= 0 ? prec_override : P->opt.prec;
    if ((prec == LS_FP32 || prec == LS_MIXED) && !P->have32) throw LsError(LS_ENOTSUP, "FP32 operator not built");
    P->kf.ensure((size_t)N * nrhs * 16);
    P->kx.ensure((size_t)N * nrhs * 16);
    P->kdx.ensure((size_t)N * nrhs * 16);
    double2* fm = P->kf.as<double2>();
    double2* xm = P->kx.as<double2>();
    double2* dm = P->kdx.as<double2>();
    lsk::launch_permute((const double2*)f, ld, fm, N, P->m2c.as<int>(), N, nrhs, false, s);
    std::vector<double> fn;
    norms(P, fm, nrhs, fn, s);
    std::vector<ColState> st(nrhs);
    std::vector<int> warm_rejected(nrhs, 0);
    for (int c = 0; c < nrhs; ++c) {
      st[c].fnorm = fn[c] > 0 ? fn[c] : 1.0;
      st[c].tol = tol;
    }
    std::vector<double> rel0(nrhs, 1.0);
    if (x0_given) {
      lsk::launch_permute((const double2*)psi, ld, xm, N, P->m2c.as<int>(), N, nrhs, false, s);
      // minimal-residual scaling of the guess g: x0 = xi g, xi = (A g)^H f / ||A g||^2, which
      // leaves ||f - A x0||^2 = ||f||^2 - |(A g)^H f|^2 / ||A g||^2
      ensure_ws(P, nrhs);
      double2* w = P->w_y.as<double2>();
      op_apply(P, false, xm, w, nrhs, s);
      std::vector<double> an;
      norms(P, w, nrhs, an, s);
      const int nch = nchunks_for(P);
      P->kpart.ensure((size_t)nrhs * nch * 16);
      P->kh.ensure((size_t)nrhs * 16);
      double2* part = P->kpart.as<double2>();
      double2* hd = P->kh.as<double2>();
      lsk::launch_gs_dot(w, N, N, 1, fm, N, part, N, nch, 1, nrhs, s);
      lsk::launch_gs_finish(part, nch, 1, 1, hd, 0, nrhs, s);
      std::vector<zd> dot(nrhs);
      hip_check(hipMemcpyAsync(dot.data(), hd, nrhs * 16, hipMemcpyDeviceToHost, s), "dot d2h");
      hip_check(hipStreamSynchronize(s), "sync");
      std::vector<zd> xi(nrhs, zd(0));
      for (int c = 0; c < nrhs; ++c) {
        const double a2 = an[c] * an[c];
        const double drop = a2 > 0 ? std::norm(dot[c]) / a2 : 0.0;
        const bool ok = std::isfinite(a2) && std::isfinite(drop) && a2 > 0 && fn[c] > 0 && drop > 1e-24 * fn[c] * fn[c];
        if (ok) xi[c] = dot[c] / a2;
        warm_rejected[c] = !ok;
      }
      hip_check(hipMemcpyAsync(hd, xi.data(), nrhs * 16, hipMemcpyHostToDevice, s), "xi h2d");
      // starting residual f - xi A g (reported), then x0 = xi g
      lsk::launch_axpby(1.0, fm, N, 0.0, fm, N, dm, N, N, nrhs, s);
      lsk::launch_gs_axpy(w, N, N, 1, hd, 1, -1.0, dm, N, N, nrhs, s);
      std::vector<double> r0;
      norms(P, dm, nrhs, r0, s);
      for (int c = 0; c < nrhs; ++c)
        if (!warm_rejected[c]) rel0[c] = r0[c] / fn[c];
      hip_check(hipMemsetAsync(w, 0, (size_t)N * nrhs * 16, s), "memset");
      lsk::launch_gs_axpy(xm, N, N, 1, hd, 1, 1.0, w, N, N, nrhs, s);
      lsk::launch_axpby(1.0, w, N, 0.0, w, N, xm, N, N, nrhs, s);
      for (int c = 0; c < nrhs; ++c)
        if (warm_rejected[c]) hip_check(hipMemsetAsync(xm + (long long)c * N, 0, N * 16, s), "memset");
    } else {
      hip_check(hipMemsetAsync(xm, 0, (size_t)N * nrhs * 16, s), "memset");
    }
    for (int c = 0; c < nrhs; ++c)
      if (fn[c] == 0) {
        st[c].done = true;
        st[c].status = LS_CONVERGED;
        hip_check(hipMemsetAsync(xm + (long long)c * N, 0, N * 16, s), "memset");
      }
    GmresCfg cfg;
    cfg.restart = P->opt.restart;
    cfg.dcgs2 = P->opt.dcgs2 != 0;
    cfg.maxit = P->opt.maxit;
    cfg.pc = P->have_hodlr;
    std::vector<int> nref(nrhs, 0);
    if (prec == LS_FP64 || prec == LS_FP32) {
      cfg.op32 = prec == LS_FP32;
      cfg.pcf = prec == LS_FP32 ? 1 : 0;
      if (graph_iters > 0)
        gmres_graph(P, cfg, fm, xm, nrhs, st, graph_iters, s);
      else
        gmres(P, cfg, fm, xm, nrhs, st, s);
    } else {
      // mixed: flexible GMRES whose products switch from the FP64 to the FP32 operator once
      // every residual estimate is below tol / delta32 (relaxation of inexact Krylov methods),
      // FP32 off-diagonal HODLR factors throughout; each restart recomputes the true FP64
      // residual f - A x (iterative refinement); after max_refine such cycles, or once a
      // cycle fails to lower the true residual by 10%, the products stay FP64.
      cfg.op32 = false;
      cfg.pcf = P->hod.have16 ? 2 : 1;
      cfg.flexible = true;
      cfg.relax = std::min(0.5, tol / P->opt.inner_tol);
      cfg.max_refine = P->opt.max_refine;
      if (graph_iters > 0)
        gmres_graph(P, cfg, fm, xm, nrhs, st, graph_iters, s);
      else
        gmres(P, cfg, fm, xm, nrhs, st, s);
      for (int c = 0; c < nrhs; ++c) {
        nref[c] = st[c].cycles;
        if (st[c].fell_back && st[c].status == LS_CONVERGED) st[c].status = LS_REFINE_STAGNATED;
      }
    }
    // final true residual with the FP64 operator
    ensure_ws(P, nrhs);
    double2* w = P->w_y.as<double2>();
    op_apply(P, false, xm, w, nrhs, s);
    lsk::launch_axpby(1.0, fm, N, -1.0, w, N, w, N, N, nrhs, s);
    std::vector<double> rn;
    norms(P, w, nrhs, rn, s);
    lsk::launch_permute(xm, N, (double2*)psi, ld, P->m2c.as<int>(), N, nrhs, true, s);
    hip_check(hipStreamSynchronize(s), "solve");
    double t1 = now_ms();
    if (info)
      for (int c = 0; c < nrhs; ++c) {
        info[c].iters = st[c].its;
        info[c].relres = fn[c] > 0 ? rn[c] / fn[c] : 0.0;
        info[c].status = st[c].status;
        if (warm_rejected[c] && st[c].status == LS_CONVERGED) info[c].status = LS_WARMSTART_REJECTED;
        info[c].n_refine = nref[c];
        info[c].t_solve_ms = t1 - t0;
        info[c].relres0 = fn[c] > 0 ? rel0[c] : 0.0;
      }
  }
}

}  // namespace lsi

using namespace lsi;

extern "C" {


ls_status ls_matvec(ls_problem* P, const void* x, void* y, int nrhs, int64_t ld, int prec, void* stream) {
  try {
    check_vec_args(P, x, y, nrhs, ld);
    if (prec != LS_FP64 && prec != LS_FP32 && prec != LS_MIXED)
      throw LsError(LS_EINVAL, "prec must be LS_FP64, LS_FP32 or LS_MIXED");
    if (x == y) throw LsError(LS_EINVAL, "x and y must not overlap");
    fmm_apply(P, prec == LS_FP32, (const double2*)x, ld, (double2*)y, ld, nrhs, 1.0, P->coef, true,
              (hipStream_t)stream);
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}

ls_status ls_apply_V(ls_problem* P, const void* x, void* y, int nrhs, int64_t ld, int prec, void* stream) {
  try {
    check_vec_args(P, x, y, nrhs, ld);
    if (prec != LS_FP64 && prec != LS_FP32 && prec != LS_MIXED)
      throw LsError(LS_EINVAL, "prec must be LS_FP64, LS_FP32 or LS_MIXED");
    if (x == y) throw LsError(LS_EINVAL, "x and y must not overlap");
    // y = V x: the epilogue with alpha = 0, coef = 1 and no contrast
    fmm_apply(P, prec == LS_FP32, (const double2*)x, ld, (double2*)y, ld, nrhs, 0.0, 1.0, true, (hipStream_t)stream,
              false);
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}


ls_status ls_precond_apply(ls_problem* P, const void* r, void* z, int nrhs, int64_t ld, int prec, void* stream) {
  try {
    check_vec_args(P, r, z, nrhs, ld);
    if (prec != LS_FP64 && prec != LS_FP32 && prec != LS_MIXED)
      throw LsError(LS_EINVAL, "prec must be LS_FP64, LS_FP32 or LS_MIXED");
    if (!P->have_hodlr) throw LsError(LS_ENOTSUP, "no HODLR preconditioner (hodlr_rank = 0)");
    hipStream_t s = (hipStream_t)stream;
    ensure_ws(P, nrhs);
    const long long N = P->N;
    double2* a = P->w_x.as<double2>();
    lsk::launch_permute((const double2*)r, ld, a, N, P->m2c.as<int>(), N, nrhs, false, s);
    const int fmt = prec == LS_FP64 ? 0 : (prec == LS_MIXED && P->hod.have16 ? 2 : 1);
    hodlr_apply(P, fmt, a, N, a, N, nrhs, 0, s);
    lsk::launch_permute(a, N, (double2*)z, ld, P->m2c.as<int>(), N, nrhs, true, s);
    hip_check(hipGetLastError(), "precond");
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}

ls_status ls_precond_apply_noalloc(ls_problem* P, const void* r, void* z, int nrhs, int64_t ld, int prec,
                                   void* stream) {
  try {
    check_vec_args(P, r, z, nrhs, ld);
    if (prec != LS_FP64 && prec != LS_FP32 && prec != LS_MIXED)
      throw LsError(LS_EINVAL, "prec must be LS_FP64, LS_FP32 or LS_MIXED");
    if (!P->have_hodlr) throw LsError(LS_ENOTSUP, "no HODLR preconditioner (hodlr_rank = 0)");
    int dev = -1;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (dev != P->device) throw LsError(LS_EINVAL, "the current device is not the problem's device");
    const HodlrDev& H = P->hod;
    const long long N = P->N;
    size_t np = 0, ns = 0;
    hodlr_ws_elems(H, &np, &ns);
    // layout: Morton copy of r (N x nrhs), chunk partials, s vectors; each 256-byte aligned
    const size_t b_vec = align256((size_t)N * nrhs * 16), b_part = align256(np * nrhs * 16),
                 b_svec = align256(ns * nrhs * 16);
    const size_t need = b_vec + b_part + b_svec;
    if (need > kScratchBytes)
      throw LsError(LS_EINVAL, "ls_precond_apply_noalloc: needs " + std::to_string(need) + " bytes of scratch for N = " +
                                   std::to_string(N) + ", nrhs = " + std::to_string(nrhs) + "; the maximum is " +
                                   std::to_string(kScratchBytes));
    char* base = (char*)P->scratch;
    double2* a = (double2*)base;
    HodlrWs ws;
    ws.partial = (double2*)(base + b_vec);
    ws.svec = (double2*)(base + b_vec + b_part);
    ws.timers = false;
    hipStream_t s = (hipStream_t)stream;
    lsk::launch_permute((const double2*)r, ld, a, N, P->m2c.as<int>(), N, nrhs, false, s);
    const int fmt = prec == LS_FP64 ? 0 : (prec == LS_MIXED && H.have16 ? 2 : 1);
    hodlr_apply(P, fmt, a, N, a, N, nrhs, 0, s, nullptr, 0, nullptr, 0, 0, &ws);
    lsk::launch_permute(a, N, (double2*)z, ld, P->m2c.as<int>(), N, nrhs, true, s);
    hip_check(hipGetLastError(), "precond (no allocation)");
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}

ls_status ls_direct_solve(ls_problem* P, const void* f, void* psi, int nrhs, int64_t ld, double tol, int max_refine,
                          ls_solve_info* info, void* stream) {
  try {
    const double t0 = now_ms();
    check_vec_args(P, f, psi, nrhs, ld);
    if (!P->have_hodlr) throw LsError(LS_ENOTSUP, "no HODLR factorisation (hodlr_rank = 0)");
    if (!(tol >= 0 && tol < 1)) throw LsError(LS_EINVAL, "tol must be in [0, 1)");
    if (max_refine < 0) throw LsError(LS_EINVAL, "max_refine must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    const long long N = P->N;
    P->kf.ensure((size_t)N * nrhs * 16);
    P->kx.ensure((size_t)N * nrhs * 16);
    P->kdx.ensure((size_t)N * nrhs * 16);
    ensure_ws(P, nrhs);
    double2* fm = P->kf.as<double2>();
    double2* xm = P->kx.as<double2>();
    double2* dm = P->kdx.as<double2>();
    double2* w = P->w_y.as<double2>();
    lsk::launch_permute((const double2*)f, ld, fm, N, P->m2c.as<int>(), N, nrhs, false, s);
    std::vector<double> fn, rn;
    norms(P, fm, nrhs, fn, s);
    // x = A~^{-1} f, then refinement x += A~^{-1} (f - A x) with FP64 DAFMM products
    hodlr_apply(P, 0, fm, N, xm, N, nrhs, 0, s);
    int steps = 0;
    for (;;) {
      op_apply(P, false, xm, w, nrhs, s);
      lsk::launch_axpby(1.0, fm, N, -1.0, w, N, w, N, N, nrhs, s);
      norms(P, w, nrhs, rn, s);
      bool ok = true;
      for (int c = 0; c < nrhs; ++c) ok &= !(rn[c] > tol * (fn[c] > 0 ? fn[c] : 1.0));
      if (ok || steps >= max_refine) break;
      hodlr_apply(P, 0, w, N, dm, N, nrhs, 0, s);
      lsk::launch_axpby(1.0, xm, N, 1.0, dm, N, xm, N, N, nrhs, s);
      ++steps;
    }
    lsk::launch_permute(xm, N, (double2*)psi, ld, P->m2c.as<int>(), N, nrhs, true, s);
    hip_check(hipStreamSynchronize(s), "direct solve");
    const double t1 = now_ms();
    if (info)
      for (int c = 0; c < nrhs; ++c) {
        const double rel = fn[c] > 0 ? rn[c] / fn[c] : 0.0;
        info[c].iters = steps;
        info[c].relres = rel;
        info[c].status = !std::isfinite(rel) ? LS_NAN : (rel <= tol ? LS_CONVERGED : LS_MAXIT);
        info[c].n_refine = steps;
        info[c].t_solve_ms = t1 - t0;
        info[c].relres0 = 1.0;
      }
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}

ls_status ls_rhs_planewave(ls_problem* P, const double* angles, int nrhs, void* f, int64_t ld, void* stream) {
  try {
    if (!P || !angles || !f) throw LsError(LS_EINVAL, "NULL argument");
    if (nrhs <= 0) throw LsError(LS_EINVAL, "nrhs must be positive");
    if (ld < P->N) throw LsError(LS_EINVAL, "ld must be >= N");
    for (int i = 0; i < nrhs; ++i)
      if (!std::isfinite(angles[i])) throw LsError(LS_EINVAL, "non-finite angle");
    hipStream_t s = (hipStream_t)stream;
    DevBuf ang;
    ang.upload(std::vector<double>(angles, angles + nrhs));
    lsk::launch_planewave(P->px.as<double>(), P->py.as<double>(), P->q_c.as<double>(), ang.as<double>(), P->kappa,
                          -P->coef, (double2*)f, ld, P->N, nrhs, s);
    hip_check(hipStreamSynchronize(s), "planewave");
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}


ls_status ls_solve(ls_problem* P, const void* f, void* psi, int nrhs, int64_t ld, double tol, int x0_given,
                   int prec_override, ls_solve_info* info, void* stream) {
  try {
    if (!P) throw LsError(LS_EINVAL, "NULL problem");
    solve_impl(P, f, psi, nrhs, ld, tol, x0_given, prec_override, info, (hipStream_t)stream, P->opt.graph_iters);
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}


namespace {

// Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on P_n
void gauss_legendre(int n, double* t, double* w) {
  for (int i = 0; i < n; ++i) {
    double x = std::cos(lsk::kPi * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    t[i] = x;
    w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
}

const lsk::FieldRules& field_rules() {
  static lsk::FieldRules R = [] {
    lsk::FieldRules r{};
    const int orders[lsk::kFieldRules] = {3, 4, 5, 6, 8, 10, 12, 16, 24, 10};
    int off = 0;
    for (int k = 0; k < lsk::kFieldRules; ++k) {
      r.off[k] = off;
      r.n[k] = orders[k];
      gauss_legendre(orders[k], r.t + off, r.w + off);
      off += orders[k];
    }
    return r;
  }();
  return R;
}

void field_impl(ls_problem* P, const double* targets, int64_t M, const void* psi, int mode, const double* q_t,
                double theta, void* u, double* E, void* stream) {
  if (!P) throw LsError(LS_EINVAL, "NULL problem");
  if (M < 0) throw LsError(LS_EINVAL, "M must be >= 0");
  if (M == 0) return;
  if (!targets || !psi || (mode == 0 && !u) || (mode == 1 && (!q_t || !E)))
    throw LsError(LS_EINVAL, "NULL buffer");
  if (!std::isfinite(theta)) throw LsError(LS_EINVAL, "theta must be finite");
  if (M > (int64_t)INT32_MAX) throw LsError(LS_EINVAL, "too many targets");
  lsk::launch_field_eval(targets, M, P->n, P->gx0, P->gy0, P->gh, P->kappa, psi, P->g2c.as<int>(), field_rules(),
                         mode, q_t, theta, (double)P->opt.sign, u, E, (hipStream_t)stream);
  hip_check(hipGetLastError(), "field kernel");
}

}  // namespace

ls_status ls_field_eval(ls_problem* P, const double* targets, int64_t M, const void* psi, void* u, void* stream) {
  try {
    field_impl(P, targets, M, psi, 0, nullptr, 0.0, u, nullptr, stream);
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}

ls_status ls_error_eval(ls_problem* P, const double* targets, int64_t M, const double* q_t, double theta,
                        const void* psi, double* E, void* stream) {
  try {
    field_impl(P, targets, M, psi, 1, q_t, theta, nullptr, E, stream);
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}

ls_status ls_green_table(int n, double h, double kappa, void* out, void* stream) {
  try {
    if (n < 1 || !(h > 0) || !std::isfinite(h)) throw LsError(LS_EINVAL, "n must be >= 1 and h > 0");
    if (!(kappa > 0) || !std::isfinite(kappa)) throw LsError(LS_EINVAL, "kappa must be positive and finite");
    if (!out) throw LsError(LS_EINVAL, "out is NULL");
    if (kappa * h * 0.7072 >= 4.0) throw LsError(LS_ENOTSUP, "kappa * h too large for the self-cell series");
    hipStream_t s = (hipStream_t)stream;
    lsk::launch_wtable((double2*)out, n, h, kappa, s);
    hip_check(hipGetLastError(), "wtable");
    zd w0 = self_cell(h, kappa);
    double2 v = make_double2(w0.real(), w0.imag());
    hip_check(hipMemcpyAsync((double2*)out + (size_t)(n - 1) * (2 * n - 1) + (n - 1), &v, 16, hipMemcpyHostToDevice, s),
              "w0");
    hip_check(hipStreamSynchronize(s), "sync");
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}


ls_status ls_profile_enable(ls_problem* P, int cls, int every) {
  if (!P || cls < 0 || cls >= kProfClasses || every < 0) {
    g_last_error = "bad arguments";
    return LS_EINVAL;
  }
  ProfileClass& pc = P->prof[cls];
  pc.enabled = every != 0;
  if (every) {
    pc.every = every;
    pc.used = 0;
    pc.count = 0;
  }
  return LS_OK;
}

ls_status ls_profile_read_each(ls_problem* P, int cls, double* ms, int* tags, int64_t cap, int64_t* n) {
  try {
    if (!P || cls < 0 || cls >= kProfClasses || cap < 0 || (cap > 0 && (!ms || !tags)) || !n)
      throw LsError(LS_EINVAL, "bad arguments");
    ProfileClass& pc = P->prof[cls];
    const size_t m = std::min(pc.used, (size_t)cap);
    for (size_t i = 0; i < m; ++i) {
      hip_check(hipEventSynchronize(pc.ev[i].second), "event sync");
      float t = 0;
      hip_check(hipEventElapsedTime(&t, pc.ev[i].first, pc.ev[i].second), "elapsed");
      ms[i] = t;
      tags[i] = i < pc.tag.size() ? pc.tag[i] : -1;
    }
    *n = (int64_t)pc.used;
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}

ls_status ls_profile_read(ls_problem* P, int cls, double* total_ms, int64_t* launches, int64_t* all_launches) {
  try {
    if (!P || cls < 0 || cls >= kProfClasses || !total_ms || !launches) throw LsError(LS_EINVAL, "bad arguments");
    ProfileClass& pc = P->prof[cls];
    double tot = 0;
    for (size_t i = 0; i < pc.used; ++i) {
      hip_check(hipEventSynchronize(pc.ev[i].second), "event sync");
      float ms = 0;
      hip_check(hipEventElapsedTime(&ms, pc.ev[i].first, pc.ev[i].second), "elapsed");
      tot += ms;
    }
    *total_ms = tot;
    *launches = (int64_t)pc.used;
    if (all_launches) *all_launches = pc.count;
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}

}  // extern "C"
