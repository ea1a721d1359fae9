// GMRES of libls (Section 6): host-driven restarted / flexible GMRES and the device-driven
// Arnoldi steps replayed from captured HIP graphs.
#include "api_internal.h"

namespace lsi {

// ---------------------------------------------------------------------------------------
// GMRES (Section 6): restarted, right-preconditioned, classical Gram-Schmidt with one
// reorthogonalisation, Givens rotations on the host.  All vectors in Morton order.
// ---------------------------------------------------------------------------------------
void op_apply(ls_problem* P, bool op32, const double2* x, double2* y, int nrhs, hipStream_t s) {
  fmm_apply(P, op32, x, P->N, y, P->N, nrhs, 1.0, P->coef, false, s);
}

// z (ld N) = M^{-1} x (ld ldx)
void pc_apply(ls_problem* P, const GmresCfg& cfg, const double2* x, long long ldx, double2* z, int nrhs,
              hipStream_t s) {
  if (cfg.pc)
    hodlr_apply(P, cfg.pcf, x, ldx, z, P->N, nrhs, 0, s);
  else
    lsk::launch_axpby(1.0, x, ldx, 0.0, x, ldx, z, P->N, P->N, nrhs, s);
}

// row chunks of the Arnoldi reductions (rows per chunk chosen by ls_autotune, default 1024)
int nchunks_for(const ls_problem* P) {
  const long long rows = std::max(1, P->tune.gs_rows);
  return (int)std::max<long long>(1, std::min<long long>(1024, (P->N + rows - 1) / rows));
}

void norms(ls_problem* P, const double2* v, int nrhs, std::vector<double>& out, hipStream_t s) {
  const long long N = P->N;
  int nch = nchunks_for(P);
  P->knp.ensure((size_t)nch * nrhs * 8);
  P->kno.ensure((size_t)nrhs * 8);
  lsk::launch_norm2(v, N, P->knp.as<double>(), N, nch, nrhs, s);
  lsk::launch_norm2_finish(P->knp.as<double>(), nch, P->kno.as<double>(), nrhs, s);
  out.resize(nrhs);
  hip_check(hipMemcpyAsync(out.data(), P->kno.p, nrhs * 8, hipMemcpyDeviceToHost, s), "norm d2h");
  hip_check(hipStreamSynchronize(s), "sync");
  for (auto& x : out) x = std::sqrt(x);
}

// Solve op(A) x = f (Morton order, ld = N) from the x given; per-column tolerances.
void gmres(ls_problem* P, const GmresCfg& cfg, const double2* f, double2* x, int nrhs, std::vector<ColState>& st,
           hipStream_t s) {
  const long long N = P->N;
  const int m = std::max(1, cfg.restart);
  const int maxv = m + 1;
  const int nch = nchunks_for(P);
  P->kQ.ensure((size_t)nrhs * maxv * N * 16);
  P->kw.ensure((size_t)nrhs * N * 16);
  P->kz.ensure((size_t)nrhs * N * 16);
  P->kr.ensure((size_t)nrhs * N * 16);
  P->kh.ensure((size_t)nrhs * maxv * 16);
  P->kpart.ensure((size_t)nrhs * nch * maxv * 16);
  P->kalpha.ensure((size_t)nrhs * 8);
  P->ky.ensure((size_t)nrhs * maxv * 16);
  if (cfg.flexible) P->kZ.ensure((size_t)nrhs * m * N * 16);
  double2* Q = P->kQ.as<double2>();
  double2* Zb = cfg.flexible ? P->kZ.as<double2>() : nullptr;
  const long long ldzr = (long long)m * N;
  double2* w = P->kw.as<double2>();
  double2* z = P->kz.as<double2>();
  double2* r = P->kr.as<double2>();
  double2* hd = P->kh.as<double2>();
  double2* part = P->kpart.as<double2>();
  const long long ldqv = N, ldqr = (long long)maxv * N;
  std::vector<std::vector<zd>> H(nrhs), g(nrhs), sn(nrhs);
  std::vector<std::vector<double>> cs(nrhs);
  std::vector<double> beta, alpha(nrhs), hnorm;
  std::vector<zd> hh((size_t)nrhs * maxv);
  std::vector<int> kcol(nrhs);
  bool first = true;
  bool relax_enabled = cfg.relax > 0;
  for (;;) {
    bool all_done = true;
    for (int c = 0; c < nrhs; ++c) all_done &= st[c].done;
    if (all_done) return;
    // true residual r = f - A x
    if (first && cfg.x_zero) {
      lsk::launch_axpby(1.0, f, N, 0.0, f, N, r, N, N, nrhs, s);
    } else {
      op_apply(P, cfg.op32, x, w, nrhs, s);
      lsk::launch_axpby(1.0, f, N, -1.0, w, N, r, N, N, nrhs, s);
    }
    first = false;
    norms(P, r, nrhs, beta, s);
    bool any = false;
    for (int c = 0; c < nrhs; ++c) {
      if (st[c].done) continue;
      st[c].relres = beta[c] / st[c].fnorm;
      if (!std::isfinite(beta[c])) {
        st[c].done = true;
        st[c].status = LS_NAN;
      } else if (st[c].relres <= st[c].tol) {
        st[c].done = true;
        st[c].status = LS_CONVERGED;
      } else if (st[c].its >= cfg.maxit) {
        st[c].done = true;
        st[c].status = LS_MAXIT;
      } else {
        any = true;
        st[c].cycles++;
        // FP32 products stopped reducing the true residual, or the refinement budget is spent
        if (relax_enabled && st[c].cycles > 1 &&
            (beta[c] > 0.9 * st[c].prev_true || st[c].cycles > cfg.max_refine)) {
          relax_enabled = false;
          st[c].fell_back = true;
        }
        st[c].prev_true = beta[c];
      }
    }
    if (!any) return;
    std::vector<char> active(nrhs, 0);
    for (int c = 0; c < nrhs; ++c) {
      active[c] = !st[c].done;
      alpha[c] = active[c] ? 1.0 / beta[c] : 0.0;
      H[c].assign((size_t)maxv * m, zd(0));
      g[c].assign(maxv, zd(0));
      g[c][0] = active[c] ? beta[c] : 0.0;
      cs[c].assign(m, 0.0);
      sn[c].assign(m, zd(0));
      kcol[c] = 0;
    }
    hip_check(hipMemcpyAsync(P->kalpha.p, alpha.data(), nrhs * 8, hipMemcpyHostToDevice, s), "alpha");
    lsk::launch_scale(r, N, P->kalpha.as<double>(), Q, ldqr, N, nrhs, s);
    bool relaxed = false;
    for (int j = 0; j < m; ++j) {
      // w = A M^{-1} q_j  (flexible: z_j kept for the update)
      if (cfg.flexible) {
        double2* zj = Zb + (long long)j * N;
        if (cfg.pc)
          hodlr_apply(P, cfg.pcf, Q + (long long)j * ldqv, ldqr, zj, ldzr, nrhs, 0, s);
        else
          lsk::launch_axpby(1.0, Q + (long long)j * ldqv, ldqr, 0.0, Q, ldqr, zj, ldzr, N, nrhs, s);
        fmm_apply(P, cfg.op32 || relaxed, zj, ldzr, w, N, nrhs, 1.0, P->coef, false, s);
      } else {
        pc_apply(P, cfg, Q + (long long)j * ldqv, ldqr, z, nrhs, s);
        op_apply(P, cfg.op32 || relaxed, z, w, nrhs, s);
      }
      // CGS2
      {
        ProfScope ps(P, 3, s);
        lsk::launch_gs_dot(Q, ldqv, ldqr, j + 1, w, N, part, N, nch, maxv, nrhs, s);
      }
      lsk::launch_gs_finish(part, nch, j + 1, maxv, hd, 0, nrhs, s);
      lsk::launch_gs_axpy(Q, ldqv, ldqr, j + 1, hd, maxv, -1.0, w, N, N, nrhs, s);
      lsk::launch_gs_dot(Q, ldqv, ldqr, j + 1, w, N, part, N, nch, maxv, nrhs, s);
      // second pass: store correction in the y buffer, then accumulate into hd
      lsk::launch_gs_finish(part, nch, j + 1, maxv, P->ky.as<double2>(), 0, nrhs, s);
      lsk::launch_gs_axpy(Q, ldqv, ldqr, j + 1, P->ky.as<double2>(), maxv, -1.0, w, N, N, nrhs, s);
      lsk::launch_axpby(1.0, hd, maxv, 1.0, P->ky.as<double2>(), maxv, hd, maxv, j + 1, nrhs, s);
      hip_check(hipMemcpyAsync(hh.data(), hd, (size_t)nrhs * maxv * 16, hipMemcpyDeviceToHost, s), "h d2h");
      norms(P, w, nrhs, hnorm, s);
      bool any_active = false;
      for (int c = 0; c < nrhs; ++c) {
        if (!active[c]) {
          alpha[c] = 0.0;
          continue;
        }
        zd* Hc = H[c].data();
        for (int i = 0; i <= j; ++i) Hc[(size_t)i * m + j] = hh[(size_t)c * maxv + i];
        Hc[(size_t)(j + 1) * m + j] = hnorm[c];
        for (int i = 0; i < j; ++i) {
          zd a = Hc[(size_t)i * m + j], b = Hc[(size_t)(i + 1) * m + j];
          Hc[(size_t)i * m + j] = cs[c][i] * a + sn[c][i] * b;
          Hc[(size_t)(i + 1) * m + j] = -std::conj(sn[c][i]) * a + cs[c][i] * b;
        }
        zd a = Hc[(size_t)j * m + j], b = Hc[(size_t)(j + 1) * m + j];
        double cc;
        zd ss;
        if (b == zd(0)) {
          cc = 1.0;
          ss = 0.0;
        } else if (a == zd(0)) {
          cc = 0.0;
          ss = std::conj(b) / std::abs(b);
        } else {
          double t = std::hypot(std::abs(a), std::abs(b));
          cc = std::abs(a) / t;
          ss = (a / std::abs(a)) * std::conj(b) / t;
        }
        cs[c][j] = cc;
        sn[c][j] = ss;
        Hc[(size_t)j * m + j] = cc * a + ss * b;
        Hc[(size_t)(j + 1) * m + j] = 0.0;
        g[c][j + 1] = -std::conj(ss) * g[c][j];
        g[c][j] = cc * g[c][j];
        st[c].its++;
        kcol[c] = j + 1;
        double est = std::abs(g[c][j + 1]) / st[c].fnorm;
        bool stop = est <= st[c].tol || st[c].its >= cfg.maxit || hnorm[c] == 0.0 || !std::isfinite(est);
        if (est <= st[c].tol) st[c].est_converged = true;
        st[c].last_est = est;
        if (stop) {
          active[c] = 0;
          alpha[c] = 0.0;
        } else {
          alpha[c] = 1.0 / hnorm[c];
          any_active = true;
        }
      }
      if (!any_active || j + 1 == m) break;
      if (relax_enabled && !relaxed) {
        bool all_small = true;
        for (int c = 0; c < nrhs; ++c)
          if (active[c] && st[c].last_est > cfg.relax) all_small = false;
        relaxed = all_small;
      }
      hip_check(hipMemcpyAsync(P->kalpha.p, alpha.data(), nrhs * 8, hipMemcpyHostToDevice, s), "alpha");
      lsk::launch_scale(w, N, P->kalpha.as<double>(), Q + (long long)(j + 1) * ldqv, ldqr, N, nrhs, s);
    }
    // y = R^{-1} g per column, x += M^{-1} (Q y)
    std::vector<zd> y((size_t)nrhs * maxv, zd(0));
    for (int c = 0; c < nrhs; ++c) {
      int k = kcol[c];
      const zd* Hc = H[c].data();
      for (int i = k - 1; i >= 0; --i) {
        zd acc = g[c][i];
        for (int jj = i + 1; jj < k; ++jj) acc -= Hc[(size_t)i * m + jj] * y[(size_t)c * maxv + jj];
        y[(size_t)c * maxv + i] = acc / Hc[(size_t)i * m + i];
      }
    }
    hip_check(hipMemcpyAsync(P->ky.p, y.data(), y.size() * 16, hipMemcpyHostToDevice, s), "y h2d");
    int kmaxc = 0;
    for (int c = 0; c < nrhs; ++c) kmaxc = std::max(kmaxc, kcol[c]);
    if (cfg.flexible) {
      lsk::launch_gs_axpy(Zb, N, ldzr, kmaxc, P->ky.as<double2>(), maxv, 1.0, x, N, N, nrhs, s);
    } else {
      hip_check(hipMemsetAsync(w, 0, (size_t)nrhs * N * 16, s), "memset");
      lsk::launch_gs_axpy(Q, ldqv, ldqr, kmaxc, P->ky.as<double2>(), maxv, 1.0, w, N, N, nrhs, s);
      pc_apply(P, cfg, w, N, z, nrhs, s);
      lsk::launch_axpby(1.0, x, N, 1.0, z, N, x, N, N, nrhs, s);
    }
    hip_check(hipStreamSynchronize(s), "gmres cycle");
    if (cfg.trust_estimate)
      for (int c = 0; c < nrhs; ++c)
        if (!st[c].done && st[c].est_converged) {
          st[c].done = true;
          st[c].status = LS_CONVERGED;
        }
  }
}

// ---------------------------------------------------------------------------------------
// GMRES with device-driven Arnoldi steps, graph_iters of them captured into one HIP graph.
// Same method as gmres() above (right preconditioning, CGS2, Givens, restarts from the true
// residual, flexible variant with precision relaxation); the Arnoldi index, the rotations and
// the stop test live on the device, so the host synchronises once per replay instead of
// once per iteration.  Steps replayed after a column has stopped leave it untouched.
// ---------------------------------------------------------------------------------------
struct KdView {
  long long N;
  int nrhs, m, maxv, nch;
  int *jd, *state, *its, *kfin;
  double *fnorm, *tol, *est, *alpha;
};

KdView kd_view(ls_problem* P, int nrhs, int m) {
  KdView v;
  v.N = P->N;
  v.nrhs = nrhs;
  v.m = m;
  v.maxv = m + 1;
  v.nch = nchunks_for(P);
  int* ic = P->kd.ictl.as<int>();
  v.jd = ic;
  v.state = ic + 1;
  v.its = ic + 1 + nrhs;
  v.kfin = ic + 1 + 2 * nrhs;
  double* dc = P->kd.dctl.as<double>();
  v.fnorm = dc;
  v.tol = dc + nrhs;
  v.est = dc + 2 * nrhs;
  v.alpha = dc + 3 * nrhs;
  return v;
}

void kd_ensure(ls_problem* P, const GmresCfg& cfg, int nrhs) {
  const long long N = P->N;
  const int m = std::max(1, cfg.restart), maxv = m + 1, nch = nchunks_for(P);
  P->kQ.ensure((size_t)nrhs * maxv * N * 16);
  if (cfg.flexible) P->kZ.ensure((size_t)nrhs * (cfg.dcgs2 ? maxv : m) * N * 16);
  P->kw.ensure((size_t)nrhs * N * 16);
  P->kz.ensure((size_t)nrhs * N * 16);
  P->kr.ensure((size_t)nrhs * N * 16);
  P->kpart.ensure((size_t)nrhs * nch * maxv * 16);
  if (cfg.dcgs2) {
    const long long nblk = (N + P->tune.dot2_rows - 1) / P->tune.dot2_rows;
    P->kpart.ensure((size_t)nrhs * (nblk + 1) * 2 * maxv * 16);
    P->kd.Hr.ensure((size_t)nrhs * maxv * maxv * 16);
    P->kd.T.ensure((size_t)nrhs * maxv * maxv * 16);
    P->kd.coef.ensure((size_t)nrhs * 2 * maxv * 16);
  }
  P->knp.ensure((size_t)nch * nrhs * 8);
  P->ky.ensure((size_t)nrhs * maxv * 16);
  P->kalpha.ensure((size_t)nrhs * 8);
  KrylovDev& K = P->kd;
  K.ictl.ensure((size_t)(1 + 3 * nrhs) * 4);
  K.dctl.ensure((size_t)4 * nrhs * 8);
  K.H.ensure((size_t)nrhs * m * maxv * 16);
  K.cs.ensure((size_t)nrhs * m * 8);
  K.sn.ensure((size_t)nrhs * m * 16);
  K.g.ensure((size_t)nrhs * maxv * 16);
  K.vin.ensure((size_t)nrhs * N * 16);
  K.tmp.ensure((size_t)nrhs * maxv * 16);
  const size_t hb = (size_t)(1 + 3 * nrhs) * 4 + 8 + (size_t)nrhs * 8;
  if (K.host_bytes < hb) {
    if (K.host) hip_check(hipHostFree(K.host), "hipHostFree");
    K.host = nullptr;
    K.host_bytes = 0;
    hip_check(hipHostMalloc((void**)&K.host, hb, hipHostMallocDefault), "hipHostMalloc");
    K.host_bytes = hb;
  }
  ensure_fmm_capacity(P, P->f64, nrhs);
  if (P->have32) ensure_fmm_capacity(P, P->f32, nrhs);
  if (P->have_hodlr) hodlr_ensure_ws(P, nrhs);
  if (!K.cap) hip_check(hipStreamCreateWithFlags(&K.cap, hipStreamNonBlocking), "hipStreamCreate");
}

void kd_key_phase(std::vector<uintptr_t>& k, const Phase& ph) {
  k.push_back((uintptr_t)ph.tasks.p);
  k.push_back((uintptr_t)ph.terms.p);
  k.push_back((uintptr_t)ph.blk.p);
  k.push_back((uintptr_t)ph.sk.p);
  k.push_back((uintptr_t)ph.nsk);
}

void kd_key_fmm(std::vector<uintptr_t>& k, const FmmDev& F) {
  for (const DevBuf* b : {&F.ops, &F.mult, &F.loc, &F.xs, &F.ys}) k.push_back((uintptr_t)b->p);
  k.push_back((uintptr_t)F.nrhs_cap);
  for (const Passes* S : {&F.narrow, &F.wide}) {
    kd_key_phase(k, S->p2m);
    kd_key_phase(k, S->nearm2l);
    kd_key_phase(k, S->l2p);
    for (const Phase& ph : S->up) kd_key_phase(k, ph);
    for (const Phase& ph : S->down) kd_key_phase(k, ph);
    k.push_back((uintptr_t)S->io_fold);
  }
  kd_key_phase(k, F.fused);
  for (const DevBuf* b : {&F.fneed, &F.fctr}) k.push_back((uintptr_t)b->p);
  k.push_back((uintptr_t)F.fused_wg);
}

// everything a captured step depends on: sizes, modes and every device address it touches
std::vector<uintptr_t> kd_key(ls_problem* P, const GmresCfg& cfg, bool op32, int nrhs, int steps) {
  std::vector<uintptr_t> k = {(uintptr_t)nrhs, (uintptr_t)cfg.restart, (uintptr_t)steps, (uintptr_t)cfg.flexible,
                              (uintptr_t)cfg.pc, (uintptr_t)cfg.pcf, (uintptr_t)op32, (uintptr_t)cfg.maxit,
                              (uintptr_t)cfg.dcgs2, (uintptr_t)P->tune.gs_rows, (uintptr_t)P->tune.hodlr_rows,
                              (uintptr_t)P->tune.dot2_rows};
  for (const DevBuf* b : {&P->kQ, &P->kZ, &P->kw, &P->kz, &P->kpart, &P->knp, &P->kd.ictl, &P->kd.dctl, &P->kd.H,
                          &P->kd.cs, &P->kd.sn, &P->kd.g, &P->kd.vin, &P->kd.tmp, &P->kd.Hr, &P->kd.T, &P->kd.coef})
    k.push_back((uintptr_t)b->p);
  kd_key_fmm(k, op32 ? P->f32 : P->f64);
  if (P->have_hodlr) {
    k.push_back((uintptr_t)P->hod.partial.p);
    k.push_back((uintptr_t)P->hod.svec.p);
  }
  return k;
}

// one Arnoldi step: q_j -> (z_j) -> w = A M^{-1} q_j, CGS2, Givens, q_{j+1}
void kd_step(ls_problem* P, const GmresCfg& cfg, bool op32, const KdView& v, hipStream_t s) {
  const long long N = v.N;
  const int nrhs = v.nrhs, m = v.m, maxv = v.maxv, nch = v.nch;
  double2* Q = P->kQ.as<double2>();
  const long long ldqv = N, ldqr = (long long)maxv * N;
  double2* w = P->kw.as<double2>();
  double2* z = P->kz.as<double2>();
  double2* vin = P->kd.vin.as<double2>();
  double2* H = P->kd.H.as<double2>();
  double2* part = P->kpart.as<double2>();
  const long long hr = (long long)m * maxv;
  if (cfg.pc) {
    // the leaf solves read q_j straight from the basis (column index on the device)
    // and the last level's update also stores z~_j into Z (flexible)
    hodlr_apply(P, cfg.pcf, Q, ldqr, z, N, nrhs, 0, s, v.jd, ldqv, cfg.flexible ? P->kZ.as<double2>() : nullptr,
                (long long)(cfg.dcgs2 ? maxv : m) * N, N);
  } else {
    lsk::launch_kd_copy(Q, ldqr, ldqv, vin, N, 0, N, v.jd, v.state, nrhs, s);
    lsk::launch_axpby(1.0, vin, N, 0.0, vin, N, z, N, N, nrhs, s);
    if (cfg.flexible)
      lsk::launch_kd_copy(z, N, 0, P->kZ.as<double2>(), (long long)(cfg.dcgs2 ? maxv : m) * N, N, N, v.jd, v.state,
                          nrhs, s);
  }
  fmm_apply(P, op32, z, N, w, N, nrhs, 1.0, P->coef, false, s);
  if (cfg.dcgs2) {
    // delayed CGS2: slot j holds u_j; one pass of inner products, the small O(j^2) update of
    // the Hessenberg column, one pass writing q_j and u_{j+1}
    {
      ProfScope ps(P, 3, s);
      lsk::launch_kd_dot2(Q, ldqv, ldqr, maxv, w, N, part, N, P->tune.dot2_rows, v.jd, v.state, nrhs, s);
    }
    const long long nblk = (N + P->tune.dot2_rows - 1) / P->tune.dot2_rows;
    const double2* cd = part + (long long)nrhs * nblk * 2 * maxv;
    lsk::launch_kd_dcgs2(cd, P->kd.Hr.as<double2>(), H, m, maxv, P->kd.cs.as<double>(), P->kd.sn.as<double2>(),
                         P->kd.g.as<double2>(), P->kd.T.as<double2>(), P->kd.coef.as<double2>(), v.jd, v.state,
                         v.its, v.kfin, v.est, v.fnorm, v.tol, cfg.maxit, v.alpha, nrhs, s);
    lsk::launch_kd_dcgs2_axpy(Q, ldqv, ldqr, w, N, P->kd.coef.as<double2>(), maxv, v.alpha, N, v.jd, v.state, nrhs,
                              s);
    return;
  }
  {
    ProfScope ps(P, 3, s);
    lsk::launch_kd_dot(Q, ldqv, ldqr, maxv, w, N, part, N, nch, v.jd, v.state, nrhs, s);
  }
  lsk::launch_kd_finish(part, nch, maxv, H, hr, maxv, 0, v.jd, v.state, nrhs, s);
  lsk::launch_kd_axpy(Q, ldqv, ldqr, H, hr, maxv, -1.0, w, N, N, v.jd, v.state, nrhs, s);
  lsk::launch_kd_dot(Q, ldqv, ldqr, maxv, w, N, part, N, nch, v.jd, v.state, nrhs, s);
  double2* t = P->kd.tmp.as<double2>();
  lsk::launch_kd_finish(part, nch, maxv, t, maxv, 0, 0, v.jd, v.state, nrhs, s);
  lsk::launch_kd_axpy(Q, ldqv, ldqr, t, maxv, 0, -1.0, w, N, N, v.jd, v.state, nrhs, s);
  lsk::launch_kd_finish(part, nch, maxv, H, hr, maxv, 1, v.jd, v.state, nrhs, s);
  lsk::launch_norm2(w, N, P->knp.as<double>(), N, nch, nrhs, s);
  lsk::launch_kd_givens(P->knp.as<double>(), nch, H, m, maxv, P->kd.cs.as<double>(), P->kd.sn.as<double2>(),
                        P->kd.g.as<double2>(), v.jd, v.state, v.its, v.kfin, v.est, v.fnorm, v.tol, cfg.maxit,
                        v.alpha, nrhs, s);
  lsk::launch_kd_next(w, N, v.alpha, Q, ldqv, ldqr, N, v.jd, v.state, nrhs, s);
}

hipGraphExec_t kd_graph(ls_problem* P, const GmresCfg& cfg, bool op32, const KdView& v, int steps) {
  KrylovDev& K = P->kd;
  const int slot = op32 ? 1 : 0;
  std::vector<uintptr_t> key = kd_key(P, cfg, op32, v.nrhs, steps);
  if (K.exec[slot] && K.key[slot] == key) return K.exec[slot];
  K.drop(slot);
  hipGraph_t g = nullptr;
  hip_check(hipStreamBeginCapture(K.cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  P->capturing = true;
  try {
    for (int i = 0; i < steps; ++i) kd_step(P, cfg, op32, v, K.cap);
  } catch (...) {
    P->capturing = false;
    (void)hipStreamEndCapture(K.cap, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  P->capturing = false;
  hip_check(hipStreamEndCapture(K.cap, &g), "hipStreamEndCapture");
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  hip_check(e, "hipGraphInstantiate");
  K.exec[slot] = ex;
  K.key[slot] = std::move(key);
  return ex;
}

void gmres_graph(ls_problem* P, const GmresCfg& cfg, const double2* f, double2* x, int nrhs,
                 std::vector<ColState>& st, int steps_in, hipStream_t s) {
  const long long N = P->N;
  const int m = std::max(1, cfg.restart);
  const int maxv = m + 1;
  const int steps = std::max(1, steps_in);
  kd_ensure(P, cfg, nrhs);
  const KdView v = kd_view(P, nrhs, m);
  KrylovDev& K = P->kd;
  double2* w = P->kw.as<double2>();
  double2* z = P->kz.as<double2>();
  double2* r = P->kr.as<double2>();
  double2* Q = P->kQ.as<double2>();
  const long long ldqr = (long long)maxv * N;
  std::vector<double> beta;
  std::vector<int> hi(1 + 3 * nrhs);
  std::vector<double> hd(4 * nrhs);
  bool first = true;
  bool timed = false;
  for (const ProfileClass& pc : P->prof) timed |= pc.enabled;
  bool relax_enabled = cfg.relax > 0;
  for (;;) {
    bool all_done = true;
    for (int c = 0; c < nrhs; ++c) all_done &= st[c].done;
    if (all_done) return;
    if (first && cfg.x_zero) {
      lsk::launch_axpby(1.0, f, N, 0.0, f, N, r, N, N, nrhs, s);
    } else {
      op_apply(P, cfg.op32, x, w, nrhs, s);
      lsk::launch_axpby(1.0, f, N, -1.0, w, N, r, N, N, nrhs, s);
    }
    first = false;
    norms(P, r, nrhs, beta, s);
    bool any = false;
    for (int c = 0; c < nrhs; ++c) {
      if (st[c].done) continue;
      st[c].relres = beta[c] / st[c].fnorm;
      if (!std::isfinite(beta[c])) {
        st[c].done = true;
        st[c].status = LS_NAN;
      } else if (st[c].relres <= st[c].tol) {
        st[c].done = true;
        st[c].status = LS_CONVERGED;
      } else if (st[c].its >= cfg.maxit) {
        st[c].done = true;
        st[c].status = LS_MAXIT;
      } else {
        any = true;
        st[c].cycles++;
        // FP32 products stopped reducing the true residual, or the refinement budget is spent
        if (relax_enabled && st[c].cycles > 1 &&
            (beta[c] > 0.9 * st[c].prev_true || st[c].cycles > cfg.max_refine)) {
          relax_enabled = false;
          st[c].fell_back = true;
        }
        st[c].prev_true = beta[c];
      }
    }
    if (!any) return;
    // cycle start on the device: j = 0, g = (beta, 0, ...), q_0 = r / beta
    hi.assign(1 + 3 * nrhs, 0);
    std::vector<zd> g0((size_t)nrhs * maxv, zd(0));
    for (int c = 0; c < nrhs; ++c) {
      const bool act = !st[c].done;
      hi[1 + c] = act ? 0 : 2;
      hi[1 + nrhs + c] = st[c].its;
      hd[c] = st[c].fnorm;
      hd[nrhs + c] = st[c].tol;
      hd[2 * nrhs + c] = 1.0;
      hd[3 * nrhs + c] = act ? 1.0 / beta[c] : 0.0;
      g0[(size_t)c * maxv] = act ? beta[c] : 0.0;
    }
    hip_check(hipMemcpyAsync(K.ictl.p, hi.data(), hi.size() * 4, hipMemcpyHostToDevice, s), "ctl h2d");
    hip_check(hipMemcpyAsync(K.dctl.p, hd.data(), hd.size() * 8, hipMemcpyHostToDevice, s), "ctl h2d");
    hip_check(hipMemcpyAsync(K.g.p, g0.data(), g0.size() * 16, hipMemcpyHostToDevice, s), "g h2d");
    lsk::launch_scale(r, N, v.alpha, Q, ldqr, N, nrhs, s);
    bool relaxed = false;
    std::vector<double> est(nrhs, 1.0);
    for (;;) {
      const bool use32 = cfg.op32 || relaxed;
      if (timed) {
        // kernel timers are on: the same steps enqueued eagerly, so every launch has its events
        for (int i = 0; i < steps; ++i) kd_step(P, cfg, use32, v, s);
      } else {
        hip_check(hipGraphLaunch(kd_graph(P, cfg, use32, v, steps), s), "hipGraphLaunch");
      }
      hip_check(hipMemcpyAsync(K.host, K.ictl.p, (size_t)(1 + 3 * nrhs) * 4, hipMemcpyDeviceToHost, s), "ctl d2h");
      // the estimates into the pinned mirror too (after the control words, 8-byte aligned): a
      // pageable destination would make the copy a staged, blocking one
      double* hest = reinterpret_cast<double*>(reinterpret_cast<char*>(K.host) +
                                               ((size_t)(1 + 3 * nrhs) * 4 + 7) / 8 * 8);
      hip_check(hipMemcpyAsync(hest, v.est, (size_t)nrhs * 8, hipMemcpyDeviceToHost, s), "est d2h");
      hip_check(hipStreamSynchronize(s), "gmres steps");
      for (int c = 0; c < nrhs; ++c) est[c] = hest[c];
      bool active = false;
      for (int c = 0; c < nrhs; ++c) active |= K.host[1 + c] == 0;
      if (!active) break;
      if (relax_enabled && !relaxed) {
        bool all_small = true;
        for (int c = 0; c < nrhs; ++c)
          if (K.host[1 + c] == 0 && est[c] > cfg.relax) all_small = false;
        relaxed = all_small;
      }
    }
    // y = R^{-1} g per column (host), x += Z y (flexible) or x += M^{-1} (Q y)
    std::vector<zd> y((size_t)nrhs * maxv, zd(0));
    int kmaxc = 0;
    std::vector<zd> R, gh(maxv);
    for (int c = 0; c < nrhs; ++c) {
      st[c].its = K.host[1 + nrhs + c];
      st[c].last_est = est[c];
      if (st[c].done) continue;
      const int k = K.host[1 + 2 * nrhs + c];
      if (est[c] <= st[c].tol) st[c].est_converged = true;
      if (k <= 0) continue;
      kmaxc = std::max(kmaxc, k);
      R.resize((size_t)k * maxv);
      hip_check(hipMemcpyAsync(R.data(), K.H.as<double2>() + (size_t)c * m * maxv, (size_t)k * maxv * 16,
                               hipMemcpyDeviceToHost, s),
                "R d2h");
      hip_check(hipMemcpyAsync(gh.data(), K.g.as<double2>() + (size_t)c * maxv, (size_t)maxv * 16,
                               hipMemcpyDeviceToHost, s),
                "g d2h");
      hip_check(hipStreamSynchronize(s), "sync");
      // R column jj holds rows 0..jj at R[jj*maxv + i]
      for (int i = k - 1; i >= 0; --i) {
        zd acc = gh[i];
        for (int jj = i + 1; jj < k; ++jj) acc -= R[(size_t)jj * maxv + i] * y[(size_t)c * maxv + jj];
        y[(size_t)c * maxv + i] = acc / R[(size_t)i * maxv + i];
      }
      if (cfg.dcgs2 && cfg.flexible) {
        // the stored z~ are Z T (T upper triangular, column jj = (c, beta) of step jj):
        // x += Z y = Z~ (T^{-1} y)
        std::vector<zd> Tc((size_t)k * maxv);
        hip_check(hipMemcpyAsync(Tc.data(), P->kd.T.as<double2>() + (size_t)c * maxv * maxv, Tc.size() * 16,
                                 hipMemcpyDeviceToHost, s),
                  "T d2h");
        hip_check(hipStreamSynchronize(s), "sync");
        zd* yc = &y[(size_t)c * maxv];
        for (int i = k - 1; i >= 0; --i) {
          zd acc = yc[i];
          for (int jj = i + 1; jj < k; ++jj) acc -= Tc[(size_t)jj * maxv + i] * yc[jj];
          yc[i] = acc / Tc[(size_t)i * maxv + i];
        }
      }
    }
    if (kmaxc > 0) {
      hip_check(hipMemcpyAsync(P->ky.p, y.data(), y.size() * 16, hipMemcpyHostToDevice, s), "y h2d");
      if (cfg.flexible) {
        lsk::launch_gs_axpy(P->kZ.as<double2>(), N, (long long)(cfg.dcgs2 ? maxv : m) * N, kmaxc,
                            P->ky.as<double2>(), maxv, 1.0, x, N, N, nrhs, s);
      } else {
        hip_check(hipMemsetAsync(w, 0, (size_t)nrhs * N * 16, s), "memset");
        lsk::launch_gs_axpy(Q, N, ldqr, kmaxc, P->ky.as<double2>(), maxv, 1.0, w, N, N, nrhs, s);
        pc_apply(P, cfg, w, N, z, nrhs, s);
        lsk::launch_axpby(1.0, x, N, 1.0, z, N, x, N, N, nrhs, s);
      }
    }
    hip_check(hipStreamSynchronize(s), "gmres cycle");
    if (cfg.trust_estimate)
      for (int c = 0; c < nrhs; ++c)
        if (!st[c].done && st[c].est_converged) {
          st[c].done = true;
          st[c].status = LS_CONVERGED;
        }
  }
}

}  // namespace lsi
