// High-order leaf panels (paper, Section 2.2, Eqs. (eq:7)-(eq:13)) on a uniform tree: the C ABI
// (ls_panels_*).  The host forms the Chebyshev nodes, the basis, the interpolation matrix Q and
// its pseudo-inverse, and the Gauss-Legendre rules; the device forms the moment tables, the
// operator blocks and the products (panels.hip).
#include <algorithm>
#include <cmath>
#include <memory>
#include <vector>

#include "api_internal.h"
#include "panels.h"

struct ls_panels {
  lsp::PanelGeom g{};
  double L = 1.0;
  int sign = -1;
  int64_t N = 0;       // unknowns
  bool dense = false;  // leaves of a general tree: the dense V instead of per-offset blocks
  int nboxes = 0;
  lsi::DevBuf V, X, boxes;
  lsi::DevBuf ref, far_x, far_w, qdag, M, T, q;
  lsi::DevBuf part;  // partial planes of the matrix-core product (one stream at a time)
  bool mfma = true;
  lsi::DevBuf kq, kw, kr, kpart, kc;  // GMRES basis, work vectors, dot partials, coefficients
};

namespace {



// n-point Gauss-Legendre rule on [-1, 1]: Newton's method on P_n from the Chebyshev-like
// initial guesses, weights 2 / ((1 - x^2) P_n'(x)^2)
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double pn = n == 1 ? z : p1, pm = n == 1 ? 1.0 : p0;
      dp = n * (z * pn - pm) / (z * z - 1.0);
      const double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double pn = n == 1 ? z : p1, pm = n == 1 ? 1.0 : p0;
      dp = n * (z * pn - pm) / (z * z - 1.0);
    }
    x[n - 1 - i] = z;  // ascending
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

double cheb(int n, double x) {
  double t0 = 1.0, t1 = x;
  if (n == 0) return t0;
  for (int k = 1; k < n; ++k) {
    const double t2 = 2.0 * x * t1 - t0;
    t0 = t1;
    t1 = t2;
  }
  return t1;
}

void check_vec(const ls_panels* P, const void* x, const void* y, int nrhs, int64_t ld) {
  if (!P) throw LsError(LS_EINVAL, "panels handle is NULL");
  if (!x || !y) throw LsError(LS_EINVAL, "x or y is NULL");
  const int64_t N = P->N;
  if (nrhs < 1 || ld < N) throw LsError(LS_EINVAL, "nrhs must be >= 1 and ld >= the number of unknowns");
}

// Chebyshev nodes (first kind, ascending), the basis (by total degree, then first index) and
// the Gauss-Legendre rules on [0, 1] along the ray and across the triangles; uploads them with
// Qdag = (Q^T Q)^-1 Q^T.  Q (n2 x np): Q[i][l] = b_l(node i); its columns are orthogonal at the
// Chebyshev points of the first kind (discrete orthogonality of T_0..T_{p-1}), so Qdag is the
// transpose scaled by the diagonal of Q^T Q.
lsp::PanelRef reference_data(ls_panels* P) {
  const lsp::PanelGeom& g = P->g;
  const int p = g.p;
  lsp::PanelRef R{};
  for (int i = 0; i < p; ++i) R.node[i] = std::cos((2.0 * (p - 1 - i) + 1.0) * M_PI / (2.0 * p));
  int l = 0;
  for (int dgr = 0; dgr < p; ++dgr)
    for (int a = 0; a <= dgr; ++a, ++l) {
      R.ba[l] = a;
      R.bb[l] = dgr - a;
    }
  std::vector<double> gx, gw;
  gauss_legendre(lsp::kRay, gx, gw);
  for (int i = 0; i < lsp::kRay; ++i) {
    R.ray_t[i] = 0.5 * (gx[i] + 1.0);
    R.ray_w[i] = 0.5 * gw[i];
  }
  gauss_legendre(lsp::kAcross, gx, gw);
  for (int i = 0; i < lsp::kAcross; ++i) {
    R.acr_t[i] = 0.5 * (gx[i] + 1.0);
    R.acr_w[i] = 0.5 * gw[i];
  }
  const int n2 = g.n2, np = g.np;
  std::vector<double> Q((size_t)n2 * np), Qd((size_t)np * n2);
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j)
      for (int k = 0; k < np; ++k) Q[(size_t)(i * p + j) * np + k] = cheb(R.ba[k], R.node[i]) * cheb(R.bb[k], R.node[j]);
  for (int k = 0; k < np; ++k) {
    double dkk = 0;
    for (int i = 0; i < n2; ++i) dkk += Q[(size_t)i * np + k] * Q[(size_t)i * np + k];
    for (int k2 = 0; k2 < np; ++k2) {
      if (k2 == k) continue;
      double off = 0;
      for (int i = 0; i < n2; ++i) off += Q[(size_t)i * np + k] * Q[(size_t)i * np + k2];
      if (std::fabs(off) > 1e-12 * dkk) throw LsError(LS_ENOTSUP, "interpolation matrix without orthogonal columns");
    }
    for (int i = 0; i < n2; ++i) Qd[(size_t)k * n2 + i] = Q[(size_t)i * np + k] / dkk;
  }
  P->ref.alloc(sizeof(R));
  lsi::hip_check(hipMemcpy(P->ref.p, &R, sizeof(R), hipMemcpyHostToDevice), "panels ref");
  P->qdag.upload(Qd);
  return R;
}

}  // namespace

extern "C" {

ls_status ls_panels_setup(int nside, double L, int p, double kappa, const double* q, int sign, ls_panels** out) {
  try {
    if (!out) throw LsError(LS_EINVAL, "out is NULL");
    *out = nullptr;
    if (nside < 1 || nside > 1024) throw LsError(LS_EINVAL, "nside must be in 1..1024");
    if (p < 1 || p > lsp::kMaxP) throw LsError(LS_EINVAL, "p must be in 1..8");
    if (!(L > 0) || !std::isfinite(L)) throw LsError(LS_EINVAL, "L must be positive and finite");
    if (!(kappa > 0) || !std::isfinite(kappa)) throw LsError(LS_EINVAL, "kappa must be positive and finite");
    if (sign != 1 && sign != -1) throw LsError(LS_EINVAL, "sign must be +1 or -1");
    if (!q) throw LsError(LS_EINVAL, "q is NULL");
    const int64_t N = (int64_t)nside * nside * p * p;
    for (int64_t i = 0; i < N; ++i)
      if (!std::isfinite(q[i])) throw LsError(LS_EINVAL, "q has a non-finite value");
    const int w2 = 2 * nside - 1;
    if ((double)w2 * w2 * p * p * p * p * 16.0 > 64e9) throw LsError(LS_ENOTSUP, "operator table above 64 GB");
    auto P = std::make_unique<ls_panels>();
    lsp::PanelGeom& g = P->g;
    g.nside = nside;
    g.p = p;
    g.np = p * (p + 1) / 2;
    g.n2 = p * p;
    g.beta = L / nside;
    g.kappa = kappa;
    g.nfar = std::max(16, (int)std::ceil(2.0 * kappa * g.beta) + 12);
    P->L = L;
    P->sign = sign;
    P->N = N;
    const int n2 = g.n2, np = g.np;
    reference_data(P.get());
    std::vector<double> fx, fw;
    gauss_legendre(g.nfar, fx, fw);
    P->far_x.upload(fx);
    P->far_w.upload(fw);
    std::vector<double> qv(q, q + N);
    P->q.upload(qv);
    const size_t noff = (size_t)w2 * w2;
    P->M.alloc(noff * n2 * np * 16);
    P->T.alloc(noff * n2 * n2 * 16);
    hipStream_t s = nullptr;
    lsp::launch_panel_moments(g, P->ref.as<lsp::PanelRef>(), P->far_x.as<double>(), P->far_w.as<double>(),
                              P->M.as<double2>(), s);
    lsi::hip_check(hipGetLastError(), "panel moments");
    lsp::launch_panel_blocks(g, P->M.as<double2>(), P->qdag.as<double>(), P->T.as<double2>(), s);
    lsi::hip_check(hipGetLastError(), "panel blocks");
    lsi::hip_check(hipDeviceSynchronize(), "panels setup");
    *out = P.release();
    return LS_OK;
  } catch (const LsError& e) {
    return lsi::fail(e);
  }
}

ls_status ls_panels_setup_leaves(int nboxes, const double* boxes, int p, double kappa, const double* q, int sign,
                                 ls_panels** out) {
  try {
    if (!out) throw LsError(LS_EINVAL, "out is NULL");
    *out = nullptr;
    if (nboxes < 1 || !boxes) throw LsError(LS_EINVAL, "nboxes must be >= 1 and boxes not NULL");
    if (p < 1 || p > lsp::kMaxP) throw LsError(LS_EINVAL, "p must be in 1..8");
    if (!(kappa > 0) || !std::isfinite(kappa)) throw LsError(LS_EINVAL, "kappa must be positive and finite");
    if (sign != 1 && sign != -1) throw LsError(LS_EINVAL, "sign must be +1 or -1");
    if (!q) throw LsError(LS_EINVAL, "q is NULL");
    const int64_t N = (int64_t)nboxes * p * p;
    if (N > lsp::kDenseMaxN) throw LsError(LS_ENOTSUP, "more unknowns than the dense operator takes (20000)");
    for (int B = 0; B < nboxes; ++B)
      if (!std::isfinite(boxes[3 * B]) || !std::isfinite(boxes[3 * B + 1]) || !(boxes[3 * B + 2] > 0) ||
          !std::isfinite(boxes[3 * B + 2]))
        throw LsError(LS_EINVAL, "box centres must be finite and half-widths positive");
    for (int64_t i = 0; i < N; ++i)
      if (!std::isfinite(q[i])) throw LsError(LS_EINVAL, "q has a non-finite value");
    auto P = std::make_unique<ls_panels>();
    lsp::PanelGeom& g = P->g;
    g.nside = 0;
    g.p = p;
    g.np = p * (p + 1) / 2;
    g.n2 = p * p;
    g.kappa = kappa;
    g.beta = 0;
    g.nfar = 0;
    P->sign = sign;
    P->N = N;
    P->dense = true;
    P->nboxes = nboxes;
    const lsp::PanelRef R = reference_data(P.get());
    // per box: its far rule (one Gauss-Legendre rule per distinct point count) and its nodes
    std::vector<double> fx, fw, bx((size_t)5 * nboxes);
    std::vector<double2> X((size_t)N);
    std::vector<int> rule_n;
    std::vector<size_t> rule_off;
    for (int B = 0; B < nboxes; ++B) {
      const double cx = boxes[3 * B], cy = boxes[3 * B + 1], be = boxes[3 * B + 2];
      const int nf = std::max(16, (int)std::ceil(2.0 * kappa * be) + 12);
      size_t r = 0;
      while (r < rule_n.size() && rule_n[r] != nf) ++r;
      if (r == rule_n.size()) {
        std::vector<double> x1, w1;
        gauss_legendre(nf, x1, w1);
        rule_n.push_back(nf);
        rule_off.push_back(fx.size());
        fx.insert(fx.end(), x1.begin(), x1.end());
        fw.insert(fw.end(), w1.begin(), w1.end());
      }
      g.nfar = std::max(g.nfar, nf);
      bx[5 * B] = cx;
      bx[5 * B + 1] = cy;
      bx[5 * B + 2] = be;
      bx[5 * B + 3] = (double)rule_off[r];
      bx[5 * B + 4] = (double)nf;
      for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j)
          X[(size_t)B * g.n2 + i * p + j] = make_double2(cx + be * R.node[i], cy + be * R.node[j]);
    }
    P->far_x.upload(fx);
    P->far_w.upload(fw);
    P->boxes.upload(bx);
    P->X.upload(X);
    std::vector<double> qv(q, q + N);
    P->q.upload(qv);
    P->M.alloc((size_t)N * nboxes * g.np * 16);
    P->V.alloc((size_t)N * N * 16);
    hipStream_t s = nullptr;
    lsp::launch_panel_moments_leaves(P->ref.as<lsp::PanelRef>(), p, g.np, kappa, P->boxes.as<double>(), nboxes,
                                     P->X.as<double2>(), N, P->far_x.as<double>(), P->far_w.as<double>(),
                                     P->M.as<double2>(), s);
    lsi::hip_check(hipGetLastError(), "panel moments (leaves)");
    lsp::launch_panel_dense_V(P->M.as<double2>(), P->qdag.as<double>(), nboxes, g.np, g.n2, P->V.as<double2>(), s);
    lsi::hip_check(hipGetLastError(), "panel dense V");
    lsi::hip_check(hipDeviceSynchronize(), "panels setup (leaves)");
    *out = P.release();
    return LS_OK;
  } catch (const LsError& e) {
    return lsi::fail(e);
  }
}

ls_status ls_panels_apply(ls_panels* P, const void* x, void* y, int nrhs, int64_t ld, int op, void* stream) {
  try {
    check_vec(P, x, y, nrhs, ld);
    if (op != 0 && op != 1) throw LsError(LS_EINVAL, "op must be 0 (A) or 1 (V)");
    if (x == y) throw LsError(LS_EINVAL, "x and y must not overlap");
    const double k2 = P->g.kappa * P->g.kappa;
    const double* q = op == 0 ? P->q.as<double>() : nullptr;
    const double alpha = op == 0 ? 1.0 : 0.0, coef = op == 0 ? P->sign * k2 : 1.0;
    if (P->dense) {
      lsp::launch_panel_dense_apply(P->V.as<double2>(), P->N, q, (const double2*)x, ld, (double2*)y, ld, nrhs, alpha,
                                    coef, (hipStream_t)stream);
    } else if (P->mfma && P->g.p <= lsp::kMfmaMaxP) {
      const int nc = lsp::panel_chunks(P->g, nrhs);
      const int64_t N = P->N;
      P->part.ensure((size_t)nc * nrhs * N * 16);
      lsp::launch_panel_apply_mfma(P->g, P->T.as<double2>(), q, (const double2*)x, ld, (double2*)y, ld, nrhs, alpha,
                                   coef, P->part.as<double2>(), nc, (hipStream_t)stream);
    } else {
      lsp::launch_panel_apply(P->g, P->T.as<double2>(), q, (const double2*)x, ld, (double2*)y, ld, nrhs, alpha,
                              coef, (hipStream_t)stream);
    }
    lsi::hip_check(hipGetLastError(), "panel apply");
    return LS_OK;
  } catch (const LsError& e) {
    return lsi::fail(e);
  }
}

// Restarted GMRES (Section 6 without the preconditioner) on A psi = f from psi = 0: classical
// Gram-Schmidt with one reorthogonalisation, Givens rotations and the triangular solve on the
// host, every vector operation on the device; each restart (and the end) recomputes the true
// residual f - A psi.
ls_status ls_panels_solve(ls_panels* P, const void* f, void* psi, double tol, int restart, int maxit,
                          ls_solve_info* info, void* stream) {
  try {
    if (!P || !f || !psi || !info) throw LsError(LS_EINVAL, "handle, f, psi or info is NULL");
    if (!(tol > 0 && tol < 1)) throw LsError(LS_EINVAL, "tol must be in (0, 1)");
    if (restart < 1 || restart > 2000 || maxit < 1) throw LsError(LS_EINVAL, "restart in 1..2000 and maxit >= 1");
    if (f == psi) throw LsError(LS_EINVAL, "f and psi must not overlap");
    const double t0 = lsi::now_ms();
    hipStream_t s = (hipStream_t)stream;
    const long long N = P->N;
    const int m = restart;
    const int nch = (int)std::max(1LL, std::min(1024LL, (N + 4095) / 4096));
    P->kq.ensure((size_t)(m + 1) * N * 16);
    P->kw.ensure((size_t)N * 16);
    P->kr.ensure((size_t)N * 16);
    P->kpart.ensure((size_t)(m + 1) * nch * 16);
    P->kc.ensure((size_t)(m + 1) * 16);
    double2* Q = P->kq.as<double2>();
    double2* w = P->kw.as<double2>();
    double2* r = P->kr.as<double2>();
    double2* x = (double2*)psi;
    const double2* fd = (const double2*)f;
    std::vector<double2> hp((size_t)(m + 1) * nch);
    // Q_0..Q_{nvec-1} (or v itself) against v, chunks added in order
    auto dots = [&](const double2* base, int nvec, const double2* v, std::vector<zd>& out) {
      lsp::launch_panel_dots(base, N, nvec, v, N, P->kpart.as<double2>(), nch, s);
      lsi::hip_check(hipMemcpyAsync(hp.data(), P->kpart.p, (size_t)nvec * nch * 16, hipMemcpyDeviceToHost, s), "dots");
      lsi::hip_check(hipStreamSynchronize(s), "dots");
      out.assign(nvec, zd(0));
      for (int i = 0; i < nvec; ++i)
        for (int c = 0; c < nch; ++c) out[i] += zd(hp[(size_t)i * nch + c].x, hp[(size_t)i * nch + c].y);
    };
    auto norm = [&](const double2* v) {
      std::vector<zd> d;
      dots(v, 1, v, d);
      return std::sqrt(std::max(d[0].real(), 0.0));
    };
    // w -= sum_i c_i Q_i (c on the host)
    std::vector<double2> ch(m + 1);
    auto update = [&](double2* v, int nvec, const std::vector<zd>& c, double sgn) {
      for (int i = 0; i < nvec; ++i) ch[i] = make_double2(sgn * c[i].real(), sgn * c[i].imag());
      lsi::hip_check(hipMemcpy(P->kc.p, ch.data(), (size_t)nvec * 16, hipMemcpyHostToDevice), "coefficients");
      lsp::launch_panel_update(v, Q, N, nvec, P->kc.as<double2>(), N, s);
    };
    const double k2 = P->g.kappa * P->g.kappa;
    auto applyA = [&](const double2* in, double2* out) {
      if (P->dense) {
        lsp::launch_panel_dense_apply(P->V.as<double2>(), N, P->q.as<double>(), in, N, out, N, 1, 1.0, P->sign * k2,
                                      s);
      } else if (P->mfma && P->g.p <= lsp::kMfmaMaxP) {
        const int nc = lsp::panel_chunks(P->g, 1);
        P->part.ensure((size_t)nc * N * 16);
        lsp::launch_panel_apply_mfma(P->g, P->T.as<double2>(), P->q.as<double>(), in, N, out, N, 1, 1.0,
                                     P->sign * k2, P->part.as<double2>(), nc, s);
      } else {
        lsp::launch_panel_apply(P->g, P->T.as<double2>(), P->q.as<double>(), in, N, out, N, 1, 1.0, P->sign * k2, s);
      }
    };
    lsp::launch_panel_combo(x, fd, 0.0, fd, 0.0, N, s);  // x0 = 0
    lsp::launch_panel_combo(r, fd, 1.0, fd, 0.0, N, s);  // r0 = f
    const double fnorm = norm(fd);
    info->iters = 0;
    info->n_refine = 0;
    info->relres0 = 1.0;
    info->relres = 0.0;
    info->status = LS_CONVERGED;
    if (!(fnorm > 0)) {
      if (!std::isfinite(fnorm)) info->status = LS_NAN;
      info->t_solve_ms = lsi::now_ms() - t0;
      return LS_OK;
    }
    std::vector<zd> H((size_t)(m + 1) * m), g(m + 1), sn(m), h, h2;
    std::vector<double> cs(m);
    int it = 0;
    for (;;) {
      const double beta = norm(r);
      const double rel = beta / fnorm;
      info->relres = rel;
      if (!std::isfinite(rel)) {
        info->status = LS_NAN;
        break;
      }
      if (rel <= tol) {
        info->status = LS_CONVERGED;
        break;
      }
      if (it >= maxit) {
        info->status = LS_MAXIT;
        break;
      }
      info->n_refine += 1;
      lsp::launch_panel_combo(Q, r, 1.0 / beta, r, 0.0, N, s);
      std::fill(H.begin(), H.end(), zd(0));
      std::fill(g.begin(), g.end(), zd(0));
      g[0] = beta;
      int k = 0;
      for (int j = 0; j < m && it < maxit; ++j) {
        applyA(Q + (size_t)j * N, w);
        ++it;
        dots(Q, j + 1, w, h);
        update(w, j + 1, h, 1.0);
        dots(Q, j + 1, w, h2);
        update(w, j + 1, h2, 1.0);
        for (int i = 0; i <= j; ++i) h[i] += h2[i];
        const double hn = norm(w);
        if (hn > 0) lsp::launch_panel_combo(Q + (size_t)(j + 1) * N, w, 1.0 / hn, w, 0.0, N, s);
        // rotations of the previous columns, then the one that removes the subdiagonal entry
        zd hj1 = hn;
        for (int i = 0; i < j; ++i) {
          const zd a = h[i], b = h[i + 1];
          h[i] = cs[i] * a + sn[i] * b;
          h[i + 1] = -std::conj(sn[i]) * a + cs[i] * b;
        }
        const zd a = h[j];
        const double rho = std::sqrt(std::norm(a) + std::norm(hj1));
        if (rho == 0) {
          cs[j] = 1.0;
          sn[j] = 0.0;
        } else if (std::abs(a) == 0) {
          cs[j] = 0.0;
          sn[j] = std::conj(hj1) / rho;
        } else {
          cs[j] = std::abs(a) / rho;
          sn[j] = (a / std::abs(a)) * std::conj(hj1) / rho;
        }
        h[j] = cs[j] * a + sn[j] * hj1;
        for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h[i];
        g[j + 1] = -std::conj(sn[j]) * g[j];
        g[j] = cs[j] * g[j];
        k = j + 1;
        if (std::abs(g[j + 1]) <= tol * fnorm || hn == 0) break;
      }
      // psi += Q y with R y = g
      std::vector<zd> y(k);
      for (int i = k - 1; i >= 0; --i) {
        zd acc = g[i];
        for (int jj = i + 1; jj < k; ++jj) acc -= H[(size_t)i * m + jj] * y[jj];
        y[i] = acc / H[(size_t)i * m + i];
      }
      update(x, k, y, -1.0);
      applyA(x, w);
      lsp::launch_panel_combo(r, fd, 1.0, w, -1.0, N, s);
    }
    info->iters = it;
    lsi::hip_check(hipGetLastError(), "panel solve");
    lsi::hip_check(hipStreamSynchronize(s), "panel solve");
    info->t_solve_ms = lsi::now_ms() - t0;
    return LS_OK;
  } catch (const LsError& e) {
    return lsi::fail(e);
  }
}

ls_status ls_panels_moments(const ls_panels* P, int dx, int dy, double* out) {
  try {
    if (!P || !out) throw LsError(LS_EINVAL, "handle or out is NULL");
    if (P->dense) throw LsError(LS_ENOTSUP, "moment table rows exist for uniform trees only");
    const int n = P->g.nside;
    if (dx <= -n || dx >= n || dy <= -n || dy >= n) throw LsError(LS_EINVAL, "box offset outside the grid");
    const size_t row = (size_t)P->g.n2 * P->g.np;
    const size_t d = (size_t)(dx + n - 1) * (2 * n - 1) + (dy + n - 1);
    lsi::hip_check(hipMemcpy(out, P->M.as<double2>() + d * row, row * 16, hipMemcpyDeviceToHost), "moments d2h");
    return LS_OK;
  } catch (const LsError& e) {
    return lsi::fail(e);
  }
}

ls_status ls_panels_info(const ls_panels* P, int64_t* n_unknowns, int* np, int* nfar) {
  if (!P || !n_unknowns || !np || !nfar) {
    lsi::g_last_error = "bad arguments";
    return LS_EINVAL;
  }
  *n_unknowns = P->N;
  *np = P->g.np;
  *nfar = P->g.nfar;
  return LS_OK;
}

void ls_panels_destroy(ls_panels* P) { delete P; }

}  // extern "C"
