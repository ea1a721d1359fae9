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
  lsi::DevBuf ref, far_x, far_w, qdag, M, T, q;
  lsi::DevBuf part;  // partial planes of the matrix-core product (one stream at a time)
  bool mfma = true;
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
  const int64_t N = (int64_t)P->g.nside * P->g.nside * P->g.n2;
  if (nrhs < 1 || ld < N) throw LsError(LS_EINVAL, "nrhs must be >= 1 and ld >= the number of unknowns");
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
    // reference data: nodes (first kind, ascending), basis by total degree then first index,
    // Gauss-Legendre rules on [0, 1] along the ray and across the triangles
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
    std::vector<double> fx, fw;
    gauss_legendre(g.nfar, fx, fw);
    // Q (n2 x np): Q[i][l] = b_l(node i); its columns are orthogonal at the Chebyshev points of the
    // first kind (discrete orthogonality of T_0..T_{p-1}), so Qdag = (Q^T Q)^-1 Q^T is the
    // transpose scaled by the diagonal of Q^T Q
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
    P->far_x.upload(fx);
    P->far_w.upload(fw);
    P->qdag.upload(Qd);
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

ls_status ls_panels_apply(ls_panels* P, const void* x, void* y, int nrhs, int64_t ld, int op, void* stream) {
  try {
    check_vec(P, x, y, nrhs, ld);
    if (op != 0 && op != 1) throw LsError(LS_EINVAL, "op must be 0 (A) or 1 (V)");
    if (x == y) throw LsError(LS_EINVAL, "x and y must not overlap");
    const double k2 = P->g.kappa * P->g.kappa;
    const double* q = op == 0 ? P->q.as<double>() : nullptr;
    const double alpha = op == 0 ? 1.0 : 0.0, coef = op == 0 ? P->sign * k2 : 1.0;
    if (P->mfma && P->g.p <= lsp::kMfmaMaxP) {
      const int nc = lsp::panel_chunks(P->g, nrhs);
      const int64_t N = (int64_t)P->g.nside * P->g.nside * P->g.n2;
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

ls_status ls_panels_moments(const ls_panels* P, int dx, int dy, double* out) {
  try {
    if (!P || !out) throw LsError(LS_EINVAL, "handle or out is NULL");
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
  *n_unknowns = (int64_t)P->g.nside * P->g.nside * P->g.n2;
  *np = P->g.np;
  *nfar = P->g.nfar;
  return LS_OK;
}

void ls_panels_destroy(ls_panels* P) { delete P; }

}  // extern "C"
