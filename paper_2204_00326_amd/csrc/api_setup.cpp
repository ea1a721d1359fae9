// Setup entry points of libls: default options, option validation, the host plan summary,
// ls_setup (grid, quadtree, NCA, operators, HODLR), statistics and destruction.
#include "api_internal.h"
#include "nca_device.h"

namespace lsi {

// Exact integral of G = (i/4) H0(kappa |y|) over the square cell [-h/2, h/2]^2 (the diagonal
// entry of Eq. (eq:13) at p = 1):  8 int_0^{pi/4} (i/4) [R H1(kappa R)/kappa + 2i/(pi kappa^2)] dtheta,
// R = h / (2 cos theta), by 64-point Gauss-Legendre quadrature in theta.
zd self_cell(double h, double kappa) {
  const int nq = 64;
  std::vector<double> xg(nq), wg(nq);
  for (int i = 0; i < nq; ++i) {  // Gauss-Legendre nodes by Newton iteration on P_nq
    double x = std::cos(lsk::kPi * (i + 0.75) / (nq + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1, p1 = x;
      for (int k = 2; k <= nq; ++k) {
        double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = nq * (x * p1 - p0) / (x * x - 1);
      double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double p0 = 1, p1 = x;
    for (int k = 2; k <= nq; ++k) {
      double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = nq * (x * p1 - p0) / (x * x - 1);
    xg[i] = x;
    wg[i] = 2.0 / ((1 - x * x) * dp * dp);
  }
  zd acc(0);
  for (int i = 0; i < nq; ++i) {
    double th = (xg[i] + 1.0) * (lsk::kPi / 8.0);
    double R = 0.5 * h / std::cos(th);
    lsk::cplx H1 = lsk::hankel1_small(kappa * R);
    zd radial = R * zd(H1.re, H1.im) / kappa + zd(0, 2.0 / (lsk::kPi * kappa * kappa));
    acc += wg[i] * (lsk::kPi / 8.0) * zd(0, 0.25) * radial;
  }
  return 8.0 * acc;
}

}  // namespace lsi

using namespace lsi;

extern "C" {

void ls_default_options(ls_options* o) {
  if (!o) return;
  o->leaf_max = 64;
  o->T = 16.0;
  o->sign = -1;
  o->hodlr_rank = 15;
  o->eps_inner = 1e-7;
  o->restart = 200;
  o->maxit = 2000;
  o->prec = LS_FP64;
  o->inner_tol = 1e-5;
  o->max_refine = 10;
  o->build_fp32 = 1;
  o->hodlr_rank_div = 0;
  o->graph_iters = 0;
  o->stencil_mfma = 1;
  o->fmm_fused = 0;
  o->nca_device = 1;
  o->pc_bf16 = 1;
  o->pc_lowp_solves = 0;
  o->hodlr_tol = 0.0;
  o->dcgs2 = 1;
}

const char* ls_last_error(void) { return g_last_error.c_str(); }

static void validate_options(const ls_options& o) {
  if (o.leaf_max < 1) throw LsError(LS_EINVAL, "leaf_max must be >= 1");
  if (!(o.T > 0) || !std::isfinite(o.T)) throw LsError(LS_EINVAL, "T must be positive");
  if (o.sign != -1 && o.sign != 1) throw LsError(LS_EINVAL, "sign must be -1 or +1");
  if (o.hodlr_rank < 0 || o.hodlr_rank > 256) throw LsError(LS_EINVAL, "hodlr_rank must be in [0, 256]");
  if (o.restart < 1) throw LsError(LS_EINVAL, "restart must be >= 1");
  if (o.maxit < 0) throw LsError(LS_EINVAL, "maxit must be >= 0");
  if (o.prec < 0 || o.prec > 2) throw LsError(LS_EINVAL, "prec must be LS_FP64, LS_FP32 or LS_MIXED");
  if (!(o.inner_tol > 0) || o.inner_tol >= 1) throw LsError(LS_EINVAL, "inner_tol must be in (0, 1)");
  if (o.max_refine < 1) throw LsError(LS_EINVAL, "max_refine must be >= 1");
  if (o.hodlr_rank_div < 0) throw LsError(LS_EINVAL, "hodlr_rank_div must be >= 0");
  if (o.graph_iters < 0 || o.graph_iters > 64) throw LsError(LS_EINVAL, "graph_iters must be in [0, 64]");
  if (o.stencil_mfma != 0 && o.stencil_mfma != 1) throw LsError(LS_EINVAL, "stencil_mfma must be 0 or 1");
  if (o.fmm_fused != 0 && o.fmm_fused != 1) throw LsError(LS_EINVAL, "fmm_fused must be 0 or 1");
  if (o.pc_bf16 != 0 && o.pc_bf16 != 1) throw LsError(LS_EINVAL, "pc_bf16 must be 0 or 1");
  if (o.pc_lowp_solves != 0 && o.pc_lowp_solves != 1) throw LsError(LS_EINVAL, "pc_lowp_solves must be 0 or 1");
  if (!(o.hodlr_tol >= 0 && o.hodlr_tol < 1)) throw LsError(LS_EINVAL, "hodlr_tol must be in [0, 1)");
  if (o.dcgs2 != 0 && o.dcgs2 != 1) throw LsError(LS_EINVAL, "dcgs2 must be 0 or 1");
  if (o.nca_device != 0 && o.nca_device != 1) throw LsError(LS_EINVAL, "nca_device must be 0 or 1");
}

ls_status ls_plan_describe(int n, double L, double kappa, const ls_options* opt, ls_plan_info* out) {
  try {
    if (!out) throw LsError(LS_EINVAL, "out is NULL");
    ls_options o;
    ls_default_options(&o);
    if (opt) o = *opt;
    validate_options(o);
    if (!(L > 0) || !std::isfinite(L)) throw LsError(LS_EINVAL, "L must be positive");
    ls::PlanOptions po;
    po.leaf_max = o.leaf_max;
    po.T = o.T;
    ls::Plan p = ls::make_plan(n, L, kappa, po);
    if (p.leaf >= 32) throw LsError(LS_ENOTSUP, "too many levels");
    std::memset(out, 0, sizeof(*out));
    out->levels = p.leaf;
    out->leaf_side = p.leaf_side;
    out->top_level = p.top;
    for (int nu = 0; nu <= p.leaf; ++nu) {
      out->hf[nu] = p.lv[nu].hf;
      out->ndir[nu] = p.lv[nu].ndir;
      out->il_pairs[nu] = p.lv[nu].il_pairs;
      out->max_il[nu] = p.lv[nu].max_il;
    }
    out->near_pairs = p.near_pairs;
    ls::plan_coverage(p, out->coverage_min, out->coverage_max);
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return LS_EINVAL;
  }
}

ls_status ls_setup(const double* points, int64_t N, const double* q, double kappa, double tol, const ls_options* opt,
                   ls_problem** out) {
  if (out) *out = nullptr;
  std::unique_ptr<ls_problem> P;
  try {
    double t0 = now_ms();
    if (!out) throw LsError(LS_EINVAL, "out is NULL");
    if (!points || !q) throw LsError(LS_EINVAL, "points and q must not be NULL");
    if (N <= 0) throw LsError(LS_EINVAL, "N must be positive");
    if (!(kappa > 0) || !std::isfinite(kappa)) throw LsError(LS_EINVAL, "kappa must be positive and finite");
    if (!(tol > 0 && tol < 1)) throw LsError(LS_EINVAL, "tol must be in (0, 1)");
    P.reset(new ls_problem());
    ls_default_options(&P->opt);
    if (opt) P->opt = *opt;
    validate_options(P->opt);
    for (int64_t i = 0; i < 2 * N; ++i)
      if (!std::isfinite(points[i])) throw LsError(LS_EINVAL, "non-finite point coordinate");
    for (int64_t i = 0; i < N; ++i)
      if (!std::isfinite(q[i])) throw LsError(LS_EINVAL, "non-finite contrast value");
    // ---- recognise the uniform cell-centred grid ----
    int n = (int)std::llround(std::sqrt((double)N));
    if ((int64_t)n * n != N) throw LsError(LS_ENOTSUP, "points do not form a square n x n grid (N not a square)");
    double xmin = points[0], xmax = points[0], ymin = points[1], ymax = points[1];
    for (int64_t i = 0; i < N; ++i) {
      xmin = std::min(xmin, points[2 * i]);
      xmax = std::max(xmax, points[2 * i]);
      ymin = std::min(ymin, points[2 * i + 1]);
      ymax = std::max(ymax, points[2 * i + 1]);
    }
    if (n < 2) throw LsError(LS_ENOTSUP, "grid side must be at least 2");
    double h = (xmax - xmin) / (n - 1);
    if (!(h > 0) || std::fabs((ymax - ymin) / (n - 1) - h) > 1e-9 * h)
      throw LsError(LS_ENOTSUP, "points do not form a square grid with equal spacing");
    std::vector<int> ca(N), cb(N), grid2caller((size_t)N, -1);
    for (int64_t i = 0; i < N; ++i) {
      double fa = (points[2 * i] - xmin) / h, fb = (points[2 * i + 1] - ymin) / h;
      long a = std::lround(fa), b = std::lround(fb);
      if (std::fabs(fa - a) > 1e-6 || std::fabs(fb - b) > 1e-6 || a < 0 || a >= n || b < 0 || b >= n)
        throw LsError(LS_ENOTSUP, "points do not lie on a uniform grid");
      int64_t g = (int64_t)a * n + b;
      if (grid2caller[g] >= 0) throw LsError(LS_EINVAL, "duplicate points");
      grid2caller[g] = (int)i;
      ca[i] = (int)a;
      cb[i] = (int)b;
    }
    P->N = N;
    P->n = n;
    P->gx0 = xmin;
    P->gy0 = ymin;
    P->gh = h;
    // the inputs are valid: from here on the setup works on the current device
    hip_check(hipGetDevice(&P->device), "hipGetDevice");
    P->scratch = scratch_address(P->device);
    P->g2c.upload(grid2caller);
    P->kappa = kappa;
    P->tol = tol;
    P->coef = P->opt.sign * kappa * kappa;
    const double L = 0.5 * n * h;
    ls::PlanOptions po;
    po.leaf_max = P->opt.leaf_max;
    po.T = P->opt.T;
    P->plan = ls::make_plan(n, L, kappa, po);
    const ls::Plan& p = P->plan;
    if (P->opt.hodlr_rank > 0 && p.leaf_side * p.leaf_side > 64)
      throw LsError(LS_ENOTSUP, "the HODLR preconditioner needs quadtree leaves of at most 64 points (leaf_max)");
    double t_plan = now_ms();
    // ---- orders: Morton (solver) and S (DAFMM leaf arrays) ----
    const int side = p.leaf_side, nbL = p.lv[p.leaf].nb, nhL = nbL / 2;
    std::vector<int> mort_a(N), mort_b(N), m2c(N), c2m(N);
    {
      std::vector<std::pair<uint64_t, int>> leaves;
      for (int la = 0; la < nbL; ++la)
        for (int lb = 0; lb < nbL; ++lb) {
          uint64_t code = 0;
          for (int bit = 0; bit < 16; ++bit) {
            code |= (uint64_t)((lb >> bit) & 1) << (2 * bit);
            code |= (uint64_t)((la >> bit) & 1) << (2 * bit + 1);
          }
          leaves.push_back({code, la * nbL + lb});
        }
      std::sort(leaves.begin(), leaves.end());
      int64_t t = 0;
      for (auto& lf : leaves) {
        int la = lf.second / nbL, lb = lf.second % nbL;
        for (int a = 0; a < side; ++a)
          for (int b = 0; b < side; ++b) {
            int ga = la * side + a, gb = lb * side + b;
            mort_a[t] = ga;
            mort_b[t] = gb;
            m2c[t] = grid2caller[(int64_t)ga * n + gb];
            c2m[m2c[t]] = (int)t;
            ++t;
          }
      }
    }
    std::vector<int> s2c(N), c2s(N), s2m(N), m2s(N);
    {
      const long long plane = (long long)nhL * nhL;
      for (int ba = 0; ba < nbL; ++ba)
        for (int bb = 0; bb < nbL; ++bb) {
          int c = (ba & 1) * 2 + (bb & 1);
          int ha = ba >> 1, hb = bb >> 1;
          for (int pa = 0; pa < side; ++pa)
            for (int pb = 0; pb < side; ++pb) {
              long long sidx = (long long)(pa * side + pb) * 4 * plane + c * plane + (long long)ha * nhL + hb;
              int ga = ba * side + pa, gb = bb * side + pb;
              int ci = grid2caller[(int64_t)ga * n + gb];
              s2c[sidx] = ci;
              c2s[ci] = (int)sidx;
              s2m[sidx] = c2m[ci];
              m2s[c2m[ci]] = (int)sidx;
            }
        }
    }
    P->s2c.upload(s2c);
    P->c2s.upload(c2s);
    P->s2m.upload(s2m);
    P->m2s.upload(m2s);
    P->m2c.upload(m2c);
    std::vector<double> qc(q, q + N), qm(N), pxv(N), pyv(N);
    for (int64_t t = 0; t < N; ++t) qm[t] = q[m2c[t]];
    for (int64_t i = 0; i < N; ++i) {
      pxv[i] = points[2 * i];
      pyv[i] = points[2 * i + 1];
    }
    P->q_c.upload(qc);
    P->q_m.upload(qm);
    P->px.upload(pxv);
    P->py.upload(pyv);
    // ---- W table on the device (H0 evaluator), self-cell term on the host ----
    ls::WTable W;
    W.n = n;
    {
      DevBuf wt;
      size_t cnt = (size_t)(2 * n - 1) * (2 * n - 1);
      wt.alloc(cnt * 16);
      lsk::launch_wtable(wt.as<double2>(), n, h, kappa, nullptr);
      hip_check(hipGetLastError(), "wtable");
      W.w.resize(cnt);
      hip_check(hipMemcpy(W.w.data(), wt.p, cnt * 16, hipMemcpyDeviceToHost), "wtable d2h");
      W.w[(size_t)(n - 1) * (2 * n - 1) + (n - 1)] = self_cell(h, kappa);
    }
    // ---- NCA factors and device operators ----
    double t_w = now_ms();
    DevBuf wdev;  // the table with the self-cell term, for the NCA on the device
    if (P->opt.nca_device) wdev.upload(W.w);
    auto nca = [&](double eps) {
      return P->opt.nca_device ? ls::build_nca_device(p, W, wdev.as<double2>(), eps, nullptr)
                               : ls::build_nca(p, W, eps);
    };
    P->nca64 = nca(tol);
    build_fmm_ops(P.get(), P->nca64, P->f64, false);
    if (P->opt.build_fp32) {
      if (P->opt.eps_inner > 0 && P->opt.eps_inner > tol)
        P->nca32 = nca(P->opt.eps_inner);
      else
        P->nca32 = P->nca64;
      build_fmm_ops(P.get(), P->nca32, P->f32, true);
      P->have32 = true;
    }
    ensure_fmm_capacity(P.get(), P->f64, 1);
    if (P->have32) ensure_fmm_capacity(P.get(), P->f32, 1);
    double t_nca = now_ms();
    // ---- HODLR preconditioner ----
    if (P->opt.hodlr_rank > 0) {
      build_hodlr(P.get(), W, mort_a, mort_b, qm);
      P->have_hodlr = true;
    }
    double t_h = now_ms();
    hip_check(hipDeviceSynchronize(), "setup");
    // ---- stats ----
    ls_stats_t& S = P->stats;
    std::memset(&S, 0, sizeof(S));
    S.N = N;
    S.n = n;
    S.levels = p.leaf;
    S.leaf_side = side;
    S.top_level = p.top;
    for (int nu = p.top; nu <= p.leaf; ++nu)
      if (p.lv[nu].hf) S.nlevels_hf++;
    for (int nu = p.top; nu <= p.leaf; ++nu) {
      S.rank_max64 = std::max(S.rank_max64, P->f64.kmax.empty() ? 0 : P->f64.kmax[nu]);
      if (P->have32) S.rank_max32 = std::max(S.rank_max32, P->f32.kmax[nu]);
      S.m2l_pairs += p.lv[nu].il_pairs;
    }
    S.entries_near = p.near_pairs * (int64_t)side * side * side * side;
    S.entries_far64 = P->f64.entries_far;
    S.entries_far32 = P->have32 ? P->f32.entries_far : 0;
    S.entries_m2l64 = P->f64.entries_m2l;
    S.entries_m2l32 = P->have32 ? P->f32.entries_m2l : 0;
    S.entries_mid64 = (int64_t)P->f64.entries_mid;
    S.entries_mid32 = P->have32 ? (int64_t)P->f32.entries_mid : 0;
    S.stored_bytes64 = P->f64.stored_bytes;
    S.stored_bytes32 = P->have32 ? P->f32.stored_bytes : 0;
    S.hodlr_bytes = P->hod.bytes;
    S.hodlr_levels = P->have_hodlr ? P->hod.Lb : 0;
    for (int l = 0; P->have_hodlr && l < P->hod.Lb; ++l) S.hodlr_rank_sum += P->hod.rank[l];
    S.hodlr_dense_leaves = P->have_hodlr ? P->hod.dense_leaves : 0;
    S.hodlr_rank_used_sum = P->have_hodlr ? P->hod.used_rank_sum : 0;
    S.hodlr_blocks = P->have_hodlr ? P->hod.blocks : 0;
    S.hodlr_rank_used_max = P->have_hodlr ? P->hod.used_rank_max : 0;
    S.hodlr_rows_active = P->have_hodlr ? P->hod.rows_active : 0;
    for (int l = 0; P->have_hodlr && l < P->hod.Lb && l < 32; ++l) {
      S.hodlr_dot_rows[l] = l < (int)P->hod.dot_rows.size() ? P->hod.dot_rows[l] : P->N;
      S.hodlr_core_nodes[l] = l < (int)P->hod.core_nodes.size() ? P->hod.core_nodes[l] : (1 << l);
    }
    S.hodlr_subtree_level =
        P->have_hodlr && P->hod.sub_rows ? P->hod.Lb - (P->hod.sub_rows == 512 ? 3 : 2) : -1;
    S.t_hodlr_aca_ms = P->hod.t_aca_ms;
    S.t_hodlr_apply_ms = P->hod.t_apply_ms;
    S.t_hodlr_cores_ms = P->hod.t_cores_ms;
    S.t_plan_ms = t_plan - t0;
    S.t_nca_ms = t_nca - t_w;
    S.t_hodlr_ms = t_h - t_nca;
    S.t_setup_ms = now_ms() - t0;
    *out = P.release();
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return LS_EINVAL;
  }
}


ls_status ls_stats(const ls_problem* P, ls_stats_t* out) {
  if (!P || !out) {
    g_last_error = "NULL argument";
    return LS_EINVAL;
  }
  *out = P->stats;
  return LS_OK;
}

void ls_destroy(ls_problem* P) {
  if (!P) return;
  for (auto& pc : P->prof)
    for (auto& e : pc.ev) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  delete P;
}

}  // extern "C"
