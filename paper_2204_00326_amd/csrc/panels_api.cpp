// High-order leaf panels (paper, Section 2.2, Eqs. (eq:7)-(eq:13)) on a uniform tree: the C ABI
// (ls_panels_*).  The host forms the Chebyshev nodes, the basis, the interpolation matrix Q and
// its pseudo-inverse, and the Gauss-Legendre rules; the device forms the moment tables, the
// operator blocks and the products (panels.hip).
#include <algorithm>
#include <cmath>
#include <memory>
#include <vector>

#include "api_internal.h"
#include "hodlr_setup.h"
#include "kernels.h"
#include "panels.h"

// HODLR approximation of the panel system (Section 6 for the discretisation of Section 2.2):
// unknowns in HODLR order (boxes in Morton order, nodes inside a box in their own order, padding
// unknowns after the last box up to 2^L leaves), leaves of lp <= 64 unknowns (whole boxes), a
// binary tree that halves the index range.  Factors as for the cell-centred grid over the M =
// 2^L lp positions: U, W per binary level (column c of block b at c * M + its row / column
// offset), Y = (the levels below)^-1 U, SMW core inverses per node, leaf inverses column-major.
struct PanelHodlr {
  int Lb = 0, lp = 0, nleaves = 0, r = 0;
  std::vector<int> rank;           // per binary level: min(r, half of a node)
  std::vector<long long> chunk;    // rows per chunk of the W^T z reductions
  std::vector<int> nchunks, cpc;
  lsi::DevBuf perm;                // perm[t] = the caller's index of HODLR position t (-1: padding)
  lsi::DevBuf qh;                  // contrast in HODLR order
  lsi::DevBuf Dinv, ident;
  std::vector<lsi::DevBuf> Y, W, core;
  lsi::DevBuf partial, svec, zh;
  int64_t used_rank_sum = 0, blocks = 0;
  int used_rank_max = 0;
  double t_setup_ms = 0;
};

struct ls_panels {
  lsp::PanelGeom g{};
  double L = 1.0;
  int sign = -1;
  int64_t N = 0;       // unknowns
  bool dense = false;  // leaves of a general tree: the dense V instead of per-offset blocks
  int nboxes = 0;
  lsi::DevBuf V, X, boxes;
  lsi::DevBuf ref, far_x, far_w, qdag, M, T, q;
  lsi::DevBuf Tt;    // column-major copies of the blocks (matrix-core product)
  lsi::DevBuf part;  // partial planes of the matrix-core product (one stream at a time)
  lsi::DevBuf xt;    // node-major copy of the product's input (one stream at a time)
  bool mfma = true;
  lsi::DevBuf kq, kw, kr, kpart, kc;  // GMRES basis, work vectors, dot partials, coefficients
  lsi::DevBuf kz;                     // preconditioned vector of the GMRES
  std::unique_ptr<PanelHodlr> hod;    // HODLR preconditioner, when built
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
// Qdag = (Q^T Q)^-1 Q^T.  Q (n2 x np): Q[i][l] = b_l(node i); its columns are orthogonal at the
// Chebyshev points of the first kind (discrete orthogonality of T_0..T_{p-1}), so Qdag is the
// transpose scaled by the diagonal of Q^T Q.
void basis_tables(int p, lsp::PanelRef& R, std::vector<double>& Qd) {
  for (int i = 0; i < p; ++i) R.node[i] = std::cos((2.0 * (p - 1 - i) + 1.0) * M_PI / (2.0 * p));
  int l = 0;
  for (int dgr = 0; dgr < p; ++dgr)
    for (int a = 0; a <= dgr; ++a, ++l) {
      R.ba[l] = a;
      R.bb[l] = dgr - a;
    }
  const int n2 = p * p, np = p * (p + 1) / 2;
  std::vector<double> Q((size_t)n2 * np);
  Qd.assign((size_t)np * n2, 0.0);
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
}

// The reference data above with the Gauss-Legendre rules on [0, 1] along the ray and across the
// triangles, uploaded (Qdag too).
lsp::PanelRef reference_data(ls_panels* P) {
  const lsp::PanelGeom& g = P->g;
  lsp::PanelRef R{};
  std::vector<double> Qd;
  basis_tables(g.p, R, Qd);
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
  P->ref.alloc(sizeof(R));
  lsi::hip_check(hipMemcpy(P->ref.p, &R, sizeof(R), hipMemcpyHostToDevice), "panels ref");
  P->qdag.upload(Qd);
  return R;
}

// Adaptive, level-restricted quadtree of Section 2.1 on [-L, L]^2.  A box is split below
// min_level, and up to max_level while it is in the high-frequency regime ((kappa w)^2 > T, w the
// half-width) or while q or the incident field is not resolved: the p-th order interpolant of the
// function on the box (Qdag applied to its node values), evaluated at the nodes of its four
// children, differs from the function there by more than eps relative to the largest magnitude
// among those values and the box's own.  Then every leaf with a neighbour (a shared boundary
// segment) more than one level finer is split, pass after pass, until none is.  Leaves are
// returned depth first, children in the order (-x, -y), (-x, +y), (+x, -y), (+x, +y).
struct TreeNode {
  double cx, cy, beta;
  int level, child;  // child: index of the first of four children, -1 for a leaf
};

bool box_resolved(ls_point_fn fn, void* ctx, const TreeNode& b, int p, double eps, const lsp::PanelRef& R,
                  const std::vector<double>& Qd) {
  const int n2 = p * p, np = p * (p + 1) / 2;
  std::vector<double> x((size_t)5 * n2), y((size_t)5 * n2), re((size_t)5 * n2, 0.0), im((size_t)5 * n2, 0.0);
  // the box's nodes, then its children's (in the child order above)
  for (int c = 0; c < 5; ++c) {
    const double h = c == 0 ? b.beta : 0.5 * b.beta;
    const double ox = c == 0 ? b.cx : b.cx + (c <= 2 ? -h : h);
    const double oy = c == 0 ? b.cy : b.cy + (c % 2 == 1 ? -h : h);
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < p; ++j) {
        x[(size_t)c * n2 + i * p + j] = ox + h * R.node[i];
        y[(size_t)c * n2 + i * p + j] = oy + h * R.node[j];
      }
  }
  fn(5 * n2, x.data(), y.data(), re.data(), im.data(), ctx);
  std::vector<zd> coef(np, zd(0));
  double scale = 0;
  for (int k = 0; k < np; ++k)
    for (int i = 0; i < n2; ++i) coef[k] += Qd[(size_t)k * n2 + i] * zd(re[i], im[i]);
  for (int i = 0; i < 5 * n2; ++i) {
    if (!std::isfinite(re[i]) || !std::isfinite(im[i])) throw LsError(LS_EINVAL, "a field value is not finite");
    scale = std::max(scale, std::abs(zd(re[i], im[i])));
  }
  scale = std::max(scale, 1e-300);
  double err = 0;
  for (int i = n2; i < 5 * n2; ++i) {
    const double u = (x[i] - b.cx) / b.beta, v = (y[i] - b.cy) / b.beta;
    zd a(0);
    for (int k = 0; k < np; ++k) a += coef[k] * (cheb(R.ba[k], u) * cheb(R.bb[k], v));
    err = std::max(err, std::abs(a - zd(re[i], im[i])));
  }
  return err <= eps * scale;
}

bool neighbours(const TreeNode& a, const TreeNode& b) {
  const double dx = std::fabs(a.cx - b.cx), dy = std::fabs(a.cy - b.cy), sw = a.beta + b.beta;
  const double tol = 1e-12 * sw;
  return (std::fabs(dx - sw) <= tol && dy < sw - tol) || (std::fabs(dy - sw) <= tol && dx < sw - tol);
}

void split_node(std::vector<TreeNode>& t, int i) {
  const TreeNode b = t[i];
  const double h = 0.5 * b.beta;
  t[i].child = (int)t.size();
  for (int sx = -1; sx <= 1; sx += 2)
    for (int sy = -1; sy <= 1; sy += 2) t.push_back({b.cx + sx * h, b.cy + sy * h, h, b.level + 1, -1});
}

std::vector<TreeNode> build_quadtree(double L, int p, double kappa, double eps, double T, int min_level,
                                     int max_level, ls_point_fn q, ls_point_fn uinc, void* ctx) {
  lsp::PanelRef R{};
  std::vector<double> Qd;
  basis_tables(p, R, Qd);
  std::vector<TreeNode> t{{0.0, 0.0, L, 0, -1}};
  for (size_t i = 0; i < t.size(); ++i) {
    const TreeNode b = t[i];
    if (b.level >= max_level) continue;
    bool split = b.level < min_level;
    if (!split) {
      const double kw = kappa * b.beta;
      split = kw * kw > T || !box_resolved(q, ctx, b, p, eps, R, Qd) || !box_resolved(uinc, ctx, b, p, eps, R, Qd);
    }
    if (split) split_node(t, (int)i);
  }
  // level restriction, pass after pass against the leaves at the start of the pass
  for (;;) {
    std::vector<int> leaves, to_split;
    for (size_t i = 0; i < t.size(); ++i)
      if (t[i].child < 0) leaves.push_back((int)i);
    for (int a : leaves)
      for (int o : leaves)
        if (t[o].level > t[a].level + 1 && neighbours(t[a], t[o])) {
          to_split.push_back(a);
          break;
        }
    if (to_split.empty()) break;
    for (int a : to_split) split_node(t, a);
  }
  // leaves depth first
  std::vector<TreeNode> out;
  std::vector<int> stack{0};
  while (!stack.empty()) {
    const int i = stack.back();
    stack.pop_back();
    if (t[i].child < 0) {
      out.push_back(t[i]);
      continue;
    }
    for (int c = 3; c >= 0; --c) stack.push_back(t[i].child + c);
  }
  return out;
}

// Morton (Z) order of the nside x nside boxes (nside a power of two): box k = ix * nside + iy has
// the code with the bits of iy at the even and those of ix at the odd positions; boxes sorted by it.
std::vector<int> morton_boxes(int nside) {
  std::vector<std::pair<unsigned long long, int>> c;
  c.reserve((size_t)nside * nside);
  for (int ix = 0; ix < nside; ++ix)
    for (int iy = 0; iy < nside; ++iy) {
      unsigned long long code = 0;
      for (int bit = 0; bit < 16; ++bit) {
        code |= (unsigned long long)((iy >> bit) & 1) << (2 * bit);
        code |= (unsigned long long)((ix >> bit) & 1) << (2 * bit + 1);
      }
      c.push_back({code, ix * nside + iy});
    }
  std::sort(c.begin(), c.end());
  std::vector<int> out(c.size());
  for (size_t i = 0; i < c.size(); ++i) out[i] = c[i].second;
  return out;
}

// In-place inverse of the n x n row-major matrix a by Gauss-Jordan elimination with partial
// pivoting; false when a pivot is exactly zero.
bool invert_dense(std::vector<zd>& a, int n) {
  std::vector<int> piv(n);
  for (int k = 0; k < n; ++k) {
    int pr = k;
    for (int i = k + 1; i < n; ++i)
      if (std::abs(a[(size_t)i * n + k]) > std::abs(a[(size_t)pr * n + k])) pr = i;
    if (a[(size_t)pr * n + k] == zd(0)) return false;
    piv[k] = pr;
    if (pr != k)
      for (int j = 0; j < n; ++j) std::swap(a[(size_t)k * n + j], a[(size_t)pr * n + j]);
    const zd d = zd(1) / a[(size_t)k * n + k];
    a[(size_t)k * n + k] = zd(1);
    for (int j = 0; j < n; ++j) a[(size_t)k * n + j] *= d;
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const zd f = a[(size_t)i * n + k];
      if (f == zd(0)) continue;
      a[(size_t)i * n + k] = zd(0);
      for (int j = 0; j < n; ++j) a[(size_t)i * n + j] -= f * a[(size_t)k * n + j];
    }
  }
  // undo the row exchanges as column exchanges, last first
  for (int k = n - 1; k >= 0; --k)
    if (piv[k] != k)
      for (int i = 0; i < n; ++i) std::swap(a[(size_t)i * n + k], a[(size_t)i * n + piv[k]]);
  return true;
}

void phod_ws(PanelHodlr& H, long long N, int nrhs) {
  size_t np = 1, ns = 1;
  for (int l = 0; l < H.Lb; ++l) {
    np = std::max(np, (size_t)H.nchunks[l] * H.rank[l]);
    ns = std::max(ns, (size_t)(1LL << l) * 2 * H.rank[l]);
  }
  H.partial.ensure(np * nrhs * 16);
  H.svec.ensure(ns * nrhs * 16);
  (void)N;
}

// z = (the HODLR levels lstop .. Lb-1 and the leaves)^-1 b in HODLR order, nrhs columns of
// leading dimension N; b and z may be the same buffer.
void phod_apply(PanelHodlr& H, long long N, const double2* b, double2* z, int nrhs, int lstop, hipStream_t s) {
  phod_ws(H, N, nrhs);
  double2* partial = H.partial.as<double2>();
  double2* svec = H.svec.as<double2>();
  lsk::launch_leaf_apply(0, H.Dinv.p, H.ident.as<unsigned char>(), b, N, z, N, H.lp, H.nleaves, nrhs, s);
  for (int l = H.Lb - 1; l >= lstop; --l) {
    const int rl = H.rank[l];
    if (rl == 0) continue;
    lsk::launch_hodlr_dot(0, H.W[l].p, z, N, partial, N, rl, H.chunk[l], H.nchunks[l], nrhs, s);
    lsk::launch_hodlr_core(0, H.core[l].p, partial, svec, rl, 1 << l, H.cpc[l], H.nchunks[l], true, nrhs, s);
    lsk::launch_hodlr_update(0, H.Y[l].p, svec, z, N, N, rl, N >> l, 1 << l, nrhs, s);
  }
}

// z = A~^-1 r in the caller's order (ld per column), through the padded HODLR order
void phod_apply_user(ls_panels* P, const double2* r, long long ldr, double2* z, long long ldz, int nrhs,
                     hipStream_t s) {
  PanelHodlr& H = *P->hod;
  const long long M = (long long)H.nleaves * H.lp;
  H.zh.ensure((size_t)M * nrhs * 16);
  double2* zh = H.zh.as<double2>();
  lsp::launch_panel_permute(r, ldr, zh, M, H.perm.as<int>(), M, nrhs, false, s);
  phod_apply(H, M, zh, zh, nrhs, 0, s);
  lsp::launch_panel_permute(zh, M, z, ldz, H.perm.as<int>(), M, nrhs, true, s);
}

// HODLR factors of A = I + sign kappa^2 diag(q) V in the HODLR order perm (M = nleaves * lp
// positions, nleaves a power of two; perm[t] = the caller's index of position t, -1 for a padding
// unknown: an identity row and column).  Vij(i, j): V between the caller's unknowns i and j.
// The off-diagonal blocks by partially pivoted ACA on the host at rank min(r, block side), leaf
// inverses on the host, Y and the SMW cores on the device.
template <class VFn>
void build_panel_hodlr(ls_panels* P, int r, int lp, const std::vector<int>& perm, VFn Vij) {
  const double t0 = lsi::now_ms();
  const long long M = (long long)perm.size();
  auto H = std::make_unique<PanelHodlr>();
  H->r = r;
  H->lp = lp;
  H->nleaves = (int)(M / lp);
  H->Lb = 0;
  while ((1 << H->Lb) < H->nleaves) ++H->Lb;
  if ((long long)H->nleaves * lp != M || (1 << H->Lb) != H->nleaves)
    throw LsError(LS_EINVAL, "HODLR order: 2^L leaves of lp positions");
  const int Lb = H->Lb;
  std::vector<double> qd((size_t)P->N), qh((size_t)M, 0.0);
  lsi::hip_check(hipMemcpy(qd.data(), P->q.p, (size_t)P->N * 8, hipMemcpyDeviceToHost), "q d2h");
  for (long long t = 0; t < M; ++t)
    if (perm[t] >= 0) qh[t] = qd[perm[t]];
  const double coef = P->sign * P->g.kappa * P->g.kappa;
  // A - I at HODLR positions (zero in the rows and columns of the padding)
  auto Aoff = [&](long long i, long long j) {
    return perm[i] < 0 || perm[j] < 0 || qh[i] == 0.0 ? zd(0) : coef * qh[i] * Vij(perm[i], perm[j]);
  };
  // leaf inverses (column-major per leaf); leaves without contrast are the identity
  std::vector<zd> Dinv((size_t)H->nleaves * lp * lp);
  std::vector<unsigned char> ident(H->nleaves, 0);
  std::vector<char> bad(H->nleaves, 0);
  lsi::parallel_for(H->nleaves, [&](int k) {
    const long long o = (long long)k * lp;
    bool any = false;
    for (int i = 0; i < lp; ++i) any |= qh[o + i] != 0.0;
    if (!any) {
      ident[k] = 1;
      return;
    }
    std::vector<zd> a((size_t)lp * lp);
    for (int i = 0; i < lp; ++i)
      for (int j = 0; j < lp; ++j) a[(size_t)i * lp + j] = (i == j ? zd(1) : zd(0)) + Aoff(o + i, o + j);
    if (!invert_dense(a, lp)) {
      bad[k] = 1;
      return;
    }
    zd* D = Dinv.data() + (size_t)k * lp * lp;
    for (int i = 0; i < lp; ++i)
      for (int j = 0; j < lp; ++j) D[(size_t)j * lp + i] = a[(size_t)i * lp + j];
  });
  for (char b : bad)
    if (b) throw LsError(LS_EINVAL, "singular HODLR leaf block of the panel system");
  // off-diagonal blocks of every binary level
  H->rank.assign(Lb, 0);
  for (int l = 0; l < Lb; ++l) H->rank[l] = (int)std::min<long long>(r, M >> (l + 1));
  std::vector<std::vector<zd>> Uh(Lb), Wh(Lb);
  for (int l = 0; l < Lb; ++l) {
    Uh[l].assign((size_t)M * H->rank[l], zd(0));
    Wh[l].assign((size_t)M * H->rank[l], zd(0));
  }
  std::vector<std::pair<int, int>> work;
  for (int l = 0; l < Lb; ++l)
    for (int b = 0; b < (1 << l); ++b) work.push_back({l, b});
  std::vector<int> used(work.size() * 2, 0);
  lsi::parallel_for((int)work.size() * 2, [&](int wi) {
    const int l = work[wi / 2].first, b = work[wi / 2].second, which = wi % 2;
    const long long sz = M >> l, lo = (long long)b * sz, mid = lo + sz / 2;
    // which = 0: A[I1, I2] ~ U W^T (U rows in the first child); which = 1: A[I2, I1]
    const long long r0 = which ? mid : lo, c0 = which ? lo : mid;
    const int m = (int)(sz / 2), n = (int)(sz / 2);
    std::vector<char> rz(m);
    for (int i = 0; i < m; ++i) rz[i] = qh[r0 + i] == 0.0;
    auto rowfn = [&](int i, zd* out) {
      for (int j = 0; j < n; ++j) out[j] = Aoff(r0 + i, c0 + j);
    };
    auto colfn = [&](int j, zd* out) {
      for (int i = 0; i < m; ++i) out[i] = Aoff(r0 + i, c0 + j);
    };
    ls::ACAResult R = ls::aca(m, n, H->rank[l], 0.0, &rz, rowfn, colfn);
    const int k = (int)R.u.size();
    used[wi] = k;
    for (int c = 0; c < k; ++c) {
      for (int i = 0; i < m; ++i) Uh[l][(size_t)c * M + r0 + i] = R.u[c][i];
      for (int j = 0; j < n; ++j) Wh[l][(size_t)c * M + c0 + j] = R.v[c][j];
    }
  });
  for (int k : used) {
    H->used_rank_sum += k;
    H->used_rank_max = std::max(H->used_rank_max, k);
  }
  H->blocks = (int64_t)used.size();
  // device factors
  H->perm.upload(perm);
  H->qh.upload(qh);
  H->Dinv.upload(Dinv);
  H->ident.upload(ident);
  H->chunk.assign(Lb, 0);
  H->nchunks.assign(Lb, 0);
  H->cpc.assign(Lb, 0);
  for (int l = 0; l < Lb; ++l) {
    const long long cs = M >> (l + 1);
    long long ch = cs;
    while (ch > 1024 && ch % 2 == 0) ch /= 2;
    H->chunk[l] = ch;
    H->nchunks[l] = (int)(M / ch);
    H->cpc[l] = (int)(cs / ch);
  }
  H->Y.resize(Lb);
  H->W.resize(Lb);
  H->core.resize(Lb);
  int rmax = 1;
  size_t kel = 1;
  for (int l = 0; l < Lb; ++l) {
    H->Y[l].upload(Uh[l]);
    H->W[l].upload(Wh[l]);
    Uh[l] = std::vector<zd>();
    Wh[l] = std::vector<zd>();
    rmax = std::max(rmax, H->rank[l]);
    kel = std::max(kel, (size_t)(1LL << l) * 4 * H->rank[l] * H->rank[l]);
  }
  phod_ws(*H, M, rmax);
  lsi::DevBuf kA, kB, kbad;
  kA.alloc(kel * 16);
  kB.alloc(kel * 16);
  kbad.alloc((size_t)std::max(1, 1 << std::max(Lb - 1, 0)) * 4);
  std::vector<int> hb((size_t)std::max(1, 1 << std::max(Lb - 1, 0)));
  hipStream_t s = nullptr;
  for (int l = Lb - 1; l >= 0; --l) {
    const int rl = H->rank[l], nodes = 1 << l;
    double2* Y = H->Y[l].as<double2>();
    phod_apply(*H, M, Y, Y, rl, l + 1, s);  // Y = (levels below)^-1 U
    lsk::launch_zero_rows(Y, M, rl, H->qh.as<double>(), s);
    lsk::launch_hodlr_dot(0, H->W[l].p, Y, M, H->partial.as<double2>(), M, rl, H->chunk[l], H->nchunks[l], rl, s);
    lsk::launch_hodlr_core(0, nullptr, H->partial.as<double2>(), H->svec.as<double2>(), rl, nodes, H->cpc[l],
                           H->nchunks[l], false, rl, s);
    H->core[l].alloc((size_t)nodes * lsk::hodlr_core_elems(rl) * 16);
    lsi::hip_check(hipMemsetAsync(kbad.p, 0, (size_t)nodes * 4, s), "memset");
    lsk::launch_core_invert(H->svec.as<double2>(), rl, nodes, kA.as<double2>(), kB.as<double2>(),
                            H->core[l].as<double2>(), kbad.as<int>(), s);
    lsi::hip_check(hipGetLastError(), "panel HODLR cores");
    lsi::hip_check(hipMemcpyAsync(hb.data(), kbad.p, (size_t)nodes * 4, hipMemcpyDeviceToHost, s), "core status");
    lsi::hip_check(hipStreamSynchronize(s), "panel HODLR cores");
    for (int k = 0; k < nodes; ++k)
      if (hb[k]) throw LsError(LS_EINVAL, "singular HODLR core of the panel system");
  }
  lsi::hip_check(hipDeviceSynchronize(), "panel HODLR setup");
  H->t_setup_ms = lsi::now_ms() - t0;
  P->hod = std::move(H);
}

// Uniform tree (nside a power of two): boxes in Morton order, leaves of 4^j whole boxes with at
// most 64 unknowns, no padding; V from the per-offset blocks T (copied to the host).
void build_panel_hodlr_uniform(ls_panels* P, int r) {
  const lsp::PanelGeom& g = P->g;
  const int ns = g.nside, n2 = g.n2, w2 = 2 * ns - 1;
  const long long N = P->N;
  int lb = 1;
  while ((long long)lb * 4 * n2 <= 64 && (long long)lb * 4 <= (long long)ns * ns) lb *= 4;
  const std::vector<int> mb = morton_boxes(ns);
  std::vector<int> perm((size_t)N);
  for (long long t = 0; t < N; ++t) perm[t] = mb[t / n2] * n2 + (int)(t % n2);
  const size_t tsz = (size_t)w2 * w2 * n2 * n2;
  std::vector<zd> T(tsz);
  lsi::hip_check(hipMemcpy(T.data(), P->T.p, tsz * 16, hipMemcpyDeviceToHost), "operator blocks d2h");
  auto Vij = [&](int i, int j) {
    const int A = i / n2, B = j / n2;
    const long long d = (long long)(A / ns - B / ns + ns - 1) * w2 + (A % ns - B % ns + ns - 1);
    return T[(size_t)((d * n2 + i % n2) * n2 + j % n2)];
  };
  build_panel_hodlr(P, r, lb * n2, perm, Vij);
}

// Leaves of any tree: boxes sorted by the Morton code of their lower-left corner on the grid of
// the smallest half-width, leaves of floor(64 / p^2) whole boxes, padding up to 2^L leaves; V from
// the dense device matrix (copied to the host).
void build_panel_hodlr_leaves(ls_panels* P, int r) {
  const int n2 = P->g.n2, nb = P->nboxes;
  const long long N = P->N;
  std::vector<double> bx((size_t)5 * nb);
  lsi::hip_check(hipMemcpy(bx.data(), P->boxes.p, bx.size() * 8, hipMemcpyDeviceToHost), "boxes d2h");
  double xmin = 1e300, ymin = 1e300, hmin = 1e300;
  for (int B = 0; B < nb; ++B) {
    xmin = std::min(xmin, bx[5 * B] - bx[5 * B + 2]);
    ymin = std::min(ymin, bx[5 * B + 1] - bx[5 * B + 2]);
    hmin = std::min(hmin, bx[5 * B + 2]);
  }
  std::vector<std::pair<unsigned long long, int>> key((size_t)nb);
  for (int B = 0; B < nb; ++B) {
    const double fx = std::floor((bx[5 * B] - bx[5 * B + 2] - xmin) / (2.0 * hmin) + 0.5);
    const double fy = std::floor((bx[5 * B + 1] - bx[5 * B + 2] - ymin) / (2.0 * hmin) + 0.5);
    const unsigned ix = (unsigned)std::min(fx, 1e9), iy = (unsigned)std::min(fy, 1e9);
    unsigned long long code = 0;
    for (int bit = 0; bit < 31; ++bit) {
      code |= (unsigned long long)((iy >> bit) & 1) << (2 * bit);
      code |= (unsigned long long)((ix >> bit) & 1) << (2 * bit + 1);
    }
    key[B] = {code, B};
  }
  std::stable_sort(key.begin(), key.end());
  const int per = std::max(1, 64 / n2);
  const int lp = per * n2;
  long long nleaves = 1;
  while (nleaves * lp < N) nleaves *= 2;
  std::vector<int> perm((size_t)(nleaves * lp), -1);
  for (int t = 0; t < nb; ++t)
    for (int a = 0; a < n2; ++a) perm[(size_t)t * n2 + a] = key[t].second * n2 + a;
  std::vector<zd> V((size_t)N * N);
  lsi::hip_check(hipMemcpy(V.data(), P->V.p, V.size() * 16, hipMemcpyDeviceToHost), "dense V d2h");
  auto Vij = [&](int i, int j) { return V[(size_t)i * N + j]; };
  build_panel_hodlr(P, r, lp, perm, Vij);
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
    if (p <= lsp::kMfmaMaxP) {
      P->Tt.alloc(noff * n2 * n2 * 16);
      lsp::launch_panel_blocks_t(g, P->T.as<double2>(), P->Tt.as<double2>(), s);
      lsi::hip_check(hipGetLastError(), "panel blocks (column-major)");
    }
    lsi::hip_check(hipDeviceSynchronize(), "panels setup");
    *out = P.release();
    return LS_OK;
  } catch (const LsError& e) {
    return lsi::fail(e);
  }
}

ls_status ls_panels_build_tree(double L, int p, double kappa, double eps_grid, double T, int min_level, int max_level,
                               ls_point_fn q, ls_point_fn uinc, void* ctx, int max_boxes, double* boxes,
                               int* nboxes) {
  try {
    if (!q || !uinc || !nboxes) throw LsError(LS_EINVAL, "q, uinc or nboxes is NULL");
    if (p < 1 || p > lsp::kMaxP) throw LsError(LS_EINVAL, "p must be in 1..8");
    if (!(L > 0) || !std::isfinite(L) || !(kappa > 0) || !std::isfinite(kappa))
      throw LsError(LS_EINVAL, "L and kappa must be positive and finite");
    if (!(eps_grid > 0) || !std::isfinite(eps_grid) || !(T > 0) || !std::isfinite(T))
      throw LsError(LS_EINVAL, "eps_grid and T must be positive and finite");
    if (min_level < 0 || max_level < min_level || max_level > 12)
      throw LsError(LS_EINVAL, "levels must satisfy 0 <= min_level <= max_level <= 12");
    if (max_boxes < 0 || (max_boxes > 0 && !boxes)) throw LsError(LS_EINVAL, "boxes is NULL");
    const std::vector<TreeNode> lv = build_quadtree(L, p, kappa, eps_grid, T, min_level, max_level, q, uinc, ctx);
    *nboxes = (int)lv.size();
    if ((int)lv.size() > max_boxes) throw LsError(LS_EINVAL, "more leaves than max_boxes (nboxes holds the count)");
    for (size_t i = 0; i < lv.size(); ++i) {
      boxes[4 * i] = lv[i].cx;
      boxes[4 * i + 1] = lv[i].cy;
      boxes[4 * i + 2] = lv[i].beta;
      boxes[4 * i + 3] = lv[i].level;
    }
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
      P->xt.ensure((size_t)nrhs * N * 16);
      lsp::launch_panel_apply_mfma(P->g, P->Tt.as<double2>(), q, (const double2*)x, ld, (double2*)y, ld, nrhs, alpha,
                                   coef, P->part.as<double2>(), P->xt.as<double2>(), nc, (hipStream_t)stream);
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

// HODLR preconditioner of the panel system (Section 6): fixed off-diagonal rank, uniform trees
// whose side is a power of two.  rank <= 0 drops the factors.
ls_status ls_panels_precond_setup(ls_panels* P, int rank) {
  try {
    if (!P) throw LsError(LS_EINVAL, "panels handle is NULL");
    if (rank <= 0) {
      P->hod.reset();
      return LS_OK;
    }
    if (rank > 256) throw LsError(LS_EINVAL, "rank must be <= 256");
    P->hod.reset();
    if (P->dense) {
      build_panel_hodlr_leaves(P, rank);
    } else {
      const int ns = P->g.nside;
      if ((ns & (ns - 1)) != 0) throw LsError(LS_ENOTSUP, "the HODLR preconditioner needs nside a power of two");
      build_panel_hodlr_uniform(P, rank);
    }
    return LS_OK;
  } catch (const LsError& e) {
    return lsi::fail(e);
  }
}

ls_status ls_panels_precond_apply(ls_panels* P, const void* r, void* z, int nrhs, int64_t ld, void* stream) {
  try {
    check_vec(P, r, z, nrhs, ld);
    if (!P->hod) throw LsError(LS_EINVAL, "no HODLR preconditioner (ls_panels_precond_setup)");
    phod_apply_user(P, (const double2*)r, ld, (double2*)z, ld, nrhs, (hipStream_t)stream);
    lsi::hip_check(hipGetLastError(), "panel HODLR apply");
    return LS_OK;
  } catch (const LsError& e) {
    return lsi::fail(e);
  }
}

ls_status ls_panels_precond_info(const ls_panels* P, int* rank, int* leaf, int* levels, double* mean_rank,
                                 int* max_rank, double* setup_ms) {
  if (!P || !rank || !leaf || !levels || !mean_rank || !max_rank || !setup_ms) {
    lsi::g_last_error = "bad arguments";
    return LS_EINVAL;
  }
  const PanelHodlr* H = P->hod.get();
  *rank = H ? H->r : 0;
  *leaf = H ? H->lp : 0;
  *levels = H ? H->Lb : 0;
  *mean_rank = H && H->blocks ? (double)H->used_rank_sum / (double)H->blocks : 0.0;
  *max_rank = H ? H->used_rank_max : 0;
  *setup_ms = H ? H->t_setup_ms : 0.0;
  return LS_OK;
}

// Restarted GMRES (Section 6) on A psi = f from psi = 0, right-preconditioned by the HODLR
// approximation when one is built (A A~^-1 u = f, psi = A~^-1 u): classical Gram-Schmidt with
// one reorthogonalisation, Givens rotations and the triangular solve on the host, every vector
// operation on the device; each restart (and the end) recomputes the true residual f - A psi.
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
    const bool pc = P->hod != nullptr;
    if (pc) P->kz.ensure((size_t)N * 16);
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
        P->xt.ensure((size_t)N * 16);
        lsp::launch_panel_apply_mfma(P->g, P->Tt.as<double2>(), P->q.as<double>(), in, N, out, N, 1, 1.0,
                                     P->sign * k2, P->part.as<double2>(), P->xt.as<double2>(), nc, s);
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
        if (pc) {
          phod_apply_user(P, Q + (size_t)j * N, N, P->kz.as<double2>(), N, 1, s);
          applyA(P->kz.as<double2>(), w);
        } else {
          applyA(Q + (size_t)j * N, w);
        }
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
      if (pc) {
        // psi += A~^-1 (Q y)
        double2* z = P->kz.as<double2>();
        lsp::launch_panel_combo(z, fd, 0.0, fd, 0.0, N, s);
        update(z, k, y, -1.0);
        phod_apply_user(P, z, N, z, N, 1, s);
        lsp::launch_panel_combo(x, x, 1.0, z, 1.0, N, s);
      } else {
        update(x, k, y, -1.0);
      }
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
