// Quadtree, regimes, cones, lists and NCA factors on a uniform grid (host code).
//
// Section 2.1 builds a quadtree; Section 3 classifies a box of half-width w as
// high-frequency when (kappa w)^2 > T and defines the low-frequency (LF) and
// directional high-frequency (HF) admissibility conditions; Section 3.2.1 builds the
// cone hierarchy; Table "notations" of Section 4.1 defines N(B), IL(B) and IL(B, l);
// Section 4 builds nested bases and pivots with NCA.
//
// On a uniform grid with the translation-invariant p = 1 kernel, the interaction list
// of a box depends only on its position inside its parent (its class) and on clipping
// at the domain boundary.  The pivots of a level (and direction) are therefore chosen
// once, for a box whose far-field candidate region is the union of all interaction
// offsets occurring at that level, and shared by every box of the level: the
// resulting bases approximate every (clipped) interaction list of the level, and the
// L2L/M2M/M2L operators become a small set of matrices shared across boxes.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <thread>

namespace ls {

static const double kPi = 3.14159265358979323846;

int cone_of(int da, int db, int ndir, double phi0) {
  if (ndir <= 1) return 0;
  double phi = std::atan2((double)db, (double)da);
  double t = (phi - phi0) / (2.0 * kPi / ndir);
  long j = (long)std::floor(t);
  j %= ndir;
  if (j < 0) j += ndir;
  return (int)j;
}

Plan make_plan(int n, double L, double kappa, const PlanOptions& opt) {
  if (n <= 0) throw LsError(-1, "grid side must be positive");
  if (!(kappa > 0) || !std::isfinite(kappa)) throw LsError(-1, "kappa must be positive and finite");
  if (opt.leaf_max < 1) throw LsError(-1, "leaf_max must be >= 1");
  if (!(opt.T > 0)) throw LsError(-1, "T must be positive");
  Plan p;
  p.n = n;
  p.L = L;
  p.h = 2.0 * L / n;
  p.kappa = kappa;
  // leaf level: the shallowest level whose boxes split n evenly, hold <= leaf_max points
  // and are low-frequency (leaves are always LF)
  int leaf = -1;
  for (int lvl = 1; lvl <= 20; ++lvl) {
    if (n % (1 << lvl) != 0) break;
    int side = n >> lvl;
    double w = 0.5 * side * p.h;
    if ((int64_t)side * side <= opt.leaf_max && (kappa * w) * (kappa * w) <= opt.T) {
      leaf = lvl;
      break;
    }
  }
  if (leaf < 0)
    throw LsError(-4, "grid side " + std::to_string(n) + " cannot be split into low-frequency leaves of <= leaf_max points");
  p.leaf = leaf;
  p.leaf_side = n >> leaf;
  p.lv.resize(leaf + 1);
  for (int nu = 0; nu <= leaf; ++nu) {
    Level& l = p.lv[nu];
    l.nu = nu;
    l.nb = 1 << nu;
    l.side = n >> nu;
    l.w = L / l.nb;
    l.hf = (kappa * l.w) * (kappa * l.w) > opt.T;
    l.nbr_r2 = l.hf ? 0.25 * (kappa * l.w) * (kappa * l.w) : 4.0;
  }
  // cone counts: 2^ceil(log2(pi kappa w)) at the finest HF level, doubling upwards
  int finest_hf = -1;
  for (int nu = leaf; nu >= 0; --nu)
    if (p.lv[nu].hf) {
      finest_hf = nu;
      break;
    }
  if (finest_hf >= 0) {
    int nd = 1;
    while (nd < kPi * kappa * p.lv[finest_hf].w) nd *= 2;
    if (nd < 8) nd = 8;
    for (int nu = finest_hf; nu >= 0; --nu) {
      p.lv[nu].ndir = nd;
      nd *= 2;
    }
  }
  // stencils: children of the parent's neighbours that are not neighbours
  auto build_stencils = [&](int nu, double phi0) {
    Level& l = p.lv[nu];
    l.stencil.assign(4 * l.ndir, {});
    if (nu == 0) return;
    const Level& pl = p.lv[nu - 1];
    int R = pl.nb - 1;
    for (int c = 0; c < 4; ++c) {
      int ca = c >> 1, cb = c & 1;
      for (int Da = -R; Da <= R; ++Da)
        for (int Db = -R; Db <= R; ++Db) {
          if ((double)(Da * Da + Db * Db) >= pl.nbr_r2) continue;
          for (int c2 = 0; c2 < 4; ++c2) {
            int da = 2 * Da + (c2 >> 1) - ca, db = 2 * Db + (c2 & 1) - cb;
            if ((double)(da * da + db * db) < l.nbr_r2) continue;
            int dir = cone_of(da, db, l.ndir, phi0);
            l.stencil[c * l.ndir + dir].push_back({da, db});
          }
        }
    }
  };
  auto clip_and_count = [&](int nu) {
    Level& l = p.lv[nu];
    l.farset.assign(l.ndir, {});
    l.terms.assign(4 * l.ndir, {});
    l.il_pairs = 0;
    l.max_il = 0;
    int nh = l.nb / 2;
    for (int c = 0; c < 4 && nu > 0; ++c) {
      int ca = c >> 1, cb = c & 1;
      for (int dir = 0; dir < l.ndir; ++dir) {
        for (const Off& d : l.stencil[c * l.ndir + dir]) {
          // boxes of class c: ba = 2 ha + ca, 0 <= ha < nh
          int cnt_a = 0, cnt_b = 0;
          for (int ha = 0; ha < nh; ++ha) {
            int s = 2 * ha + ca + d.a;
            if (s >= 0 && s < l.nb) ++cnt_a;
          }
          for (int hb = 0; hb < nh; ++hb) {
            int s = 2 * hb + cb + d.b;
            if (s >= 0 && s < l.nb) ++cnt_b;
          }
          if (cnt_a && cnt_b) {
            l.terms[c * l.ndir + dir].push_back(d);
            l.il_pairs += (int64_t)cnt_a * cnt_b;
            bool seen = false;
            for (const Off& e : l.farset[dir])
              if (e.a == d.a && e.b == d.b) {
                seen = true;
                break;
              }
            if (!seen) l.farset[dir].push_back(d);
          }
        }
      }
    }
    // per-box maximum list length
    if (nu > 0) {
      for (int ba = 0; ba < l.nb; ++ba)
        for (int bb = 0; bb < l.nb; ++bb) {
          int c = (ba & 1) * 2 + (bb & 1);
          for (int dir = 0; dir < l.ndir; ++dir) {
            int cnt = 0;
            for (const Off& d : l.terms[c * l.ndir + dir]) {
              int sa = ba + d.a, sb = bb + d.b;
              if (sa >= 0 && sa < l.nb && sb >= 0 && sb < l.nb) ++cnt;
            }
            l.max_il = std::max(l.max_il, cnt);
          }
        }
    }
    l.has_il = l.il_pairs > 0;
  };
  // first pass with phi0 = 0 to find the coarsest level with an interaction list
  for (int nu = 1; nu <= leaf; ++nu) {
    build_stencils(nu, 0.0);
    clip_and_count(nu);
  }
  p.top = leaf + 1;
  for (int nu = 1; nu <= leaf; ++nu)
    if (p.lv[nu].has_il) {
      p.top = nu;
      break;
    }
  // cone boundaries phi0 + 2 pi j / n with phi0 = pi / n_top, n_top the cone count of the
  // coarsest HF level holding interactions: boundaries are odd multiples of pi / n_top, so
  // no lattice direction lies on one and the cones of consecutive levels nest exactly
  p.phi0 = 0.0;
  for (int nu = p.top; nu <= leaf; ++nu)
    if (p.lv[nu].hf) {
      p.phi0 = kPi / p.lv[nu].ndir;
      break;
    }
  for (int nu = 1; nu <= leaf; ++nu) {
    build_stencils(nu, p.phi0);
    clip_and_count(nu);
  }
  // levels above the top carry no interactions
  for (int nu = 0; nu < p.top && nu <= leaf; ++nu) {
    p.lv[nu].il_pairs = 0;
    p.lv[nu].max_il = 0;
  }
  // near field: ordered neighbouring leaf pairs (LF rule at the leaf level)
  const Level& ll = p.lv[leaf];
  p.near_pairs = 0;
  for (int ba = 0; ba < ll.nb; ++ba)
    for (int bb = 0; bb < ll.nb; ++bb)
      for (int da = -1; da <= 1; ++da)
        for (int db = -1; db <= 1; ++db) {
          int sa = ba + da, sb = bb + db;
          if (sa >= 0 && sa < ll.nb && sb >= 0 && sb < ll.nb) ++p.near_pairs;
        }
  return p;
}

void plan_coverage(const Plan& p, int& cmin, int& cmax) {
  // For every ordered pair of leaves (X, Y): near-field membership plus the number of
  // (level, direction) interaction lists of X's ancestors containing Y's ancestor.
  const Level& ll = p.lv[p.leaf];
  int nb = ll.nb;
  // per level and class: count grid over offsets
  struct Lookup {
    int R = 0;
    std::vector<int> cnt[4];
    int get(int c, int da, int db) const {
      if (da < -R || da > R || db < -R || db > R) return 0;
      return cnt[c][(da + R) * (2 * R + 1) + (db + R)];
    }
  };
  std::vector<Lookup> lk(p.leaf + 1);
  for (int nu = std::max(1, p.top); nu <= p.leaf; ++nu) {
    const Level& l = p.lv[nu];
    Lookup& L = lk[nu];
    L.R = 2 * l.nb + 2;
    for (int c = 0; c < 4; ++c) {
      L.cnt[c].assign((2 * L.R + 1) * (2 * L.R + 1), 0);
      for (int dir = 0; dir < l.ndir; ++dir)
        for (const Off& d : l.stencil[c * l.ndir + dir]) L.cnt[c][(d.a + L.R) * (2 * L.R + 1) + (d.b + L.R)]++;
    }
  }
  int mn = 1 << 30, mx = 0;
  int nthreads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<int> tmn(nthreads, 1 << 30), tmx(nthreads, 0);
  std::vector<std::thread> th;
  for (int t = 0; t < nthreads; ++t)
    th.emplace_back([&, t]() {
      for (int xa = t; xa < nb; xa += nthreads)
        for (int xb = 0; xb < nb; ++xb)
          for (int ya = 0; ya < nb; ++ya)
            for (int yb = 0; yb < nb; ++yb) {
              int cnt = (std::abs(xa - ya) <= 1 && std::abs(xb - yb) <= 1) ? 1 : 0;
              for (int nu = std::max(1, p.top); nu <= p.leaf; ++nu) {
                int sh = p.leaf - nu;
                int Xa = xa >> sh, Xb = xb >> sh, Ya = ya >> sh, Yb = yb >> sh;
                int c = (Xa & 1) * 2 + (Xb & 1);
                cnt += lk[nu].get(c, Ya - Xa, Yb - Xb);
              }
              tmn[t] = std::min(tmn[t], cnt);
              tmx[t] = std::max(tmx[t], cnt);
            }
    });
  for (auto& x : th) x.join();
  for (int t = 0; t < nthreads; ++t) {
    mn = std::min(mn, tmn[t]);
    mx = std::max(mx, tmx[t]);
  }
  cmin = mn;
  cmax = mx;
}

// ---- dense helpers --------------------------------------------------------------------

// X (r x k, row-major) := X * B^{-1}, B (k x k row-major), by LU with partial pivoting of
// B^T applied to the columns of X^T.
void lu_solve_transposed(const std::vector<zd>& B, int k, std::vector<zd>& X, int r) {
  std::vector<zd> Bt((size_t)k * k);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) Bt[(size_t)i * k + j] = B[(size_t)j * k + i];
  std::vector<int> perm(k);
  for (int i = 0; i < k; ++i) perm[i] = i;
  for (int col = 0; col < k; ++col) {
    int pr = col;
    double best = std::abs(Bt[(size_t)col * k + col]);
    for (int rr = col + 1; rr < k; ++rr) {
      double v = std::abs(Bt[(size_t)rr * k + col]);
      if (v > best) {
        best = v;
        pr = rr;
      }
    }
    if (best == 0.0) throw LsError(-1, "singular pivot block in NCA");
    if (pr != col) {
      for (int j = 0; j < k; ++j) std::swap(Bt[(size_t)pr * k + j], Bt[(size_t)col * k + j]);
      std::swap(perm[pr], perm[col]);
    }
    for (int rr = col + 1; rr < k; ++rr) {
      zd f = Bt[(size_t)rr * k + col] / Bt[(size_t)col * k + col];
      Bt[(size_t)rr * k + col] = f;
      for (int j = col + 1; j < k; ++j) Bt[(size_t)rr * k + j] -= f * Bt[(size_t)col * k + j];
    }
  }
  std::vector<zd> y(k);
  for (int row = 0; row < r; ++row) {
    zd* x = &X[(size_t)row * k];
    for (int i = 0; i < k; ++i) y[i] = x[perm[i]];
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < i; ++j) y[i] -= Bt[(size_t)i * k + j] * y[j];
    for (int i = k - 1; i >= 0; --i) {
      for (int j = i + 1; j < k; ++j) y[i] -= Bt[(size_t)i * k + j] * y[j];
      y[i] /= Bt[(size_t)i * k + i];
    }
    for (int i = 0; i < k; ++i) x[i] = y[i];
  }
}

// ---- NCA (Section 4) -------------------------------------------------------------------

// V(leaf points, leaf points + d * side) for the 9 neighbour offsets d of a leaf (near field)
void nca_near_tiles(const Plan& p, const WTable& W, NCA& out) {
  const int s = p.leaf_side;
  std::vector<Off> leafpts = nca_leaf_points(p);
  out.near.resize(9);
  for (int da = -1; da <= 1; ++da)
    for (int db = -1; db <= 1; ++db) {
      auto& T = out.near[(da + 1) * 3 + (db + 1)];
      T.resize((size_t)s * s * s * s);
      for (int i = 0; i < s * s; ++i)
        for (int j = 0; j < s * s; ++j)
          T[(size_t)i * s * s + j] = W(leafpts[i].a - (leafpts[j].a + da * s), leafpts[i].b - (leafpts[j].b + db * s));
    }
}

std::vector<Off> nca_leaf_points(const Plan& p) {
  std::vector<Off> leafpts;
  for (int a = 0; a < p.leaf_side; ++a)
    for (int b = 0; b < p.leaf_side; ++b) leafpts.push_back({a, b});
  return leafpts;
}

// candidate sets of level nu, direction dir (Section 4.2.2, step 1): targets are the leaf
// points, or the self pivots of the four children; sources are the same sets translated by
// every offset of the direction's far set (the antipodal cone's child pivots)
void nca_candidates(const Plan& p, const NCA& out, int nu, int dir, std::vector<Off>& tcand,
                    std::vector<Off>& scand) {
  const Level& l = p.lv[nu];
  const bool is_leaf = (nu == p.leaf);
  const int s = p.leaf_side;
  const LevelNCA* CL = is_leaf ? nullptr : &out.lv[nu + 1];
  const Level* cl = is_leaf ? nullptr : &p.lv[nu + 1];
  const int cs = is_leaf ? 0 : cl->side;
  auto child_dir = [&](int d) { return (!is_leaf && cl->hf) ? d / 2 : 0; };
  tcand.clear();
  scand.clear();
  std::vector<Off> leafpts = is_leaf ? nca_leaf_points(p) : std::vector<Off>();
  if (is_leaf) {
    tcand = leafpts;
  } else {
    int cd = child_dir(dir);
    for (int c = 0; c < 4; ++c)
      for (const Off& q : CL->self[cd]) tcand.push_back({(c >> 1) * cs + q.a, (c & 1) * cs + q.b});
  }
  int ad = antipodal(dir, l.ndir);
  for (const Off& d : l.farset[dir]) {
    if (is_leaf) {
      for (const Off& q : leafpts) scand.push_back({d.a * s + q.a, d.b * s + q.b});
    } else {
      int cd = child_dir(ad);
      for (int c = 0; c < 4; ++c)
        for (const Off& q : CL->self[cd])
          scand.push_back({d.a * l.side + (c >> 1) * cs + q.a, d.b * l.side + (c & 1) * cs + q.b});
    }
  }
}

// M2L operators (Section 5, transverse pass): K = V(self pivots of B, self pivots of B + d)
void nca_m2l(const Plan& p, const WTable& W, NCA& out) {
  for (int nu = p.top; nu <= p.leaf; ++nu) {
    const Level& l = p.lv[nu];
    LevelNCA& L = out.lv[nu];
    const int nd = l.ndir;
    L.kofs.assign(nd, {});
    L.K.assign(nd, {});
    for (int dir = 0; dir < nd; ++dir) {
      int ad = antipodal(dir, nd);
      const std::vector<Off>& P = L.self[dir];
      const std::vector<Off>& Q = L.self[ad];
      for (const Off& d : l.farset[dir]) {
        std::vector<zd> K(P.size() * Q.size());
        for (size_t i = 0; i < P.size(); ++i)
          for (size_t j = 0; j < Q.size(); ++j)
            K[i * Q.size() + j] = W(P[i].a - (Q[j].a + d.a * l.side), P[i].b - (Q[j].b + d.b * l.side));
        L.kofs[dir].push_back(d);
        L.K[dir].push_back(std::move(K));
      }
    }
  }
}

NCA build_nca(const Plan& p, const WTable& W, double tol) {
  NCA out;
  out.lv.resize(p.leaf + 1);
  const int leaf = p.leaf;
  const int s = p.leaf_side;
  auto Vent = [&](const Off& t, const Off& src) { return W(t.a - src.a, t.b - src.b); };
  std::vector<Off> leafpts = nca_leaf_points(p);
  nca_near_tiles(p, W, out);
  if (p.top > leaf) return out;  // no far field
  int nthreads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  for (int nu = leaf; nu >= p.top; --nu) {
    const Level& l = p.lv[nu];
    LevelNCA& L = out.lv[nu];
    const int nd = l.ndir;
    L.self.assign(nd, {});
    L.far.assign(nd, {});
    L.rank.assign(nd, 0);
    L.C.assign(nd, {});
    const bool is_leaf = (nu == leaf);
    const LevelNCA* CL = is_leaf ? nullptr : &out.lv[nu + 1];
    const Level* cl = is_leaf ? nullptr : &p.lv[nu + 1];
    const int cs = is_leaf ? 0 : cl->side;
    auto child_dir = [&](int dir) { return (!is_leaf && cl->hf) ? dir / 2 : 0; };
    std::vector<std::string> errs(nd);
    auto work = [&](int dir) {
      try {
        std::vector<Off> tcand, scand;
        nca_candidates(p, out, nu, dir, tcand, scand);
        int m = (int)tcand.size(), nn = (int)scand.size();
        // step 2: ACA with accuracy tol on A(tcand, scand)
        ACAResult R = aca(
            m, nn, std::min(m, nn), tol, nullptr,
            [&](int i, zd* row) {
              for (int j = 0; j < nn; ++j) row[j] = Vent(tcand[i], scand[j]);
            },
            [&](int j, zd* col) {
              for (int i = 0; i < m; ++i) col[i] = Vent(tcand[i], scand[j]);
            });
        int k = (int)R.rows.size();
        std::vector<Off>& P = L.self[dir];
        std::vector<Off>& F = L.far[dir];
        for (int t = 0; t < k; ++t) {
          P.push_back(tcand[R.rows[t]]);
          F.push_back(scand[R.cols[t]]);
        }
        L.rank[dir] = k;
        if (k == 0) return;
        std::vector<zd> B((size_t)k * k);
        for (int i = 0; i < k; ++i)
          for (int j = 0; j < k; ++j) B[(size_t)i * k + j] = Vent(P[i], F[j]);
        if (is_leaf) {
          std::vector<zd> X((size_t)s * s * k);
          for (int i = 0; i < s * s; ++i)
            for (int j = 0; j < k; ++j) X[(size_t)i * k + j] = Vent(leafpts[i], F[j]);
          lu_solve_transposed(B, k, X, s * s);
          out.U = std::move(X);
        } else {
          int cd = child_dir(dir);
          const std::vector<Off>& PC = CL->self[cd];
          int kc = (int)PC.size();
          L.C[dir].resize(4);
          for (int c = 0; c < 4; ++c) {
            std::vector<zd> X((size_t)kc * k);
            for (int i = 0; i < kc; ++i) {
              Off t{(c >> 1) * cs + PC[i].a, (c & 1) * cs + PC[i].b};
              for (int j = 0; j < k; ++j) X[(size_t)i * k + j] = Vent(t, F[j]);
            }
            lu_solve_transposed(B, k, X, kc);
            L.C[dir][c] = std::move(X);
          }
        }
      } catch (const std::exception& e) {
        errs[dir] = e.what();
      }
    };
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t)
      th.emplace_back([&, t]() {
        for (int dir = t; dir < nd; dir += nthreads) work(dir);
      });
    for (auto& x : th) x.join();
    for (int dir = 0; dir < nd; ++dir)
      if (!errs[dir].empty()) throw LsError(-1, errs[dir]);
    L.kmax = 0;
    for (int dir = 0; dir < nd; ++dir) L.kmax = std::max(L.kmax, L.rank[dir]);
    if (is_leaf) out.kleaf = L.rank[0];
  }
  nca_m2l(p, W, out);
  return out;
}

}  // namespace ls
