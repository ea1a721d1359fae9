// Host-side planning for the DAFMM on a uniform cell-centred grid: quadtree levels,
// frequency regimes, directional cones, neighbour and interaction-list stencils, and
// the Nested Cross Approximation (NCA) factors.
#pragma once
#include <complex>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace ls {

using zd = std::complex<double>;

struct LsError : std::runtime_error {
  int code;
  LsError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

struct Off {
  int a, b;
};

struct PlanOptions {
  int leaf_max = 64;
  double T = 16.0;
};

// One quadtree level.  Boxes at level nu form an nb x nb grid; box (ba, bb) covers the
// cells a in [ba*side, (ba+1)*side), b in [bb*side, (bb+1)*side).  The class of a box is
// c = (ba & 1) * 2 + (bb & 1), its position inside its parent.
struct Level {
  int nu = 0, nb = 1, side = 0;
  double w = 0;        // half-width of a box
  bool hf = false;     // (kappa w)^2 > T  (Section 3)
  int ndir = 1;        // cones (HF) or 1 (LF)
  double nbr_r2 = 4;   // neighbour iff |d|^2 < nbr_r2, d in box widths (Section 3.1 / 3.2)
  // interaction-list stencils: stencil[c * ndir + dir] = offsets d with B + d in IL(B[, dir])
  // for an interior box of class c (before clipping at the domain boundary)
  std::vector<std::vector<Off>> stencil;
  // per direction: offsets that occur in the domain for at least one box (far-field
  // candidate region of the NCA pivot search)
  std::vector<std::vector<Off>> farset;
  // per class and direction: stencil offsets that occur in the domain for that class
  std::vector<std::vector<Off>> terms;
  int64_t il_pairs = 0;
  int max_il = 0;
  bool has_il = false;
};

struct Plan {
  int n = 0;           // grid side
  double h = 0, L = 0; // cell size, half-width of the domain
  double kappa = 0;
  int leaf = 0;        // leaf level
  int leaf_side = 0;
  int top = 0;         // coarsest level with a non-empty interaction list (leaf+1 if none)
  double phi0 = 0;     // cone boundaries at phi0 + 2 pi j / ndir
  std::vector<Level> lv;
  int64_t near_pairs = 0;
};

Plan make_plan(int n, double L, double kappa, const PlanOptions& opt);
int cone_of(int da, int db, int ndir, double phi0);
inline int antipodal(int dir, int ndir) { return ndir > 1 ? (dir + ndir / 2) % ndir : 0; }
void plan_coverage(const Plan& p, int& cmin, int& cmax);

// ---- NCA ----------------------------------------------------------------------------
// Offsets are in cells relative to the lower-left cell of the box the pivots belong to.
struct LevelNCA {
  std::vector<std::vector<Off>> self;  // self pivots per direction (incoming = outgoing)
  std::vector<std::vector<Off>> far;   // far-field pivots per direction
  std::vector<int> rank;               // per direction
  int kmax = 0;
  // L2L for parent (this level) -> child: C[dir][c] is (k_child x k_dir), row-major.
  std::vector<std::vector<std::vector<zd>>> C;
  // M2L: K[dir][t] for terms list `kofs[dir]`, (k_dir x k_antipodal) row-major.
  std::vector<std::vector<Off>> kofs;
  std::vector<std::vector<std::vector<zd>>> K;
};

struct NCA {
  std::vector<LevelNCA> lv;  // indexed by level; only levels top..leaf are filled
  std::vector<zd> U;         // leaf L2P: (side^2 x k_leaf) row-major; P2M = U^T
  int kleaf = 0;
  std::vector<std::vector<zd>> near;  // 9 tiles (da,db) in {-1,0,1}^2, index (da+1)*3+(db+1), side^2 x side^2
};

// W(da, db) = V entry for grid offset (da, db); table of (2n-1)^2 values.
struct WTable {
  int n = 0;
  std::vector<zd> w;
  zd operator()(int da, int db) const { return w[(size_t)(da + n - 1) * (2 * n - 1) + (db + n - 1)]; }
};

NCA build_nca(const Plan& p, const WTable& W, double tol);

// Pieces of the NCA shared by the host and the device builds: the leaf's points (grid offsets
// inside a leaf), the 9 near-field tiles, the candidate sets of one level and direction
// (targets: leaf points or the children's self pivots; sources: the far set's translates), and
// the M2L operators from the self pivots of every level.  The interpolation operator of a
// level and direction has one row per target candidate (the leaf points at the leaf level,
// child c's self pivots in rows c * k_child ... at the others).
std::vector<Off> nca_leaf_points(const Plan& p);
void nca_near_tiles(const Plan& p, const WTable& W, NCA& out);
void nca_candidates(const Plan& p, const NCA& out, int nu, int dir, std::vector<Off>& tcand, std::vector<Off>& scand);
void nca_m2l(const Plan& p, const WTable& W, NCA& out);

// Partially pivoted ACA on an m x n block given by entry(i, j), row(i, out), col(j, out).
struct ACAResult {
  std::vector<int> rows, cols;
  std::vector<std::vector<zd>> u, v;  // u_k (m), v_k (n)
};
template <class RowFn, class ColFn>
ACAResult aca(int m, int n, int max_rank, double eps, const std::vector<char>* row_zero, RowFn rowfn, ColFn colfn);

// Dense complex helpers
void lu_solve_transposed(const std::vector<zd>& B, int k, std::vector<zd>& X, int r);  // X (r x k) := X B^{-1}

}  // namespace ls

#include "aca_impl.h"
