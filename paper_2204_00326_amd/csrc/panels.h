// High-order leaf panels (paper, Section 2.2, Eqs. (eq:7)-(eq:13)) on a uniform tree: device
// tables of the box moments of G against the Chebyshev basis, the blocks of the discrete volume
// operator, and its product.
//
// Geometry: nside x nside leaf boxes of half-width beta tile [-L, L]^2; box k = ix * nside + iy
// has centre (-L + (2 ix + 1) beta, -L + (2 iy + 1) beta).  Each box carries the p x p tensor
// Chebyshev points of the first kind (ascending), node a = i * p + j at centre + beta (x_i, x_j).
// The basis b_l(u, v) = T_a(u) T_b(v), a + b < p, is ordered by total degree, then by a
// (N_p = p (p + 1) / 2 members).  On a uniform tree the moment of source box B at a node of
// box A depends only on the box offset d = A - B, so one table row per offset serves every pair.
#pragma once
#include <hip/hip_runtime.h>

namespace lsp {

constexpr int kMaxP = 8;                        // nodes per box side
constexpr int kMaxNp = kMaxP * (kMaxP + 1) / 2;  // basis functions
constexpr int kRay = 48;                        // Gauss-Legendre points along a Duffy ray
constexpr int kAcross = 48;                     // points across a triangle, per side of the foot
constexpr long long kDenseMaxN = 20000;         // unknowns of the dense operator of a general tree

struct PanelGeom {
  int nside, p, np, n2;  // n2 = p * p
  double beta, kappa;
  int nfar;               // Gauss-Legendre points per direction of the far rule
};

// Reference data the host computes once (Gauss-Legendre rules, Chebyshev nodes, the basis
// exponents), uploaded as one buffer.
struct PanelRef {
  double node[kMaxP];               // Chebyshev points of the first kind, ascending
  int ba[kMaxNp], bb[kMaxNp];       // basis l = T_ba(u) T_bb(v)
  double ray_t[kRay], ray_w[kRay];  // Gauss-Legendre on [0, 1]
  double acr_t[kAcross], acr_w[kAcross];
};

// M[d][a][l] (complex, interleaved) for every offset d = (dx + nside - 1) * (2 nside - 1) +
// (dy + nside - 1).  far_x / far_w: the nfar-point Gauss-Legendre rule on [-1, 1].
void launch_panel_moments(const PanelGeom& g, const PanelRef* ref, const double* far_x, const double* far_w,
                          double2* M, hipStream_t s);
// T[d] = M[d] Qdag (n2 x n2 per offset, row = target node, column = source node); Qdag: N_p x n2.
void launch_panel_blocks(const PanelGeom& g, const double2* M, const double* Qdag, double2* T, hipStream_t s);
// y = alpha x + coef diag(q) (V x) for nrhs columns (leading dimension ld); q may be NULL (= 1).
void launch_panel_apply(const PanelGeom& g, const double2* T, const double* q, const double2* x, long long ldx,
                        double2* y, long long ldy, int nrhs, double alpha, double coef, hipStream_t s);

// The same product on the matrix cores (FP64 MFMA, p <= kMfmaMaxP) from the column-major blocks
// Tt[d] = T[d]^T (launch_panel_blocks_t): x copied node-major into xt (nrhs x N), partial planes
// of nchunks chunks of the offsets (part: nchunks x nrhs x N complex), then their sum in chunk
// order.  Tiles of 16 target boxes, panel_tile_y(g) of them along y.
constexpr int kMfmaMaxP = 5;
int panel_tile_y(const PanelGeom& g);
int panel_chunks(const PanelGeom& g, int nrhs);
void launch_panel_blocks_t(const PanelGeom& g, const double2* T, double2* Tt, hipStream_t s);
void launch_panel_apply_mfma(const PanelGeom& g, const double2* Tt, const double* q, const double2* x, long long ldx,
                             double2* y, long long ldy, int nrhs, double alpha, double coef, double2* part,
                             double2* xt, int nchunks, hipStream_t s);

// Leaves of any tree (an adaptive, level-restricted one included): boxes[5 B ..] = (cx, cy, beta,
// offset of the box's far rule in far_x / far_w, its points per direction); X: the N nodes (x, y).
// M[i][B][l] for every target node i and box B (same rules as launch_panel_moments), then the
// dense V (N x N row-major, column B * n2 + b) and its product.
void launch_panel_moments_leaves(const PanelRef* ref, int p, int np, double kappa, const double* boxes, int nboxes,
                                 const double2* X, long long N, const double* far_x, const double* far_w, double2* M,
                                 hipStream_t s);
void launch_panel_dense_V(const double2* M, const double* Qdag, int nboxes, int np, int n2, double2* V, hipStream_t s);
void launch_panel_dense_apply(const double2* V, long long N, const double* q, const double2* x, long long ldx,
                              double2* y, long long ldy, int nrhs, double alpha, double coef, hipStream_t s);

// Krylov vectors of the panel solver: part[i * nch + c] = chunk c of Q_i^H w (the host adds the
// chunks in order); w -= sum_i c[i] Q_i (c on the device); y = alpha a + beta b.
void launch_panel_dots(const double2* Q, long long ldq, int nvec, const double2* w, long long N, double2* part,
                       int nch, hipStream_t s);
void launch_panel_update(double2* w, const double2* Q, long long ldq, int nvec, const double2* c, long long N,
                         hipStream_t s);
// HODLR order with padding (perm[t] < 0: a padding unknown): gather into M rows (zeros at the
// padding) or scatter back (padding rows dropped)
void launch_panel_permute(const double2* x, long long ldx, double2* y, long long ldy, const int* perm, long long M,
                          int nrhs, bool scatter, hipStream_t s);
void launch_panel_combo(double2* y, const double2* a, double alpha, const double2* b, double beta, long long N,
                        hipStream_t s);

}  // namespace lsp
