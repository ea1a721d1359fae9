// HODLR factorisation on the device: batched ACA of the off-diagonal blocks, leaf and SMW core inverses.
#pragma once
#include <hip/hip_runtime.h>

namespace lsk {

// One binary level: nb = 2^(l+1) blocks of S x S (block b: node b/2; b even = rows of the first
// child against columns of the second, b odd = the transpose pair).  All arrays are device
// arrays; U, V are the level's factors (column k of block b at k*N + its row / column offset).
struct AcaLevel {
  const double2* W;                // table of V entries, (2n-1)^2, offset (da, db) at (da+n-1)(2n-1)+db+n-1
  const int *ma, *mb;              // grid coordinates of the Morton-ordered points
  const double* q;                 // contrast, Morton order
  double coef;                     // s kappa^2
  int n;                           // grid side
  long long N, S;
  int nb;
  double2 *U, *V;
  unsigned char *row_used, *col_used;  // N each; rows with q = 0 start used
  double2* rbuf;                   // N: residual pivot rows at their blocks' column ranges
  double* pmax;                    // nb * ceil(S / 256): per 256-entry tile, the largest magnitude
                                   // over its unused entries (-1 when it has none)
  int *ib, *jb, *state, *kcur, *retry;  // nb each
};

void launch_aca_start(const AcaLevel& L, hipStream_t s);
// residual pivot rows and their column pivots (a block whose row is exactly zero marks it used,
// moves to its next unused row and sets retry: the column kernels skip it in this step)
void launch_aca_row(const AcaLevel& L, hipStream_t s);
// v_k, u_k and the next pivot rows; blocks stop at kmax or when no row is left
void launch_aca_col(const AcaLevel& L, int kmax, hipStream_t s);
// SMW core inverses of one level (2r <= 512) from t (svec layout: [c][node][2r], the r-column
// W^T Y products) into out (hodlr_core_elems(r) entries per node, 16-row blocks), by the Schur
// complement of the identity block; A: nodes x 4r^2 and B: nodes x r^2 workspaces (at least);
// bad[node] set to 1 where a pivot of the Schur complement is exactly zero
void launch_core_invert(const double2* t, int r, int nodes, double2* A, double2* B, double2* out, int* bad,
                        hipStream_t s);
// inverses of the listed dense leaves (diagonal blocks I + coef diag(q) V of lp <= 512 points,
// V from the table W of an n_grid x n_grid grid) into Dinv (column-major lp x lp at each leaf's
// index); A, B: nleaves x lp^2 workspaces; bad[k] set to 1 where a pivot is exactly zero
void launch_leaf_invert(const double2* W, int n_grid, const int* ma, const int* mb, const double* q, double coef,
                        int lp, const int* leaves, int nleaves, double2* A, double2* B, double2* Dinv, int* bad,
                        hipStream_t s);
// Y[c][i] = 0 for every column c where q[i] == 0 (Y: N x r column-major)
void launch_zero_rows(double2* Y, long long N, int r, const double* q, hipStream_t s);
// identity blocks at the listed leaves of Dinv
void launch_leaf_identity(const int* leaves, int nleaves, int lp, double2* Dinv, hipStream_t s);

}  // namespace lsk
