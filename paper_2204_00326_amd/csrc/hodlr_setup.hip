// HODLR factorisation on the device (Section 6).
//
// Batched partially pivoted ACA for the off-diagonal blocks of one level (fixed-rank compression
// of the off-diagonal blocks), with the pivoting rules of the host routine in aca_impl.h: start at
// the first row not known to be zero, the column pivot is the largest residual entry of the pivot
// row over unused columns, the next row pivot the largest entry of the new residual column over
// unused rows, an exactly zero residual row moves on to the first unused row, magnitudes within a
// relative 1e-9 of the maximum are ties won by the lowest index.  Every step runs for all blocks
// of the level at once (a block whose pivot row was exactly zero only moves to its next row in
// that step, and adds its term in a later one); the residual row and column are formed from the
// table of V entries, the contrast and the factors found so far, in the host routine's order of
// operations, and the factors land directly in the device arrays U, V.  The pivot searches are
// two-stage: the kernels that form a residual row or column also write the largest magnitude over
// the unused entries of each 256-entry tile; the pivot kernel takes the maximum over the tiles,
// finds the first tile that reaches the tie threshold and scans only that tile for the first
// index that does (the first tile reaching it holds the first such index), so a block of 131072
// entries costs one workgroup a few hundred reads.
//
// Inverses of the dense leaf blocks (Gauss-Jordan) and of the SMW cores (through the Schur
// complement of their identity block), written in the layouts the apply kernels read.
#include <hip/hip_runtime.h>

#include <climits>
#include <stdexcept>

#include "hodlr_setup.h"

namespace lsk {

namespace {

constexpr double kTie = 1e-9;

struct BlockGeom {
  long long r0, c0;
};

__device__ inline BlockGeom geom(const AcaLevel& L, int b) {
  const long long node = b >> 1, lo = node * 2 * L.S, mid = lo + L.S;
  return (b & 1) ? BlockGeom{mid, lo} : BlockGeom{lo, mid};
}

// coef q[gi] W(a_i - a_j, b_i - b_j)
__device__ inline double2 entry(const AcaLevel& L, long long gi, long long gj) {
  const double cq = L.coef * L.q[gi];
  const double2 w = L.W[(long long)(L.ma[gi] - L.ma[gj] + L.n - 1) * (2 * L.n - 1) + (L.mb[gi] - L.mb[gj] + L.n - 1)];
  return make_double2(cq * w.x, cq * w.y);
}

__device__ inline double cabs_(double2 a) { return hypot(a.x, a.y); }

// (a / b) by Smith's scaling
__device__ inline double2 cdiv(double2 a, double2 b) {
  if (fabs(b.y) <= fabs(b.x)) {
    const double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  }
  const double r = b.x / b.y, d = b.y + b.x * r;
  return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}

// block-wide max (and, below, min) over 256 threads; LLONG_MAX stands for "none"
__device__ inline double block_max(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ inline long long block_min(long long v, long long* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s && red[threadIdx.x + s] < red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + s];
    __syncthreads();
  }
  const long long r = red[0];
  __syncthreads();
  return r;
}

}  // namespace

// first unused row of every block (rows with q = 0 are marked used beforehand)
__global__ __launch_bounds__(256) void k_aca_start(AcaLevel L) {
  __shared__ long long ri[256];
  const int b = blockIdx.x;
  const BlockGeom g = geom(L, b);
  long long first = LLONG_MAX;
  for (long long i = threadIdx.x; i < L.S; i += 256)
    if (!L.row_used[g.r0 + i] && i < first) first = i;
  first = block_min(first, ri);
  if (threadIdx.x != 0) return;
  L.kcur[b] = 0;
  L.retry[b] = 0;
  if (first == LLONG_MAX) {
    L.state[b] = 1;
  } else {
    L.state[b] = 0;
    L.ib[b] = (int)first;
  }
}

// largest magnitude over the unused entries of this workgroup's tile (-1: none), to pmax
__device__ inline void tile_max(const AcaLevel& L, int b, double v, bool use, double* red) {
  const double m = block_max(use ? v : -1.0, red);
  if (threadIdx.x == 0) L.pmax[(long long)b * gridDim.x + blockIdx.x] = m;
}

// pivot of a block from its tile maxima and the values: the first index (lowest) among unused
// entries whose magnitude reaches (1 - kTie) * max, or, with max == 0 and allow_zero, the first
// unused entry; LLONG_MAX when there is none (or max == 0 without allow_zero).  mx_out: the max.
__device__ long long pick_pivot(const AcaLevel& L, int b, long long ntiles, const double2* vals,
                                const unsigned char* used, bool allow_zero, double* mx_out, double* rd,
                                long long* ri) {
  const double* pm = L.pmax + (long long)b * ntiles;
  double mx = -1.0;
  for (long long w = threadIdx.x; w < ntiles; w += 256) mx = fmax(mx, pm[w]);
  mx = block_max(mx, rd);
  *mx_out = mx;
  if (mx < 0.0 || (mx == 0.0 && !allow_zero)) return LLONG_MAX;
  const double thr = mx == 0.0 ? 0.0 : (1.0 - kTie) * mx;
  long long wf = LLONG_MAX;
  for (long long w = threadIdx.x; w < ntiles; w += 256)
    if (pm[w] >= thr && w < wf) wf = w;
  wf = block_min(wf, ri);
  if (wf == LLONG_MAX) return LLONG_MAX;
  const long long j = wf * 256 + threadIdx.x;
  long long first = LLONG_MAX;
  if (j < L.S && !used[j] && (mx == 0.0 || cabs_(vals[j]) >= thr)) first = j;
  return block_min(first, ri);
}

// residual of the pivot row: r[j] = entry(i, j) - sum_{l < k} U_l[i] V_l[j]
__global__ __launch_bounds__(256) void k_aca_row(AcaLevel L) {
  __shared__ double rd[256];
  const int b = blockIdx.y;
  if (L.state[b] != 0) return;
  const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
  const BlockGeom g = geom(L, b);
  double2 r = make_double2(0.0, 0.0);
  const bool in = j < L.S;
  if (in) {
    const long long gi = g.r0 + L.ib[b], gj = g.c0 + j;
    r = entry(L, gi, gj);
    const int k = L.kcur[b];
    for (int l = 0; l < k; ++l) {
      const double2 u = L.U[(long long)l * L.N + gi];
      if (u.x == 0.0 && u.y == 0.0) continue;
      const double2 v = L.V[(long long)l * L.N + gj];
      r.x -= u.x * v.x - u.y * v.y;
      r.y -= u.x * v.y + u.y * v.x;
    }
    L.rbuf[gj] = r;
  }
  tile_max(L, b, cabs_(r), in && !L.col_used[g.c0 + j], rd);
}

// column pivot of the residual row (or, for an exactly zero row, the next unused row to try)
__global__ __launch_bounds__(256) void k_aca_colpivot(AcaLevel L) {
  __shared__ double rd[256];
  __shared__ long long ri[256];
  const int b = blockIdx.x;
  if (L.state[b] != 0) return;
  const BlockGeom g = geom(L, b);
  double mx;
  const long long first = pick_pivot(L, b, (L.S + 255) / 256, L.rbuf + g.c0, L.col_used + g.c0, false, &mx, rd, ri);
  if (mx > 0.0) {
    if (threadIdx.x == 0) {
      L.row_used[g.r0 + L.ib[b]] = 1;
      L.jb[b] = (int)first;
      L.retry[b] = 0;
    }
    return;
  }
  // zero residual row (or no unused column): mark the row used and move to the first unused row
  if (threadIdx.x == 0) L.row_used[g.r0 + L.ib[b]] = 1;
  __syncthreads();
  long long fr = LLONG_MAX;
  for (long long i = threadIdx.x; i < L.S; i += 256)
    if (!L.row_used[g.r0 + i] && i < fr) fr = i;
  fr = block_min(fr, ri);
  if (threadIdx.x != 0) return;
  if (fr == LLONG_MAX) {
    L.state[b] = 1;
    L.retry[b] = 0;
  } else {
    L.ib[b] = (int)fr;
    L.retry[b] = 1;
  }
}

// v_k = r / r[j_piv] and the residual of the pivot column u_k[i] = entry(i, j) - sum_l V_l[j] U_l[i]
__global__ __launch_bounds__(256) void k_aca_col(AcaLevel L) {
  __shared__ double rd[256];
  const int b = blockIdx.y;
  if (L.state[b] != 0 || L.retry[b]) return;  // retry: the row was zero, the next step tries another
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const BlockGeom g = geom(L, b);
  const bool in = i < L.S;
  double2 u = make_double2(0.0, 0.0);
  if (in) {
    const int k = L.kcur[b];
    const long long gjp = g.c0 + L.jb[b];
    const double2 piv = L.rbuf[gjp];
    L.V[(long long)k * L.N + g.c0 + i] = cdiv(L.rbuf[g.c0 + i], piv);
    const long long gi = g.r0 + i;
    u = entry(L, gi, gjp);
    for (int l = 0; l < k; ++l) {
      const double2 v = L.V[(long long)l * L.N + gjp];
      if (v.x == 0.0 && v.y == 0.0) continue;
      const double2 w = L.U[(long long)l * L.N + gi];
      u.x -= v.x * w.x - v.y * w.y;
      u.y -= v.x * w.y + v.y * w.x;
    }
    L.U[(long long)k * L.N + gi] = u;
  }
  tile_max(L, b, cabs_(u), in && !L.row_used[g.r0 + i], rd);
}

// mark the pivot column, count the rank, and pick the next pivot row from the new column
__global__ __launch_bounds__(256) void k_aca_rowpivot(AcaLevel L, int kmax) {
  __shared__ double rd[256];
  __shared__ long long ri[256];
  const int b = blockIdx.x;
  if (L.state[b] != 0 || L.retry[b]) return;
  const BlockGeom g = geom(L, b);
  const int k = L.kcur[b];
  double mx;
  const long long first = pick_pivot(L, b, (L.S + 255) / 256, L.U + (long long)k * L.N + g.r0, L.row_used + g.r0, true,
                                     &mx, rd, ri);
  if (threadIdx.x != 0) return;
  L.col_used[g.c0 + L.jb[b]] = 1;
  L.kcur[b] = k + 1;
  if (k + 1 >= kmax || first == LLONG_MAX) {
    L.state[b] = 1;
  } else {
    L.ib[b] = (int)first;
  }
}

// Gauss-Jordan inversion of the n x n matrix A (row-major, n <= 512) by one workgroup of 1024
// threads, B = A^-1 on return (B must hold the identity on entry).  Per column: the pivot is the
// largest magnitude at or below the diagonal (the lowest row among equals), the pivot row is
// swapped up and scaled, and multiples of it are subtracted from every other row.  Columns left
// of the pivot are already unit columns and are skipped.  Returns false (for every thread) on
// an exactly zero pivot.
__device__ bool gj_invert(double2* A, double2* B, int n) {
  constexpr int NT = 1024;
  __shared__ double rv[512];
  __shared__ int rix[512];
  __shared__ double2 f[512], arow[512], brow[512];
  __shared__ int pivr;
  __shared__ double2 pinv;
  const int tid = threadIdx.x;
  const int tr = tid >> 6, tj = tid & 63;  // 16 row groups x 64 columns
  for (int col = 0; col < n; ++col) {
    if (tid < 512) {
      rv[tid] = (tid >= col && tid < n) ? cabs_(A[(long long)tid * n + col]) : -1.0;
      rix[tid] = tid;
    }
    __syncthreads();
    for (int st = 256; st > 0; st >>= 1) {
      if (tid < st) {
        const double v2 = rv[tid + st];
        const int i2 = rix[tid + st];
        if (v2 > rv[tid] || (v2 == rv[tid] && i2 < rix[tid])) {
          rv[tid] = v2;
          rix[tid] = i2;
        }
      }
      __syncthreads();
    }
    if (rv[0] <= 0.0) return false;  // the same value for every thread: all leave together
    if (tid == 0) pivr = rix[0];
    __syncthreads();
    const int pr = pivr;
    // swap rows pr and col (A: columns >= col; B: all)
    for (int j = tid; j < n; j += NT) {
      if (pr != col) {
        if (j >= col) {
          const double2 a1 = A[(long long)pr * n + j], a2 = A[(long long)col * n + j];
          A[(long long)pr * n + j] = a2;
          A[(long long)col * n + j] = a1;
        }
        const double2 b1 = B[(long long)pr * n + j], b2 = B[(long long)col * n + j];
        B[(long long)pr * n + j] = b2;
        B[(long long)col * n + j] = b1;
      }
    }
    __syncthreads();
    if (tid == 0) pinv = cdiv(make_double2(1.0, 0.0), A[(long long)col * n + col]);
    // multipliers of every other row (before the pivot row changes)
    for (int i = tid; i < n; i += NT) f[i] = A[(long long)i * n + col];
    __syncthreads();
    const double2 iv = pinv;
    for (int j = tid; j < n; j += NT) {
      double2 bb = B[(long long)col * n + j];
      bb = make_double2(bb.x * iv.x - bb.y * iv.y, bb.x * iv.y + bb.y * iv.x);
      B[(long long)col * n + j] = bb;
      brow[j] = bb;
      if (j >= col) {
        double2 a = A[(long long)col * n + j];
        a = make_double2(a.x * iv.x - a.y * iv.y, a.x * iv.y + a.y * iv.x);
        A[(long long)col * n + j] = a;
        arow[j] = a;
      }
    }
    __syncthreads();
    for (int i = tr; i < n; i += NT / 64) {
      if (i == col) continue;
      const double2 fi = f[i];
      if (fi.x == 0.0 && fi.y == 0.0) continue;
      for (int j = col + tj; j < n; j += 64) {
        const double2 p = arow[j];
        double2 a = A[(long long)i * n + j];
        a.x -= fi.x * p.x - fi.y * p.y;
        a.y -= fi.x * p.y + fi.y * p.x;
        A[(long long)i * n + j] = a;
      }
      for (int j = tj; j < n; j += 64) {
        const double2 p = brow[j];
        double2 bb = B[(long long)i * n + j];
        bb.x -= fi.x * p.x - fi.y * p.y;
        bb.y -= fi.x * p.y + fi.y * p.x;
        B[(long long)i * n + j] = bb;
      }
    }
    __syncthreads();
  }
  return true;
}

// Batched complex n x n products C = alpha A B (+ I), one 16 x 16 tile of C per workgroup and
// node (grid: tiles x nodes).  Element (i, k) of A is at A[node aN + i aI + k aK], likewise B and
// C, so the operands can be read in place from the t layout; a tile is loaded along whichever
// index has unit stride.
__global__ __launch_bounds__(256) void k_bgemm(const double2* __restrict__ A, long long aI, long long aK, long long aN,
                                               const double2* __restrict__ B, long long bK, long long bJ,
                                               long long bN, double2* __restrict__ C, long long cI, long long cJ,
                                               long long cN, int n, double alpha, int add_identity) {
  __shared__ double2 As[16][17], Bs[16][17];
  const int nt = (n + 15) / 16;
  const int ti = blockIdx.x / nt, tj = blockIdx.x - ti * nt;
  const long long node = blockIdx.y;
  const int li = threadIdx.x >> 4, lj = threadIdx.x & 15;
  double re = 0, im = 0;
  for (int k0 = 0; k0 < n; k0 += 16) {
    {
      const int x = aI == 1 ? lj : li, y = aI == 1 ? li : lj;  // As[x][y] = A(16 ti + x, k0 + y)
      const int ai = ti * 16 + x, ak = k0 + y;
      As[x][y] = (ai < n && ak < n) ? A[node * aN + ai * aI + ak * aK] : make_double2(0.0, 0.0);
    }
    {
      const int x = bK == 1 ? lj : li, y = bK == 1 ? li : lj;  // Bs[x][y] = B(k0 + x, 16 tj + y)
      const int bk = k0 + x, bj = tj * 16 + y;
      Bs[x][y] = (bk < n && bj < n) ? B[node * bN + bk * bK + bj * bJ] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const double2 u = As[li][kk], v = Bs[kk][lj];
      re = fma(u.x, v.x, re);
      re = fma(-u.y, v.y, re);
      im = fma(u.x, v.y, im);
      im = fma(u.y, v.x, im);
    }
    __syncthreads();
  }
  const int i = ti * 16 + li, j = tj * 16 + lj;
  if (i < n && j < n)
    C[node * cN + i * cI + j * cJ] = make_double2(alpha * re + (add_identity && i == j ? 1.0 : 0.0), alpha * im);
}

// S^-1 for every node (S row-major n x n, destroyed), one workgroup per node
__global__ __launch_bounds__(1024) void k_gj_batch(double2* __restrict__ Sw, double2* __restrict__ Siw, int n,
                                                   int* __restrict__ bad) {
  const long long node = blockIdx.x;
  double2* S = Sw + node * n * n;
  double2* Si = Siw + node * n * n;
  for (int idx = threadIdx.x; idx < n * n; idx += 1024)
    Si[idx] = make_double2(idx % (n + 1) == 0 ? 1.0 : 0.0, 0.0);
  __syncthreads();
  if (!gj_invert(S, Si, n) && threadIdx.x == 0) bad[node] = 1;
}

// K^-1 from its blocks, in the 16-row-block layout of the apply:
// [[TL, -P], [-Q, S^-1]] with P = X S^-1, Q = S^-1 Z, TL = I + P Z (all r x r row-major per node)
__global__ __launch_bounds__(256) void k_core_assemble(const double2* __restrict__ Si, const double2* __restrict__ P,
                                                       const double2* __restrict__ Q, const double2* __restrict__ TL,
                                                       int r, double2* __restrict__ out) {
  const long long node = blockIdx.x;
  const int n = 2 * r, nb = (n + 15) / 16;
  const long long rr = (long long)r * r;
  double2* D = out + node * nb * 16 * n;
  for (int idx = threadIdx.x; idx < nb * 16 * n; idx += 256) {
    const int blk = idx / (16 * n), rem = idx - blk * 16 * n;
    const int j = rem >> 4, i = blk * 16 + (rem & 15);
    double2 v = make_double2(0.0, 0.0);
    if (i < r && j < r) {
      v = TL[node * rr + (long long)i * r + j];
    } else if (i < r && j < n) {
      const double2 p = P[node * rr + (long long)i * r + (j - r)];
      v = make_double2(-p.x, -p.y);
    } else if (i < n && j < r) {
      const double2 q = Q[node * rr + (long long)(i - r) * r + j];
      v = make_double2(-q.x, -q.y);
    } else if (i < n) {
      v = Si[node * rr + (long long)(i - r) * r + (j - r)];
    }
    D[idx] = v;
  }
}

// Dense HODLR leaves (diagonal blocks I + s kappa^2 diag(q) V of lp points), one workgroup per
// listed leaf: formed from the table of V entries, inverted by gj_invert, written column-major to
// Dinv at the leaf's index.  A, B: per-listed-leaf workspaces; bad[k] = 1 for a zero pivot.
__global__ __launch_bounds__(1024) void k_leaf_invert(const double2* __restrict__ Wt, int n_grid,
                                                      const int* __restrict__ ma, const int* __restrict__ mb,
                                                      const double* __restrict__ q, double coef, int lp,
                                                      const int* __restrict__ leaves, double2* __restrict__ Aw,
                                                      double2* __restrict__ Bw, double2* __restrict__ Dinv,
                                                      int* __restrict__ bad) {
  const int k = blockIdx.x, tid = threadIdx.x;
  const long long leaf = leaves[k], base = leaf * lp;
  double2* A = Aw + (long long)k * lp * lp;
  double2* B = Bw + (long long)k * lp * lp;
  for (int idx = tid; idx < lp * lp; idx += 1024) {
    const int m = idx / lp, c = idx - m * lp;
    const double2 w = Wt[(long long)(ma[base + m] - ma[base + c] + n_grid - 1) * (2 * n_grid - 1) +
                         (mb[base + m] - mb[base + c] + n_grid - 1)];
    const double cq = coef * q[base + m];
    A[idx] = make_double2((m == c ? 1.0 : 0.0) + cq * w.x, cq * w.y);
    B[idx] = make_double2(m == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  if (!gj_invert(A, B, lp)) {
    if (tid == 0) bad[k] = 1;
    return;
  }
  double2* D = Dinv + leaf * lp * lp;  // column-major: (m, c) at c * lp + m
  for (int idx = tid; idx < lp * lp; idx += 1024) {
    const int c = idx / lp, m = idx - c * lp;
    D[idx] = B[(long long)m * lp + c];
  }
}

// identity blocks (leaves without contrast)
__global__ __launch_bounds__(256) void k_leaf_identity(const int* __restrict__ leaves, int lp, double2* __restrict__ Dinv) {
  double2* D = Dinv + (long long)leaves[blockIdx.x] * lp * lp;
  for (int idx = threadIdx.x; idx < lp * lp; idx += 256) D[idx] = make_double2(idx % (lp + 1) == 0 ? 1.0 : 0.0, 0.0);
}

void launch_leaf_identity(const int* leaves, int nleaves, int lp, double2* Dinv, hipStream_t s) {
  if (nleaves > 0) k_leaf_identity<<<nleaves, 256, 0, s>>>(leaves, lp, Dinv);
}

void launch_leaf_invert(const double2* W, int n_grid, const int* ma, const int* mb, const double* q, double coef,
                        int lp, const int* leaves, int nleaves, double2* A, double2* B, double2* Dinv, int* bad,
                        hipStream_t s) {
  if (lp > 512) throw std::runtime_error("HODLR leaves need at most 512 points");
  if (nleaves > 0) k_leaf_invert<<<nleaves, 1024, 0, s>>>(W, n_grid, ma, mb, q, coef, lp, leaves, A, B, Dinv, bad);
}

// K = I + [0, X; Z, 0], X[i][c] = t[c][node][i], Z[i][c] = t[c][node][r + i] (t: [c][node][2r]).
// By the Schur complement of the identity block, S = I - Z X and
//   K^-1 = [[I + X S^-1 Z, -X S^-1], [-S^-1 Z, S^-1]]:
// four batched r x r products and one batched Gauss-Jordan of order r instead of order 2r.
void launch_core_invert(const double2* t, int r, int nodes, double2* A, double2* B, double2* out, int* bad,
                        hipStream_t s) {
  if (2 * r > 512) throw std::runtime_error("HODLR cores need rank <= 256");
  if (r <= 0 || nodes <= 0) return;
  const long long rr = (long long)r * r, r2 = 2 * r, tn = (long long)nodes * r2;
  double2 *S = A, *P = A + nodes * rr, *Q = A + 2 * nodes * rr, *TL = A + 3 * nodes * rr, *Si = B;
  const int nt = (r + 15) / 16;
  const dim3 grid((unsigned)(nt * nt), (unsigned)nodes);
  const double2 *X = t, *Z = t + r;  // X(i, k) at X[node r2 + i + k tn], Z likewise
  // S = I - Z X
  k_bgemm<<<grid, 256, 0, s>>>(Z, 1, tn, r2, X, 1, tn, r2, S, r, 1, rr, r, -1.0, 1);
  // S^-1 (S destroyed)
  k_gj_batch<<<nodes, 1024, 0, s>>>(S, Si, r, bad);
  // P = X S^-1, Q = S^-1 Z, TL = I + P Z
  k_bgemm<<<grid, 256, 0, s>>>(X, 1, tn, r2, Si, r, 1, rr, P, r, 1, rr, r, 1.0, 0);
  k_bgemm<<<grid, 256, 0, s>>>(Si, r, 1, rr, Z, 1, tn, r2, Q, r, 1, rr, r, 1.0, 0);
  k_bgemm<<<grid, 256, 0, s>>>(P, r, 1, rr, Z, 1, tn, r2, TL, r, 1, rr, r, 1.0, 1);
  k_core_assemble<<<nodes, 256, 0, s>>>(Si, P, Q, TL, r, out);
}

// rows of a factor (N x r, column-major) that belong to points without contrast set to zero
__global__ __launch_bounds__(256) void k_zero_rows(double2* __restrict__ Y, long long N, int r,
                                                   const double* __restrict__ q) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= N || q[i] != 0.0) return;
  for (int c = 0; c < r; ++c) Y[(long long)c * N + i] = make_double2(0.0, 0.0);
}

void launch_zero_rows(double2* Y, long long N, int r, const double* q, hipStream_t s) {
  if (N > 0 && r > 0) k_zero_rows<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(Y, N, r, q);
}

void launch_aca_start(const AcaLevel& L, hipStream_t s) { k_aca_start<<<L.nb, 256, 0, s>>>(L); }

void launch_aca_row(const AcaLevel& L, hipStream_t s) {
  dim3 grid((unsigned)((L.S + 255) / 256), L.nb);
  k_aca_row<<<grid, 256, 0, s>>>(L);
  k_aca_colpivot<<<L.nb, 256, 0, s>>>(L);
}

void launch_aca_col(const AcaLevel& L, int kmax, hipStream_t s) {
  dim3 grid((unsigned)((L.S + 255) / 256), L.nb);
  k_aca_col<<<grid, 256, 0, s>>>(L);
  k_aca_rowpivot<<<L.nb, 256, 0, s>>>(L, kmax);
}

}  // namespace lsk
