// Batched partially pivoted ACA for the off-diagonal blocks of one HODLR level on the device
// (Section 5: fixed-rank compression of the off-diagonal blocks; the pivoting rules of the
// host routine in aca_impl.h: start at the first row not known to be zero, the column pivot is
// the largest residual entry of the pivot row over unused columns, the next row pivot the largest
// entry of the new residual column over unused rows, an exactly zero residual row moves on to the
// first unused row, magnitudes within a relative 1e-9 of the maximum are ties won by the lowest
// index).  Every step runs for all blocks of the level at once; the residual row and column are
// formed from the table of V entries, the contrast and the factors found so far, in the host
// routine's order of operations, and the factors land directly in the device arrays U, V.
// The pivot searches are two-stage: the kernels that form a residual row or column also write
// the largest magnitude over the unused entries of each 256-entry tile; the pivot kernel takes
// the maximum over the tiles, finds the first tile that reaches the tie threshold and scans
// only that tile for the first index that does (the first tile reaching it holds the first
// such index), so a block of 131072 entries costs one workgroup a few hundred reads.
#include <hip/hip_runtime.h>

#include <climits>

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
__global__ __launch_bounds__(256) void k_aca_row(AcaLevel L, int only_retry) {
  __shared__ double rd[256];
  const int b = blockIdx.y;
  if (L.state[b] != 0 || (only_retry && !L.retry[b])) return;
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
__global__ __launch_bounds__(256) void k_aca_colpivot(AcaLevel L, int only_retry) {
  __shared__ double rd[256];
  __shared__ long long ri[256];
  const int b = blockIdx.x;
  if (L.state[b] != 0 || (only_retry && !L.retry[b])) return;
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
  if (L.state[b] != 0) return;
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
  if (L.state[b] != 0) return;
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

void launch_aca_start(const AcaLevel& L, hipStream_t s) { k_aca_start<<<L.nb, 256, 0, s>>>(L); }

void launch_aca_row(const AcaLevel& L, bool only_retry, hipStream_t s) {
  dim3 grid((unsigned)((L.S + 255) / 256), L.nb);
  k_aca_row<<<grid, 256, 0, s>>>(L, only_retry ? 1 : 0);
  k_aca_colpivot<<<L.nb, 256, 0, s>>>(L, only_retry ? 1 : 0);
}

void launch_aca_col(const AcaLevel& L, int kmax, hipStream_t s) {
  dim3 grid((unsigned)((L.S + 255) / 256), L.nb);
  k_aca_col<<<grid, 256, 0, s>>>(L);
  k_aca_rowpivot<<<L.nb, 256, 0, s>>>(L, kmax);
}

}  // namespace lsk
