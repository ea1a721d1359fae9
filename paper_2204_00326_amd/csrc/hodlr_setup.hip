// Batched partially pivoted ACA for the off-diagonal blocks of one HODLR level on the device
// (Section 5: fixed-rank compression of the off-diagonal blocks; the pivoting rules of the
// host routine in aca_impl.h: start at the first row not known to be zero, the column pivot is
// the largest residual entry of the pivot row over unused columns, the next row pivot the largest
// entry of the new residual column over unused rows, an exactly zero residual row moves on to the
// first unused row, magnitudes within a relative 1e-9 of the maximum are ties won by the lowest
// index).  Every step runs for all blocks of the level at once; the residual row and column are
// formed from the table of V entries, the contrast and the factors found so far, in the host
// routine's order of operations, and the factors land directly in the device arrays U, V.
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

// residual of the pivot row: r[j] = entry(i, j) - sum_{l < k} U_l[i] V_l[j]
__global__ __launch_bounds__(256) void k_aca_row(AcaLevel L, int only_retry) {
  const int b = blockIdx.y;
  if (L.state[b] != 0 || (only_retry && !L.retry[b])) return;
  const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
  if (j >= L.S) return;
  const BlockGeom g = geom(L, b);
  const long long gi = g.r0 + L.ib[b], gj = g.c0 + j;
  double2 r = entry(L, gi, gj);
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

// column pivot of the residual row (or, for an exactly zero row, the next unused row to try)
__global__ __launch_bounds__(256) void k_aca_colpivot(AcaLevel L, int only_retry) {
  __shared__ double rd[256];
  __shared__ long long ri[256];
  const int b = blockIdx.x;
  if (L.state[b] != 0 || (only_retry && !L.retry[b])) return;
  const BlockGeom g = geom(L, b);
  double mx = 0.0;
  for (long long j = threadIdx.x; j < L.S; j += 256)
    if (!L.col_used[g.c0 + j]) mx = fmax(mx, cabs_(L.rbuf[g.c0 + j]));
  mx = block_max(mx, rd);
  if (mx > 0.0) {
    const double thr = (1.0 - kTie) * mx;
    long long first = LLONG_MAX;
    for (long long j = threadIdx.x; j < L.S; j += 256)
      if (!L.col_used[g.c0 + j] && cabs_(L.rbuf[g.c0 + j]) >= thr && j < first) first = j;
    first = block_min(first, ri);
    if (threadIdx.x == 0) {
      L.row_used[g.r0 + L.ib[b]] = 1;
      L.jb[b] = (int)first;
      L.retry[b] = 0;
    }
    return;
  }
  // zero residual row: mark it used and move to the first unused row
  if (threadIdx.x == 0) L.row_used[g.r0 + L.ib[b]] = 1;
  __syncthreads();
  long long first = LLONG_MAX;
  for (long long i = threadIdx.x; i < L.S; i += 256)
    if (!L.row_used[g.r0 + i] && i < first) first = i;
  first = block_min(first, ri);
  if (threadIdx.x != 0) return;
  if (first == LLONG_MAX) {
    L.state[b] = 1;
    L.retry[b] = 0;
  } else {
    L.ib[b] = (int)first;
    L.retry[b] = 1;
  }
}

// v_k = r / r[j_piv] and the residual of the pivot column u_k[i] = entry(i, j) - sum_l V_l[j] U_l[i]
__global__ __launch_bounds__(256) void k_aca_col(AcaLevel L) {
  const int b = blockIdx.y;
  if (L.state[b] != 0) return;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= L.S) return;
  const BlockGeom g = geom(L, b);
  const int k = L.kcur[b];
  const long long gjp = g.c0 + L.jb[b];
  const double2 piv = L.rbuf[gjp];
  L.V[(long long)k * L.N + g.c0 + i] = cdiv(L.rbuf[g.c0 + i], piv);
  const long long gi = g.r0 + i;
  double2 u = entry(L, gi, gjp);
  for (int l = 0; l < k; ++l) {
    const double2 v = L.V[(long long)l * L.N + gjp];
    if (v.x == 0.0 && v.y == 0.0) continue;
    const double2 w = L.U[(long long)l * L.N + gi];
    u.x -= v.x * w.x - v.y * w.y;
    u.y -= v.x * w.y + v.y * w.x;
  }
  L.U[(long long)k * L.N + gi] = u;
}

// mark the pivot column, count the rank, and pick the next pivot row from the new column
__global__ __launch_bounds__(256) void k_aca_rowpivot(AcaLevel L, int kmax) {
  __shared__ double rd[256];
  __shared__ long long ri[256];
  const int b = blockIdx.x;
  if (L.state[b] != 0) return;
  const BlockGeom g = geom(L, b);
  const int k = L.kcur[b];
  const double2* u = L.U + (long long)k * L.N + g.r0;
  double mx = 0.0;
  for (long long i = threadIdx.x; i < L.S; i += 256)
    if (!L.row_used[g.r0 + i]) mx = fmax(mx, cabs_(u[i]));
  mx = block_max(mx, rd);
  const double thr = (1.0 - kTie) * mx;
  long long first = LLONG_MAX;
  for (long long i = threadIdx.x; i < L.S; i += 256)
    if (!L.row_used[g.r0 + i] && (mx == 0.0 || cabs_(u[i]) >= thr) && i < first) first = i;
  first = block_min(first, ri);
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
