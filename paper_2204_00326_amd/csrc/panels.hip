// High-order leaf panels on a uniform tree (paper, Section 2.2, Eqs. (eq:7)-(eq:13); the moment
// tables of Section 2.3): device kernels.  Layouts and geometry are described in panels.h.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "h0.h"
#include "panels.h"

namespace lsp {

static_assert(sizeof(PanelRef) % sizeof(double) == 0, "PanelRef is copied as doubles");

namespace {

// G(r) = (i/4) H0^(1)(kappa r)
__device__ inline double2 green(double kappa, double r) {
  const lsk::cplx h = lsk::hankel0(kappa * r);
  return make_double2(-0.25 * h.im, 0.25 * h.re);
}

// T_0..T_{p-1} at x by the three-term recurrence
__device__ inline void cheb_all(int p, double x, double* T) {
  T[0] = 1.0;
  if (p > 1) T[1] = x;
  for (int n = 2; n < p; ++n) T[n] = 2.0 * x * T[n - 1] - T[n - 2];
}

// acc[l] += g * b_l(u, v)
__device__ inline void add_basis(const PanelRef& R, int p, int np, double u, double v, double2 g, double2* acc) {
  double Tu[kMaxP], Tv[kMaxP];
  cheb_all(p, u, Tu);
  cheb_all(p, v, Tv);
#pragma unroll
  for (int l = 0; l < kMaxNp; ++l) {
    if (l < np) {
      const double b = Tu[R.ba[l]] * Tv[R.bb[l]];
      acc[l].x = fma(g.x, b, acc[l].x);
      acc[l].y = fma(g.y, b, acc[l].y);
    }
  }
}

}  // namespace

// One workgroup per (offset d, target node a): M[d][a][l] = int_B G(|x - y|) b_l((y - c_B) / beta) dy
// with x the target node relative to the source box centre c_B.  Targets at least beta away from
// the box take the tensor Gauss-Legendre rule (nfar points per direction); nearer ones split the
// box into the four signed triangles with apex at the target, each mapped to the unit square with
// y = x + s (a + t (b - a) - x), s = u^2 (the Jacobian s ds = 2 u^3 du removes the logarithmic
// singularity at the apex), Gauss-Legendre in u and, across the triangle, Gauss-Legendre after
// t = t0 + mu sinh(tau) on each side of the foot t0 of the perpendicular from the apex (mu: the
// apex's distance to the edge line over the edge length), which spreads the peak of the integrand
// at the foot (the sinh transformation for nearly singular integrals, Johnston and Elliott 2005).
// One thread's share of the moments of a box of half-width be at the target (tx, ty) taken
// relative to the box centre, added into acc[0..np): the far rule's points or the near rule's
// (triangle, side of the foot, point across) items, strided over the 256 threads.
__device__ void moment_part(const PanelRef& R, int p, int np, double kappa, double be, double tx, double ty,
                            const double* __restrict__ far_x, const double* __restrict__ far_w, int nfar, int t,
                            double2* acc) {
  const double ox = fmax(fabs(tx) - be, 0.0), oy = fmax(fabs(ty) - be, 0.0);
  if (sqrt(ox * ox + oy * oy) >= be) {
    const int nq = nfar * nfar;
    for (int q = t; q < nq; q += 256) {
      const double u = far_x[q / nfar], v = far_x[q % nfar];
      const double w = far_w[q / nfar] * far_w[q % nfar] * be * be;
      const double rx = tx - be * u, ry = ty - be * v;
      const double2 G = green(kappa, sqrt(rx * rx + ry * ry));
      add_basis(R, p, np, u, v, make_double2(G.x * w, G.y * w), acc);
    }
    return;
  }
  for (int it = t; it < 4 * 2 * kAcross; it += 256) {
    const int k = it / (2 * kAcross), side = (it / kAcross) & 1, ia = it % kAcross;
    const double cxk[4] = {-be, be, be, -be}, cyk[4] = {-be, -be, be, be};
    const double ax = cxk[k], ay = cyk[k], bx = cxk[(k + 1) & 3], by = cyk[(k + 1) & 3];
    const double ex = bx - ax, ey = by - ay;
    const double J = (ax - tx) * ey - (ay - ty) * ex;
    if (fabs(J) <= 1e-15 * be * be) continue;
    const double dd = ex * ex + ey * ey;
    const double t0 = ((tx - ax) * ex + (ty - ay) * ey) / dd;
    const double mu = fabs(J) / dd;
    // the two sides of the foot inside [0, 1] (one empty when the foot lies outside)
    const double f = fmin(fmax(t0, 0.0), 1.0);
    const double lo = side ? f : 0.0, hi = side ? 1.0 : f;
    if (hi <= lo) continue;
    const double tl = asinh((lo - t0) / mu), th = asinh((hi - t0) / mu);
    const double tau = tl + (th - tl) * R.acr_t[ia];
    const double tt = t0 + mu * sinh(tau);
    const double wt = (th - tl) * R.acr_w[ia] * mu * cosh(tau) * J;
    const double px = ax + tt * ex - tx, py = ay + tt * ey - ty;
    const double rho = sqrt(px * px + py * py);
    for (int iu = 0; iu < kRay; ++iu) {
      const double u = R.ray_t[iu], s = u * u, ws = 2.0 * u * u * u * R.ray_w[iu] * wt;
      const double2 G = green(kappa, s * rho);
      add_basis(R, p, np, (tx + s * px) / be, (ty + s * py) / be, make_double2(G.x * ws, G.y * ws), acc);
    }
  }
}

// workgroup sum in a fixed order (butterfly within each wave, then the four waves) into out[0..np)
__device__ void moment_reduce(double2* acc, int np, double2 (*red)[kMaxNp], double2* out) {
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
#pragma unroll
  for (int l = 0; l < kMaxNp; ++l) {
    if (l < np) {
      double re = acc[l].x, im = acc[l].y;
      for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_xor(re, off, 64);
        im += __shfl_xor(im, off, 64);
      }
      if (lane == 0) red[wave][l] = make_double2(re, im);
    }
  }
  __syncthreads();
  if (t < np) {
    double2 o = red[0][t];
    for (int w = 1; w < 4; ++w) {
      o.x += red[w][t].x;
      o.y += red[w][t].y;
    }
    out[t] = o;
  }
}

__device__ void load_ref(const PanelRef* __restrict__ ref, PanelRef& R) {
  for (int i = threadIdx.x; i < (int)(sizeof(PanelRef) / sizeof(double)); i += 256)
    reinterpret_cast<double*>(&R)[i] = reinterpret_cast<const double*>(ref)[i];
  __syncthreads();
}

// One workgroup per (offset d, target node a): M[d][a][l] = int_B G(|x - y|) b_l((y - c_B) / beta) dy
// with x the target node relative to the source box centre c_B.  Targets at least beta away from
// the box take the tensor Gauss-Legendre rule (nfar points per direction); nearer ones split the
// box into the four signed triangles with apex at the target, each mapped to the unit square with
// y = x + s (a + t (b - a) - x), s = u^2 (the Jacobian s ds = 2 u^3 du removes the logarithmic
// singularity at the apex), Gauss-Legendre in u and, across the triangle, Gauss-Legendre after
// t = t0 + mu sinh(tau) on each side of the foot t0 of the perpendicular from the apex (mu: the
// apex's distance to the edge line over the edge length), which spreads the peak of the integrand
// at the foot (the sinh transformation for nearly singular integrals, Johnston and Elliott 2005).
__global__ __launch_bounds__(256) void k_panel_moments(PanelGeom g, const PanelRef* __restrict__ ref,
                                                       const double* __restrict__ far_x,
                                                       const double* __restrict__ far_w, double2* __restrict__ M) {
  __shared__ PanelRef R;
  __shared__ double2 red[4][kMaxNp];
  const int d = blockIdx.x, a = blockIdx.y;
  load_ref(ref, R);
  const int w2 = 2 * g.nside - 1;
  const int dx = d / w2 - (g.nside - 1), dy = d % w2 - (g.nside - 1);
  const double be = g.beta;
  const double tx = 2.0 * be * dx + be * R.node[a / g.p], ty = 2.0 * be * dy + be * R.node[a % g.p];
  double2 acc[kMaxNp];
#pragma unroll
  for (int l = 0; l < kMaxNp; ++l) acc[l] = make_double2(0.0, 0.0);
  moment_part(R, g.p, g.np, g.kappa, be, tx, ty, far_x, far_w, g.nfar, threadIdx.x, acc);
  moment_reduce(acc, g.np, red, M + ((long long)d * g.n2 + a) * g.np);
}

// Leaves of any tree (boxes[B] = (cx, cy, beta, far rule offset, far rule points)): one workgroup
// per (source box B, target node i at X[i]): M[i][B][l], same rules as k_panel_moments
__global__ __launch_bounds__(256) void k_panel_moments_leaves(const PanelRef* __restrict__ ref, int p, int np,
                                                              double kappa, const double* __restrict__ boxes,
                                                              int nboxes, const double2* __restrict__ X,
                                                              const double* __restrict__ far_x,
                                                              const double* __restrict__ far_w,
                                                              double2* __restrict__ M) {
  __shared__ PanelRef R;
  __shared__ double2 red[4][kMaxNp];
  const int B = blockIdx.x, i = blockIdx.y;
  load_ref(ref, R);
  const double* bx = boxes + 5 * B;
  const double be = bx[2];
  const int off = (int)bx[3], nfar = (int)bx[4];
  const double2 xi = X[i];
  double2 acc[kMaxNp];
#pragma unroll
  for (int l = 0; l < kMaxNp; ++l) acc[l] = make_double2(0.0, 0.0);
  moment_part(R, p, np, kappa, be, xi.x - bx[0], xi.y - bx[1], far_x + off, far_w + off, nfar, threadIdx.x, acc);
  moment_reduce(acc, np, red, M + ((long long)i * nboxes + B) * np);
}

// V[i][B * n2 + b] = sum_l M[i][B][l] Qdag[l][b] (row-major, N x N)
__global__ __launch_bounds__(256) void k_panel_dense_V(const double2* __restrict__ M, const double* __restrict__ Qdag,
                                                       int nboxes, int np, int n2, double2* __restrict__ V) {
  const long long i = blockIdx.x;
  const int ncol = nboxes * n2;
  for (int c = threadIdx.x; c < ncol; c += 256) {
    const int B = c / n2, b = c % n2;
    const double2* m = M + (i * nboxes + B) * np;
    double re = 0, im = 0;
    for (int l = 0; l < np; ++l) {
      const double q = Qdag[l * n2 + b];
      re = fma(m[l].x, q, re);
      im = fma(m[l].y, q, im);
    }
    V[i * ncol + c] = make_double2(re, im);
  }
}

// y = alpha x + coef q (V x) with the dense V: one wave per row and right-hand side, its lanes
// striding over the columns (coalesced), butterfly sum
__global__ __launch_bounds__(256) void k_panel_dense_apply(const double2* __restrict__ V, long long N,
                                                           const double* __restrict__ q,
                                                           const double2* __restrict__ x, long long ldx,
                                                           double2* __restrict__ y, long long ldy, double alpha,
                                                           double coef) {
  const long long i = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, rhs = blockIdx.y;
  if (i >= N) return;
  const double2* row = V + i * N;
  const double2* xr = x + rhs * ldx;
  double re = 0, im = 0;
  for (long long j = lane; j < N; j += 64) {
    const double2 a = row[j], v = xr[j];
    re = fma(a.x, v.x, re);
    re = fma(-a.y, v.y, re);
    im = fma(a.x, v.y, im);
    im = fma(a.y, v.x, im);
  }
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  if (lane == 0) {
    const double2 xi = xr[i];
    const double c = q ? coef * q[i] : coef;
    y[rhs * ldy + i] = make_double2(alpha * xi.x + c * re, alpha * xi.y + c * im);
  }
}

// T[d][a][b] = sum_l M[d][a][l] Qdag[l][b]
__global__ __launch_bounds__(256) void k_panel_blocks(PanelGeom g, const double2* __restrict__ M,
                                                      const double* __restrict__ Qdag, double2* __restrict__ T) {
  const long long d = blockIdx.x;
  for (int e = threadIdx.x; e < g.n2 * g.n2; e += 256) {
    const int a = e / g.n2, b = e % g.n2;
    const double2* m = M + (d * g.n2 + a) * g.np;
    double re = 0, im = 0;
    for (int l = 0; l < g.np; ++l) {
      const double q = Qdag[l * g.n2 + b];
      re = fma(m[l].x, q, re);
      im = fma(m[l].y, q, im);
    }
    T[(d * g.n2 + a) * g.n2 + b] = make_double2(re, im);
  }
}

// One workgroup per (target box A, right-hand side): thread (a, part) sums the source boxes
// B = part, part + S, ... (S = 256 / n2 parts) over the source nodes b of T[A - B][a][b] x_B[b];
// the parts are added in a fixed order, then y = alpha x + coef q (V x).
__global__ __launch_bounds__(256) void k_panel_apply(PanelGeom g, const double2* __restrict__ T,
                                                     const double* __restrict__ q, const double2* __restrict__ x,
                                                     long long ldx, double2* __restrict__ y, long long ldy,
                                                     double alpha, double coef) {
  __shared__ double2 part[256];
  const int A = blockIdx.x, rhs = blockIdx.y, t = threadIdx.x;
  const int n2 = g.n2, S = 256 / n2, nb = g.nside * g.nside, w2 = 2 * g.nside - 1;
  const int a = t % n2, sp = t / n2;
  const int ax = A / g.nside, ay = A % g.nside;
  const double2* xr = x + rhs * ldx;
  double re = 0, im = 0;
  if (sp < S) {
    for (int B = sp; B < nb; B += S) {
      const int dx = ax - B / g.nside, dy = ay - B % g.nside;
      const long long d = (long long)(dx + g.nside - 1) * w2 + (dy + g.nside - 1);
      const double2* Tr = T + (d * n2 + a) * n2;
      const double2* xb = xr + (long long)B * n2;
      for (int b = 0; b < n2; ++b) {
        const double2 m = Tr[b], v = xb[b];
        re = fma(m.x, v.x, re);
        re = fma(-m.y, v.y, re);
        im = fma(m.x, v.y, im);
        im = fma(m.y, v.x, im);
      }
    }
  }
  part[t] = make_double2(re, im);
  __syncthreads();
  if (t < n2) {
    for (int k = 1; k < S; ++k) {
      re += part[k * n2 + t].x;
      im += part[k * n2 + t].y;
    }
    const long long i = (long long)A * n2 + t;
    const double2 xi = xr[i];
    const double c = q ? coef * q[i] : coef;
    y[rhs * ldy + i] = make_double2(alpha * xi.x + c * re, alpha * xi.y + c * im);
  }
}

// The same product on the matrix cores: for a tile of TX x TY = 16 target boxes and an offset d,
// the sources are the tile shifted by d (boxes outside the grid masked), and the products of
// that offset are one (n2 x n2) by (n2 x 16 boxes) complex GEMM, RT 16-row tiles by KB 4-deep
// k-blocks of 16 x 16 x 4 FP64 MFMAs (four real ones per complex product; rows and k past n2
// padded with zeros).  The operands are read from node-major copies, so that the 64 lanes of
// every load take consecutive addresses: the blocks column by column (Tt[d][b][a] = T[d][a][b])
// and the densities node by node (xt[b][B] = x[B n2 + b]).  A workgroup takes one tile and a
// chunk of the tile's offsets, its 4 waves every 4th offset of the chunk, with the next offset's
// operands loaded before the current products; the waves' sums are added through LDS in a fixed
// order into the chunk's partial plane, and k_panel_reduce adds the chunks in order.  Lane l:
// T element (row l % 16, k l / 16), x element (k l / 16, box l % 16); accumulator element v:
// row l / 16 + 4 v, box l % 16.  Box j of a tile sits at (x0 + j / TY, y0 + j % TY).
typedef double pf64x4 __attribute__((ext_vector_type(4)));

template <int RT, int KB>
__global__ __launch_bounds__(256) void k_panel_apply_mfma(PanelGeom g, const double2* __restrict__ Tt,
                                                          const double2* __restrict__ xt,
                                                          double2* __restrict__ part, int nchunks, long long N,
                                                          int TY) {
  __shared__ double2 red[4][RT][4][64];
  const int tile = blockIdx.x, chunk = blockIdx.y, rhs = blockIdx.z;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int n2 = g.n2, nside = g.nside, nb = nside * nside, w2 = 2 * nside - 1;
  const int TX = 16 / TY, nty = (nside + TY - 1) / TY;
  // the offsets that pair some box of the tile with a box of the grid: a rectangle of
  // (x extent + nside - 1) x (y extent + nside - 1) offsets; chunk c of the launch takes its share
  const int x0 = (tile / nty) * TX, y0 = (tile % nty) * TY;
  const int x1 = min(x0 + TX, nside) - 1, y1 = min(y0 + TY, nside) - 1;
  const int wx = x1 - x0 + nside, wy = y1 - y0 + nside;
  const int dxlo = x0 - (nside - 1), dylo = y0 - (nside - 1);
  const int nrect = wx * wy;
  const int d0 = (int)((long long)nrect * chunk / nchunks), d1 = (int)((long long)nrect * (chunk + 1) / nchunks);
  const int j = lane & 15, kq = lane >> 4;
  const int ax = x0 + j / TY, ay = y0 + j % TY;
  const bool aok = ax < nside && ay < nside;
  const double2* xr = xt + rhs * N;
  pf64x4 accr[RT], acci[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    accr[rt] = pf64x4{0, 0, 0, 0};
    acci[rt] = pf64x4{0, 0, 0, 0};
  }
  // operands of offset (dx, dy): T fragments (row rt * 16 + j, k kb * 4 + kq) and x fragments
  // (k kb * 4 + kq, box j shifted by the offset)
  auto load = [&](int dx, int dy, double2 (&ta)[RT][KB], double2 (&xa)[KB]) -> bool {
    const long long d = (long long)(dx + nside - 1) * w2 + (dy + nside - 1);
    const int bx = ax - dx, by = ay - dy;
    const bool ok = aok && bx >= 0 && bx < nside && by >= 0 && by < nside;
    const long long B = ok ? (long long)bx * nside + by : 0;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      const int b = kb * 4 + kq;
      xa[kb] = ok && b < n2 ? xr[(long long)b * nb + B] : make_double2(0.0, 0.0);
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const int a = rt * 16 + j;
        ta[rt][kb] = a < n2 && b < n2 ? Tt[(d * n2 + b) * n2 + a] : make_double2(0.0, 0.0);
      }
    }
    return __any(ok);
  };
  double2 ta[RT][KB], xa[KB], tb[RT][KB], xb[KB];
  // offset e of the rectangle = (dxlo + e / wy, dylo + e % wy), stepped without divisions
  int e = d0 + wave;
  int ex = e / wy, ey = e % wy;
  bool live = e < d1 ? load(dxlo + ex, dylo + ey, ta, xa) : false;
  while (e < d1) {
    e += 4;
    ey += 4;
    while (ey >= wy) {
      ey -= wy;
      ++ex;
    }
    const bool nlive = e < d1 ? load(dxlo + ex, dylo + ey, tb, xb) : false;
    if (live) {
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
          accr[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ta[rt][kb].x, xa[kb].x, accr[rt], 0, 0, 0);
          accr[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ta[rt][kb].y, xa[kb].y, accr[rt], 0, 0, 0);
          acci[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ta[rt][kb].x, xa[kb].y, acci[rt], 0, 0, 0);
          acci[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ta[rt][kb].y, xa[kb].x, acci[rt], 0, 0, 0);
        }
    }
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      xa[kb] = xb[kb];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) ta[rt][kb] = tb[rt][kb];
    }
    live = nlive;
  }
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wave][rt][v][lane] = make_double2(accr[rt][v], acci[rt][v]);
  __syncthreads();
  if (wave == 0 && aok) {
    const long long A = (long long)ax * nside + ay;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = rt * 16 + kq + 4 * v;
        if (a >= n2) continue;
        double2 o = red[0][rt][v][lane];
        for (int w = 1; w < 4; ++w) {
          o.x += red[w][rt][v][lane].x;
          o.y += red[w][rt][v][lane].y;
        }
        part[((long long)chunk * gridDim.z + rhs) * N + A * n2 + a] = o;
      }
  }
}

// xt[rhs][b][B] = x[rhs * ldx + B n2 + b]
__global__ __launch_bounds__(256) void k_panel_node_major(const double2* __restrict__ x, long long ldx,
                                                          double2* __restrict__ xt, int nb, int n2) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x, N = (long long)nb * n2;
  const int rhs = blockIdx.y;
  if (i >= N) return;
  const long long b = i / nb, B = i - b * nb;
  xt[rhs * N + i] = x[rhs * ldx + B * n2 + b];
}

// Tt[d][b][a] = T[d][a][b]
__global__ __launch_bounds__(256) void k_panel_blocks_t(const double2* __restrict__ T, double2* __restrict__ Tt,
                                                        int n2) {
  const long long d = blockIdx.x;
  for (int e = threadIdx.x; e < n2 * n2; e += 256) {
    const int b = e / n2, a = e % n2;
    Tt[(d * n2 + b) * n2 + a] = T[(d * n2 + a) * n2 + b];
  }
}

// y = alpha x + coef q (sum over the chunks of the partial planes, in chunk order)
__global__ __launch_bounds__(256) void k_panel_reduce(const double2* __restrict__ part, int nchunks, int nrhs,
                                                      long long N, const double* __restrict__ q,
                                                      const double2* __restrict__ x, long long ldx,
                                                      double2* __restrict__ y, long long ldy, double alpha,
                                                      double coef) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const int rhs = blockIdx.y;
  if (i >= N) return;
  double re = 0, im = 0;
  for (int c = 0; c < nchunks; ++c) {
    const double2 v = part[((long long)c * nrhs + rhs) * N + i];
    re += v.x;
    im += v.y;
  }
  const double2 xi = x[rhs * ldx + i];
  const double cf = q ? coef * q[i] : coef;
  y[rhs * ldy + i] = make_double2(alpha * xi.x + cf * re, alpha * xi.y + cf * im);
}

int panel_tile_y(const PanelGeom& g) {
  int ty = 1;
  while (ty < 4 && ty * 2 <= g.nside) ty *= 2;
  return ty;
}

int panel_chunks(const PanelGeom& g, int nrhs) {
  const int ty = panel_tile_y(g), tx = 16 / ty;
  const int ntiles = ((g.nside + tx - 1) / tx) * ((g.nside + ty - 1) / ty);
  const long long N = (long long)g.nside * g.nside * g.n2;
  const int rect = (std::min(tx, g.nside) - 1 + g.nside) * (std::min(ty, g.nside) - 1 + g.nside);
  int c = std::max(1, std::min(rect / 4, (2048 + ntiles - 1) / ntiles));
  // partial planes of at most 512 MB
  while (c > 1 && (long long)c * nrhs * N * 16 > (512LL << 20)) c /= 2;
  return c;
}

template <int RT, int KB>
static void apply_mfma(const PanelGeom& g, const double2* Tt, const double* q, const double2* x, long long ldx,
                       double2* y, long long ldy, int nrhs, double alpha, double coef, double2* part, double2* xt,
                       int nchunks, hipStream_t s) {
  const int nb = g.nside * g.nside, ty = panel_tile_y(g), tx = 16 / ty;
  const int ntiles = ((g.nside + tx - 1) / tx) * ((g.nside + ty - 1) / ty);
  const long long N = (long long)nb * g.n2;
  k_panel_node_major<<<dim3((unsigned)((N + 255) / 256), (unsigned)nrhs), 256, 0, s>>>(x, ldx, xt, nb, g.n2);
  k_panel_apply_mfma<RT, KB><<<dim3((unsigned)ntiles, (unsigned)nchunks, (unsigned)nrhs), 256, 0, s>>>(
      g, Tt, xt, part, nchunks, N, ty);
  k_panel_reduce<<<dim3((unsigned)((N + 255) / 256), (unsigned)nrhs), 256, 0, s>>>(part, nchunks, nrhs, N, q, x, ldx,
                                                                                 y, ldy, alpha, coef);
}

void launch_panel_blocks_t(const PanelGeom& g, const double2* T, double2* Tt, hipStream_t s) {
  const int w2 = 2 * g.nside - 1;
  k_panel_blocks_t<<<(unsigned)(w2 * w2), 256, 0, s>>>(T, Tt, g.n2);
}

void launch_panel_apply_mfma(const PanelGeom& g, const double2* Tt, const double* q, const double2* x, long long ldx,
                             double2* y, long long ldy, int nrhs, double alpha, double coef, double2* part,
                             double2* xt, int nchunks, hipStream_t s) {
  switch (g.p) {
    case 1: apply_mfma<1, 1>(g, Tt, q, x, ldx, y, ldy, nrhs, alpha, coef, part, xt, nchunks, s); break;
    case 2: apply_mfma<1, 1>(g, Tt, q, x, ldx, y, ldy, nrhs, alpha, coef, part, xt, nchunks, s); break;
    case 3: apply_mfma<1, 3>(g, Tt, q, x, ldx, y, ldy, nrhs, alpha, coef, part, xt, nchunks, s); break;
    case 4: apply_mfma<1, 4>(g, Tt, q, x, ldx, y, ldy, nrhs, alpha, coef, part, xt, nchunks, s); break;
    case 5: apply_mfma<2, 7>(g, Tt, q, x, ldx, y, ldy, nrhs, alpha, coef, part, xt, nchunks, s); break;
    default: break;  // p > 5: the double-buffered operands would not fit the registers (VALU form)
  }
}

// ---- Krylov vector kernels of the panel solver (complex128, one right-hand side) ----
// part[i * nch + c] = sum over chunk c of conj(Q_i[k]) w[k]; workgroup sums in a fixed order
__global__ __launch_bounds__(256) void k_panel_dots(const double2* __restrict__ Q, long long ldq, int nvec,
                                                    const double2* __restrict__ w, long long N,
                                                    double2* __restrict__ part, int nch) {
  __shared__ double2 red[4];
  const int c = blockIdx.x, i = blockIdx.y, t = threadIdx.x;
  const long long k0 = N * c / nch, k1 = N * (c + 1) / nch;
  const double2* q = Q + i * ldq;
  double re = 0, im = 0;
  for (long long k = k0 + t; k < k1; k += 256) {
    const double2 a = q[k], b = w[k];
    re = fma(a.x, b.x, re);
    re = fma(a.y, b.y, re);
    im = fma(a.x, b.y, im);
    im = fma(-a.y, b.x, im);
  }
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  if ((t & 63) == 0) red[t >> 6] = make_double2(re, im);
  __syncthreads();
  if (t == 0) {
    double2 o = red[0];
    for (int w2 = 1; w2 < 4; ++w2) {
      o.x += red[w2].x;
      o.y += red[w2].y;
    }
    part[(long long)i * nch + c] = o;
  }
}

// w[k] -= sum_i c[i] Q_i[k]
__global__ __launch_bounds__(256) void k_panel_update(double2* __restrict__ w, const double2* __restrict__ Q,
                                                      long long ldq, int nvec, const double2* __restrict__ c,
                                                      long long N) {
  const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
  if (k >= N) return;
  double2 o = w[k];
  for (int i = 0; i < nvec; ++i) {
    const double2 a = c[i], q = Q[i * ldq + k];
    o.x -= a.x * q.x - a.y * q.y;
    o.y -= a.x * q.y + a.y * q.x;
  }
  w[k] = o;
}

// y = alpha a + beta b (real coefficients)
// y may be a or b (each thread reads its entries before it writes)
__global__ __launch_bounds__(256) void k_panel_combo(double2* y, const double2* a, double alpha, const double2* b,
                                                     double beta, long long N) {
  const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
  if (k >= N) return;
  const double2 u = a[k], v = b[k];
  y[k] = make_double2(alpha * u.x + beta * v.x, alpha * u.y + beta * v.y);
}

void launch_panel_dots(const double2* Q, long long ldq, int nvec, const double2* w, long long N, double2* part,
                       int nch, hipStream_t s) {
  k_panel_dots<<<dim3((unsigned)nch, (unsigned)nvec), 256, 0, s>>>(Q, ldq, nvec, w, N, part, nch);
}
void launch_panel_update(double2* w, const double2* Q, long long ldq, int nvec, const double2* c, long long N,
                         hipStream_t s) {
  k_panel_update<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(w, Q, ldq, nvec, c, N);
}
// gather: y[rhs * ldy + t] = x[rhs * ldx + perm[t]], zero where perm[t] < 0 (padding);
// scatter: y[rhs * ldy + perm[t]] = x[rhs * ldx + t] where perm[t] >= 0.  t < M.
__global__ __launch_bounds__(256) void k_panel_permute(const double2* __restrict__ x, long long ldx,
                                                       double2* __restrict__ y, long long ldy,
                                                       const int* __restrict__ perm, long long M, int scatter) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  const int rhs = blockIdx.y;
  if (t >= M) return;
  const int k = perm[t];
  if (scatter) {
    if (k >= 0) y[rhs * ldy + k] = x[rhs * ldx + t];
  } else {
    y[rhs * ldy + t] = k >= 0 ? x[rhs * ldx + k] : make_double2(0.0, 0.0);
  }
}

void launch_panel_permute(const double2* x, long long ldx, double2* y, long long ldy, const int* perm, long long M,
                          int nrhs, bool scatter, hipStream_t s) {
  if (M > 0 && nrhs > 0)
    k_panel_permute<<<dim3((unsigned)((M + 255) / 256), (unsigned)nrhs), 256, 0, s>>>(x, ldx, y, ldy, perm, M,
                                                                                       scatter ? 1 : 0);
}

void launch_panel_combo(double2* y, const double2* a, double alpha, const double2* b, double beta, long long N,
                        hipStream_t s) {
  k_panel_combo<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(y, a, alpha, b, beta, N);
}

void launch_panel_moments_leaves(const PanelRef* ref, int p, int np, double kappa, const double* boxes, int nboxes,
                                 const double2* X, long long N, const double* far_x, const double* far_w, double2* M,
                                 hipStream_t s) {
  k_panel_moments_leaves<<<dim3((unsigned)nboxes, (unsigned)N), 256, 0, s>>>(ref, p, np, kappa, boxes, nboxes, X,
                                                                             far_x, far_w, M);
}

void launch_panel_dense_V(const double2* M, const double* Qdag, int nboxes, int np, int n2, double2* V, hipStream_t s) {
  k_panel_dense_V<<<(unsigned)((long long)nboxes * n2), 256, 0, s>>>(M, Qdag, nboxes, np, n2, V);
}

void launch_panel_dense_apply(const double2* V, long long N, const double* q, const double2* x, long long ldx,
                              double2* y, long long ldy, int nrhs, double alpha, double coef, hipStream_t s) {
  k_panel_dense_apply<<<dim3((unsigned)((N + 3) / 4), (unsigned)nrhs), 256, 0, s>>>(V, N, q, x, ldx, y, ldy, alpha,
                                                                                   coef);
}

void launch_panel_moments(const PanelGeom& g, const PanelRef* ref, const double* far_x, const double* far_w,
                          double2* M, hipStream_t s) {
  const int w2 = 2 * g.nside - 1;
  k_panel_moments<<<dim3((unsigned)(w2 * w2), (unsigned)g.n2), 256, 0, s>>>(g, ref, far_x, far_w, M);
}

void launch_panel_blocks(const PanelGeom& g, const double2* M, const double* Qdag, double2* T, hipStream_t s) {
  const int w2 = 2 * g.nside - 1;
  k_panel_blocks<<<(unsigned)(w2 * w2), 256, 0, s>>>(g, M, Qdag, T);
}

void launch_panel_apply(const PanelGeom& g, const double2* T, const double* q, const double2* x, long long ldx,
                        double2* y, long long ldy, int nrhs, double alpha, double coef, hipStream_t s) {
  k_panel_apply<<<dim3((unsigned)(g.nside * g.nside), (unsigned)nrhs), 256, 0, s>>>(g, T, q, x, ldx, y, ldy, alpha,
                                                                                    coef);
}

}  // namespace lsp
