// Off-grid volume potential and the error function E(x) (paper, Section 6: u_scat = V[psi]
// from the discrete density; Section 6.2, Eq. (eq:error)).  At p = 1 the density is constant
// on each cell, so (V psi)(x) = sum_j psi_j int_{cell j} G(|x - y|) dy for any point x.
//
// One workgroup per target.  Cells at Chebyshev distance d >= 2 (in cells) from the cell that
// contains x are integrated with a tensor Gauss-Legendre rule whose order is set by the nearest
// singularity (distance >= (d - 1) h: 6 points at d = 2, 5 up to d = 4, 4 beyond) and by the
// oscillation across a cell (at least 4 points for kappa h <= 0.6, 5 up to 1.5, 6 up to 2, 8 up
// to 3, then 10, 12, 16), two more at d = 2 when kappa h > 1.5: measured below 3e-11 relative
// for kappa h <= 3 with the target at the worst place in its cell.  The 3 x 3 cells around x are integrated in polar coordinates about x: a cell is the
// signed sum over its edges of the triangles (x, edge), and with A the distance from x to the
// edge's line and y the coordinate along the edge from the foot of the perpendicular,
//   int_triangle G dy = sign * int_{y1}^{y2} A F(sqrt(A^2 + y^2)) / (A^2 + y^2) dy,
//   F(rho) = int_0^rho G(kappa r) r dr = 2 rho^2 int_0^1 G(kappa rho s^2) s^3 ds.
// The y-integrand has its singularities at y = +-iA, so [0, |y|] is cut into pieces
// [b_k, b_{k+1}], b_{k+1} = 2 b_k + A, each at least its own half-length away from them
// (Gauss-Legendre converges like 3.1^(-2n) on every piece, whatever A), and F is done by
// Gauss-Legendre in s.
#include <hip/hip_runtime.h>

#include "field.h"
#include "h0.h"

namespace lsk {

namespace {

__device__ inline double2 green_d(double kappa, double r) {
  const cplx h = hankel0(kappa * r);
  return make_double2(-0.25 * h.im, 0.25 * h.re);  // (i/4) H0
}

__device__ inline double2 gl_rect(const FieldRules& R, int which, double kappa, double x1, double x2, double a0,
                                  double b0, double h) {
  const int off = R.off[which], np = R.n[which];
  double re = 0, im = 0;
  for (int p = 0; p < np; ++p) {
    const double ya = a0 + 0.5 * h * (1.0 + R.t[off + p]);
    const double wa = 0.5 * h * R.w[off + p];
    for (int q = 0; q < np; ++q) {
      const double yb = b0 + 0.5 * h * (1.0 + R.t[off + q]);
      const double wgt = wa * 0.5 * h * R.w[off + q];
      const double2 g = green_d(kappa, hypot(ya - x1, yb - x2));
      re += wgt * g.x;
      im += wgt * g.y;
    }
  }
  return make_double2(re, im);
}

// F(rho) = int_0^rho G(kappa r) r dr = 2 rho^2 int_0^1 G(kappa rho s^2) s^3 ds
__device__ inline double2 radial(const FieldRules& R, double kappa, double rho) {
  const int off = R.off[kRuleRadial], np = R.n[kRuleRadial];
  double re = 0, im = 0;
  for (int p = 0; p < np; ++p) {
    const double s = 0.5 * (1.0 + R.t[off + p]);
    const double w = 0.5 * R.w[off + p] * s * s * s;
    const double2 g = green_d(kappa, rho * s * s);
    re += w * g.x;
    im += w * g.y;
  }
  return make_double2(2.0 * rho * rho * re, 2.0 * rho * rho * im);
}

}  // namespace

__global__ __launch_bounds__(256) void k_field_eval(const double2* __restrict__ targets, int n, double x0, double y0,
                                                    double h, double kappa, const double2* __restrict__ psi,
                                                    const int* __restrict__ g2c, FieldRules R, int mode,
                                                    const double* __restrict__ q_t, double theta, double sign,
                                                    double2* __restrict__ u_out, double* __restrict__ e_out) {
  __shared__ double red[2][256];
  const int t = blockIdx.x, tid = threadIdx.x;
  const double2 x = targets[t];
  const long long ax = (long long)floor((x.x - x0) / h + 0.5), bx = (long long)floor((x.y - y0) / h + 0.5);
  const long long N = (long long)n * n;
  const double kh = kappa * h;
  const int osc = kh <= 0.6 ? 4 : kh <= 1.5 ? 5 : kh <= 2.0 ? 6 : kh <= 3.0 ? 8 : kh <= 4.0 ? 10 : kh <= 6.0 ? 12 : 16;
  double re = 0, im = 0;
  // cells at distance >= 2: tensor Gauss-Legendre
  for (long long j = tid; j < N; j += 256) {
    const long long a = j / n, b = j - a * n;
    const long long da = a > ax ? a - ax : ax - a, db = b > bx ? b - bx : bx - b;
    const long long d = da > db ? da : db;
    if (d <= 1) continue;
    const double2 p = psi[g2c[j]];
    if (p.x == 0.0 && p.y == 0.0) continue;
    int np = d == 2 ? 6 : (d <= 4 ? 5 : 4);
    np = np > osc ? np : osc;
    if (d == 2 && kh > 1.5) np += 2;
    const int which = np <= 3 ? 0 : np <= 4 ? 1 : np <= 5 ? 2 : np <= 6 ? 3 : np <= 8 ? 4 : np <= 10 ? 5 : np <= 12 ? 6 : 7;
    const double2 I = gl_rect(R, which, kappa, x.x, x.y, x0 + (a - 0.5) * h, y0 + (b - 0.5) * h, h);
    re += I.x * p.x - I.y * p.y;
    im += I.x * p.y + I.y * p.x;
  }
  // the 3 x 3 cells around x: signed triangles about x; one (cell, edge, half, piece) per item
  const int npc = R.n[kRulePiece], ofp = R.off[kRulePiece];
  for (int k = tid; k < 9 * 4 * 2 * kMaxPieces; k += 256) {
    const int piece = k % kMaxPieces, half = (k / kMaxPieces) & 1, e = (k / (2 * kMaxPieces)) & 3;
    const int c = k / (8 * kMaxPieces);
    const long long a = ax + c / 3 - 1, b = bx + c % 3 - 1;
    if (a < 0 || a >= n || b < 0 || b >= n) continue;
    const double2 p = psi[g2c[a * n + b]];
    if (p.x == 0.0 && p.y == 0.0) continue;
    // corners counter-clockwise; edge e runs from corner e to corner e+1
    const double ca0 = x0 + (a - 0.5) * h, ca1 = ca0 + h, cb0 = y0 + (b - 0.5) * h, cb1 = cb0 + h;
    const double px[4] = {ca0, ca1, ca1, ca0}, py[4] = {cb0, cb0, cb1, cb1};
    const double v1x = px[e] - x.x, v1y = py[e] - x.y;
    const double ex = px[(e + 1) & 3] - px[e], ey = py[(e + 1) & 3] - py[e], el = hypot(ex, ey);
    const double cr = v1x * ey - v1y * ex;  // twice the signed area of (x, p_e, p_e+1)
    const double A = fabs(cr) / el;
    if (A <= 1e-12 * h) continue;  // x on the edge's line: a triangle of no area
    const double y1 = (v1x * ex + v1y * ey) / el, y2 = y1 + el;
    double lo, hi;
    if (y1 >= 0.0) {
      if (half) continue;
      lo = y1;
      hi = y2;
    } else if (y2 <= 0.0) {
      if (half) continue;
      lo = -y2;
      hi = -y1;
    } else {
      lo = 0.0;
      hi = half ? y2 : -y1;
    }
    const double bk = ldexp(lo + A, piece) - A;
    if (bk >= hi) continue;
    const double bk1 = fmin(hi, 2.0 * bk + A);
    double sr = 0, si = 0;
    for (int q = 0; q < npc; ++q) {
      const double y = bk + 0.5 * (bk1 - bk) * (1.0 + R.t[ofp + q]);
      const double r2 = A * A + y * y;
      const double2 F = radial(R, kappa, sqrt(r2));
      const double wq = 0.5 * (bk1 - bk) * R.w[ofp + q] * A / r2;
      sr += wq * F.x;
      si += wq * F.y;
    }
    const double sg = cr > 0 ? 1.0 : -1.0;
    sr *= sg;
    si *= sg;
    re += sr * p.x - si * p.y;
    im += sr * p.y + si * p.x;
  }
  red[0][tid] = re;
  red[1][tid] = im;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) {
      red[0][tid] += red[0][tid + st];
      red[1][tid] += red[1][tid + st];
    }
    __syncthreads();
  }
  if (tid != 0) return;
  const double2 u = make_double2(red[0][0], red[1][0]);
  if (mode == 0) {
    u_out[t] = u;
    return;
  }
  // E(x) = |psi(x) + s kappa^2 q(x) u(x) - f(x)| / kappa^2, f = -s kappa^2 q u_inc
  double2 px_ = make_double2(0.0, 0.0);
  if (ax >= 0 && ax < n && bx >= 0 && bx < n) px_ = psi[g2c[ax * n + bx]];
  const double k2 = kappa * kappa, q = q_t[t];
  const double ph = kappa * (cos(theta) * x.x + sin(theta) * x.y);
  const double2 uinc = make_double2(cos(ph), sin(ph));
  const double rr = px_.x + sign * k2 * q * u.x + sign * k2 * q * uinc.x;
  const double ri = px_.y + sign * k2 * q * u.y + sign * k2 * q * uinc.y;
  e_out[t] = hypot(rr, ri) / k2;
}

void launch_field_eval(const double* targets, long long M, int n, double x0, double y0, double h, double kappa,
                       const void* psi, const int* g2c, const FieldRules& R, int mode, const double* q_t,
                       double theta, double sign, void* u_out, double* e_out, hipStream_t s) {
  if (M <= 0) return;
  k_field_eval<<<(unsigned)M, 256, 0, s>>>((const double2*)targets, n, x0, y0, h, kappa, (const double2*)psi, g2c, R,
                                           mode, q_t, theta, sign, (double2*)u_out, e_out);
}

}  // namespace lsk
