// Partially pivoted adaptive cross approximation (ACA).
//
// The paper chooses NCA pivots with partially pivoted ACA stopped by Rjasanow's
// criterion at accuracy eps_NCA (Section 4.2.2, step 2, and the notation table of
// Section 6.2); the same routine, capped at a fixed rank, compresses the off-diagonal
// blocks of the HODLR preconditioner (Section 6).  Rules: start at the first row
// that is not known to be zero; the column pivot is the largest residual entry of the
// pivot row over unused columns; the next row pivot is the largest entry of the new
// residual column over unused rows; an exactly zero residual row is skipped in favour
// of the next unused row; magnitudes within a relative 1e-9 of the maximum are ties,
// won by the lowest index; stop at max_rank, at min(m, n), when no nonzero row is
// left, or when ||u_k|| ||v_k|| <= eps ||S_k||_F.
#pragma once
#include <cmath>

namespace ls {

static constexpr double kAcaTie = 1e-9;

// x[0..n) -= a * y[0..n) in plain real arithmetic (vectorisable; the same products and sums as
// the complex operators for finite values)
inline void axpy_sub(zd* x, zd a, const zd* y, int n) {
  double* xd = reinterpret_cast<double*>(x);
  const double* yd = reinterpret_cast<const double*>(y);
  const double ar = a.real(), ai = a.imag();
  for (int k = 0; k < n; ++k) {
    const double yr = yd[2 * k], yi = yd[2 * k + 1];
    xd[2 * k] -= ar * yr - ai * yi;
    xd[2 * k + 1] -= ar * yi + ai * yr;
  }
}

template <class RowFn, class ColFn>
ACAResult aca(int m, int n, int max_rank, double eps, const std::vector<char>* row_zero, RowFn rowfn,
              ColFn colfn) {
  ACAResult R;
  std::vector<char> row_used(m, 0), col_used(n, 0);
  if (row_zero)
    for (int i = 0; i < m; ++i)
      if ((*row_zero)[i]) row_used[i] = 1;
  int kmax = std::min(max_rank, std::min(m, n));
  double normS2 = 0.0;
  std::vector<zd> r(n), c(m);
  auto next_unused = [&](int from) {
    for (int i = from; i < m; ++i)
      if (!row_used[i]) return i;
    for (int i = 0; i < from; ++i)
      if (!row_used[i]) return i;
    return -1;
  };
  int i = next_unused(0);
  while ((int)R.u.size() < kmax && i >= 0) {
    int j = -1;
    for (;;) {
      rowfn(i, r.data());
      for (size_t l = 0; l < R.u.size(); ++l) {
        const zd ui = R.u[l][i];
        if (ui != zd(0)) axpy_sub(r.data(), ui, R.v[l].data(), n);
      }
      row_used[i] = 1;
      double mx = 0.0;
      for (int jj = 0; jj < n; ++jj)
        if (!col_used[jj]) mx = std::max(mx, std::abs(r[jj]));
      if (mx > 0.0) {
        const double thr = (1.0 - kAcaTie) * mx;
        for (int jj = 0; jj < n; ++jj)
          if (!col_used[jj] && std::abs(r[jj]) >= thr) {
            j = jj;
            break;
          }
        break;
      }
      // first unused row (lowest index) after an exactly zero residual row
      int nxt = -1;
      for (int ii = 0; ii < m; ++ii)
        if (!row_used[ii]) {
          nxt = ii;
          break;
        }
      if (nxt < 0) return R;
      i = nxt;
    }
    const zd piv = r[j];
    std::vector<zd> v(n), u(m);
    for (int jj = 0; jj < n; ++jj) v[jj] = r[jj] / piv;
    colfn(j, c.data());
    for (int ii = 0; ii < m; ++ii) u[ii] = c[ii];
    for (size_t l = 0; l < R.u.size(); ++l) {
      const zd vj = R.v[l][j];
      if (vj != zd(0)) axpy_sub(u.data(), vj, R.u[l].data(), m);
    }
    col_used[j] = 1;
    R.rows.push_back(i);
    R.cols.push_back(j);
    // Rjasanow's stopping test needs ||S_k||_F; a fixed-rank run (eps = 0) skips it
    if (eps > 0.0) {
      double cross = 0.0;
      for (size_t l = 0; l < R.u.size(); ++l) {
        zd a(0), b(0);
        const zd* ul = R.u[l].data();
        const zd* vl = R.v[l].data();
        for (int ii = 0; ii < m; ++ii) a += std::conj(ul[ii]) * u[ii];
        for (int jj = 0; jj < n; ++jj) b += std::conj(v[jj]) * vl[jj];
        cross += 2.0 * (a * b).real();
      }
      double nu2 = 0, nv2 = 0;
      for (int ii = 0; ii < m; ++ii) nu2 += std::norm(u[ii]);
      for (int jj = 0; jj < n; ++jj) nv2 += std::norm(v[jj]);
      normS2 += cross + nu2 * nv2;
      R.u.push_back(std::move(u));
      R.v.push_back(std::move(v));
      if (std::sqrt(nu2 * nv2) <= eps * std::sqrt(std::max(normS2, 0.0))) break;
    } else {
      R.u.push_back(std::move(u));
      R.v.push_back(std::move(v));
    }
    if ((int)R.u.size() >= kmax) break;
    const std::vector<zd>& uk = R.u.back();
    double mx = 0.0;
    for (int ii = 0; ii < m; ++ii)
      if (!row_used[ii]) mx = std::max(mx, std::abs(uk[ii]));
    int inext = -1;
    if (mx > 0.0) {
      const double thr = (1.0 - kAcaTie) * mx;
      for (int ii = 0; ii < m; ++ii)
        if (!row_used[ii] && std::abs(uk[ii]) >= thr) {
          inext = ii;
          break;
        }
    } else {
      for (int ii = 0; ii < m; ++ii)
        if (!row_used[ii]) {
          inext = ii;
          break;
        }
    }
    i = inext;
  }
  return R;
}

}  // namespace ls
