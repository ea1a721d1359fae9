// Complex Hankel function H0^(1)(z) = J0(z) + i Y0(z) for real z > 0, FP64,
// usable from host and device code.  The Green's function of the 2D Helmholtz
// equation is G = (i/4) H0^(1)(kappa r) (paper, Section 1, below Eq. (eq:5)).
//
// Three branches, each accurate to about 1e-15 relative in |H0|:
//   z < 4        ascending series (Abramowitz & Stegun 9.1.12, 9.1.13);
//   4 <= z < 20  Miller's backward recurrence for J_k(z), normalised with
//                J0 + 2 sum J_2k = 1, and the Neumann series
//                Y0 = (2/pi)(ln(z/2) + gamma) J0 - (4/pi) sum_k (-1)^k J_2k / k   (A&S 9.1.88);
//   z >= 20      Hankel's asymptotic expansion
//                H0 = sqrt(2/(pi z)) e^{i(z - pi/4)} sum_k i^k a_k / z^k,
//                a_k = prod_{j<=k} (-(2j-1)^2) / (k! 8^k)        (A&S 9.2.7).
// H1^(1) is provided on the ascending-series branch only (used for the
// self-cell integral, whose arguments are below kappa*h).
#pragma once
#include <math.h>

#ifndef LS_HD
#if defined(__HIPCC__) || defined(__HIP__)
#define LS_HD __host__ __device__
#else
#define LS_HD
#endif
#endif

namespace lsk {

constexpr double kPi = 3.14159265358979323846;
constexpr double kEulerGamma = 0.57721566490153286061;

struct cplx {
  double re, im;
};

LS_HD inline cplx h0_series(double z) {
  const double t = 0.25 * z * z;
  double term = 1.0, J = 1.0, S = 0.0, H = 0.0;
  for (int k = 1; k < 60; ++k) {
    term *= -t / ((double)k * (double)k);
    H += 1.0 / (double)k;
    J += term;
    S -= term * H;
    if (fabs(term) < 1e-18 * fabs(J) && fabs(term * H) < 1e-18 * (fabs(S) + 1e-300)) break;
  }
  const double Y = (2.0 / kPi) * (log(0.5 * z) + kEulerGamma) * J + (2.0 / kPi) * S;
  return {J, Y};
}

LS_HD inline cplx h0_miller(double z) {
  // start order: even, well above z so that J_M(z) is negligible
  int M = 2 * (int)((z + 40.0) * 0.5) + 2;
  double jp1 = 0.0, j = 1e-30, norm = 0.0, ysum = 0.0;
  for (int n = M; n >= 1; --n) {
    const double jm1 = (2.0 * n / z) * j - jp1;
    jp1 = j;
    j = jm1;  // j = J_{n-1} (unnormalised)
    const int m = n - 1;
    if (m > 0 && (m & 1) == 0) {
      norm += 2.0 * j;
      const int k = m >> 1;
      ysum += ((k & 1) ? -j : j) / (double)k;
    }
  }
  norm += j;
  const double J0 = j / norm;
  const double Y0 = (2.0 / kPi) * (log(0.5 * z) + kEulerGamma) * J0 - (4.0 / kPi) * (ysum / norm);
  return {J0, Y0};
}

LS_HD inline cplx h0_asymptotic(double z) {
  // P + i Q = sum_k i^k a_k / z^k
  double P = 0.0, Q = 0.0, a = 1.0;
  for (int k = 0; k < 200; ++k) {
    switch (k & 3) {
      case 0: P += a; break;
      case 1: Q += a; break;
      case 2: P -= a; break;
      default: Q -= a; break;
    }
    const double kk = (double)(k + 1);
    const double an = a * (-(2.0 * kk - 1.0) * (2.0 * kk - 1.0)) / (kk * 8.0 * z);
    if (fabs(an) < 1e-18 || fabs(an) > fabs(a)) break;
    a = an;
  }
  const double chi = z - 0.25 * kPi;
  double s, c;
  s = sin(chi);
  c = cos(chi);
  const double amp = sqrt(2.0 / (kPi * z));
  // (c + i s)(P + i Q)
  return {amp * (c * P - s * Q), amp * (s * P + c * Q)};
}

// H0^(1)(z) = J0 + i Y0, z > 0.
LS_HD inline cplx hankel0(double z) {
  if (z < 4.0) return h0_series(z);
  if (z < 20.0) return h0_miller(z);
  return h0_asymptotic(z);
}

// H1^(1)(z) for 0 < z < 4 by the ascending series (A&S 9.1.10, 9.1.11 with n = 1).
LS_HD inline cplx hankel1_small(double z) {
  const double t = 0.25 * z * z;
  const double half = 0.5 * z;
  // J1 = (z/2) sum (-t)^k / (k!(k+1)!)
  // Y1 = -2/(pi z) + (2/pi) ln(z/2) J1 - (1/pi)(z/2) sum (psi(k+1)+psi(k+2)) (-t)^k/(k!(k+1)!)
  double term = 1.0;  // (-t)^k / (k! (k+1)!)
  double psi1 = -kEulerGamma;         // psi(k+1)
  double psi2 = 1.0 - kEulerGamma;    // psi(k+2)
  double sJ = 0.0, sY = 0.0;
  for (int k = 0; k < 60; ++k) {
    sJ += term;
    sY += (psi1 + psi2) * term;
    const double kk = (double)k;
    term *= -t / ((kk + 1.0) * (kk + 2.0));
    psi1 += 1.0 / (kk + 1.0);
    psi2 += 1.0 / (kk + 2.0);
    if (fabs(term) < 1e-18 * fabs(sJ)) break;
  }
  const double J1 = half * sJ;
  const double Y1 = -2.0 / (kPi * z) + (2.0 / kPi) * log(half) * J1 - (1.0 / kPi) * half * sY;
  return {J1, Y1};
}

}  // namespace lsk
