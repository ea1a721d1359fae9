// Off-grid volume potential and error function (see field.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace lsk {

// Gauss-Legendre rules on [-1, 1]: the tensor rules of 3, 4, 5, 6, 8, 10, 12 and 16 points per
// axis (index 0..7), the radial rule and the rule per edge piece of the polar integration; at
// most kMaxPieces graded pieces per half edge (enough for A >= 1e-12 h)
constexpr int kTensorRules = 8, kRuleRadial = 8, kRulePiece = 9, kFieldRules = 10, kMaxPieces = 48;
struct FieldRules {
  double t[104], w[104];
  int off[kFieldRules], n[kFieldRules];
};

// mode 0: u_out[t] = (V psi)(x_t); mode 1: e_out[t] = E(x_t) with q_t[t] = q(x_t), incidence
// angle theta and sign s.  targets: device, M x 2 doubles; psi: device complex128 in the order
// g2c maps grid index a*n + b to; (x0, y0) is the centre of cell (0, 0), h the cell side.
void launch_field_eval(const double* targets, long long M, int n, double x0, double y0, double h, double kappa,
                       const void* psi, const int* g2c, const FieldRules& R, int mode, const double* q_t,
                       double theta, double sign, void* u_out, double* e_out, hipStream_t s);

}  // namespace lsk
