// Neural-operator warm start (device network state and launchers).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

namespace lsk {
namespace nop {

// Parameter layout (one flat float array): P [C][nin], p [C], per layer R [C][C][2M][M] (complex,
// interleaved), W [C][C], b [C]; Q [nout][C], q [nout].
struct Net {
  int n = 0, C = 0, M = 0, L = 0, nin = 6, nout = 2, Bmax = 0;
  long long nparams = 0;
  long long OFF_P = 0, OFF_p = 0, OFF_Q = 0, OFF_q = 0;
  std::vector<long long> off_R, off_W, off_b;
  float *params = nullptr, *grads = nullptr, *adam_m = nullptr, *adam_v = nullptr;
  float2 *tw_w = nullptr, *tw_h = nullptr;
  std::vector<float*> act_V, act_Z;  // V_0..V_L, Z_0..Z_{L-1}
  std::vector<float2*> act_A2;       // A2 of each layer (kept for the weight gradient)
  float2 *buf_A1 = nullptr, *buf_S = nullptr, *buf_G = nullptr;
  float *buf_dV = nullptr, *buf_dZ = nullptr;
  float* buf_wpart = nullptr;  // BF16 mode: split partials of the channel-mixing weight gradients
  bool bf16 = false;           // channel mixing on the matrix cores with BF16 inputs
  const float* X_last = nullptr;
  int B_last = 0;
  int step_count = 0;

  float* param(long long off) const { return params + off; }
  float* grad(long long off) const { return grads + off; }
  float2* cparam(long long off) const { return reinterpret_cast<float2*>(params + off); }
  float2* cgrad(long long off) const { return reinterpret_cast<float2*>(grads + off); }

  void init_twiddles(hipStream_t s);
  void pointwise(const float* W, const float* bias, const float* X, float* Z, int Cin, int Cout, int B,
                 hipStream_t s);
  void pointwise_bwd(const float* W, const float* dZ, float* dX, int Cin, int Cout, int B, hipStream_t s);
  void wgrad(const float* dZ, const float* X, float* dW, float* db, int B, int Cin, int Cout, hipStream_t s);
  void forward(const float* X, float* O, int B, hipStream_t s);
  void backward(const float* dO, hipStream_t s);
  void loss(const float* O, const float2* w, const float2* t, const float* snorm2, float* dO, float* lossb, int B,
            hipStream_t s);
  void adam(float lr, float b1, float b2, float eps, hipStream_t s);
};

void launch_features(const double* q, int n, double L, double kappa, double theta, float* X, hipStream_t s);
void launch_warmstart(const double* q, int n, double L, double kappa, double theta, const float* O,
                      const double2* f, double2* psi0, hipStream_t s);

}  // namespace nop
}  // namespace lsk
