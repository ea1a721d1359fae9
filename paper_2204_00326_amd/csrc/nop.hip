// Neural-operator warm start for GMRES: forward, backward and Adam on the GPU.
//
// FNO-style network on an n x n image (channels first, FP32): lift 6 -> C, L layers of
// (truncated-DFT spectral convolution with M modes per axis + 1x1 convolution + bias,
// exact GELU except after the last layer), projection C -> 2.  The spectral convolution:
//   A1[c,h,kw] = sum_w V[c,h,w] e^{-2 pi i kw w/n},  A2[c,j,kw] = sum_h A1 e^{-2 pi i f(j) h/n},
//   S[o,j,kw] = sum_c A2[c,j,kw] R[c,o,j,kw],        B1[o,h,kw] = sum_j S e^{+2 pi i f(j) h/n},
//   Y[o,h,w]  = (1/n^2) sum_kw c_kw Re(B1 e^{+2 pi i kw w/n}),  c_0 = 1, c_kw = 2,
// with f(j) = j for j < M and n - 2M + j otherwise.  The backward kernels apply the adjoint
// of each step; complex gradients are stored as (d/dRe, d/dIm).
#include <hip/hip_runtime.h>

#include <cmath>

#include "nop.h"

namespace lsk {
namespace nop {

__device__ inline float2 cmul(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline float2 cmulc(float2 a, float2 b) {  // conj(a) * b
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// ---- twiddles ----------------------------------------------------------------------------
__global__ void k_twiddles(float2* tw_w, float2* tw_h, int n, int M) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n * M) {
    const int w = i / M, k = i % M;
    const double a = -2.0 * 3.14159265358979323846 * (double)((long long)k * w % n) / n;
    tw_w[i] = make_float2((float)cos(a), (float)sin(a));
  }
  if (i < n * 2 * M) {
    const int h = i / (2 * M), j = i % (2 * M);
    const int f = j < M ? j : n - 2 * M + j;
    const double a = -2.0 * 3.14159265358979323846 * (double)((long long)f * h % n) / n;
    tw_h[i] = make_float2((float)cos(a), (float)sin(a));
  }
}

// ---- pointwise (1x1 convolution) -----------------------------------------------------------
// Z[b][o][p] (+)= sum_c W[o][c] V[b][c][p] + bias[o]
__global__ void k_pointwise(const float* __restrict__ W, const float* __restrict__ bias, const float* __restrict__ V,
                            float* __restrict__ Z, int Cin, int Cout, int P, int accumulate) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int o = blockIdx.y, b = blockIdx.z;
  if (p >= P) return;
  const float* v = V + (long long)b * Cin * P + p;
  float acc = bias ? bias[o] : 0.f;
  for (int c = 0; c < Cin; ++c) acc = fmaf(W[o * Cin + c], v[(long long)c * P], acc);
  float* z = Z + ((long long)b * Cout + o) * P + p;
  *z = accumulate ? *z + acc : acc;
}

// dV[b][c][p] (+)= sum_o W[o][c] dZ[b][o][p]
__global__ void k_pointwise_bwd(const float* __restrict__ W, const float* __restrict__ dZ, float* __restrict__ dV,
                                int Cin, int Cout, int P, int accumulate) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y, b = blockIdx.z;
  if (p >= P) return;
  const float* dz = dZ + (long long)b * Cout * P + p;
  float acc = 0.f;
  for (int o = 0; o < Cout; ++o) acc = fmaf(W[o * Cin + c], dz[(long long)o * P], acc);
  float* d = dV + ((long long)b * Cin + c) * P + p;
  *d = accumulate ? *d + acc : acc;
}

// dW[o][c] = sum_{b,p} dZ[b][o][p] V[b][c][p]  (c < Cin);  db[o] = sum dZ[b][o][p]  (c == Cin)
__global__ __launch_bounds__(256) void k_wgrad(const float* __restrict__ dZ, const float* __restrict__ V,
                                               float* __restrict__ dW, float* __restrict__ db, int B, int Cin,
                                               int Cout, int P, int c0) {
  __shared__ float red[4];
  const int o = blockIdx.y, c = blockIdx.x + c0;  // c == Cin -> bias
  float acc = 0.f;
  for (int b = 0; b < B; ++b) {
    const float* dz = dZ + ((long long)b * Cout + o) * P;
    const float* v = c < Cin ? V + ((long long)b * Cin + c) * P : nullptr;
    for (int p = threadIdx.x; p < P; p += blockDim.x) acc += v ? dz[p] * v[p] : dz[p];
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    if (c < Cin)
      dW[o * Cin + c] = s;
    else
      db[o] = s;
  }
}

// ---- GELU ---------------------------------------------------------------------------------
// ---- channel mixing on the matrix cores (BF16 inputs, FP32 accumulation) ----------------
// v_mfma_f32_16x16x16_bf16: lane l supplies A[l % 16][4 (l / 16) + t] and B[4 (l / 16) + t][l % 16]
// (t < 4) and receives D[4 (l / 16) + v][l % 16] (v < 4).  FP32 values are rounded to bfloat16
// (nearest even) as they are loaded; weights stay FP32 in memory.
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ inline short f2bf(float f) {
  const unsigned u = __float_as_uint(f);
  return (short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// Z_b[o][p] = (accumulate ? Z_b[o][p] : 0) + bias[o] + sum_c A[o*sao + c*sac] X_b[c][p]; a wave owns
// 16 pixels and every output row (tiles of 16), a workgroup 64 pixels of one sample.
__global__ __launch_bounds__(256) void k_pw_mfma(const float* __restrict__ A, int sao, int sac,
                                                 const float* __restrict__ bias, const float* __restrict__ X,
                                                 float* __restrict__ Z, int K, int M, int P, int accumulate) {
  constexpr int MT = 16;  // at most 256 output rows
  const int b = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int p0 = (blockIdx.x * 4 + wave) * 16;
  const int p = p0 + li;
  const bool pin = p < P;
  const float* Xb = X + (long long)b * K * P;
  const int mt = (M + 15) / 16;
  f32x4 acc[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) acc[t] = (f32x4){0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    bf16x4 bx;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = k0 + 4 * lg + t;
      bx[t] = f2bf((pin && k < K) ? Xb[(long long)k * P + p] : 0.f);
    }
#pragma unroll
    for (int ti = 0; ti < MT; ++ti) {
      if (ti >= mt) break;
      const int o = ti * 16 + li;
      bf16x4 ax;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int k = k0 + 4 * lg + t;
        ax[t] = f2bf((o < M && k < K) ? A[(long long)o * sao + (long long)k * sac] : 0.f);
      }
      acc[ti] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ax, bx, acc[ti], 0, 0, 0);
    }
  }
  if (!pin) return;
  float* Zb = Z + (long long)b * M * P;
#pragma unroll
  for (int ti = 0; ti < MT; ++ti) {
    if (ti >= mt) break;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int o = ti * 16 + 4 * lg + v;
      if (o >= M) continue;
      float r = acc[ti][v] + (bias ? bias[o] : 0.f);
      float* z = Zb + (long long)o * P + p;
      *z = accumulate ? *z + r : r;
    }
  }
}

// partial[split][o][c] = sum over the split's pixels of dZ_b[o][p] V_b[c][p]; split = (sample,
// range of KS pixels); the waves of a workgroup take the 16x16 tiles of the (o, c) block in turn
__global__ __launch_bounds__(256) void k_wgrad_mfma(const float* __restrict__ dZ, const float* __restrict__ V,
                                                    float* __restrict__ part, int Cin, int Cout, int P, int KS,
                                                    int nsp) {
  const int split = blockIdx.x;
  const int b = split / nsp, sp = split - b * nsp;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int mt = (Cout + 15) / 16, nt = (Cin + 15) / 16;
  const int pb = sp * KS, pe = pb + KS < P ? pb + KS : P;
  const float* dZb = dZ + (long long)b * Cout * P;
  const float* Vb = V + (long long)b * Cin * P;
  float* out = part + (long long)split * Cout * Cin;
  for (int tile = wave; tile < mt * nt; tile += 4) {
    const int o = (tile / nt) * 16 + li, c = (tile % nt) * 16 + li;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = pb; k0 < pe; k0 += 16) {
      const int k = k0 + 4 * lg;  // 4 consecutive pixels
      bf16x4 ax, bx;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const bool kin = k + t < pe;
        ax[t] = f2bf((o < Cout && kin) ? dZb[(long long)o * P + k + t] : 0.f);
        bx[t] = f2bf((c < Cin && kin) ? Vb[(long long)c * P + k + t] : 0.f);
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ax, bx, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int oo = (tile / nt) * 16 + 4 * lg + v;
      if (oo < Cout && c < Cin) out[(long long)oo * Cin + c] = acc[v];
    }
  }
}

// dW[e] = sum_s part[s][e] in split order (deterministic)
__global__ void k_wgrad_reduce(const float* __restrict__ part, int nsplit, float* __restrict__ dW, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  float acc = 0.f;
  for (int q = 0; q < nsplit; ++q) acc += part[(long long)q * n + e];
  dW[e] = acc;
}

__global__ void k_gelu(const float* __restrict__ Z, float* __restrict__ V, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float x = Z[i];
  V[i] = 0.5f * x * (1.f + erff(x * 0.70710678118654752f));
}

__global__ void k_gelu_bwd(const float* __restrict__ Z, const float* __restrict__ dV, float* __restrict__ dZ,
                           long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float x = Z[i];
  const float g = 0.5f * (1.f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.3989422804014327f;
  dZ[i] = dV[i] * g;
}

// ---- spectral convolution, forward ------------------------------------------------------------
// A1[r][kw] = sum_w V[r][w] tw_w[w][kw],  r = (b, c, h)
__global__ void k_dft_w(const float* __restrict__ V, const float2* __restrict__ tw_w, float2* __restrict__ A1,
                        long long rows, int n, int M) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * M) return;
  const long long r = t / M;
  const int k = (int)(t % M);
  const float* v = V + r * n;
  float2 acc = make_float2(0.f, 0.f);
  for (int w = 0; w < n; ++w) {
    const float x = v[w];
    const float2 tw = tw_w[w * M + k];
    acc.x = fmaf(x, tw.x, acc.x);
    acc.y = fmaf(x, tw.y, acc.y);
  }
  A1[t] = acc;
}

// A2[bc][j][kw] = sum_h A1[bc][h][kw] tw_h[h][j]
__global__ void k_dft_h(const float2* __restrict__ A1, const float2* __restrict__ tw_h, float2* __restrict__ A2,
                        long long BC, int n, int M) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int JK = 2 * M * M;
  if (t >= BC * JK) return;
  const long long bc = t / JK;
  const int jk = (int)(t % JK), j = jk / M, k = jk % M;
  const float2* a = A1 + bc * n * M + k;
  float2 acc = make_float2(0.f, 0.f);
  for (int h = 0; h < n; ++h) {
    const float2 p = cmul(a[(long long)h * M], tw_h[h * 2 * M + j]);
    acc.x += p.x;
    acc.y += p.y;
  }
  A2[t] = acc;
}

// S[b][o][mode] = sum_c A2[b][c][mode] R[c][o][mode]
__global__ void k_mix(const float2* __restrict__ A2, const float2* __restrict__ R, float2* __restrict__ S, int B,
                      int C, int NM) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)B * C * NM) return;
  const int mode = (int)(t % NM);
  const int o = (int)((t / NM) % C);
  const int b = (int)(t / ((long long)NM * C));
  float2 acc = make_float2(0.f, 0.f);
  for (int c = 0; c < C; ++c) {
    const float2 p = cmul(A2[((long long)b * C + c) * NM + mode], R[((long long)c * C + o) * NM + mode]);
    acc.x += p.x;
    acc.y += p.y;
  }
  S[t] = acc;
}

// B1[bo][h][kw] = sum_j S[bo][j][kw] conj(tw_h[h][j])
__global__ void k_idft_h(const float2* __restrict__ S, const float2* __restrict__ tw_h, float2* __restrict__ B1,
                         long long BO, int n, int M) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= BO * n * M) return;
  const long long bo = t / (n * M);
  const int hk = (int)(t % (n * M)), h = hk / M, k = hk % M;
  const float2* s = S + bo * 2 * M * M + k;
  float2 acc = make_float2(0.f, 0.f);
  for (int j = 0; j < 2 * M; ++j) {
    const float2 p = cmulc(tw_h[h * 2 * M + j], s[j * M]);
    acc.x += p.x;
    acc.y += p.y;
  }
  B1[t] = acc;
}

// Z[bo][h][w] += (1/n^2) sum_kw c_kw Re(B1[bo][h][kw] conj(tw_w[w][kw]))
__global__ void k_idft_w(const float2* __restrict__ B1, const float2* __restrict__ tw_w, float* __restrict__ Z,
                         long long rows, int n, int M) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * n) return;
  const long long r = t / n;
  const int w = (int)(t % n);
  const float2* b1 = B1 + r * M;
  float acc = 0.f;
  for (int k = 0; k < M; ++k) {
    const float2 a = b1[k], tw = tw_w[w * M + k];
    const float re = a.x * tw.x + a.y * tw.y;  // Re(a * conj(tw))
    acc += (k == 0 ? 1.f : 2.f) * re;
  }
  Z[t] += acc / ((float)n * (float)n);
}

// ---- spectral convolution, adjoint --------------------------------------------------------------
// gB1[r][kw] = (c_kw / n^2) sum_w dY[r][w] tw_w[w][kw]
__global__ void k_adj_idft_w(const float* __restrict__ dY, const float2* __restrict__ tw_w, float2* __restrict__ gB1,
                             long long rows, int n, int M) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * M) return;
  const long long r = t / M;
  const int k = (int)(t % M);
  const float* d = dY + r * n;
  float2 acc = make_float2(0.f, 0.f);
  for (int w = 0; w < n; ++w) {
    const float x = d[w];
    const float2 tw = tw_w[w * M + k];
    acc.x = fmaf(x, tw.x, acc.x);
    acc.y = fmaf(x, tw.y, acc.y);
  }
  const float s = (k == 0 ? 1.f : 2.f) / ((float)n * (float)n);
  gB1[t] = make_float2(acc.x * s, acc.y * s);
}

// gS[bo][j][kw] = sum_h gB1[bo][h][kw] tw_h[h][j]   (same contraction as k_dft_h)
// gA2[b][c][mode] = sum_o conj(R[c][o][mode]) gS[b][o][mode]
__global__ void k_mix_bwd_in(const float2* __restrict__ gS, const float2* __restrict__ R, float2* __restrict__ gA2,
                             int B, int C, int NM) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)B * C * NM) return;
  const int mode = (int)(t % NM);
  const int c = (int)((t / NM) % C);
  const int b = (int)(t / ((long long)NM * C));
  float2 acc = make_float2(0.f, 0.f);
  for (int o = 0; o < C; ++o) {
    const float2 p = cmulc(R[((long long)c * C + o) * NM + mode], gS[((long long)b * C + o) * NM + mode]);
    acc.x += p.x;
    acc.y += p.y;
  }
  gA2[t] = acc;
}

// gR[c][o][mode] = sum_b conj(A2[b][c][mode]) gS[b][o][mode]
__global__ void k_mix_bwd_w(const float2* __restrict__ A2, const float2* __restrict__ gS, float2* __restrict__ gR,
                            int B, int C, int NM) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)C * C * NM) return;
  const int mode = (int)(t % NM);
  const int o = (int)((t / NM) % C);
  const int c = (int)(t / ((long long)NM * C));
  float2 acc = make_float2(0.f, 0.f);
  for (int b = 0; b < B; ++b) {
    const float2 p = cmulc(A2[((long long)b * C + c) * NM + mode], gS[((long long)b * C + o) * NM + mode]);
    acc.x += p.x;
    acc.y += p.y;
  }
  gR[t] = acc;
}

// gA1[bc][h][kw] = sum_j conj(tw_h[h][j]) gA2[bc][j][kw]   (same contraction as k_idft_h)
// dV[r][w] += sum_kw Re(conj(tw_w[w][kw]) gA1[r][kw])
__global__ void k_adj_dft_w(const float2* __restrict__ gA1, const float2* __restrict__ tw_w, float* __restrict__ dV,
                            long long rows, int n, int M) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * n) return;
  const long long r = t / n;
  const int w = (int)(t % n);
  const float2* g = gA1 + r * M;
  float acc = 0.f;
  for (int k = 0; k < M; ++k) {
    const float2 a = g[k], tw = tw_w[w * M + k];
    acc += tw.x * a.x + tw.y * a.y;
  }
  dV[t] += acc;
}

// ---- loss, Adam, features, warm start ------------------------------------------------------------
// per sample b: loss_b = |w O - t|^2 / snorm2_b ; dO = 2 conj(w) (w O - t) / snorm2_b / B
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ O, const float2* __restrict__ wgt,
                                              const float2* __restrict__ t, const float* __restrict__ snorm2,
                                              float* __restrict__ dO, float* __restrict__ lossb, int B, int P) {
  __shared__ float red[4];
  const int b = blockIdx.x;
  const float sn = snorm2[b];
  float acc = 0.f;
  for (int p = threadIdx.x; p < P; p += blockDim.x) {
    const float2 w = wgt[(long long)b * P + p];
    const float2 tt = t[(long long)b * P + p];
    const float ore = O[((long long)b * 2) * P + p], oim = O[((long long)b * 2 + 1) * P + p];
    const float rre = w.x * ore - w.y * oim - tt.x, rim = w.x * oim + w.y * ore - tt.y;
    acc += rre * rre + rim * rim;
    const float s = 2.f / sn / (float)B;
    dO[((long long)b * 2) * P + p] = s * (w.x * rre + w.y * rim);
    dO[((long long)b * 2 + 1) * P + p] = s * (w.x * rim - w.y * rre);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) lossb[b] = (red[0] + red[1] + red[2] + red[3]) / sn;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long long n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// X[6][n][n]: q, Re u_inc, Im u_inc, kappa/60, x1, x2 at the cell centres of [-L, L]^2 (grid order)
// WKB phase added along the incoming ray: kappa h sum_k g(x - (k + 1/2) h d) over k < 2n, with
// g = sqrt(max(1 + q, 0)) - 1 bilinear between cell centres and zero outside them.  The backward
// ray leaves the padded index box [-1, n]^2 for good once it is outside, so the sum stops there.
__device__ double ray_phase(const double* __restrict__ q, int n, double L, double kappa, double d1, double d2, int a,
                            int b) {
  const double h = 2.0 * L / n;
  const double u0 = (double)a, v0 = (double)b;  // fractional index of the cell centre itself
  double acc = 0.0;
  for (int k = 0; k < 2 * n; ++k) {
    const double t = k + 0.5;  // in units of h
    const double u = u0 - t * d1, v = v0 - t * d2;
    if (u <= -1.0 || v <= -1.0 || u >= (double)n || v >= (double)n) break;
    const int i0 = (int)floor(u), j0 = (int)floor(v);
    const double fu = u - i0, fv = v - j0;
    double val = 0.0;
#pragma unroll
    for (int di = 0; di < 2; ++di)
#pragma unroll
      for (int dj = 0; dj < 2; ++dj) {
        const int i = i0 + di, j = j0 + dj;
        if (i >= 0 && i < n && j >= 0 && j < n) {
          const double w = (di ? fu : 1.0 - fu) * (dj ? fv : 1.0 - fv);
          val += w * (sqrt(fmax(1.0 + q[(long long)i * n + j], 0.0)) - 1.0);
        }
      }
    acc += val;
  }
  return kappa * h * acc;
}

// channels: q, cos and sin of kappa d.x + phi, kappa/60, x1, x2
__global__ void k_features(const double* __restrict__ q, int n, double L, double kappa, double theta,
                           float* __restrict__ X) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int P = n * n;
  if (i >= P) return;
  const int a = i / n, b = i % n;
  const double h = 2.0 * L / n;
  const double x1 = -L + (a + 0.5) * h, x2 = -L + (b + 0.5) * h;
  const double d1 = cos(theta), d2 = sin(theta);
  const double ph = kappa * (d1 * x1 + d2 * x2) + ray_phase(q, n, L, kappa, d1, d2, a, b);
  X[i] = (float)q[i];
  X[P + i] = (float)cos(ph);
  X[2 * P + i] = (float)sin(ph);
  X[3 * P + i] = (float)(kappa / 60.0);
  X[4 * P + i] = (float)x1;
  X[5 * P + i] = (float)x2;
}

// psi0 = f exp(i phi) (1 + O_re + i O_im); O may be NULL (the WKB start alone)
__global__ void k_warmstart(const double* __restrict__ q, int n, double L, double kappa, double theta,
                            const float* __restrict__ O, const double2* __restrict__ f, double2* __restrict__ psi0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int P = n * n;
  if (i >= P) return;
  const double ph = ray_phase(q, n, L, kappa, cos(theta), sin(theta), i / n, i % n);
  const double c = cos(ph), sn = sin(ph);
  const double2 fv = f[i];
  const double br = fv.x * c - fv.y * sn, bi = fv.x * sn + fv.y * c;
  const double a = 1.0 + (O ? (double)O[i] : 0.0), b = O ? (double)O[P + i] : 0.0;
  psi0[i] = make_double2(br * a - bi * b, br * b + bi * a);
}

// ==============================================================================================
static inline unsigned nblk(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

void Net::init_twiddles(hipStream_t s) {
  k_twiddles<<<nblk((long long)n * 2 * M), 256, 0, s>>>(tw_w, tw_h, n, M);
}

// Z_b = W X_b + bias for each sample (W: Cout x Cin), on the matrix cores in BF16 mode
void Net::pointwise(const float* W, const float* bias, const float* X, float* Z, int Cin, int Cout, int B,
                    hipStream_t s) {
  const int P = n * n;
  if (bf16)
    k_pw_mfma<<<dim3((P + 63) / 64, B), 256, 0, s>>>(W, Cin, 1, bias, X, Z, Cin, Cout, P, 0);
  else
    k_pointwise<<<dim3(nblk(P), Cout, B), 256, 0, s>>>(W, bias, X, Z, Cin, Cout, P, 0);
}

// dX_b = W^T dZ_b
void Net::pointwise_bwd(const float* W, const float* dZ, float* dX, int Cin, int Cout, int B, hipStream_t s) {
  const int P = n * n;
  if (bf16)
    k_pw_mfma<<<dim3((P + 63) / 64, B), 256, 0, s>>>(W, 1, Cin, nullptr, dZ, dX, Cout, Cin, P, 0);
  else
    k_pointwise_bwd<<<dim3(nblk(P), Cin, B), 256, 0, s>>>(W, dZ, dX, Cin, Cout, P, 0);
}

// dW = sum_b dZ_b X_b^T, db = sum_b sum_p dZ_b
void Net::wgrad(const float* dZ, const float* X, float* dW, float* db, int B, int Cin, int Cout, hipStream_t s) {
  const int P = n * n;
  if (bf16) {
    const int KS = 1024, nsp = (P + KS - 1) / KS, nsplit = B * nsp;
    k_wgrad_mfma<<<nsplit, 256, 0, s>>>(dZ, X, buf_wpart, Cin, Cout, P, KS, nsp);
    k_wgrad_reduce<<<nblk((long long)Cout * Cin), 256, 0, s>>>(buf_wpart, nsplit, dW, Cout * Cin);
    k_wgrad<<<dim3(1, Cout), 256, 0, s>>>(dZ, X, dW, db, B, Cin, Cout, P, Cin);  // bias only
  } else {
    k_wgrad<<<dim3(Cin + 1, Cout), 256, 0, s>>>(dZ, X, dW, db, B, Cin, Cout, P, 0);
  }
}

void Net::forward(const float* X, float* O, int B, hipStream_t s) {
  const int P = n * n, NM = 2 * M * M;
  const long long BC = (long long)B * C;
  // lift
  pointwise(param(OFF_P), param(OFF_p), X, act_V[0], nin, C, B, s);
  for (int l = 0; l < L; ++l) {
    const float* V = act_V[l];
    float* Z = act_Z[l];
    pointwise(param(off_W[l]), param(off_b[l]), V, Z, C, C, B, s);
    k_dft_w<<<nblk(BC * n * M), 256, 0, s>>>(V, tw_w, buf_A1, BC * n, n, M);
    k_dft_h<<<nblk(BC * NM), 256, 0, s>>>(buf_A1, tw_h, act_A2[l], BC, n, M);
    k_mix<<<nblk(BC * NM), 256, 0, s>>>(act_A2[l], cparam(off_R[l]), buf_S, B, C, NM);
    k_idft_h<<<nblk(BC * n * M), 256, 0, s>>>(buf_S, tw_h, buf_A1, BC, n, M);
    k_idft_w<<<nblk(BC * P), 256, 0, s>>>(buf_A1, tw_w, Z, BC * n, n, M);
    if (l < L - 1)
      k_gelu<<<nblk(BC * P), 256, 0, s>>>(Z, act_V[l + 1], BC * P);
    else
      hipMemcpyAsync(act_V[l + 1], Z, sizeof(float) * BC * P, hipMemcpyDeviceToDevice, s);
  }
  pointwise(param(OFF_Q), param(OFF_q), act_V[L], O, C, nout, B, s);
  X_last = X;
  B_last = B;
}

void Net::backward(const float* dO, hipStream_t s) {
  const int B = B_last, P = n * n, NM = 2 * M * M;
  const long long BC = (long long)B * C;
  // projection
  wgrad(dO, act_V[L], grad(OFF_Q), grad(OFF_q), B, C, nout, s);
  pointwise_bwd(param(OFF_Q), dO, buf_dV, C, nout, B, s);
  for (int l = L - 1; l >= 0; --l) {
    // dZ
    if (l < L - 1)
      k_gelu_bwd<<<nblk(BC * P), 256, 0, s>>>(act_Z[l], buf_dV, buf_dZ, BC * P);
    else
      hipMemcpyAsync(buf_dZ, buf_dV, sizeof(float) * BC * P, hipMemcpyDeviceToDevice, s);
    const float* Vin = act_V[l];
    wgrad(buf_dZ, Vin, grad(off_W[l]), grad(off_b[l]), B, C, C, s);
    pointwise_bwd(param(off_W[l]), buf_dZ, buf_dV, C, C, B, s);
    // spectral adjoint
    k_adj_idft_w<<<nblk(BC * n * M), 256, 0, s>>>(buf_dZ, tw_w, buf_A1, BC * n, n, M);
    k_dft_h<<<nblk(BC * NM), 256, 0, s>>>(buf_A1, tw_h, buf_S, BC, n, M);  // gS
    k_mix_bwd_w<<<nblk((long long)C * C * NM), 256, 0, s>>>(act_A2[l], buf_S, cgrad(off_R[l]), B, C, NM);
    k_mix_bwd_in<<<nblk(BC * NM), 256, 0, s>>>(buf_S, cparam(off_R[l]), buf_G, B, C, NM);
    k_idft_h<<<nblk(BC * n * M), 256, 0, s>>>(buf_G, tw_h, buf_A1, BC, n, M);  // gA1
    k_adj_dft_w<<<nblk(BC * P), 256, 0, s>>>(buf_A1, tw_w, buf_dV, BC * n, n, M);
  }
  // lift
  wgrad(buf_dV, X_last, grad(OFF_P), grad(OFF_p), B, nin, C, s);
}

void Net::loss(const float* O, const float2* w, const float2* t, const float* snorm2, float* dO, float* lossb, int B,
               hipStream_t s) {
  k_loss<<<B, 256, 0, s>>>(O, w, t, snorm2, dO, lossb, B, n * n);
}

void Net::adam(float lr, float b1, float b2, float eps, hipStream_t s) {
  ++step_count;
  const float c1 = 1.f - powf(b1, (float)step_count), c2 = 1.f - powf(b2, (float)step_count);
  k_adam<<<nblk(nparams), 256, 0, s>>>(params, grads, adam_m, adam_v, nparams, lr, b1, b2, eps, c1, c2);
}

void launch_features(const double* q, int n, double L, double kappa, double theta, float* X, hipStream_t s) {
  k_features<<<nblk((long long)n * n), 256, 0, s>>>(q, n, L, kappa, theta, X);
}

void launch_warmstart(const double* q, int n, double L, double kappa, double theta, const float* O,
                      const double2* f, double2* psi0, hipStream_t s) {
  k_warmstart<<<nblk((long long)n * n), 256, 0, s>>>(q, n, L, kappa, theta, O, f, psi0);
}

}  // namespace nop
}  // namespace lsk
