// C ABI of the neural-operator warm start (ls_nop_*).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ls.h"
#include "nop.h"

namespace ls {
void set_last_error(const std::string& msg);
}

struct ls_nop {
  lsk::nop::Net net;
  std::vector<void*> allocs;
  ~ls_nop() {
    for (void* p : allocs) (void)hipFree(p);
  }
  template <class T>
  T* alloc(size_t count) {
    void* p = nullptr;
    if (hipMalloc(&p, count * sizeof(T) + 16) != hipSuccess) throw std::runtime_error("hipMalloc failed");
    allocs.push_back(p);
    return reinterpret_cast<T*>(p);
  }
};

namespace {

ls_status nfail(ls_status code, const std::string& msg) {
  ls::set_last_error(msg);
  return code;
}

// deterministic initialisation: splitmix64 + Box-Muller
struct Rng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
  }
  double uniform() { return (next() >> 11) * (1.0 / 9007199254740992.0); }
  double normal() {
    double u1 = uniform(), u2 = uniform();
    if (u1 < 1e-300) u1 = 1e-300;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};

}  // namespace

extern "C" {

ls_status ls_nop_create(const ls_nop_config* cfg, ls_nop** out) {
  if (out) *out = nullptr;
  if (!cfg || !out) return nfail(LS_EINVAL, "NULL argument");
  if (cfg->n < 8 || cfg->width < 1 || cfg->width > 256 || cfg->modes < 1 || 2 * cfg->modes > cfg->n ||
      cfg->layers < 1 || cfg->batch_max < 1 || (cfg->bf16 != 0 && cfg->bf16 != 1))
    return nfail(LS_EINVAL, "invalid network configuration");
  ls_nop* N = nullptr;
  try {
    N = new ls_nop();
    lsk::nop::Net& net = N->net;
    net.n = cfg->n;
    net.C = cfg->width;
    net.M = cfg->modes;
    net.L = cfg->layers;
    net.Bmax = cfg->batch_max;
    const int C = net.C, M = net.M, n = net.n, L = net.L;
    long long off = 0;
    net.OFF_P = off;
    off += (long long)C * net.nin;
    net.OFF_p = off;
    off += C;
    for (int l = 0; l < L; ++l) {
      net.off_R.push_back(off);
      off += 2LL * C * C * 2 * M * M;
      net.off_W.push_back(off);
      off += (long long)C * C;
      net.off_b.push_back(off);
      off += C;
    }
    net.OFF_Q = off;
    off += (long long)net.nout * C;
    net.OFF_q = off;
    off += net.nout;
    net.nparams = off;
    net.params = N->alloc<float>(off);
    net.grads = N->alloc<float>(off);
    net.adam_m = N->alloc<float>(off);
    net.adam_v = N->alloc<float>(off);
    net.tw_w = N->alloc<float2>((size_t)n * M);
    net.tw_h = N->alloc<float2>((size_t)n * 2 * M);
    const long long P = (long long)n * n, BCP = (long long)net.Bmax * C * P, BCS = (long long)net.Bmax * C * 2 * M * M;
    for (int l = 0; l <= L; ++l) net.act_V.push_back(N->alloc<float>(BCP));
    for (int l = 0; l < L; ++l) {
      net.act_Z.push_back(N->alloc<float>(BCP));
      net.act_A2.push_back(N->alloc<float2>(BCS));
    }
    net.buf_A1 = N->alloc<float2>((size_t)net.Bmax * C * n * M);
    net.buf_S = N->alloc<float2>(BCS);
    net.buf_G = N->alloc<float2>(BCS);
    net.buf_dV = N->alloc<float>(BCP);
    net.buf_dZ = N->alloc<float>(BCP);
    net.bf16 = cfg->bf16 != 0;
    if (net.bf16) {
      const long long nsplit = (long long)net.Bmax * ((P + 1023) / 1024);
      const long long cmax = std::max<long long>(C, net.nin);
      net.buf_wpart = N->alloc<float>(nsplit * cmax * C);
    }
    // initial parameters (host), same scales as a standard FNO initialisation
    std::vector<float> h(off, 0.f);
    Rng rng{cfg->seed * 0x2545F4914F6CDD1DULL + 1};
    for (long long i = 0; i < (long long)C * net.nin; ++i) h[net.OFF_P + i] = (float)(rng.normal() / std::sqrt((double)net.nin));
    for (int l = 0; l < L; ++l) {
      const double sc = 1.0 / ((double)C * C);
      for (long long i = 0; i < 2LL * C * C * 2 * M * M; ++i) h[net.off_R[l] + i] = (float)(sc * rng.uniform());
      for (long long i = 0; i < (long long)C * C; ++i) h[net.off_W[l] + i] = (float)(rng.normal() / std::sqrt((double)C));
    }
    for (long long i = 0; i < (long long)net.nout * C; ++i) h[net.OFF_Q + i] = (float)(0.1 * rng.normal() / std::sqrt((double)C));
    if (hipMemcpy(net.params, h.data(), off * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(net.adam_m, 0, off * sizeof(float)) != hipSuccess ||
        hipMemset(net.adam_v, 0, off * sizeof(float)) != hipSuccess ||
        hipMemset(net.grads, 0, off * sizeof(float)) != hipSuccess)
      throw std::runtime_error("device initialisation failed");
    net.init_twiddles(nullptr);
    if (hipDeviceSynchronize() != hipSuccess) throw std::runtime_error("twiddle kernel failed");
    *out = N;
    return LS_OK;
  } catch (const std::exception& e) {
    delete N;
    return nfail(LS_ENOMEM, e.what());
  }
}

int64_t ls_nop_param_count(const ls_nop* N) { return N ? N->net.nparams : -1; }

ls_status ls_nop_get_params(const ls_nop* N, float* host, int64_t count) {
  if (!N || !host || count != N->net.nparams) return nfail(LS_EINVAL, "bad arguments");
  if (hipMemcpy(host, N->net.params, count * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
    return nfail(LS_EDEVICE, "copy failed");
  return LS_OK;
}

ls_status ls_nop_set_params(ls_nop* N, const float* host, int64_t count) {
  if (!N || !host || count != N->net.nparams) return nfail(LS_EINVAL, "bad arguments");
  if (hipMemcpy(N->net.params, host, count * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(N->net.adam_m, 0, count * sizeof(float)) != hipSuccess ||
      hipMemset(N->net.adam_v, 0, count * sizeof(float)) != hipSuccess)
    return nfail(LS_EDEVICE, "copy failed");
  N->net.step_count = 0;
  return LS_OK;
}

ls_status ls_nop_get_grads(const ls_nop* N, float* host, int64_t count) {
  if (!N || !host || count != N->net.nparams) return nfail(LS_EINVAL, "bad arguments");
  if (hipMemcpy(host, N->net.grads, count * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
    return nfail(LS_EDEVICE, "copy failed");
  return LS_OK;
}

ls_status ls_nop_forward(ls_nop* N, const float* X, float* O, int B, void* stream) {
  if (!N || !X || !O || B < 1 || B > N->net.Bmax) return nfail(LS_EINVAL, "bad arguments");
  N->net.forward(X, O, B, (hipStream_t)stream);
  if (hipGetLastError() != hipSuccess) return nfail(LS_EDEVICE, "forward kernels failed");
  return LS_OK;
}

ls_status ls_nop_backward(ls_nop* N, const float* dO, void* stream) {
  if (!N || !dO || N->net.B_last < 1) return nfail(LS_EINVAL, "backward needs a preceding forward");
  N->net.backward(dO, (hipStream_t)stream);
  if (hipGetLastError() != hipSuccess) return nfail(LS_EDEVICE, "backward kernels failed");
  return LS_OK;
}

ls_status ls_nop_loss(ls_nop* N, const float* O, const void* w, const void* t, const float* snorm2, int B, float* dO,
                      float* loss, void* stream) {
  if (!N || !O || !w || !t || !snorm2 || !dO || !loss || B < 1) return nfail(LS_EINVAL, "bad arguments");
  N->net.loss(O, (const float2*)w, (const float2*)t, snorm2, dO, loss, B, (hipStream_t)stream);
  if (hipGetLastError() != hipSuccess) return nfail(LS_EDEVICE, "loss kernel failed");
  return LS_OK;
}

ls_status ls_nop_adam_step(ls_nop* N, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!N || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return nfail(LS_EINVAL, "bad arguments");
  N->net.adam(lr, beta1, beta2, eps, (hipStream_t)stream);
  if (hipGetLastError() != hipSuccess) return nfail(LS_EDEVICE, "adam kernel failed");
  return LS_OK;
}

ls_status ls_nop_features(int n, double L, const double* q, double kappa, double theta, float* X, void* stream) {
  if (n < 1 || !(L > 0) || !q || !X || !(kappa > 0)) return nfail(LS_EINVAL, "bad arguments");
  lsk::nop::launch_features(q, n, L, kappa, theta, X, (hipStream_t)stream);
  if (hipGetLastError() != hipSuccess) return nfail(LS_EDEVICE, "features kernel failed");
  return LS_OK;
}

ls_status ls_nop_warmstart(int n, double L, const double* q, double kappa, double theta, const float* O,
                           const void* f, void* psi0, void* stream) {
  if (n < 1 || !(L > 0) || !q || !(kappa > 0) || !f || !psi0) return nfail(LS_EINVAL, "bad arguments");
  lsk::nop::launch_warmstart(q, n, L, kappa, theta, O, (const double2*)f, (double2*)psi0, (hipStream_t)stream);
  if (hipGetLastError() != hipSuccess) return nfail(LS_EDEVICE, "warmstart kernel failed");
  return LS_OK;
}

void ls_nop_destroy(ls_nop* N) { delete N; }

}  // extern "C"
