// NCA factors of the DAFMM on the device (Section 4.2.2, steps 1 and 2; the operators of
// Section 5).
//
// For every direction of one quadtree level at once (one workgroup each), the block
// V(target candidates, source candidates) is compressed by partially pivoted ACA with Rjasanow's
// stopping test ||u_k|| ||v_k|| <= eps ||S_k||_F, under the pivoting rules of the host routine
// (aca_impl.h): start at row 0, the column pivot is the largest residual entry of the pivot row
// over unused columns, the next row pivot the largest entry of the new residual column over
// unused rows, an exactly zero residual row moves on to the first unused row, magnitudes within a
// relative 1e-9 of the maximum are ties won by the lowest index.  The row pivots are the
// direction's self pivots P, the column pivots its far pivots F.  A second launch forms the
// interpolation operator X = V(target candidates, F) B^{-1} with B = V(P, F) by Gauss-Jordan
// elimination with partial pivoting on the augmented matrix [B^T | V(targets, F)^T].
//
// Entries of V come from the table of grid offsets; residual rows, factors and the augmented
// matrix sit in a global workspace of the workgroup (a few MB, L2-resident).  Reductions are a
// wave shuffle tree followed by the waves' results in wave order, so every thread holds the same
// value and the result does not depend on timing.  Levels run from the leaf up, because a level's
// target candidates are its children's self pivots (host index work between launches).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <string>
#include <vector>

#include "nca_device.h"

namespace {

constexpr int NT = 1024, NW = NT / 64;
constexpr double kTie = 1e-9;
// workspace columns per direction: min(m, nn) (the host routine's rank limit) up to this cap; ranks at
// eps_NCA >= 1e-15 stay far below it (15-60 on the benchmark grids, 46 at eps 1e-15 on 32 x 32)
constexpr int kRankCap = 4096;

struct NcaArgs {
  const double2* W;  // (2n-1)^2 table, offset (da, db) at (da+n-1)(2n-1) + db+n-1
  int n;
  const int2* tgt;
  const int* tgt_off;  // problem p: targets tgt[tgt_off[p] .. tgt_off[p+1])
  const int2* src;
  const int* src_off;
  const int* kcap;
  const long long* ws_off;  // U (kcap x m), V (kcap x nn), residual row (nn)
  double2* ws;
  unsigned char* used;  // row flags at tgt_off[p], column flags at mtot + src_off[p]
  int mtot;
  double eps;
  int* rows;
  int* cols;
  const int* piv_off;
  int* rank;
  int* status;  // 0 ok, 1 rank cap reached before the stopping test, 2 singular B
};

__device__ inline double2 went(const double2* __restrict__ W, int n, int2 t, int2 s) {
  return W[(long long)(t.x - s.x + n - 1) * (2 * n - 1) + (t.y - s.y + n - 1)];
}
// x - a * y
__device__ inline double2 csub_mul(double2 x, double2 a, double2 y) {
  return make_double2(x.x - (a.x * y.x - a.y * y.y), x.y - (a.x * y.y + a.y * y.x));
}
__device__ inline double2 cdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ inline double cabs2(double2 a) { return hypot(a.x, a.y); }

__device__ inline double block_max(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = sh[0];
  for (int w = 1; w < NW; ++w) r = fmax(r, sh[w]);
  __syncthreads();
  return r;
}
__device__ inline double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = sh[0];
  for (int w = 1; w < NW; ++w) r += sh[w];
  __syncthreads();
  return r;
}
__device__ inline int block_min(int v, int* sh) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  int r = sh[0];
  for (int w = 1; w < NW; ++w) r = min(r, sh[w]);
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(NT) void k_nca_aca(NcaArgs A) {
  __shared__ double shd[NW];
  __shared__ int shi[NW];
  const int p = blockIdx.x, tid = threadIdx.x;
  const int2* T = A.tgt + A.tgt_off[p];
  const int m = A.tgt_off[p + 1] - A.tgt_off[p];
  const int2* S = A.src + A.src_off[p];
  const int nn = A.src_off[p + 1] - A.src_off[p];
  const int kc = A.kcap[p];
  double2* U = A.ws + A.ws_off[p];
  double2* V = U + (long long)kc * m;
  double2* r = V + (long long)kc * nn;
  unsigned char* ru = A.used + A.tgt_off[p];
  unsigned char* cu = A.used + A.mtot + A.src_off[p];
  int* rows = A.rows + A.piv_off[p];
  int* cols = A.cols + A.piv_off[p];
  for (int i = tid; i < m; i += NT) ru[i] = 0;
  for (int j = tid; j < nn; j += NT) cu[j] = 0;
  __syncthreads();
  const int kmax = min(kc, min(m, nn));
  int k = 0, i = m > 0 ? 0 : -1;
  double normS2 = 0.0;  // the same in every thread
  bool stopped = false;
  while (k < kmax && i >= 0) {
    int j = -1;
    for (;;) {
      // residual row i over every column
      for (int jj = tid; jj < nn; jj += NT) {
        double2 v = went(A.W, A.n, T[i], S[jj]);
        for (int l = 0; l < k; ++l) {
          const double2 ui = U[(long long)l * m + i];
          if (ui.x != 0.0 || ui.y != 0.0) v = csub_mul(v, ui, V[(long long)l * nn + jj]);
        }
        r[jj] = v;
      }
      double mx = 0.0;
      for (int jj = tid; jj < nn; jj += NT)
        if (!cu[jj]) mx = fmax(mx, cabs2(r[jj]));
      mx = block_max(mx, shd);
      if (tid == 0) ru[i] = 1;
      if (mx > 0.0) {
        const double thr = (1.0 - kTie) * mx;
        int jm = INT_MAX;
        for (int jj = tid; jj < nn; jj += NT)
          if (!cu[jj] && cabs2(r[jj]) >= thr) {
            jm = jj;
            break;
          }
        j = block_min(jm, shi);
        break;
      }
      // an exactly zero residual row: the first unused row
      __syncthreads();
      int nx = INT_MAX;
      for (int ii = tid; ii < m; ii += NT)
        if (!ru[ii]) {
          nx = ii;
          break;
        }
      nx = block_min(nx, shi);
      i = nx == INT_MAX ? -1 : nx;
      if (i < 0) break;
    }
    if (i < 0) break;
    // v_k = residual row / pivot, u_k = residual column j
    const double2 piv = r[j];
    double2* vk = V + (long long)k * nn;
    double2* uk = U + (long long)k * m;
    for (int jj = tid; jj < nn; jj += NT) vk[jj] = cdiv(r[jj], piv);
    for (int ii = tid; ii < m; ii += NT) {
      double2 u = went(A.W, A.n, T[ii], S[j]);
      for (int l = 0; l < k; ++l) {
        const double2 vj = V[(long long)l * nn + j];
        if (vj.x != 0.0 || vj.y != 0.0) u = csub_mul(u, vj, U[(long long)l * m + ii]);
      }
      uk[ii] = u;
    }
    if (tid == 0) {
      cu[j] = 1;
      rows[k] = i;
      cols[k] = j;
    }
    __syncthreads();
    if (A.eps > 0.0) {
      // ||S_k||_F^2 = ||S_{k-1}||_F^2 + 2 sum_l Re(<u_l, u_k> <v_k, v_l>) + ||u_k||^2 ||v_k||^2;
      // wave w takes the terms l = w, w + NW, ...
      const int w = tid >> 6, lane = tid & 63;
      double cr = 0.0;
      for (int l = w; l < k; l += NW) {
        const double2* ul = U + (long long)l * m;
        const double2* vl = V + (long long)l * nn;
        double ar = 0, ai = 0, br = 0, bi = 0;
        for (int ii = lane; ii < m; ii += 64) {
          const double2 a = ul[ii], b = uk[ii];
          ar += a.x * b.x + a.y * b.y;
          ai += a.x * b.y - a.y * b.x;
        }
        for (int jj = lane; jj < nn; jj += 64) {
          const double2 a = vk[jj], b = vl[jj];
          br += a.x * b.x + a.y * b.y;
          bi += a.x * b.y - a.y * b.x;
        }
        for (int o = 32; o > 0; o >>= 1) {
          ar += __shfl_xor(ar, o);
          ai += __shfl_xor(ai, o);
          br += __shfl_xor(br, o);
          bi += __shfl_xor(bi, o);
        }
        cr += 2.0 * (ar * br - ai * bi);
      }
      cr = block_sum(lane == 0 ? cr : 0.0, shd);
      double nu2 = 0, nv2 = 0;
      for (int ii = tid; ii < m; ii += NT) nu2 += uk[ii].x * uk[ii].x + uk[ii].y * uk[ii].y;
      for (int jj = tid; jj < nn; jj += NT) nv2 += vk[jj].x * vk[jj].x + vk[jj].y * vk[jj].y;
      nu2 = block_sum(nu2, shd);
      nv2 = block_sum(nv2, shd);
      normS2 += cr + nu2 * nv2;
      ++k;
      if (sqrt(nu2 * nv2) <= A.eps * sqrt(fmax(normS2, 0.0))) {
        stopped = true;
        break;
      }
    } else {
      ++k;
    }
    if (k >= kmax) break;
    // next row pivot: the largest entry of u_k over unused rows (else the first unused row)
    double mx = 0.0;
    for (int ii = tid; ii < m; ii += NT)
      if (!ru[ii]) mx = fmax(mx, cabs2(uk[ii]));
    mx = block_max(mx, shd);
    const double thr = (1.0 - kTie) * mx;
    int nx = INT_MAX;
    for (int ii = tid; ii < m; ii += NT)
      if (!ru[ii] && (mx == 0.0 || cabs2(uk[ii]) >= thr)) {
        nx = ii;
        break;
      }
    nx = block_min(nx, shi);
    i = nx == INT_MAX ? -1 : nx;
  }
  if (tid == 0) {
    A.rank[p] = k;
    A.status[p] = (A.eps > 0.0 && !stopped && i >= 0 && k == kc && kc < min(m, nn)) ? 1 : 0;
  }
}

// X = V(targets, F) B^{-1}: Gauss-Jordan with partial pivoting (largest magnitude, first on ties)
// on G = [B^T | V(targets, F)^T], k x (k + m), row-major in the workspace; X is m x k row-major.
__global__ __launch_bounds__(NT) void k_nca_interp(NcaArgs A, const long long* __restrict__ aug_off,
                                                   double2* __restrict__ aug, const long long* __restrict__ x_off,
                                                   double2* __restrict__ X) {
  __shared__ double shd[NW];
  __shared__ int shi[NW];
  const int p = blockIdx.x, tid = threadIdx.x;
  const int k = A.rank[p];
  if (k == 0 || A.status[p] != 0) return;
  const int2* T = A.tgt + A.tgt_off[p];
  const int m = A.tgt_off[p + 1] - A.tgt_off[p];
  const int2* S = A.src + A.src_off[p];
  const int* rows = A.rows + A.piv_off[p];
  const int* cols = A.cols + A.piv_off[p];
  const int ld = k + m;
  double2* G = aug + aug_off[p];
  for (long long idx = tid; idx < (long long)k * ld; idx += NT) {
    const int a = (int)(idx / ld), c = (int)(idx % ld);
    const int2 f = S[cols[a]];
    G[idx] = c < k ? went(A.W, A.n, T[rows[c]], f) : went(A.W, A.n, T[c - k], f);
  }
  __syncthreads();
  for (int col = 0; col < k; ++col) {
    double mx = 0.0;
    for (int rr = col + tid; rr < k; rr += NT) mx = fmax(mx, cabs2(G[(long long)rr * ld + col]));
    mx = block_max(mx, shd);
    if (mx == 0.0) {  // uniform: every thread holds the same maximum
      if (tid == 0) A.status[p] = 2;
      return;
    }
    int pr = INT_MAX;
    for (int rr = col + tid; rr < k; rr += NT)
      if (cabs2(G[(long long)rr * ld + col]) == mx) {
        pr = rr;
        break;
      }
    pr = block_min(pr, shi);
    if (pr != col)
      for (int c = tid; c < ld; c += NT) {
        const double2 t = G[(long long)pr * ld + c];
        G[(long long)pr * ld + c] = G[(long long)col * ld + c];
        G[(long long)col * ld + c] = t;
      }
    __syncthreads();
    const double2 piv = G[(long long)col * ld + col];
    __syncthreads();
    for (int c = col + 1 + tid; c < ld; c += NT) G[(long long)col * ld + c] = cdiv(G[(long long)col * ld + c], piv);
    __syncthreads();
    const int w = ld - col - 1;
    for (long long idx = tid; idx < (long long)(k - 1) * w; idx += NT) {
      int rr = (int)(idx / w);
      if (rr >= col) ++rr;
      const int c = col + 1 + (int)(idx % w);
      G[(long long)rr * ld + c] = csub_mul(G[(long long)rr * ld + c], G[(long long)rr * ld + col], G[(long long)col * ld + c]);
    }
    __syncthreads();
  }
  double2* Xp = X + x_off[p];
  for (long long idx = tid; idx < (long long)m * k; idx += NT) {
    const int q = (int)(idx / k), a = (int)(idx % k);
    Xp[idx] = G[(long long)a * ld + k + q];
  }
}

void hip_ok(hipError_t e, const char* what) {
  if (e != hipSuccess) throw ls::LsError(-1, std::string("NCA on the device: ") + what + ": " + hipGetErrorString(e));
}

// device buffer freed at scope exit
struct Dev {
  void* p = nullptr;
  Dev() = default;
  Dev(const Dev&) = delete;
  Dev& operator=(const Dev&) = delete;
  ~Dev() {
    if (p) (void)hipFree(p);
  }
  template <typename T>
  T* alloc(size_t count) {
    hip_ok(hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)), "hipMalloc");
    return static_cast<T*>(p);
  }
  template <typename T>
  T* upload(const std::vector<T>& v, hipStream_t s) {
    T* d = alloc<T>(v.size());
    if (!v.empty()) hip_ok(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s), "upload");
    return d;
  }
};

}  // namespace

namespace ls {

NCA build_nca_device(const Plan& p, const WTable& W, const double2* Wd, double tol, hipStream_t s) {
  NCA out;
  out.lv.resize(p.leaf + 1);
  nca_near_tiles(p, W, out);
  if (p.top > p.leaf) return out;  // no far field
  for (int nu = p.leaf; nu >= p.top; --nu) {
    const Level& l = p.lv[nu];
    LevelNCA& L = out.lv[nu];
    const int nd = l.ndir;
    const bool is_leaf = (nu == p.leaf);
    L.self.assign(nd, {});
    L.far.assign(nd, {});
    L.rank.assign(nd, 0);
    L.C.assign(nd, {});
    std::vector<std::vector<Off>> tc(nd), sc(nd);
    std::vector<int2> tgt, src;
    std::vector<int> toff{0}, soff{0}, kcap(nd), poff{0};
    std::vector<long long> wsoff{0}, augoff{0}, xoff{0};
    for (int dir = 0; dir < nd; ++dir) {
      nca_candidates(p, out, nu, dir, tc[dir], sc[dir]);
      const int m = (int)tc[dir].size(), nn = (int)sc[dir].size();
      for (const Off& o : tc[dir]) tgt.push_back(make_int2(o.a, o.b));
      for (const Off& o : sc[dir]) src.push_back(make_int2(o.a, o.b));
      toff.push_back(toff.back() + m);
      soff.push_back(soff.back() + nn);
      const int kc = std::min(std::min(m, nn), kRankCap);
      kcap[dir] = kc;
      poff.push_back(poff.back() + kc);
      wsoff.push_back(wsoff.back() + (long long)kc * (m + nn) + nn);
      augoff.push_back(augoff.back() + (long long)kc * (kc + m));
      xoff.push_back(xoff.back() + (long long)m * kc);
    }
    Dev dt, ds, dto, dso, dkc, dws, dpo, dused, drows, dcols, drank, dst, dao, daug, dxo, dx;
    NcaArgs A;
    A.W = Wd;
    A.n = p.n;
    A.tgt = dt.upload(tgt, s);
    A.tgt_off = dto.upload(toff, s);
    A.src = ds.upload(src, s);
    A.src_off = dso.upload(soff, s);
    A.kcap = dkc.upload(kcap, s);
    A.ws_off = dws.upload(wsoff, s);
    Dev dwork;
    A.ws = dwork.alloc<double2>((size_t)wsoff.back());
    A.mtot = toff.back();
    A.used = dused.alloc<unsigned char>((size_t)toff.back() + soff.back());
    A.eps = tol;
    A.rows = drows.alloc<int>((size_t)poff.back());
    A.cols = dcols.alloc<int>((size_t)poff.back());
    A.piv_off = dpo.upload(poff, s);
    A.rank = drank.alloc<int>(nd);
    A.status = dst.alloc<int>(nd);
    const long long* aoff = dao.upload(augoff, s);
    double2* aug = daug.alloc<double2>((size_t)augoff.back());
    const long long* xo = dxo.upload(xoff, s);
    double2* X = dx.alloc<double2>((size_t)xoff.back());
    k_nca_aca<<<nd, NT, 0, s>>>(A);
    hip_ok(hipGetLastError(), "k_nca_aca launch");
    k_nca_interp<<<nd, NT, 0, s>>>(A, aoff, aug, xo, X);
    hip_ok(hipGetLastError(), "k_nca_interp launch");
    std::vector<int> rank(nd), status(nd), rows(poff.back()), cols(poff.back());
    std::vector<double2> Xh((size_t)xoff.back());
    hip_ok(hipMemcpyAsync(rank.data(), A.rank, nd * sizeof(int), hipMemcpyDeviceToHost, s), "ranks");
    hip_ok(hipMemcpyAsync(status.data(), A.status, nd * sizeof(int), hipMemcpyDeviceToHost, s), "status");
    if (!rows.empty()) {
      hip_ok(hipMemcpyAsync(rows.data(), A.rows, rows.size() * sizeof(int), hipMemcpyDeviceToHost, s), "rows");
      hip_ok(hipMemcpyAsync(cols.data(), A.cols, cols.size() * sizeof(int), hipMemcpyDeviceToHost, s), "cols");
    }
    if (!Xh.empty())
      hip_ok(hipMemcpyAsync(Xh.data(), X, Xh.size() * sizeof(double2), hipMemcpyDeviceToHost, s), "operators");
    hip_ok(hipStreamSynchronize(s), "NCA kernels");
    for (int dir = 0; dir < nd; ++dir) {
      if (status[dir] == 1)
        throw LsError(-1, "NCA on the device: ACA reached rank " + std::to_string(kcap[dir]) + " at level " +
                              std::to_string(nu) + " before its stopping test");
      if (status[dir] == 2) throw LsError(-1, "singular pivot block in NCA");
      const int k = rank[dir];
      const int m = (int)tc[dir].size();
      L.rank[dir] = k;
      for (int t = 0; t < k; ++t) {
        L.self[dir].push_back(tc[dir][rows[poff[dir] + t]]);
        L.far[dir].push_back(sc[dir][cols[poff[dir] + t]]);
      }
      if (k == 0) continue;
      const double2* Xd = Xh.data() + xoff[dir];
      auto rows_of = [&](int r0, int nr) {
        std::vector<zd> M((size_t)nr * k);
        for (int q = 0; q < nr; ++q)
          for (int a = 0; a < k; ++a) {
            const double2 v = Xd[(size_t)(r0 + q) * k + a];
            M[(size_t)q * k + a] = zd(v.x, v.y);
          }
        return M;
      };
      if (is_leaf) {
        if (dir == 0) out.U = rows_of(0, m);
      } else {
        const int kcc = m / 4;  // rows of child c: its self pivots, c * kcc ...
        L.C[dir].resize(4);
        for (int c = 0; c < 4; ++c) L.C[dir][c] = rows_of(c * kcc, kcc);
      }
    }
    L.kmax = 0;
    for (int dir = 0; dir < nd; ++dir) L.kmax = std::max(L.kmax, L.rank[dir]);
    if (is_leaf) out.kleaf = L.rank[0];
  }
  nca_m2l(p, W, out);
  return out;
}

}  // namespace ls
