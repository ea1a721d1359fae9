// Device kernels for gfx950 (CDNA4, wave64).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <stdexcept>
#include <type_traits>

#include "h0.h"
#include "kernels.h"

namespace lsk {

// Timing of the next timed launch on this host thread (set by the caller): the launch is made
// with AMD's extended launch, which stamps `start` and `stop` from the dispatch itself.
static thread_local hipEvent_t g_next_start = nullptr, g_next_stop = nullptr;
void set_next_launch_events(hipEvent_t start, hipEvent_t stop) {
  g_next_start = start;
  g_next_stop = stop;
}
bool next_launch_events_pending() { return g_next_start != nullptr; }
void clear_next_launch_events() { g_next_start = g_next_stop = nullptr; }
static inline bool take_launch_events(hipEvent_t* a, hipEvent_t* b) {
  if (!g_next_start) return false;
  *a = g_next_start;
  *b = g_next_stop;
  g_next_start = g_next_stop = nullptr;
  return true;
}
// launch kernel K (a name, possibly a template-id) timed if events are pending
#define LSK_LAUNCH(K, GRID, BLOCK, SHM, STREAM, ...)                                   \
  do {                                                                                 \
    hipEvent_t e0_, e1_;                                                               \
    if (take_launch_events(&e0_, &e1_))                                                \
      hipExtLaunchKernelGGL(K, dim3(GRID), dim3(BLOCK), SHM, STREAM, e0_, e1_, 0, __VA_ARGS__); \
    else                                                                               \
      K<<<GRID, BLOCK, SHM, STREAM>>>(__VA_ARGS__);                                    \
  } while (0)

template <typename T>
struct V2;
template <>
struct V2<double> {
  using type = double2;
};
template <>
struct V2<float> {
  using type = float2;
};
// complex bfloat16 storage (factor matrices read at half the FP32 traffic)
struct bf16 {};
struct alignas(4) BF2 {
  unsigned short x, y;
};
template <>
struct V2<bf16> {
  using type = BF2;
};
__device__ inline double2 to_d2(const double2& v) { return v; }
__device__ inline double2 to_d2(const float2& v) { return make_double2((double)v.x, (double)v.y); }
__device__ inline double2 to_d2(const BF2& v) {
  return make_double2((double)__uint_as_float((unsigned)v.x << 16), (double)__uint_as_float((unsigned)v.y << 16));
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide sum of (re, im) for a block of `nt` threads (multiple of 64, <= 1024).
// `red` is a __shared__ buffer of 2 * 16 doubles.  Result valid in all threads.
__device__ inline double2 block_sum2(double re, double im, double* red) {
  re = wave_sum(re);
  im = wave_sum(im);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) {
    red[2 * wid] = re;
    red[2 * wid + 1] = im;
  }
  __syncthreads();
  double a = 0, b = 0;
  for (int w = 0; w < nw; ++w) {
    a += red[2 * w];
    b += red[2 * w + 1];
  }
  return make_double2(a, b);
}

// =====================================================================================
// Stencil GEMM over boxes with operators shared by all boxes of a level (DAFMM passes).
// A workgroup owns 64 boxes of one task (one output level/direction/class) and
// kRowBlock output rows; its 4 waves split the task's flattened (term, k) range evenly and
// are summed in a fixed order through LDS, so results are deterministic.  Operator
// entries are wave-uniform and read through the scalar cache; inputs are coalesced along
// the box index of the class half-grid.
// =====================================================================================
// Plain aggregates for loads through address-space-qualified pointers.
struct alignas(16) PD2 {
  double x, y;
};
struct alignas(8) PF2 {
  float x, y;
};
template <typename T>
struct P2;
template <>
struct P2<double> {
  using type = PD2;
};
template <>
struct P2<float> {
  using type = PF2;
};
template <typename T>
using ConstPtr = __attribute__((address_space(4))) const typename P2<T>::type*;
template <typename T>
using GlobalPtr = __attribute__((address_space(1))) const typename P2<T>::type*;
template <typename T>
__device__ inline typename P2<T>::type ldc(ConstPtr<T> p, long long i) {
  typename P2<T>::type v;
  v.x = p[i].x;
  v.y = p[i].y;
  return v;
}
template <typename T>
__device__ inline typename P2<T>::type ldg(GlobalPtr<T> p, long long i) {
  typename P2<T>::type v;
  v.x = p[i].x;
  v.y = p[i].y;
  return v;
}

template <typename T, int Tag>
__global__ __launch_bounds__(kStencilThreads) void k_stencil(const DTask* __restrict__ tasks,
                                                             const DTerm* __restrict__ terms,
                                                             const int* __restrict__ blk_task) {
  using C2 = typename P2<T>::type;
  __shared__ C2 red[kStencilWaves - 1][kRowBlock][kBoxBlock];
  const int blk = blockIdx.x;
  const int rhs = blockIdx.y;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int ti = __builtin_amdgcn_readfirstlane(blk_task[blk]);
  const DTask& tk = tasks[ti];
  const int local = blk - tk.blk0;
  const int rb = local % tk.nrb;
  const int bb = local / tk.nrb;
  const int nh = tk.nh;
  const int box = bb * kBoxBlock + lane;
  const bool active = box < nh * nh;
  const int ha = active ? box / nh : 0;
  const int hb = active ? box - ha * nh : 0;
  const int m0 = rb * kRowBlock;
  const int Mpad = tk.Mpad;
  T ar[kRowBlock], ai[kRowBlock];
#pragma unroll
  for (int r = 0; r < kRowBlock; ++r) {
    ar[r] = 0;
    ai[r] = 0;
  }
  // this wave's share of the flattened (term, k) range
  const int P = tk.ktot;
  const int p0 = (int)(((long long)P * wave) / kStencilWaves);
  const int p1 = (int)(((long long)P * (wave + 1)) / kStencilWaves);
  int t = tk.t0;
  while (t < tk.t1 && terms[t].kbase + terms[t].K <= p0) ++t;
  for (; t < tk.t1; ++t) {
    const DTerm& tm = terms[t];
    if (tm.kbase >= p1) break;
    const int kb = p0 > tm.kbase ? p0 - tm.kbase : 0;
    const int ke = (p1 - tm.kbase) < tm.K ? (p1 - tm.kbase) : tm.K;
    const int nhi = tm.nh_in;
    const long long plane = (long long)nhi * nhi;
    long long src = 0;
    bool ok = active;
    switch (tm.mode) {
      case MODE_SAME:
        src = (long long)tk.cout * plane + box;
        break;
      case MODE_SHIFT: {
        const int sa = ha + tm.sha, sb = hb + tm.shb;
        ok = ok && sa >= 0 && sa < nhi && sb >= 0 && sb < nhi;
        src = (long long)tm.cin * plane + (long long)sa * nhi + sb;
      } break;
      case MODE_CHILD: {
        const int pa = 2 * ha + (tk.cout >> 1), pb = 2 * hb + (tk.cout & 1);
        src = (long long)tm.cin * plane + (long long)pa * nhi + pb;
      } break;
      default: {  // MODE_PARENT: the parent of (class cout, ha, hb) has full coords (ha, hb)
        const int pc = ((ha & 1) << 1) | (hb & 1);
        src = (long long)pc * plane + (long long)(ha >> 1) * nhi + (hb >> 1);
      } break;
    }
    if (ok) {
      GlobalPtr<T> in = (GlobalPtr<T>)(reinterpret_cast<const C2*>(tm.in) + rhs * tm.in_rhs + src);
      ConstPtr<T> op = (ConstPtr<T>)(reinterpret_cast<const C2*>(tm.op) + m0);
      const long long ks = 4 * plane;
      int k = kb;
      for (; k + 2 <= ke; k += 2) {
        const C2 x0 = ldg<T>(in, (long long)k * ks);
        const C2 x1 = ldg<T>(in, (long long)(k + 1) * ks);
#pragma unroll
        for (int r = 0; r < kRowBlock; ++r) {
          const C2 a = ldc<T>(op, (long long)k * Mpad + r);
          ar[r] = fma(a.x, x0.x, ar[r]);
          ar[r] = fma(-a.y, x0.y, ar[r]);
          ai[r] = fma(a.x, x0.y, ai[r]);
          ai[r] = fma(a.y, x0.x, ai[r]);
        }
#pragma unroll
        for (int r = 0; r < kRowBlock; ++r) {
          const C2 b = ldc<T>(op, (long long)(k + 1) * Mpad + r);
          ar[r] = fma(b.x, x1.x, ar[r]);
          ar[r] = fma(-b.y, x1.y, ar[r]);
          ai[r] = fma(b.x, x1.y, ai[r]);
          ai[r] = fma(b.y, x1.x, ai[r]);
        }
      }
      if (k < ke) {
        const C2 x0 = ldg<T>(in, (long long)k * ks);
#pragma unroll
        for (int r = 0; r < kRowBlock; ++r) {
          const C2 a = ldc<T>(op, (long long)k * Mpad + r);
          ar[r] = fma(a.x, x0.x, ar[r]);
          ar[r] = fma(-a.y, x0.y, ar[r]);
          ai[r] = fma(a.x, x0.y, ai[r]);
          ai[r] = fma(a.y, x0.x, ai[r]);
        }
      }
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int r = 0; r < kRowBlock; ++r) {
      C2 v;
      v.x = ar[r];
      v.y = ai[r];
      red[wave - 1][r][lane] = v;
    }
  }
  __syncthreads();
  if (wave != 0 || !active) return;
#pragma unroll
  for (int w = 0; w < kStencilWaves - 1; ++w)
#pragma unroll
    for (int r = 0; r < kRowBlock; ++r) {
      const C2 v = red[w][r][lane];
      ar[r] += v.x;
      ai[r] += v.y;
    }
  C2* out = reinterpret_cast<C2*>(tk.out) + rhs * tk.out_rhs + (long long)tk.cout * nh * nh + box;
  const long long ks = 4LL * nh * nh;
#pragma unroll
  for (int r = 0; r < kRowBlock; ++r) {
    const int m = m0 + r;
    if (m < tk.M) {
      C2 v;
      v.x = ar[r];
      v.y = ai[r];
      if (tk.beta) {
        const C2 o = out[(long long)m * ks];
        v.x += o.x;
        v.y += o.y;
      }
      out[(long long)m * ks] = v;
    }
  }
}

template <int Tag>
static void launch_stencil_t(bool fp32, const DTask* tasks, const DTerm* terms, const int* blk_task, int nblocks,
                             int nrhs, hipStream_t s) {
  dim3 grid(nblocks, nrhs);
  if (fp32) {
    auto kern = k_stencil<float, Tag>;
    LSK_LAUNCH(kern, grid, kStencilThreads, 0, s, tasks, terms, blk_task);
  } else {
    auto kern = k_stencil<double, Tag>;
    LSK_LAUNCH(kern, grid, kStencilThreads, 0, s, tasks, terms, blk_task);
  }
}

void launch_stencil(int tag, bool fp32, const DTask* tasks, const DTerm* terms, const int* blk_task, int nblocks,
                    int nrhs, hipStream_t s) {
  if (nblocks <= 0) return;
  switch (tag) {
    case 0: launch_stencil_t<0>(fp32, tasks, terms, blk_task, nblocks, nrhs, s); break;
    case 1: launch_stencil_t<1>(fp32, tasks, terms, blk_task, nblocks, nrhs, s); break;
    case 2: launch_stencil_t<2>(fp32, tasks, terms, blk_task, nblocks, nrhs, s); break;
    case 3: launch_stencil_t<3>(fp32, tasks, terms, blk_task, nblocks, nrhs, s); break;
    default: launch_stencil_t<4>(fp32, tasks, terms, blk_task, nblocks, nrhs, s); break;
  }
}

// =====================================================================================
// Stencil GEMM on the matrix cores.  For one task (output level/direction/class) and a group of
// rpg 16-row tiles of the output, out[m][box] = sum_terms sum_k op_t[k][m] in_t[k][src_t(box)]
// is a sum of 16 x 4 by 4 x 16 products, one per 4-deep k-block of a term (a term's K is padded
// to the block by zeros); each input tile a wave loads is multiplied into all rpg row tiles.
// Complex entries: Re += Ar Xr - Ai Xi, Im += Ar Xi + Ai Xr, four real 16x16x4 MFMAs.  A
// workgroup's 4 waves cover 64 / kps boxes in sub-tiles of 16 boxes, and kps waves per sub-tile
// split the task's k-blocks; the parts are summed through LDS in a fixed order (deterministic).
// Long tasks also split their k-blocks over kgroups workgroups, each writing a partial plane that
// a separate launch adds in group order.  The host lists every k-block of a task (operator and
// input addresses, box shift, real depth), so the inner loop is a counted loop over descriptors
// read through the scalar cache, with a ring of in-flight loads (branch-free: clamped addresses,
// empty slots zeroed at use).  Lane l: A element (row l % 16, k l / 16), B element (k l / 16,
// box l % 16); the accumulator element v of lane l is (row l/16 + 4v) for FP64 and
// (row 4(l/16) + v) for FP32, box l % 16.
// =====================================================================================
typedef double mf64x4 __attribute__((ext_vector_type(4)));
typedef float mf32x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct MfmaAcc;
template <>
struct MfmaAcc<double> {
  using type = mf64x4;
  __device__ static inline mf64x4 mma(double a, double b, mf64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct MfmaAcc<float> {
  using type = mf32x4;
  __device__ static inline mf32x4 mma(float a, float b, mf32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// coherent (device-scope) loads and stores for data written and read inside one launch by
// different workgroups: relaxed agent-scope atomics, which neither hit nor leave stale copies
// in the per-CU and per-XCD caches
template <typename C2>
__device__ inline C2 ld_coh(const C2* p) {
  C2 v;
  v.x = __hip_atomic_load(&p->x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  v.y = __hip_atomic_load(&p->y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return v;
}
template <typename C2>
__device__ inline void st_coh(C2* p, const C2& v) {
  __hip_atomic_store(&p->x, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&p->y, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One block of the stencil GEMM: task ti, block `local` within the task, right-hand side rhs.
// A block covers one row group (up to four 16-row tiles: every wave multiplies each input tile it
// loads into all of them), 64 / kps boxes in sub-tiles of 16, and the k-blocks of split-K group
// grp.  COH: honour the coherence flags of the fused launch (inputs and outputs produced or
// consumed by other workgroups of the same launch).  Called by all 256 threads; contains
// barriers when the task splits its k-blocks over waves (kps > 1) or workgroups (kgroups > 1).
// IO: 0, IO_GATHER (the input is io.x read through io.gidx; the task has one same-box term, so
// the tree index of k row k of a lane's box is k * pks + lsrc; row group 0 stores the values
// into io.xs) or IO_EPILOGUE (the accumulated output is finished into io.y).
template <typename T, bool COH, int MT, int IO>
__device__ __forceinline__ void mfma_rows(const DTask& tk, const DTerm* __restrict__ terms, int rg, int bb, int grp,
                                          int rhs, T (*red)[16][64], const IoArgs& io) {
  using C2 = typename P2<T>::type;
  using GC = __attribute__((address_space(1))) const C2*;
  using MA = MfmaAcc<T>;
  using V4 = typename MA::type;
  constexpr int D = MT >= 3 ? 2 : 3;  // k-blocks in flight per wave
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int G = tk.kgroups;           // workgroups sharing the tile (split K)
  const int kps = tk.kps;             // 1, 2 or 4
  const int nsub = 4 / kps;           // box sub-tiles per workgroup
  const int sub = wave % nsub, kpart = wave / nsub;
  const int nh = tk.nh, nbox = nh * nh;
  const int li = lane & 15, lk = lane >> 4;
  const int box = (bb * nsub + sub) * 16 + li;
  const bool bact = box < nbox;
  const int ha = bact ? box / nh : 0;
  const int hb = bact ? box - ha * nh : 0;
  // operator rows of this lane in each tile (rows past M read row 0: finite, and never stored)
  int arow[MT];
#pragma unroll
  for (int r = 0; r < MT; ++r) {
    const int m = (rg * tk.rpg + r) * 16 + li;
    arow[r] = m < tk.M ? m : 0;
  }
  V4 cre[MT], cim[MT];
#pragma unroll
  for (int r = 0; r < MT; ++r) {
    cre[r] = V4{0, 0, 0, 0};
    cim[r] = V4{0, 0, 0, 0};
  }
  // this workgroup's share of the task's k-blocks, split again over its kps waves
  const int g0 = (int)(((long long)tk.ktot * grp) / G), g1 = (int)(((long long)tk.ktot * (grp + 1)) / G);
  const int nblk = g1 - g0;
  const int b0 = g0 + (int)(((long long)nblk * kpart) / kps);
  const int b1 = g0 + (int)(((long long)nblk * (kpart + 1)) / kps);
  // the lane's input box inside a plane of the input level (SHIFT adds each block's shift)
  const int nhi = tk.nh_in;
  const long long plane = (long long)nhi * nhi;
  long long lsrc = 0;
  switch (tk.mode) {
    case MODE_SAME: lsrc = (long long)tk.cout * plane + box; break;
    case MODE_SHIFT: lsrc = (long long)ha * nhi + hb; break;
    case MODE_CHILD: lsrc = (long long)(2 * ha + (tk.cout >> 1)) * nhi + 2 * hb + (tk.cout & 1); break;
    default: lsrc = (long long)(((ha & 1) << 1) | (hb & 1)) * plane + (long long)(ha >> 1) * nhi + (hb >> 1); break;
  }
  const bool shift = tk.mode == MODE_SHIFT;
  const long long Mp = tk.Mpad;
  // the descriptors are constant for the launch: read them through the scalar cache (a generic
  // pointer would be read with vector loads, whose completion the data loads would then share)
  using KC = __attribute__((address_space(4))) const KBlk*;
  const KC kbl = (KC)tk.kb;
  // ring of D in-flight k-blocks: the operator entries of every tile and the input entry.  The
  // loop is branch-free: past b1 the last block is fetched again and marked empty; an input past
  // the block's real depth or outside the domain is zeroed at use.
  C2 ra[D][MT], rx[D];
  bool rv[D];
  // IO_GATHER: the tree index of the lane's input for the next block of each slot and its index
  // in io.x (loaded one ring round before the value; a k row past the term's depth takes the
  // block's first row, inside the level), and the tree index of the value in the slot
  long long gnx[D], gcur[D];
  int enx[D];
  const int kg = IO == IO_GATHER ? terms[tk.t0].K : 0;
  auto gidx_load = [&](int s, int j) {
    const int jj = j < b1 ? j : b1 - 1;
    const int k = 4 * jj + lk < kg ? 4 * jj + lk : 4 * jj;
    gnx[s] = (long long)k * tk.pks + lsrc;
    enx[s] = bact ? io.gidx[gnx[s]] : 0;
  };
  // descriptors of the next ring round, read one round ahead so that the scalar loads complete
  // behind the matrix products instead of stalling the address computation
  struct Dsc {
    unsigned long long op, in;
    int sha, shb, klim;
  } dn[D];
  auto desc = [&](int s, int j) {
    const KC dp = kbl + (j < b1 ? j : b1 - 1);
    dn[s].op = dp->op;
    dn[s].in = dp->in;
    dn[s].sha = dp->sha;
    dn[s].shb = dp->shb;
    dn[s].klim = dp->klim;
  };
  auto fetch = [&](int s, int j) {
    const bool inr = j < b1;
    const unsigned long long d_op = dn[s].op, d_in = dn[s].in;
    const int d_sha = dn[s].sha, d_shb = dn[s].shb, d_klim = dn[s].klim;
    const int sa = ha + d_sha, sb = hb + d_shb;  // the shift is zero unless the term is shifted
    // branch-free validity (bitwise, not short-circuit): the box exists and, for a shifted term,
    // its neighbour lies inside the level
    const bool inside = ((unsigned)sa < (unsigned)nhi) & ((unsigned)sb < (unsigned)nhi);
    const bool ok = bact & (!shift | inside);
    const long long src = ok ? (long long)d_shb + (long long)d_sha * nhi + lsrc : 0;
    // a lane past the block's real depth reads row k = 0 of the block (inside the term's operator
    // and input) and is zeroed at use
    const bool kin = lk < d_klim;
    const long long lkc = kin ? lk : 0;
    const C2* pa = reinterpret_cast<const C2*>(d_op) + lkc * Mp;
#pragma unroll
    for (int r = 0; r < MT; ++r) {
      const GC q = (GC)(pa + arow[r]);
      ra[s][r].x = q->x;
      ra[s][r].y = q->y;
    }
    const C2* px = reinterpret_cast<const C2*>(d_in) + lkc * tk.pks + rhs * tk.in_rhs + src;
    if constexpr (IO == IO_GATHER) {
      const double2 xv = io.x[rhs * io.ldx + enx[s]];
      rx[s].x = (T)xv.x;
      rx[s].y = (T)xv.y;
      gcur[s] = gnx[s];
    } else if (COH && tk.coh_in) {
      rx[s] = ld_coh(px);
    } else {
      const GC q = (GC)px;
      rx[s].x = q->x;
      rx[s].y = q->y;
    }
    rv[s] = inr && ok && kin;
  };
  auto mac = [&](int s) {
    const T zr = 0;
    const T xr = rv[s] ? rx[s].x : zr, xi = rv[s] ? rx[s].y : zr;
    if constexpr (IO == IO_GATHER) {
      // the tree-order copy of the input, for the passes that read it later
      if (rg == 0 && rv[s]) reinterpret_cast<C2*>(const_cast<void*>(io.xs))[rhs * tk.in_rhs + gcur[s]] = rx[s];
    }
    // the real parts of the operator first, then the imaginary parts: an accumulator is reused
    // only 2 MT products later
#pragma unroll
    for (int r = 0; r < MT; ++r) {
      cre[r] = MA::mma(ra[s][r].x, xr, cre[r]);
      cim[r] = MA::mma(ra[s][r].x, xi, cim[r]);
    }
#pragma unroll
    for (int r = 0; r < MT; ++r) {
      cre[r] = MA::mma(-ra[s][r].y, xi, cre[r]);
      cim[r] = MA::mma(ra[s][r].y, xr, cim[r]);
    }
  };
  if (b0 < b1) {
#pragma unroll
    for (int s = 0; s < D; ++s) {
      if constexpr (IO == IO_GATHER) gidx_load(s, b0 + s);
      desc(s, b0 + s);
      fetch(s, b0 + s);
      desc(s, b0 + D + s);
      if constexpr (IO == IO_GATHER) gidx_load(s, b0 + D + s);
    }
    for (int c = b0; c < b1; c += D) {
#pragma unroll
      for (int s = 0; s < D; ++s) {
        mac(s);
        fetch(s, c + D + s);
        desc(s, c + 2 * D + s);
        if constexpr (IO == IO_GATHER) gidx_load(s, c + 2 * D + s);
      }
    }
  }
  // k-parts 1..kps-1 of each sub-tile hand their sums to part 0 through LDS; waves 1..3
  // own slots 0..2 (wave w = kpart * nsub + sub, so part 0 waves are 0..nsub-1)
  if (kps > 1) {
    // real parts, then imaginary parts, through one 16-value slot per wave
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (wave > 0 && kpart > 0) {
#pragma unroll
        for (int r = 0; r < MT; ++r)
#pragma unroll
          for (int v = 0; v < 4; ++v) red[wave - 1][4 * r + v][lane] = h ? cim[r][v] : cre[r][v];
      }
      __syncthreads();
      if (kpart == 0)
        for (int q = 1; q < kps; ++q) {
          const int w = q * nsub + sub;
#pragma unroll
          for (int r = 0; r < MT; ++r)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              if (h)
                cim[r][v] += red[w - 1][4 * r + v][lane];
              else
                cre[r][v] += red[w - 1][4 * r + v][lane];
            }
        }
      if (h == 0) __syncthreads();
    }
  }
  C2* out = reinterpret_cast<C2*>(tk.out) + rhs * tk.out_rhs + (long long)tk.cout * nbox + box;
  const long long kso = 4LL * nbox;
  if (G > 1) {
    // split K: this group's partial tile goes to its plane of part[rhs][g][m][box]; a separate
    // launch (launch_splitk_reduce) adds the planes in group order into the output
    if (kpart != 0 || !bact) return;
    using GO = __attribute__((address_space(1))) C2*;
    C2* pp = reinterpret_cast<C2*>(tk.part) + rhs * tk.part_rhs + (long long)grp * tk.M * nbox + box;
#pragma unroll
    for (int r = 0; r < MT; ++r)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = (rg * tk.rpg + r) * 16 + MA::row(lane, v);
        if (m < tk.M) {
          GO q = (GO)(pp + (long long)m * nbox);
          q->x = cre[r][v];
          q->y = cim[r][v];
        }
      }
    return;
  }
  if (kpart != 0 || !bact) return;
  const bool coh = COH && tk.coh_out;
#pragma unroll
  for (int r = 0; r < MT; ++r)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = (rg * tk.rpg + r) * 16 + MA::row(lane, v);
      if (m < tk.M) {
        C2 o;
        o.x = cre[r][v];
        o.y = cim[r][v];
        C2* po = out + (long long)m * kso;
        if (tk.beta) {
          const C2 p = COH ? ld_coh(po) : *po;
          o.x += p.x;
          o.y += p.y;
        }
        if constexpr (IO == IO_EPILOGUE) {
          // finish into the caller's vector: y[e] = alpha x[e] + coef q[e] v, e = gidx[t]
          const long long t = (po - reinterpret_cast<const C2*>(io.ys)) - rhs * tk.out_rhs;
          const int e = io.gidx[t];
          const double c = io.q ? io.coef * io.q[e] : io.coef;
          double2 r = make_double2(c * (double)o.x, c * (double)o.y);
          if (io.alpha != 0.0) {
            const double2 xv = io.x[rhs * io.ldx + e];
            r.x += io.alpha * xv.x;
            r.y += io.alpha * xv.y;
          }
          io.y[rhs * io.ldy + e] = r;
        } else if (coh) {
          st_coh(po, o);
        } else {
          *po = o;
        }
      }
    }
}

// tasks with io set have one row tile per row group (rpg = 1)
template <typename T, bool COH>
__device__ __forceinline__ void mfma_block(const DTask* __restrict__ tasks, const DTerm* __restrict__ terms, int ti,
                                           int local, int rhs, T (*red)[16][64], const IoArgs& io) {
  const DTask& tk = tasks[ti];
  const int rg = local % tk.nrb;               // row group (rpg 16-row tiles)
  const int bb = tk.bb0 + (local / tk.nrb) % tk.nbb;  // box block
  const int grp = local / (tk.nrb * tk.nbb);   // split-K group
  if constexpr (!COH) {
    if (tk.io == IO_GATHER) {
      mfma_rows<T, false, 1, IO_GATHER>(tk, terms, rg, bb, grp, rhs, red, io);
      return;
    }
    if (tk.io == IO_EPILOGUE) {
      mfma_rows<T, false, 1, IO_EPILOGUE>(tk, terms, rg, bb, grp, rhs, red, io);
      return;
    }
  }
  const int ntile = (tk.M + 15) / 16 - tk.rpg * rg;
  switch (ntile >= tk.rpg ? tk.rpg : ntile) {
    case 1: mfma_rows<T, COH, 1, 0>(tk, terms, rg, bb, grp, rhs, red, io); break;
    case 2: mfma_rows<T, COH, 2, 0>(tk, terms, rg, bb, grp, rhs, red, io); break;
    case 3: mfma_rows<T, COH, 3, 0>(tk, terms, rg, bb, grp, rhs, red, io); break;
    default: mfma_rows<T, COH, 4, 0>(tk, terms, rg, bb, grp, rhs, red, io); break;
  }
}

template <typename T>
__global__ __launch_bounds__(256, 2) void k_stencil_mfma(const DTask* __restrict__ tasks, const DTerm* __restrict__ terms,
                                                      const int* __restrict__ blk_task, IoArgs io) {
  __shared__ T red[3][16][64];
  // blk_task holds (task, block within the task) pairs in dispatch order, heaviest blocks first
  const int ti = __builtin_amdgcn_readfirstlane(blk_task[2 * blockIdx.x]);
  const int local = __builtin_amdgcn_readfirstlane(blk_task[2 * blockIdx.x + 1]);
  mfma_block<T, false>(tasks, terms, ti, local, blockIdx.y, red, io);
}

// out[m][box] (+)= sum_{g = 0..G-1} part[g][m][box] for every split-K task of a pass, the planes
// added in group order (deterministic); one thread per output element, grid.y = task, grid.z = rhs
template <typename T>
__global__ __launch_bounds__(256) void k_splitk_reduce(const SplitK* __restrict__ sk) {
  using C2 = typename P2<T>::type;
  const SplitK& k = sk[blockIdx.y];
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long ne = (long long)k.M * k.nbox;
  if (e >= ne) return;
  const int rhs = blockIdx.z;
  const long long m = e / k.nbox, box = e - m * k.nbox;
  const C2* p = reinterpret_cast<const C2*>(k.part) + rhs * k.part_rhs + e;
  C2 o = p[0];
  for (int g = 1; g < k.G; ++g) {
    const C2 q = p[(long long)g * ne];
    o.x += q.x;
    o.y += q.y;
  }
  C2* po = reinterpret_cast<C2*>(k.out) + rhs * k.out_rhs + (long long)k.cout * k.nbox + box + m * 4LL * k.nbox;
  if (k.beta) {
    const C2 q = *po;
    o.x += q.x;
    o.y += q.y;
  }
  *po = o;
}

void launch_splitk_reduce(bool fp32, const SplitK* sk, int ntask, long long max_elems, int nrhs, hipStream_t s) {
  if (ntask <= 0) return;
  dim3 grid((unsigned)((max_elems + 255) / 256), ntask, nrhs);
  if (fp32)
    k_splitk_reduce<float><<<grid, 256, 0, s>>>(sk);
  else
    k_splitk_reduce<double><<<grid, 256, 0, s>>>(sk);
}

void launch_stencil_mfma(bool fp32, const DTask* tasks, const DTerm* terms, const int* blk_task, int nblocks,
                         int nrhs, hipStream_t s, const IoArgs* io) {
  if (nblocks <= 0) return;
  dim3 grid(nblocks, nrhs);
  const IoArgs a = io ? *io : IoArgs{};
  if (fp32) {
    auto kern = k_stencil_mfma<float>;
    LSK_LAUNCH(kern, grid, 256, 0, s, tasks, terms, blk_task, a);
  } else {
    auto kern = k_stencil_mfma<double>;
    LSK_LAUNCH(kern, grid, 256, 0, s, tasks, terms, blk_task, a);
  }
}

// =====================================================================================
// All DAFMM passes in one persistent launch.  Each workgroup loops: take a ticket (an atomic
// counter), map it to (queue item, right-hand side), wait until every stage the item's task
// depends on is complete, compute the block (mfma_block with coherent loads of in-launch
// inputs and coherent stores of in-launch outputs), then count it into its stage.  The
// workgroup whose count completes a stage sets the stage's bit in 64 flag words, one per group
// of workgroups (blockIdx % 64, so each group sits on one XCD), and waiting workgroups poll
// their group's word: the polls spread over 64 cache lines instead of hammering one.
// The queue is in dependency order, so the earliest unfinished ticket never waits on a later
// one: every wait ends.  A wait is still bounded: past kSpinLimit polls bit 31 is set in every
// flag word, every later wait returns at once, and the epilogue turns the result into NaN.
// Counter block (unsigned, one 128-byte line each): line 0 the ticket, lines 1..nst the stage
// counts, lines nst+1..nst+64 the group flags.
// =====================================================================================
constexpr unsigned kSpinLimit = 1u << 20;
constexpr int kFlagGroups = 64;
constexpr int kLine = 32;  // unsigned per 128-byte line

template <typename T>
__global__ __launch_bounds__(256, 2) void k_dafmm_fused(const DTask* __restrict__ tasks,
                                                     const DTerm* __restrict__ terms, const int* __restrict__ queue,
                                                     int nitems, int nrhs, int nst, unsigned* __restrict__ ctr,
                                                     const unsigned* __restrict__ need) {
  __shared__ T red[3][16][64];
  __shared__ int s_ticket;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const unsigned one = lane == 0 ? 1u : 0u;  // a whole-wave atomic adds 1 in total
  const int total = nitems * nrhs;
  unsigned* const flags = ctr + kLine * (1 + nst);
  unsigned* const myflag = flags + kLine * (blockIdx.x % kFlagGroups);
  // Every branch below that encloses a barrier, an atomic or a loop is uniform per wave (wave 0
  // alone takes tickets, waits and counts, with all of its lanes), so all lanes of a wave stay
  // in the same iteration.  Each iteration takes a new ticket, so at most total + 1 iterations.
  for (int iter = 0; iter <= total; ++iter) {
    if (wave == 0) {
      const unsigned old = atomicAdd(&ctr[0], one);
      s_ticket = (int)__builtin_amdgcn_readfirstlane(old);
    }
    __syncthreads();
    const int tkt = __builtin_amdgcn_readfirstlane(s_ticket);
    if (tkt >= total) break;
    const int item = tkt / nrhs, rhs = tkt - item * nrhs;
    const int ti = __builtin_amdgcn_readfirstlane(queue[2 * item]);
    const int local = __builtin_amdgcn_readfirstlane(queue[2 * item + 1]);
    const DTask& tk = tasks[ti];
    if (wave == 0) {
      unsigned mask = 0;
      for (int q = 0; q < 3; ++q)
        if (tk.dep[q] >= 0) mask |= 1u << tk.dep[q];
      if (mask != 0u) {
        for (unsigned spins = 0;; ++spins) {
          const unsigned f = __builtin_amdgcn_readfirstlane(
              __hip_atomic_load(myflag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
          if ((f & mask) == mask || (f >> 31) != 0u) break;
          if (spins >= kSpinLimit) {
            __hip_atomic_fetch_or(flags + kLine * lane, 1u << 31, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          __builtin_amdgcn_s_sleep(16);
        }
      }
    }
    __syncthreads();
    mfma_block<T, true>(tasks, terms, ti, local, rhs, red, IoArgs{});
    // this wave's stores (coherent at device scope) are complete before the workgroup counts
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (wave == 0) {
      const int st = tk.stage;
      const unsigned old = __builtin_amdgcn_readfirstlane(
          __hip_atomic_fetch_add(&ctr[kLine * (1 + st)], one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      if (old + 1u == need[st] * (unsigned)nrhs)  // the stage's last block: publish it
        __hip_atomic_fetch_or(flags + kLine * lane, 1u << st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

int dafmm_fused_workgroups(bool fp32) {
  static int cached[2] = {0, 0};
  int& c = cached[fp32 ? 1 : 0];
  if (c > 0) return c;
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) throw std::runtime_error("hipGetDevice failed");
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    throw std::runtime_error("hipDeviceGetAttribute failed");
  hipError_t e = fp32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_dafmm_fused<float>, 256, 0)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_dafmm_fused<double>, 256, 0);
  if (e != hipSuccess || per <= 0) throw std::runtime_error("occupancy query failed");
  c = cus * per;
  return c;
}

void launch_dafmm_fused(bool fp32, const DTask* tasks, const DTerm* terms, const int* queue, int nitems, int nrhs,
                        int nst, unsigned* ctr, const unsigned* need, int nwg, hipStream_t s) {
  if (nitems <= 0) return;
  if (nwg <= 0) throw std::runtime_error("fused DAFMM launch needs workgroups");
  if (nst < 1 || nst > 31) throw std::runtime_error("fused DAFMM launch takes 1 to 31 stages");
  if (fp32) {
    auto kern = k_dafmm_fused<float>;
    LSK_LAUNCH(kern, dim3(nwg), 256, 0, s, tasks, terms, queue, nitems, nrhs, nst, ctr, need);
  } else {
    auto kern = k_dafmm_fused<double>;
    LSK_LAUNCH(kern, dim3(nwg), 256, 0, s, tasks, terms, queue, nitems, nrhs, nst, ctr, need);
  }
}

int dafmm_fused_counter_lines(int nst) { return 1 + nst + kFlagGroups; }

// =====================================================================================
// Offset table W(da, db) = h^2 (i/4) H0(kappa h |(da, db)|); the (0,0) entry is set on
// the host (exact self-cell integral).
// =====================================================================================
__global__ void k_wtable(double2* W, int n, double h, double kappa) {
  const int m = 2 * n - 1;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)m * m) return;
  const int da = (int)(idx / m) - (n - 1);
  const int db = (int)(idx % m) - (n - 1);
  if (da == 0 && db == 0) {
    W[idx] = make_double2(0.0, 0.0);
    return;
  }
  const double r = h * sqrt((double)da * da + (double)db * db);
  const cplx H = hankel0(kappa * r);
  // (i/4)(J0 + i Y0) = (-Y0/4) + i (J0/4)
  W[idx] = make_double2(-0.25 * H.im * h * h, 0.25 * H.re * h * h);
}

void launch_wtable(double2* W, int n, double h, double kappa, hipStream_t s) {
  const long long tot = (long long)(2 * n - 1) * (2 * n - 1);
  k_wtable<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(W, n, h, kappa);
}

// =====================================================================================
// Permutations and the operator epilogue y = alpha x + coef * q * (V x)
// =====================================================================================
template <typename T>
__global__ void k_gather(const double2* __restrict__ x, long long ldx, typename V2<T>::type* __restrict__ xs,
                         const int* __restrict__ idx, long long N) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (t >= N) return;
  const double2 v = x[rhs * ldx + idx[t]];
  typename V2<T>::type o;
  o.x = (T)v.x;
  o.y = (T)v.y;
  xs[rhs * N + t] = o;
}

void launch_gather(bool to_fp32, const double2* x, long long ldx, void* xs, const int* idx, long long N, int nrhs,
                   hipStream_t s) {
  dim3 grid((unsigned)((N + 255) / 256), nrhs);
  if (to_fp32)
    k_gather<float><<<grid, 256, 0, s>>>(x, ldx, (float2*)xs, idx, N);
  else
    k_gather<double><<<grid, 256, 0, s>>>(x, ldx, (double2*)xs, idx, N);
}

template <typename T>
__global__ void k_epilogue(const double2* __restrict__ x, long long ldx, const typename V2<T>::type* __restrict__ ys,
                           const int* __restrict__ idx, const double* __restrict__ q, double alpha, double coef,
                           double2* __restrict__ y, long long ldy, long long N) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (i >= N) return;
  const typename V2<T>::type v = ys[rhs * N + idx[i]];
  const double c = q ? coef * q[i] : coef;
  double2 o = make_double2(c * (double)v.x, c * (double)v.y);
  if (alpha != 0.0) {
    const double2 xv = x[rhs * ldx + i];
    o.x += alpha * xv.x;
    o.y += alpha * xv.y;
  }
  y[rhs * ldy + i] = o;
}

void launch_epilogue(bool from_fp32, const double2* x, long long ldx, const void* ys, const int* idx, const double* q,
                     double alpha, double coef, double2* y, long long ldy, long long N, int nrhs, hipStream_t s) {
  dim3 grid((unsigned)((N + 255) / 256), nrhs);
  if (from_fp32)
    k_epilogue<float><<<grid, 256, 0, s>>>(x, ldx, (const float2*)ys, idx, q, alpha, coef, y, ldy, N);
  else
    k_epilogue<double><<<grid, 256, 0, s>>>(x, ldx, (const double2*)ys, idx, q, alpha, coef, y, ldy, N);
}

template <typename T>
__global__ void k_gather_zero(const double2* __restrict__ x, long long ldx, typename V2<T>::type* __restrict__ xs,
                              const int* __restrict__ idx, long long N, unsigned* __restrict__ zero, int nz) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (rhs == 0 && t < nz) zero[t * kLine] = 0u;
  if (t >= N) return;
  const double2 v = x[rhs * ldx + idx[t]];
  typename V2<T>::type o;
  o.x = (T)v.x;
  o.y = (T)v.y;
  xs[rhs * N + t] = o;
}

void launch_gather_zero(bool to_fp32, const double2* x, long long ldx, void* xs, const int* idx, long long N, int nrhs,
                        unsigned* zero, int nz, hipStream_t s) {
  if (nz < 0 || nz > 1024) throw std::runtime_error("gather: at most 1024 counter lines to zero");
  const long long nt = N > nz ? N : nz;
  dim3 grid((unsigned)((nt + 255) / 256), nrhs);
  if (to_fp32)
    k_gather_zero<float><<<grid, 256, 0, s>>>(x, ldx, (float2*)xs, idx, N, zero, nz);
  else
    k_gather_zero<double><<<grid, 256, 0, s>>>(x, ldx, (double2*)xs, idx, N, zero, nz);
}

template <typename T>
__global__ void k_epilogue_checked(const double2* __restrict__ x, long long ldx,
                                   const typename V2<T>::type* __restrict__ ys, const int* __restrict__ idx,
                                   const double* __restrict__ q, double alpha, double coef, double2* __restrict__ y,
                                   long long ldy, long long N, const unsigned* __restrict__ err) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (i >= N) return;
  if ((*err >> 31) != 0u) {
    y[rhs * ldy + i] = make_double2(__builtin_nan(""), __builtin_nan(""));
    return;
  }
  const typename V2<T>::type v = ys[rhs * N + idx[i]];
  const double c = q ? coef * q[i] : coef;
  double2 o = make_double2(c * (double)v.x, c * (double)v.y);
  if (alpha != 0.0) {
    const double2 xv = x[rhs * ldx + i];
    o.x += alpha * xv.x;
    o.y += alpha * xv.y;
  }
  y[rhs * ldy + i] = o;
}

void launch_epilogue_checked(bool from_fp32, const double2* x, long long ldx, const void* ys, const int* idx,
                             const double* q, double alpha, double coef, double2* y, long long ldy, long long N,
                             int nrhs, const unsigned* err, hipStream_t s) {
  dim3 grid((unsigned)((N + 255) / 256), nrhs);
  if (from_fp32)
    k_epilogue_checked<float><<<grid, 256, 0, s>>>(x, ldx, (const float2*)ys, idx, q, alpha, coef, y, ldy, N, err);
  else
    k_epilogue_checked<double><<<grid, 256, 0, s>>>(x, ldx, (const double2*)ys, idx, q, alpha, coef, y, ldy, N, err);
}

__global__ void k_permute(const double2* __restrict__ x, long long ldx, double2* __restrict__ y, long long ldy,
                          const int* __restrict__ perm, long long N, int scatter) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (i >= N) return;
  if (scatter)
    y[rhs * ldy + perm[i]] = x[rhs * ldx + i];
  else
    y[rhs * ldy + i] = x[rhs * ldx + perm[i]];
}

void launch_permute(const double2* x, long long ldx, double2* y, long long ldy, const int* perm, long long N, int nrhs,
                    bool scatter, hipStream_t s) {
  dim3 grid((unsigned)((N + 255) / 256), nrhs);
  k_permute<<<grid, 256, 0, s>>>(x, ldx, y, ldy, perm, N, scatter ? 1 : 0);
}

__global__ void k_planewave(const double* px, const double* py, const double* q, const double* angles, double kappa,
                            double coef, double2* f, long long ldf, long long N) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (i >= N) return;
  const double th = angles[rhs];
  const double ph = kappa * (cos(th) * px[i] + sin(th) * py[i]);
  const double c = coef * q[i];
  f[rhs * ldf + i] = make_double2(c * cos(ph), c * sin(ph));
}

void launch_planewave(const double* px, const double* py, const double* q, const double* angles, double kappa,
                      double coef, double2* f, long long ldf, long long N, int nrhs, hipStream_t s) {
  dim3 grid((unsigned)((N + 255) / 256), nrhs);
  k_planewave<<<grid, 256, 0, s>>>(px, py, q, angles, kappa, coef, f, ldf, N);
}

// =====================================================================================
// Tall-skinny products  partial[(rhs*nchunks + ch)*ldp + c] = sum_{i in chunk ch} op(A_c[i]) x[i]
// with A_c = A + c*lda + rhs*lda_rhs (column c of a column-major block), op = identity or
// complex conjugate, for c < ncols.  A workgroup is 4 waves; each wave owns 16 columns and
// walks the chunk's rows with its 64 lanes (coalesced), accumulating in registers; waves of
// one column group split the rows when there are fewer than 4 groups.  One wave reduction
// per column at the end.
// =====================================================================================
// R consecutive complex entries in one 16-byte load (R = 4 bfloat16, 2 complex64, 1 complex128)
template <typename T, int R>
struct alignas(16) Pack {
  typename V2<T>::type v[R];
};

template <typename T, bool CONJ, int R = 1>
__global__ __launch_bounds__(256) void k_tsdot(const typename V2<T>::type* __restrict__ A, long long lda,
                                               long long lda_rhs, int ncols, const double2* __restrict__ x,
                                               long long ldx, double2* __restrict__ partial, int ldp, long long chunk,
                                               int nchunks, int wpg, long long nrows, const int* __restrict__ jdev,
                                               const int* __restrict__ skip) {
  constexpr int G = 16;
  __shared__ double lds[4][2 * G];
  const int ch = blockIdx.x, rhs = blockIdx.z;
  if (skip && skip[rhs] != 0) return;  // uniform per block
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int gpb = 4 / wpg;  // column groups per block (the launch's layout)
  if (jdev) {
    // a column count known only on the device (the launch is laid out for the most columns):
    // the waves of a block split among the groups that hold columns, the rest take row parts
    ncols = *jdev + 1;
    const int active = min(gpb, (ncols + G - 1) / G - (int)blockIdx.y * gpb);
    if (active <= 0) return;  // uniform per block
    wpg = active > 2 ? 1 : (active == 2 ? 2 : 4);
  }
  const int grp = blockIdx.y * gpb + w / wpg;        // this wave's column group
  const int rp = w % wpg;                            // this wave's row part
  const int c0 = grp * G;
  const long long i0 = (long long)ch * chunk;
  const long long i1 = i0 + chunk < nrows ? i0 + chunk : nrows;
  const typename V2<T>::type* Ab = A + rhs * lda_rhs;
  const double2* xb = x + rhs * ldx;
  double acc[2 * G];
#pragma unroll
  for (int c = 0; c < 2 * G; ++c) acc[c] = 0;
  if (c0 < ncols) {
    // columns past ncols re-read the last column (unconditional loads keep all 16 in
    // flight); their sums are never stored
    long long coff[G];
#pragma unroll
    for (int c = 0; c < G; ++c) coff[c] = (long long)(c0 + c < ncols ? c0 + c : ncols - 1) * lda;
    // each lane takes R consecutive rows per step (chunks and column offsets are multiples of R)
    for (long long i = i0 + (long long)(rp * 64 + lane) * R; i < i1; i += 64LL * wpg * R) {
      double2 xv[R];
#pragma unroll
      for (int q = 0; q < R; ++q) xv[q] = xb[i + q];
      Pack<T, R> a[G];
#pragma unroll
      for (int c = 0; c < G; ++c) a[c] = *reinterpret_cast<const Pack<T, R>*>(Ab + coff[c] + i);
#pragma unroll
      for (int c = 0; c < G; ++c)
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const double2 av = to_d2(a[c].v[q]);
          const double ax = av.x, ay = CONJ ? -av.y : av.y;
          acc[2 * c] = fma(ax, xv[q].x, acc[2 * c]);
          acc[2 * c] = fma(-ay, xv[q].y, acc[2 * c]);
          acc[2 * c + 1] = fma(ax, xv[q].y, acc[2 * c + 1]);
          acc[2 * c + 1] = fma(ay, xv[q].x, acc[2 * c + 1]);
        }
      // schedule all of the step's loads before its FMAs (memory-level parallelism)
      __builtin_amdgcn_sched_group_barrier(0x0020, G + R, 0);
      __builtin_amdgcn_sched_group_barrier(0x0002, 8 * G * R, 0);
    }
  }
#pragma unroll
  for (int c = 0; c < 2 * G; ++c) acc[c] = wave_sum(acc[c]);
  if (wpg > 1) {
    if (lane == 0)
#pragma unroll
      for (int c = 0; c < 2 * G; ++c) lds[w][c] = acc[c];
    __syncthreads();
    if (rp != 0) return;
    for (int q = 1; q < wpg; ++q)
#pragma unroll
      for (int c = 0; c < 2 * G; ++c) acc[c] += lds[w + q][c];
  }
  if (c0 >= ncols) return;
  if (lane < G && c0 + lane < ncols) {
    double re = 0, im = 0;
#pragma unroll
    for (int c = 0; c < G; ++c)
      if (c == lane) {
        re = acc[2 * c];
        im = acc[2 * c + 1];
      }
    partial[((long long)rhs * nchunks + ch) * ldp + c0 + lane] = make_double2(re, im);
  }
}

// ncols columns, or (jdev != NULL) *jdev + 1 of at most ncols; rhs with skip[rhs] != 0 untouched.
// fmt: storage of A, 0 complex128, 1 complex64, 2 complex bfloat16.
template <typename T>
static void tsdot_t(bool conj, const void* A, long long lda, long long lda_rhs, int ncols, const double2* x,
                    long long ldx, double2* partial, int ldp, long long chunk, int nchunks, long long nrows, int nrhs,
                    hipStream_t s, const int* jdev, const int* skip) {
  const int groups = (ncols + 15) / 16;
  const int wpg = groups >= 4 ? 1 : (groups == 1 ? 4 : 2);
  const int gpb = 4 / wpg;
  dim3 grid(nchunks, (groups + gpb - 1) / gpb, nrhs);
  using S = typename V2<T>::type;
  const S* As = (const S*)A;
  if (conj) {
    auto kern = k_tsdot<T, true>;
    LSK_LAUNCH(kern, grid, 256, 0, s, As, lda, lda_rhs, ncols, x, ldx, partial, ldp, chunk, nchunks, wpg, nrows, jdev,
               skip);
  } else {
    auto kern = k_tsdot<T, false>;
    LSK_LAUNCH(kern, grid, 256, 0, s, As, lda, lda_rhs, ncols, x, ldx, partial, ldp, chunk, nchunks, wpg, nrows, jdev,
               skip);
  }
}

static void tsdot(int fmt, bool conj, const void* A, long long lda, long long lda_rhs, int ncols, const double2* x,
                  long long ldx, double2* partial, int ldp, long long chunk, int nchunks, long long nrows, int nrhs,
                  hipStream_t s, const int* jdev = nullptr, const int* skip = nullptr) {
  if (fmt == 2)
    tsdot_t<bf16>(conj, A, lda, lda_rhs, ncols, x, ldx, partial, ldp, chunk, nchunks, nrows, nrhs, s, jdev, skip);
  else if (fmt == 1)
    tsdot_t<float>(conj, A, lda, lda_rhs, ncols, x, ldx, partial, ldp, chunk, nchunks, nrows, nrhs, s, jdev, skip);
  else
    tsdot_t<double>(conj, A, lda, lda_rhs, ncols, x, ldx, partial, ldp, chunk, nchunks, nrows, nrhs, s, jdev, skip);
}

// =====================================================================================
// HODLR apply: leaf solves, then per binary level  z -= Y core^{-1} (W^T z).
// =====================================================================================
template <typename TD>
__global__ __launch_bounds__(64) void k_leaf_apply(const typename V2<TD>::type* __restrict__ Dinv,
                                                   const unsigned char* __restrict__ ident,
                                                   const double2* b, long long ldb, double2* z, long long ldz, int lp,
                                                   int nrf, const int* __restrict__ jdev, long long bldj) {
  __shared__ double2 bl[64];
  if (jdev) b += (long long)(*jdev) * bldj;  // b = column *jdev of a basis
  // nrf > 0: the right-hand sides are the fastest grid index, so the workgroups that use one
  // factor block run back to back and find it in L2
  const int leaf = nrf ? blockIdx.x / nrf : blockIdx.x, rhs = nrf ? blockIdx.x % nrf : blockIdx.y;
  const int t = threadIdx.x;
  const long long base = (long long)leaf * lp;
  if (t < lp) bl[t] = b[rhs * ldb + base + t];
  __syncthreads();
  if (t >= lp) return;
  if (ident[leaf]) {
    z[rhs * ldz + base + t] = bl[t];
    return;
  }
  const typename V2<TD>::type* D = Dinv + (long long)leaf * lp * lp;
  double re = 0, im = 0;
  for (int k = 0; k < lp; ++k) {
    const double2 a = to_d2(D[(long long)k * lp + t]);
    const double2 x = bl[k];
    re = fma(a.x, x.x, re);
    re = fma(-a.y, x.y, re);
    im = fma(a.x, x.y, im);
    im = fma(a.y, x.x, im);
  }
  z[rhs * ldz + base + t] = make_double2(re, im);
}

void launch_leaf_apply(int dfmt, const void* Dinv, const unsigned char* ident, const double2* b, long long ldb,
                       double2* z, long long ldz, int lp, int nleaves, int nrhs, hipStream_t s, const int* jdev,
                       long long bldj) {
  const int nrf = nrhs > 1 ? nrhs : 0;
  dim3 grid(nrf ? nleaves * nrhs : nleaves, nrf ? 1 : nrhs);
  if (dfmt == 2) {
    auto kern = k_leaf_apply<bf16>;
    LSK_LAUNCH(kern, grid, 64, 0, s, (const BF2*)Dinv, ident, b, ldb, z, ldz, lp, nrf, jdev, bldj);
  } else if (dfmt == 1) {
    auto kern = k_leaf_apply<float>;
    LSK_LAUNCH(kern, grid, 64, 0, s, (const float2*)Dinv, ident, b, ldb, z, ldz, lp, nrf, jdev, bldj);
  } else {
    auto kern = k_leaf_apply<double>;
    LSK_LAUNCH(kern, grid, 64, 0, s, (const double2*)Dinv, ident, b, ldb, z, ldz, lp, nrf, jdev, bldj);
  }
}

// W^T z for the HODLR levels: partial[(rhs*nchunks + ch)*r + c] = sum_{i in chunk ch} W[c*N + i] z[i].
// A segment of lc lanes (a power of two, 16 <= lc <= 64) owns one chunk and one group of G
// columns (few columns per lane keep many waves resident); each lane takes R consecutive rows
// per step (one 16-byte pack per column), the segment is summed by butterfly shuffles, and a
// wave holds 64 / lc chunks: no LDS, no idle waves for short chunks.
template <typename T, int R, int G>
__global__ __launch_bounds__(256) void k_hodlr_dot_seg(const typename V2<T>::type* __restrict__ W, long long N, int r,
                                                       const double2* __restrict__ z, long long ldz,
                                                       double2* __restrict__ partial, long long chunk, int nchunks,
                                                       int lc, int nrf, const int* __restrict__ clist, int nk,
                                                       int cpc) {
  // nrf > 0: right-hand sides fastest in grid.x (factor tiles reused from L2 across them)
  const int rhs = nrf ? blockIdx.x % nrf : blockIdx.z, grp = blockIdx.y;
  const long long bx = nrf ? blockIdx.x / nrf : blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int spw = 64 / lc;
  const int seg = lane / lc, sl = lane - seg * lc;
  // clist: the children whose chunks are formed (cpc chunks each, nk chunks in all); else every chunk
  const long long k = (bx * 4 + wave) * spw + seg;
  const bool valid = k < nk;
  const long long ch = clist && valid ? (long long)clist[k / cpc] * cpc + k % cpc : k;
  const int c0 = grp * G;
  const double2* zb = z + rhs * ldz;
  double acc[2 * G];
#pragma unroll
  for (int c = 0; c < 2 * G; ++c) acc[c] = 0;
  if (valid) {
    long long coff[G];
#pragma unroll
    for (int c = 0; c < G; ++c) coff[c] = (long long)(c0 + c < r ? c0 + c : r - 1) * N;
    const long long i0 = ch * chunk, i1 = i0 + chunk;
    for (long long i = i0 + (long long)sl * R; i < i1; i += (long long)lc * R) {
      double2 xv[R];
#pragma unroll
      for (int q = 0; q < R; ++q) xv[q] = zb[i + q];
      Pack<T, R> a[G];
#pragma unroll
      for (int c = 0; c < G; ++c) a[c] = *reinterpret_cast<const Pack<T, R>*>(W + coff[c] + i);
#pragma unroll
      for (int c = 0; c < G; ++c)
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const double2 av = to_d2(a[c].v[q]);
          acc[2 * c] = fma(av.x, xv[q].x, acc[2 * c]);
          acc[2 * c] = fma(-av.y, xv[q].y, acc[2 * c]);
          acc[2 * c + 1] = fma(av.x, xv[q].y, acc[2 * c + 1]);
          acc[2 * c + 1] = fma(av.y, xv[q].x, acc[2 * c + 1]);
        }
      __builtin_amdgcn_sched_group_barrier(0x0020, G + R, 0);
      __builtin_amdgcn_sched_group_barrier(0x0002, 8 * G * R, 0);
    }
  }
  // butterfly inside the segment (offsets below lc keep to it); every lane takes part
  for (int off = lc >> 1; off > 0; off >>= 1)
#pragma unroll
    for (int c = 0; c < 2 * G; ++c) acc[c] += __shfl_xor(acc[c], off, 64);
  if (!valid || sl >= G || c0 + sl >= r) return;
  double re = 0, im = 0;
#pragma unroll
  for (int c = 0; c < G; ++c)
    if (c == sl) {
      re = acc[2 * c];
      im = acc[2 * c + 1];
    }
  partial[((long long)rhs * nchunks + ch) * r + c0 + sl] = make_double2(re, im);
}

// Many right-hand sides with complex128 factors: a segment owns one chunk, G columns and RB
// right-hand sides, so each factor entry is read once per RB right-hand sides and each z entry
// once per G columns.  Per (column, right-hand side) the lane and row order and the butterfly
// are those of k_hodlr_dot_seg<double, 1, G>: the same sums, bit for bit.
template <int G, int RB>
__global__ __launch_bounds__(256) void k_hodlr_dot_rb(const double2* __restrict__ W, long long N, int r,
                                                      const double2* __restrict__ z, long long ldz,
                                                      double2* __restrict__ partial, long long chunk, int nchunks,
                                                      int lc, int nrhs, int ngrp) {
  const int grp = blockIdx.x % ngrp, rb0 = (blockIdx.x / ngrp) * RB;
  const long long bx = blockIdx.y;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int spw = 64 / lc;
  const int seg = lane / lc, sl = lane - seg * lc;
  const long long ch = (bx * 4 + wave) * spw + seg;
  const bool valid = ch < nchunks;
  const int c0 = grp * G;
  const int nb = nrhs - rb0 < RB ? nrhs - rb0 : RB;
  double acc[G][RB][2];
#pragma unroll
  for (int c = 0; c < G; ++c)
#pragma unroll
    for (int b = 0; b < RB; ++b) acc[c][b][0] = acc[c][b][1] = 0;
  if (valid) {
    long long coff[G], zoff[RB];
#pragma unroll
    for (int c = 0; c < G; ++c) coff[c] = (long long)(c0 + c < r ? c0 + c : r - 1) * N;
#pragma unroll
    for (int b = 0; b < RB; ++b) zoff[b] = (long long)(rb0 + (b < nb ? b : nb - 1)) * ldz;
    const long long i0 = ch * chunk, i1 = i0 + chunk;
    for (long long i = i0 + sl; i < i1; i += lc) {
      double2 a[G], x[RB];
#pragma unroll
      for (int c = 0; c < G; ++c) a[c] = W[coff[c] + i];
#pragma unroll
      for (int b = 0; b < RB; ++b) x[b] = z[zoff[b] + i];
#pragma unroll
      for (int c = 0; c < G; ++c)
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          acc[c][b][0] = fma(a[c].x, x[b].x, acc[c][b][0]);
          acc[c][b][0] = fma(-a[c].y, x[b].y, acc[c][b][0]);
          acc[c][b][1] = fma(a[c].x, x[b].y, acc[c][b][1]);
          acc[c][b][1] = fma(a[c].y, x[b].x, acc[c][b][1]);
        }
    }
  }
  for (int off = lc >> 1; off > 0; off >>= 1)
#pragma unroll
    for (int c = 0; c < G; ++c)
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        acc[c][b][0] += __shfl_xor(acc[c][b][0], off, 64);
        acc[c][b][1] += __shfl_xor(acc[c][b][1], off, 64);
      }
  if (!valid) return;
  // output k = c * RB + b goes out from lane k mod lc of the segment
#pragma unroll
  for (int c = 0; c < G; ++c)
#pragma unroll
    for (int b = 0; b < RB; ++b)
      if ((c * RB + b) % lc == sl && c0 + c < r && b < nb)
        partial[((long long)(rb0 + b) * nchunks + ch) * r + c0 + c] = make_double2(acc[c][b][0], acc[c][b][1]);
}

constexpr int kDotCols = 8;  // columns per segment
template <typename T, int R>
static void hodlr_dot_seg(const void* W, const double2* z, long long ldz, double2* partial, long long N, int r,
                          long long chunk, int nchunks, int nrhs, hipStream_t s, const int* clist, int nlist, int cpc) {
  int lc = 64;
  while (lc > chunk / R) lc >>= 1;
  constexpr int G = kDotCols;
  const int per_wg = 4 * (64 / lc);
  const int nk = clist ? nlist * cpc : nchunks;
  const unsigned nbx = (unsigned)((nk + per_wg - 1) / per_wg);
  const int nrf = nrhs > 1 ? nrhs : 0;
  dim3 grid(nrf ? nbx * nrhs : nbx, (r + G - 1) / G, nrf ? 1 : nrhs);
  using S = typename V2<T>::type;
  const S* Ws = (const S*)W;
  auto kern = k_hodlr_dot_seg<T, R, G>;
  LSK_LAUNCH(kern, grid, 256, 0, s, Ws, N, r, z, ldz, partial, chunk, nchunks, lc, nrf, clist, nk, cpc);
}

// 16-byte packs when the chunk and N allow them (chunk a multiple of R holding at least 16
// packs), single entries otherwise
template <typename T>
static void hodlr_dot_fmt(const void* W, const double2* z, long long ldz, double2* partial, long long N, int r,
                          long long chunk, int nchunks, int nrhs, hipStream_t s, const int* clist, int nlist, int cpc) {
  constexpr int RW = 16 / (int)sizeof(typename V2<T>::type);
  if (RW == 1 && nrhs >= 8) {  // complex128 factors, many right-hand sides
    constexpr int G = 4, RB = 8;
    int lc = 64;
    while (lc > chunk) lc >>= 1;
    const int per_wg = 4 * (64 / lc);
    const int ngrp = (r + G - 1) / G;
    dim3 grid((unsigned)(ngrp * ((nrhs + RB - 1) / RB)), (unsigned)((nchunks + per_wg - 1) / per_wg));
    auto kern = k_hodlr_dot_rb<G, RB>;
    LSK_LAUNCH(kern, grid, 256, 0, s, (const double2*)W, N, r, z, ldz, partial, chunk, nchunks, lc, nrhs, ngrp);
    return;
  }
  if (RW > 1 && chunk % RW == 0 && N % RW == 0 && chunk / RW >= 16)
    hodlr_dot_seg<T, RW>(W, z, ldz, partial, N, r, chunk, nchunks, nrhs, s, clist, nlist, cpc);
  else
    hodlr_dot_seg<T, 1>(W, z, ldz, partial, N, r, chunk, nchunks, nrhs, s, clist, nlist, cpc);
}

void launch_hodlr_dot(int fmt, const void* W, const double2* z, long long ldz, double2* partial, long long N, int r,
                      long long chunk, int nchunks, int nrhs, hipStream_t s, const int* clist, int nlist, int cpc) {
  if (clist && (cpc <= 0 || nchunks % cpc != 0 || nlist < 0 || (long long)nlist * cpc > nchunks))
    throw std::runtime_error("hodlr dot: the child list needs whole children of cpc chunks");
  if (chunk < 16) {  // tiny leaves: plain tall-skinny reduction
    tsdot(fmt, false, W, N, 0, r, z, ldz, partial, r, chunk, nchunks, N, nrhs, s);
    return;
  }
  if (clist && nlist == 0) return;  // no chunk is needed on this level
  if (fmt == 2)
    hodlr_dot_fmt<bf16>(W, z, ldz, partial, N, r, chunk, nchunks, nrhs, s, clist, nlist, cpc);
  else if (fmt == 1)
    hodlr_dot_fmt<float>(W, z, ldz, partial, N, r, chunk, nchunks, nrhs, s, clist, nlist, cpc);
  else
    hodlr_dot_fmt<double>(W, z, ldz, partial, N, r, chunk, nchunks, nrhs, s, clist, nlist, cpc);
}

// t = [t_A; t_B]: t_A from the chunks of the second child (rows paired with Q), t_B from
// the first child (rows paired with S), written out as it is (the setup forms the cores from
// it; the apply form is k_hodlr_core_rows).  256 threads per node (2r <= 256): nks = 256 / 2r
// threads per entry take every nks-th chunk, then a fixed-order sum in LDS.
__global__ __launch_bounds__(256) void k_hodlr_core(const double2* __restrict__ partial, double2* __restrict__ sout,
                                                    int r, int nodes, int cpc, int nchunks) {
  __shared__ double2 t[256];
  __shared__ double2 tp[256];
  const int node = blockIdx.x, rhs = blockIdx.y;
  const int r2 = 2 * r;
  if (r2 > 256) {  // one thread per value and chunk order, several values per thread
    for (int v = threadIdx.x; v < r2; v += 256) {
      const int half = v < r ? 1 : 0;
      const int c = v < r ? v : v - r;
      const long long ch0 = (long long)node * 2 * cpc + (long long)half * cpc;
      double re = 0, im = 0;
      for (int k = 0; k < cpc; ++k) {
        const double2 p = partial[((long long)rhs * nchunks + ch0 + k) * r + c];
        re += p.x;
        im += p.y;
      }
      sout[((long long)rhs * nodes + node) * r2 + v] = make_double2(re, im);
    }
    return;
  }
  const int nks = 256 / r2;
  if ((int)threadIdx.x < r2 * nks) {
    const int v = threadIdx.x % r2, ks = threadIdx.x / r2;
    const int half = v < r ? 1 : 0;  // t_A sums the second child
    const int c = v < r ? v : v - r;
    const long long ch0 = (long long)node * 2 * cpc + (long long)half * cpc;
    double re = 0, im = 0;
    for (int k = ks; k < cpc; k += nks) {
      const double2 p = partial[((long long)rhs * nchunks + ch0 + k) * r + c];
      re += p.x;
      im += p.y;
    }
    tp[ks * r2 + v] = make_double2(re, im);
  }
  __syncthreads();
  if ((int)threadIdx.x < r2) {
    double re = 0, im = 0;
    for (int ks = 0; ks < nks; ++ks) {
      re += tp[ks * r2 + threadIdx.x].x;
      im += tp[ks * r2 + threadIdx.x].y;
    }
    t[threadIdx.x] = make_double2(re, im);
  }
  __syncthreads();
  double2* so = sout + ((long long)rhs * nodes + node) * r2;
  const int i = threadIdx.x;
  if (i >= r2) return;
  so[i] = t[i];
}

// Apply form split by rows.  The core inverses are stored in 16-row blocks: block b of a node
// holds rows 16b .. 16b+15 of every column, column after column (rows past 2r are zero), so a
// block is one contiguous run of 16 * 2r entries.  Workgroup (node, block) sums t from the
// chunk partials (every block of a node recomputes the same 2r sums, in the same order), then
// its NT threads form 16 rows of s = K^-1 t: thread (li, jp) takes row li over the columns
// jp, jp + NT/16, ..., so the lanes of a wave read one contiguous kilobyte per load and a
// thread issues all its loads before using them; the NT/16 partial sums of a row are added
// through LDS in a fixed order.  NT = 1024 for levels with many chunk partials per node.
template <typename TC, int NT, int R2MAX = 256, int RB = 1>
__global__ __launch_bounds__(NT) void k_hodlr_core_rows(const double2* __restrict__ partial,
                                                        const typename V2<TC>::type* __restrict__ coreinv,
                                                        double2* __restrict__ sout, int r, int nodes, int cpc,
                                                        int nchunks, int nrf, const unsigned char* __restrict__ cact,
                                                        int cstr) {
  constexpr int CG = NT / 16;
  constexpr int MAXU = R2MAX / CG;  // columns per thread at 2r = R2MAX
  using VT = typename V2<TC>::type;
  __shared__ double2 t[RB][R2MAX];
  __shared__ double2 tp[NT];
  __shared__ double2 part[CG][16];
  // nrf > 0: nrf right-hand sides in blocks of RB (each block of K^-1 is read once per RB of
  // them), the right-hand-side block fastest in grid.x; nrf = 0: the right-hand side is grid.z
  const int nrb = nrf ? (nrf + RB - 1) / RB : 1;
  const int node = nrf ? blockIdx.x / nrb : blockIdx.x, blk = blockIdx.y;
  const int rhs0 = nrf ? (blockIdx.x % nrb) * RB : blockIdx.z;
  const int nbr = nrf ? (nrf - rhs0 < RB ? nrf - rhs0 : RB) : 1;
  const int r2 = 2 * r;
  const int li = threadIdx.x & 15, jp = threadIdx.x >> 4;
  const int i = blk * 16 + li;
  // children with contrast (bit 0 first child, bit 1 second); the same for the whole workgroup
  const int m = cact ? (cact[2 * node] ? 1 : 0) | (cact[2 * node + 1] ? 2 : 0) : 3;
  // both Y zero, or this block's 16 rows all in the half of s that a child without contrast uses
  if (m == 0 || (m != 3 && (blk * 16 + 16 <= r ? !(m & 1) : (blk * 16 >= r && !(m & 2))))) {
    if (jp == 0 && i < r2)
      for (int b = 0; b < nbr; ++b) sout[((long long)(rhs0 + b) * nodes + node) * r2 + i] = make_double2(0.0, 0.0);
    return;
  }
  // the block of K^-1 does not depend on t: its loads go out first and overlap the sums of t
  const long long nb = (r2 + 15) / 16;
  const VT* Cb = coreinv + ((long long)node * nb + blk) * 16 * r2;  // (16 blk + li, j) at j * 16 + li
  VT a[MAXU];
  if (m == 3) {
#pragma unroll
    for (int u = 0; u < MAXU; ++u) {
      const int j = jp + u * CG;
      if (j < r2) a[u] = Cb[j * 16 + li];
    }
  }
  // t from the chunk partials: nks threads per value take every nks-th chunk, then a fixed-order sum
  const int nks = NT / r2;
  for (int b = 0; b < nbr; ++b) {
    const long long rhs = rhs0 + b;
    if ((int)threadIdx.x < r2 * nks) {
      const int v = threadIdx.x % r2, ks = threadIdx.x / r2;
      const int half = v < r ? 1 : 0;  // t_A sums the second child
      const int c = v < r ? v : v - r;
      const long long ch0 = (long long)node * 2 * cstr + (long long)half * cstr;  // cstr: chunks per child in the layout
      // a one-sided node uses only the half of t that its child with contrast multiplies; the
      // chunk partials of the other half were not formed by the masked W^T z (stale) and are not read
      const int kend = (m == 3 || (m & (v < r ? 1 : 2))) ? cpc : 0;
      double re = 0, im = 0;
#pragma unroll(NT == 1024 ? 16 : 4)
      for (int k = ks; k < kend; k += nks) {
        const double2 p = partial[(rhs * nchunks + ch0 + k) * r + c];
        re += p.x;
        im += p.y;
      }
      tp[ks * r2 + v] = make_double2(re, im);
    }
    __syncthreads();
    if ((int)threadIdx.x < r2) {
      double re = 0, im = 0;
      for (int ks = 0; ks < nks; ++ks) {
        re += tp[ks * r2 + threadIdx.x].x;
        im += tp[ks * r2 + threadIdx.x].y;
      }
      t[b][threadIdx.x] = make_double2(re, im);
    }
    __syncthreads();
  }
  if (m != 3) {  // one child with contrast: K^-1 is the identity on the half that child uses
    if (jp == 0 && i < r2)
      for (int b = 0; b < nbr; ++b)
        sout[((long long)(rhs0 + b) * nodes + node) * r2 + i] =
            (m & (i < r ? 1 : 2)) ? t[b][i] : make_double2(0.0, 0.0);
    return;
  }
  for (int b = 0; b < nbr; ++b) {
    double re = 0, im = 0;
#pragma unroll
    for (int u = 0; u < MAXU; ++u) {
      const int j = jp + u * CG;
      if (j < r2) {
        const double2 av = to_d2(a[u]);
        const double2 x = t[b][j];
        re = fma(av.x, x.x, re);
        re = fma(-av.y, x.y, re);
        im = fma(av.x, x.y, im);
        im = fma(av.y, x.x, im);
      }
    }
    part[jp][li] = make_double2(re, im);
    __syncthreads();
    if (jp == 0 && i < r2) {
      for (int q = 1; q < CG; ++q) {
        re += part[q][li].x;
        im += part[q][li].y;
      }
      sout[((long long)(rhs0 + b) * nodes + node) * r2 + i] = make_double2(re, im);
    }
    __syncthreads();
  }
}

// One right-hand side: the cpc chunk partials of W^T z over one child, summed into the child's first
// partial.  Workgroup (2 node + half, 64-column block); thread (c, ks) adds the chunks ks, ks + 16, ...
// and the 16 slices are added in slice order.  Halves that the core does not read (the child without
// contrast of a one-sided node, both of a node without contrast) are skipped.
__global__ __launch_bounds__(1024) void k_hodlr_tsum_inplace(double2* __restrict__ partial, int r, int cpc,
                                                             const unsigned char* __restrict__ cact) {
  __shared__ double2 sl[16][64];
  const int nh = blockIdx.x, node = nh >> 1, half = nh & 1;
  const int ci = threadIdx.x & 63, ks = threadIdx.x >> 6;
  const int c = blockIdx.y * 64 + ci;
  // the partials of half 1 (the second child's rows) make t_A, which the core reads when the first
  // child has contrast; those of half 0 make t_B, read when the second child has contrast
  const int m = cact ? (cact[2 * node] ? 1 : 0) | (cact[2 * node + 1] ? 2 : 0) : 3;
  if (!(m & (half ? 1 : 2))) return;
  double2* P = partial + ((long long)node * 2 * cpc + (long long)half * cpc) * r;
  double re = 0, im = 0;
  if (c < r)
#pragma unroll 4
    for (int k = ks; k < cpc; k += 16) {
      const double2 v = P[(long long)k * r + c];
      re += v.x;
      im += v.y;
    }
  sl[ks][ci] = make_double2(re, im);
  __syncthreads();
  if (ks == 0 && c < r) {
    for (int q = 1; q < 16; ++q) {
      re += sl[q][ci].x;
      im += sl[q][ci].y;
    }
    P[c] = make_double2(re, im);
  }
}

long long hodlr_core_elems(int r) { return (long long)((2 * r + 15) / 16) * 16 * (2 * r); }

template <typename TC, int RB>
static void core_rows_shape(const void* coreinv, const double2* partial, double2* sout, int r, int nodes, int cpc,
                            int nchunks, int nrhs, hipStream_t s, const unsigned char* cact, int cstr) {
  const int nrf = nrhs > 1 ? nrhs : 0;
  const int nrb = (nrhs + RB - 1) / RB;
  dim3 grid(nrf ? nodes * nrb : nodes, (2 * r + 15) / 16, nrf ? 1 : nrhs);
  const auto* C = (const typename V2<TC>::type*)coreinv;
  // ranks above 128 (up to 512 columns): 1024 threads where many chunk partials make up t, else 512
  if (2 * r > 256) {
    if (cpc >= 16) {
      auto kern = k_hodlr_core_rows<TC, 1024, 512, RB>;
      LSK_LAUNCH(kern, grid, 1024, 0, s, partial, C, sout, r, nodes, cpc, nchunks, nrf, cact, cstr);
    } else {
      auto kern = k_hodlr_core_rows<TC, 512, 512, RB>;
      LSK_LAUNCH(kern, grid, 512, 0, s, partial, C, sout, r, nodes, cpc, nchunks, nrf, cact, cstr);
    }
    return;
  }
  // many partials per node (the coarse levels): 1024 threads share the sums of t
  if (cpc >= 16) {
    auto kern = k_hodlr_core_rows<TC, 1024, 256, RB>;
    LSK_LAUNCH(kern, grid, 1024, 0, s, partial, C, sout, r, nodes, cpc, nchunks, nrf, cact, cstr);
  } else {
    auto kern = k_hodlr_core_rows<TC, 256, 256, RB>;
    LSK_LAUNCH(kern, grid, 256, 0, s, partial, C, sout, r, nodes, cpc, nchunks, nrf, cact, cstr);
  }
}

template <typename TC>
static void core_rows_pick(const void* coreinv, double2* partial, double2* sout, int r, int nodes, int cpc,
                           int nchunks, int nrhs, hipStream_t s, const unsigned char* cact) {
  // many right-hand sides: 8 per workgroup share each block of K^-1 (same sums per column)
  if (nrhs >= 8) {
    core_rows_shape<TC, 8>(coreinv, partial, sout, r, nodes, cpc, nchunks, nrhs, s, cact, cpc);
    return;
  }
  // one right-hand side and many chunk partials per child (the coarse levels): every row block of
  // a node would sum all of them again, so one launch first folds them into the first partial of
  // each child, and the core reads that one
  if (nrhs == 1 && cpc >= 16) {
    const dim3 grid((unsigned)(nodes * 2), (unsigned)((r + 63) / 64));
    LSK_LAUNCH(k_hodlr_tsum_inplace, grid, 1024, 0, s, partial, r, cpc, cact);
    core_rows_shape<TC, 1>(coreinv, partial, sout, r, nodes, 1, nchunks, nrhs, s, cact, cpc);
    return;
  }
  core_rows_shape<TC, 1>(coreinv, partial, sout, r, nodes, cpc, nchunks, nrhs, s, cact, cpc);
}

void launch_hodlr_core(int cfmt, const void* coreinv, const double2* partial, double2* sout, int r, int nodes,
                       int chunks_per_child, int nchunks, bool apply, int nrhs, hipStream_t s,
                       const unsigned char* cact) {
  if (2 * r > 512) throw std::runtime_error("HODLR cores need rank <= 256");
  if (apply) {
    // the partials are consumed here: with one right-hand side and 16 or more chunks per child they
    // are folded in place (every caller owns them as writable scratch)
    double2* pw = const_cast<double2*>(partial);
    if (cfmt == 2)
      core_rows_pick<bf16>(coreinv, pw, sout, r, nodes, chunks_per_child, nchunks, nrhs, s, cact);
    else if (cfmt == 1)
      core_rows_pick<float>(coreinv, pw, sout, r, nodes, chunks_per_child, nchunks, nrhs, s, cact);
    else
      core_rows_pick<double>(coreinv, pw, sout, r, nodes, chunks_per_child, nchunks, nrhs, s, cact);
    return;
  }
  dim3 grid(nodes, nrhs);
  k_hodlr_core<<<grid, 256, 0, s>>>(partial, sout, r, nodes, chunks_per_child, nchunks);
}

// z[i] -= sum_c Y[c*N + i] * s[node][half*r + c]
template <typename T>
__global__ __launch_bounds__(256) void k_hodlr_update(const typename V2<T>::type* __restrict__ Y,
                                                      const double2* __restrict__ sv, double2* __restrict__ z,
                                                      long long ldz, long long N, int r, long long nodesize,
                                                      int nodes) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (i >= N) return;
  const long long node = i / nodesize;
  const int half = (i - node * nodesize) >= (nodesize >> 1) ? 1 : 0;
  const double2* s = sv + ((long long)rhs * nodes + node) * 2 * r + half * r;
  double re = 0, im = 0;
  for (int c0 = 0; c0 < r; c0 += 8) {
    // unconditional loads (clamped column, zero weight past r) keep 8 loads in flight
    typename V2<T>::type y[8];
    double2 x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int cc = c0 + c < r ? c0 + c : r - 1;
      y[c] = Y[(long long)cc * N + i];
      x[c] = s[cc];
      if (c0 + c >= r) x[c] = make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const double2 yv = to_d2(y[c]);
      re = fma(yv.x, x[c].x, re);
      re = fma(-yv.y, x[c].y, re);
      im = fma(yv.x, x[c].y, im);
      im = fma(yv.y, x[c].x, im);
    }
    __builtin_amdgcn_sched_group_barrier(0x0020, 16, 0);
    __builtin_amdgcn_sched_group_barrier(0x0002, 40, 0);
  }
  double2 o = z[rhs * ldz + i];
  o.x -= re;
  o.y -= im;
  z[rhs * ldz + i] = o;
}

// Many right-hand sides with complex128 factors (the r-column applies that form the factors):
// a thread owns one row and RB right-hand sides, so each factor entry is read once per RB
// right-hand sides instead of once per right-hand side.  A wave's 64 rows lie in one node half
// (halves hold at least 64 rows), so the s entries a wave reads are the same for all its lanes:
// the wave stages them in LDS, 32 columns at a time, and reads them back as broadcasts.  Per
// (row, right-hand side) the sums run over c in the order of k_hodlr_update: same results.
template <int RB>
__global__ __launch_bounds__(256) void k_hodlr_update_rb(const double2* __restrict__ Y, const double2* __restrict__ sv,
                                                         double2* __restrict__ z, long long ldz, long long N, int r,
                                                         long long nodesize, int nodes, int nrhs) {
  constexpr int CC = 32;  // columns of s staged at a time
  __shared__ double2 sl[4][RB][CC];
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const int rhs0 = blockIdx.y * RB;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  long long i0 = (long long)blockIdx.x * 256 + wv * 64;
  if (i0 > N - 1) i0 = N - 1;  // a wave past the end still takes part in the barriers
  const long long node = i0 / nodesize;
  const int half = (i0 - node * nodesize) >= (nodesize >> 1) ? 1 : 0;
  const long long sstride = (long long)nodes * 2 * r;
  const double2* s = sv + node * 2 * r + half * r + (long long)rhs0 * sstride;
  const int nb = nrhs - rhs0 < RB ? nrhs - rhs0 : RB;
  const long long ic = i < N ? i : N - 1;
  double re[RB], im[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) re[b] = im[b] = 0;
  for (int c0 = 0; c0 < r; c0 += CC) {
    const int cw = r - c0 < CC ? r - c0 : CC;
    // each wave stages the s entries of its own node half (waves of one workgroup may differ)
    for (int e = lane; e < RB * CC; e += 64) {
      const int b = e / CC, c = e - b * CC;
      sl[wv][b][c] = (b < nb && c < cw) ? s[b * sstride + c0 + c] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int c = 0; c < cw; ++c) {
      const double2 y = Y[(long long)(c0 + c) * N + ic];
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        const double2 x = sl[wv][b][c];
        re[b] = fma(y.x, x.x, re[b]);
        re[b] = fma(-y.y, x.y, re[b]);
        im[b] = fma(y.x, x.y, im[b]);
        im[b] = fma(y.y, x.x, im[b]);
      }
    }
    __syncthreads();
  }
  if (i >= N) return;
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    if (b >= nb) break;
    double2* zp = z + (long long)(rhs0 + b) * ldz + i;
    double2 o = *zp;
    o.x -= re[b];
    o.y -= im[b];
    *zp = o;
  }
}

// 16-byte-pack form: a thread owns R consecutive rows (one node half, as halves are multiples
// of 64 rows)
template <typename T>
__global__ __launch_bounds__(256) void k_hodlr_update_wide(const typename V2<T>::type* __restrict__ Y,
                                                           const double2* __restrict__ sv, double2* __restrict__ z,
                                                           long long ldz, long long N, int r, long long nodesize,
                                                           int nodes, int nrf, double2* __restrict__ z2,
                                                           long long z2ldr, const int* __restrict__ jdev,
                                                           long long z2ldj, const unsigned char* __restrict__ ract) {
  constexpr int R = 16 / (int)sizeof(typename V2<T>::type);
  const long long bx = nrf ? blockIdx.x / nrf : blockIdx.x;
  const int rhs = nrf ? blockIdx.x % nrf : blockIdx.y;
  const long long i = (bx * blockDim.x + threadIdx.x) * R;
  if (i >= N) return;
  // a wave's 64 R rows lie in one 256-row block (N is a multiple of 128): rows without contrast
  // have zero rows of Y, so such a wave leaves z as it is and reads no Y
  const bool act = !ract || ract[__builtin_amdgcn_readfirstlane((int)(i >> 8))] != 0;
  const long long node = i / nodesize;
  const int half = (i - node * nodesize) >= (nodesize >> 1) ? 1 : 0;
  const double2* s = sv + ((long long)rhs * nodes + node) * 2 * r + half * r;
  double re[R], im[R];
#pragma unroll
  for (int q = 0; q < R; ++q) re[q] = im[q] = 0;
  for (int c0 = 0; act && c0 < r; c0 += 8) {
    Pack<T, R> y[8];
    double2 x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int cc = c0 + c < r ? c0 + c : r - 1;
      y[c] = *reinterpret_cast<const Pack<T, R>*>(Y + (long long)cc * N + i);
      x[c] = s[cc];
      if (c0 + c >= r) x[c] = make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const double2 yv = to_d2(y[c].v[q]);
        re[q] = fma(yv.x, x[c].x, re[q]);
        re[q] = fma(-yv.y, x[c].y, re[q]);
        im[q] = fma(yv.x, x[c].y, im[q]);
        im[q] = fma(yv.y, x[c].x, im[q]);
      }
    __builtin_amdgcn_sched_group_barrier(0x0020, 16, 0);
    __builtin_amdgcn_sched_group_barrier(0x0002, 32 * R, 0);
  }
  // z2 != NULL: the result also goes to column *jdev of a basis (the stored z~ of flexible GMRES)
  double2* zc = z2 ? z2 + rhs * z2ldr + (long long)(*jdev) * z2ldj : nullptr;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    double2 o = z[rhs * ldz + i + q];
    if (act) {
      o.x -= re[q];
      o.y -= im[q];
      z[rhs * ldz + i + q] = o;
    }
    if (zc) zc[i + q] = o;
  }
}

// Update of one level fused with the W^T z reduction of the next: workgroup bx owns rows
// [1024 bx, 1024 bx + 1024).  Its threads first apply z -= Y s of level "a" to 4 rows each (the
// arithmetic of k_hodlr_update_wide), keep the new rows in LDS and store them, then its waves
// form the partial sums of W^T z over the 1024 / chunk chunks of those rows for the 4-column
// groups of level "b" with the lane and row order of k_hodlr_dot_seg (64-lane segments; the
// library launches it for 1024-row chunks): the same sums, bit for bit, without a second launch
// or a second read of z.
template <int CH>
__global__ __launch_bounds__(256) void k_hodlr_upd_dot(const BF2* __restrict__ Y, int ra,
                                                       const double2* __restrict__ sv, long long nodesize, int nodes,
                                                       const BF2* __restrict__ W, int rb, double2* __restrict__ z,
                                                       long long N, double2* __restrict__ partial,
                                                       const unsigned char* __restrict__ ract) {
  constexpr int chunk = CH, NS = CH / 256;  // rows per chunk, steps per lane
  constexpr int R = 4, G = 4;
  __shared__ double2 zs[1024];
  const long long bx = blockIdx.x;
  const int t = threadIdx.x;
  {
    const long long i = bx * 1024 + (long long)t * R;
    // a wave's 256 rows: rows without contrast have zero rows of Y, so a wave whose rows all
    // lack contrast leaves z as it is and reads no Y
    const bool act = !ract || ract[__builtin_amdgcn_readfirstlane((int)(i >> 8))] != 0;
    const long long node = i / nodesize;
    const int half = (i - node * nodesize) >= (nodesize >> 1) ? 1 : 0;
    const double2* s = sv + node * 2 * ra + half * ra;
    double re[R], im[R];
#pragma unroll
    for (int q = 0; q < R; ++q) re[q] = im[q] = 0;
    for (int c0 = 0; act && c0 < ra; c0 += 8) {
      Pack<bf16, R> y[8];
      double2 x[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int cc = c0 + c < ra ? c0 + c : ra - 1;
        y[c] = *reinterpret_cast<const Pack<bf16, R>*>(Y + (long long)cc * N + i);
        x[c] = s[cc];
        if (c0 + c >= ra) x[c] = make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const double2 yv = to_d2(y[c].v[q]);
          re[q] = fma(yv.x, x[c].x, re[q]);
          re[q] = fma(-yv.y, x[c].y, re[q]);
          im[q] = fma(yv.x, x[c].y, im[q]);
          im[q] = fma(yv.y, x[c].x, im[q]);
        }
      __builtin_amdgcn_sched_group_barrier(0x0020, 16, 0);
      __builtin_amdgcn_sched_group_barrier(0x0002, 32 * R, 0);
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      double2 o = z[i + q];
      if (act) {
        o.x -= re[q];
        o.y -= im[q];
        z[i + q] = o;
      }
      zs[t * R + q] = o;
    }
  }
  __syncthreads();
  const int wave = t >> 6, sl = t & 63;
  const int ngrp = (rb + G - 1) / G;
  const int kc = 1024 / chunk;  // chunks of this workgroup
  for (int pr = wave; pr < ngrp * kc; pr += 4) {
    const int grp = pr % ngrp, kk = pr / ngrp;
    const int c0 = grp * G;
    double acc[2 * G];
#pragma unroll
    for (int c = 0; c < 2 * G; ++c) acc[c] = 0;
    long long coff[G];
#pragma unroll
    for (int c = 0; c < G; ++c) coff[c] = (long long)(c0 + c < rb ? c0 + c : rb - 1) * N;
    // every step's loads first (NS x G packs in flight), then the sums in the step order
    Pack<bf16, R> a[NS][G];
#pragma unroll
    for (int k = 0; k < NS; ++k)
#pragma unroll
      for (int c = 0; c < G; ++c)
        a[k][c] = *reinterpret_cast<const Pack<bf16, R>*>(W + coff[c] + bx * 1024 + kk * chunk + sl * R + k * 64 * R);
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const int li = kk * chunk + sl * R + k * 64 * R;
      double2 xv[R];
#pragma unroll
      for (int q = 0; q < R; ++q) xv[q] = zs[li + q];
#pragma unroll
      for (int c = 0; c < G; ++c)
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const double2 av = to_d2(a[k][c].v[q]);
          acc[2 * c] = fma(av.x, xv[q].x, acc[2 * c]);
          acc[2 * c] = fma(-av.y, xv[q].y, acc[2 * c]);
          acc[2 * c + 1] = fma(av.x, xv[q].y, acc[2 * c + 1]);
          acc[2 * c + 1] = fma(av.y, xv[q].x, acc[2 * c + 1]);
        }
    }
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
      for (int c = 0; c < 2 * G; ++c) acc[c] += __shfl_xor(acc[c], off, 64);
    if (sl < G && c0 + sl < rb) {
      double re = 0, im = 0;
#pragma unroll
      for (int c = 0; c < G; ++c)
        if (c == sl) {
          re = acc[2 * c];
          im = acc[2 * c + 1];
        }
      partial[(bx * kc + kk) * rb + c0 + sl] = make_double2(re, im);
    }
  }
}

// Fused only where the next level's chunks are 1024 rows: with shorter chunks the reduction phase
// of one workgroup per 1024 rows has too few independent items per wave, and the two separate
// launches (many workgroups each) are faster.
bool hodlr_upd_dot_ok(long long N, long long nodesize_a, long long chunk_b) {
  return N % 1024 == 0 && nodesize_a % 128 == 0 && chunk_b == 1024;
}

void launch_hodlr_upd_dot(const void* Y, int ra, const double2* sv, long long nodesize, int nodes, const void* W,
                          int rb, double2* z, long long N, double2* partial, long long chunk, hipStream_t s,
                          const unsigned char* ract) {
  const dim3 grid((unsigned)(N / 1024));
  const BF2 *Yb = (const BF2*)Y, *Wb = (const BF2*)W;
  if (chunk != 1024) throw std::runtime_error("fused HODLR update/dot needs chunks of 1024 rows");
  auto kern = k_hodlr_upd_dot<1024>;
  LSK_LAUNCH(kern, grid, 256, 0, s, Yb, ra, sv, nodesize, nodes, Wb, rb, z, N, partial, ract);
}

// One right-hand side, only the listed 256-row blocks (those with contrast; the other rows of Y
// are zero), one block per workgroup: its four waves take a quarter of the columns each over all
// 256 rows (R rows per lane, 16-byte loads), and the four partial sums of a row are added in
// wave order through LDS before z is updated.  All threads of the launch work on rows that
// change, and a wave's chain of loads is a quarter as long as in the row-per-thread kernels.
template <typename T>
__global__ __launch_bounds__(256) void k_hodlr_update_list(const typename V2<T>::type* __restrict__ Y,
                                                           const double2* __restrict__ sv, double2* __restrict__ z,
                                                           long long N, int r, long long nodesize,
                                                           const int* __restrict__ blist, int nact) {
  constexpr int R = 16 / (int)sizeof(typename V2<T>::type);
  constexpr int LR = 64 * R;  // rows of one pass of a wave
  __shared__ double2 part[4][256];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long long b0 = (long long)blist[blockIdx.x] * 256;
  const int cw = (r + 3) / 4, c_lo = w * cw, c_hi = c_lo + cw < r ? c_lo + cw : r;
  for (int pass = 0; pass < 256 / LR; ++pass) {
    const int lr = pass * LR + lane * R;  // row in the block
    long long i = b0 + lr;
    if (i > N - R) i = N - R;            // a clipped last block: in-bounds loads, rows not written
    const long long node = i / nodesize;
    const int half = (i - node * nodesize) >= (nodesize >> 1) ? 1 : 0;
    const double2* s = sv + node * 2 * r + half * r;
    double re[R], im[R];
#pragma unroll
    for (int q = 0; q < R; ++q) re[q] = im[q] = 0;
    for (int c0 = c_lo; c0 < c_hi; c0 += 8) {
      Pack<T, R> y[8];
      double2 x[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int cc = c0 + c < c_hi ? c0 + c : c_hi - 1;
        y[c] = *reinterpret_cast<const Pack<T, R>*>(Y + (long long)cc * N + i);
        x[c] = s[cc];
        if (c0 + c >= c_hi) x[c] = make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const double2 yv = to_d2(y[c].v[q]);
          re[q] = fma(yv.x, x[c].x, re[q]);
          re[q] = fma(-yv.y, x[c].y, re[q]);
          im[q] = fma(yv.x, x[c].y, im[q]);
          im[q] = fma(yv.y, x[c].x, im[q]);
        }
      __builtin_amdgcn_sched_group_barrier(0x0020, 16, 0);
      __builtin_amdgcn_sched_group_barrier(0x0002, 32 * R, 0);
    }
#pragma unroll
    for (int q = 0; q < R; ++q) part[w][lr + q] = make_double2(re[q], im[q]);
  }
  __syncthreads();
  const long long i = b0 + threadIdx.x;
  if (i >= N) return;
  const double2 p0 = part[0][threadIdx.x], p1 = part[1][threadIdx.x], p2 = part[2][threadIdx.x],
                p3 = part[3][threadIdx.x];
  double2 o = z[i];
  o.x -= ((p0.x + p1.x) + p2.x) + p3.x;
  o.y -= ((p0.y + p1.y) + p2.y) + p3.y;
  z[i] = o;
}

void launch_hodlr_update_list(int fmt, const void* Y, const double2* sv, double2* z, long long N, int r,
                              long long nodesize, const int* blist, int nact, hipStream_t s) {
  if (nact <= 0) return;
  if (N < 4) throw std::runtime_error("listed HODLR update needs N >= 4");
  if (N % 256 != 0 || nodesize % 8 != 0 || N % nodesize != 0)
    throw std::runtime_error("listed HODLR update needs N % 256 == 0 and node halves of a multiple of 4 rows");
  if (fmt == 2) {
    auto kern = k_hodlr_update_list<bf16>;
    LSK_LAUNCH(kern, dim3((unsigned)nact), 256, 0, s, (const BF2*)Y, sv, z, N, r, nodesize, blist, nact);
  } else if (fmt == 1) {
    auto kern = k_hodlr_update_list<float>;
    LSK_LAUNCH(kern, dim3((unsigned)nact), 256, 0, s, (const float2*)Y, sv, z, N, r, nodesize, blist, nact);
  } else {
    throw std::runtime_error("listed HODLR update needs complex64 or complex bfloat16 factors");
  }
}

// =====================================================================================
// The deep HODLR levels in one launch.  The leaf solves and the levels F..Lb-1 of the binary
// tree read and write only the rows of their level-F ancestor, so one workgroup per level-F
// node (SF rows, one thread per row) runs them in order with that node's rows of z in LDS:
// the leaf solves (a wave per 64-row leaf), then per level, deepest first, W^T z for both
// children of every node (4-row packs, butterfly sums over the lanes of one child), s = K^-1 t
// (one 16-row block of K^-1 per wave; the masked identity for a node with one child holding
// contrast, zero for none) and z -= Y s.  The same operations as launch_leaf_apply and the
// per-level dot, core and update launches, with every sum in FP64 (in another order).
// =====================================================================================
template <typename T, int SF>
__global__ __launch_bounds__(SF) void k_hodlr_subtree(const double2* __restrict__ Dinv,
                                                      const unsigned char* __restrict__ ident, const double2* b,
                                                      const int* __restrict__ jdev, long long bldj, double2* z,
                                                      long long N, int Lb, int F, SubtreeLevels lv,
                                                      const unsigned char* __restrict__ nodeact) {
  using VT = typename V2<T>::type;
  constexpr int NP = SF / 4;  // 4-row packs; SF / NP = 4 column groups
  constexpr int PB = 32 / (int)sizeof(VT);  // 4-row packs per batch of loads: 8 bf16, 4 complex64, 2 complex128
  constexpr int kTv = 512;    // entries of t (and s) of one level: nodes x 2r <= (SF / 128) x 128
  __shared__ double2 zl[SF];
  __shared__ double2 tv[kTv];
  __shared__ double2 sv[kTv];
  __shared__ double2 part[4][SF];
  __shared__ int mk[SF / 128];
  const int g = blockIdx.x, t = threadIdx.x;
  const long long R0 = (long long)g * SF;
  const double2* bb = jdev ? b + (long long)(*jdev) * bldj : b;
  const double2 bv = bb[R0 + t];
  if (nodeact && !nodeact[(1LL << F) + g]) {  // no contrast below this node: every step is the identity
    z[R0 + t] = bv;
    return;
  }
  zl[t] = bv;
  __syncthreads();
  {
    const long long leaf = (R0 >> 6) + (t >> 6);
    double2 o = bv;
    if (!ident[leaf]) {
      const double2* D = Dinv + leaf * 4096;
      const int row = t & 63, base = t & ~63;
      double re = 0, im = 0;
#pragma unroll 16
      for (int k = 0; k < 64; ++k) {
        const double2 a = D[k * 64 + row];
        const double2 x = zl[base + k];
        re = fma(a.x, x.x, re);
        re = fma(-a.y, x.y, re);
        im = fma(a.x, x.y, im);
        im = fma(a.y, x.x, im);
      }
      o = make_double2(re, im);
    }
    __syncthreads();
    zl[t] = o;
  }
  const int wave = t >> 6, lane = t & 63;
  for (int l = Lb - 1; l >= F; --l) {
    const int li = l - F;
    const int r = lv.r[li];
    if (r == 0) continue;
    const int nn = 1 << li;     // nodes of level l below this workgroup's node
    const int Sl = SF >> li;    // rows per node
    const int h = Sl >> 1;      // rows per child
    const int r2 = 2 * r;
    const long long J0 = (long long)g * nn;
    if (t < nn) {
      const unsigned char* c = nodeact ? nodeact + (2LL << l) + 2 * (J0 + t) : nullptr;
      mk[t] = c ? (c[0] ? 1 : 0) | (c[1] ? 2 : 0) : 3;
    }
    __syncthreads();
    const VT* W = (const VT*)lv.W[li];
    const VT* Y = (const VT*)lv.Y[li];
    const int p = t % NP, cg = t / NP;  // column group: uniform per wave
    const int row = 4 * p, j = row / Sl, half = (row % Sl) >= h ? 1 : 0;
    // t_A (entries 0..r-1) sums W^T z over the second child and feeds the first child's update,
    // t_B (r..2r-1) the first child's rows for the second.  Loads go out in batches of PB packs
    // (64 registers) before their first use; columns cg, cg + 4, ... < r <= 64
    {
      const bool need = (mk[j] & (half ? 1 : 2)) != 0;
      const int seg = h >> 2;  // lanes of one child: 16, 32 or 64
      const double2 x0 = zl[row], x1 = zl[row + 1], x2 = zl[row + 2], x3 = zl[row + 3];
#pragma unroll 1
      for (int u0 = 0; u0 < 16 && cg + 4 * u0 < r; u0 += PB) {
        Pack<T, 4> wa[PB];
#pragma unroll
        for (int u = 0; u < PB; ++u) {
          const int c = cg + 4 * (u0 + u);
          if (need && c < r) wa[u] = *reinterpret_cast<const Pack<T, 4>*>(W + (long long)c * N + R0 + row);
        }
#pragma unroll
        for (int u = 0; u < PB; ++u) {
          const int c = cg + 4 * (u0 + u);
          if (c < r) {  // uniform per wave
            double re = 0, im = 0;
            if (need) {
              const double2 a0 = to_d2(wa[u].v[0]), a1 = to_d2(wa[u].v[1]), a2 = to_d2(wa[u].v[2]),
                            a3 = to_d2(wa[u].v[3]);
              re = fma(a0.x, x0.x, re);
              re = fma(-a0.y, x0.y, re);
              im = fma(a0.x, x0.y, im);
              im = fma(a0.y, x0.x, im);
              re = fma(a1.x, x1.x, re);
              re = fma(-a1.y, x1.y, re);
              im = fma(a1.x, x1.y, im);
              im = fma(a1.y, x1.x, im);
              re = fma(a2.x, x2.x, re);
              re = fma(-a2.y, x2.y, re);
              im = fma(a2.x, x2.y, im);
              im = fma(a2.y, x2.x, im);
              re = fma(a3.x, x3.x, re);
              re = fma(-a3.y, x3.y, re);
              im = fma(a3.x, x3.y, im);
              im = fma(a3.y, x3.x, im);
            }
            for (int off = seg >> 1; off > 0; off >>= 1) {
              re += __shfl_xor(re, off, 64);
              im += __shfl_xor(im, off, 64);
            }
            if (need && (p & (seg - 1)) == 0) tv[j * r2 + (half ? c : r + c)] = make_double2(re, im);
          }
        }
      }
    }
    __syncthreads();
    // s = K^-1 t where both children hold contrast; else the half of t the child with contrast
    // uses, zeros elsewhere (no K^-1 read)
    for (int e = t; e < nn * r2; e += SF) {
      const int jj = e / r2, i = e - jj * r2;
      if (mk[jj] != 3) sv[e] = (mk[jj] & (i < r ? 1 : 2)) ? tv[e] : make_double2(0.0, 0.0);
    }
    {
      const int nb = (r2 + 15) / 16;
      const int l16 = lane & 15, jq = lane >> 4;
      for (int pr = wave; pr < nn * nb; pr += SF / 64) {
        const int jj = pr / nb, blk = pr - jj * nb;
        if (mk[jj] != 3) continue;
        const double2* Cb = lv.K[li] + ((J0 + jj) * nb + blk) * 16 * r2;
        const double2* tj = tv + jj * r2;
        double re = 0, im = 0;
        // columns jq, jq + 4, ... < 2r <= 128, 16 loads in flight
#pragma unroll 1
        for (int u0 = 0; u0 < 32 && jq + 4 * u0 < r2; u0 += 8) {
          double2 ka[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int k = jq + 4 * (u0 + u);
            if (k < r2) ka[u] = Cb[k * 16 + l16];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int k = jq + 4 * (u0 + u);
            if (k < r2) {
              const double2 x = tj[k];
              re = fma(ka[u].x, x.x, re);
              re = fma(-ka[u].y, x.y, re);
              im = fma(ka[u].x, x.y, im);
              im = fma(ka[u].y, x.x, im);
            }
          }
        }
        re += __shfl_xor(re, 16, 64);
        im += __shfl_xor(im, 16, 64);
        re += __shfl_xor(re, 32, 64);
        im += __shfl_xor(im, 32, 64);
        const int i = blk * 16 + l16;
        if (jq == 0 && i < r2) sv[jj * r2 + i] = make_double2(re, im);
      }
    }
    __syncthreads();
    // z -= Y s on the rows of children with contrast (Y is zero on the others)
    {
      double re[4] = {0, 0, 0, 0}, im[4] = {0, 0, 0, 0};
      if (mk[j] & (half ? 2 : 1)) {
        const double2* sj = sv + j * r2 + half * r;
  #pragma unroll 1
      for (int u0 = 0; u0 < 16 && cg + 4 * u0 < r; u0 += PB) {
          Pack<T, 4> ya[PB];
#pragma unroll
          for (int u = 0; u < PB; ++u) {
            const int c = cg + 4 * (u0 + u);
            if (c < r) ya[u] = *reinterpret_cast<const Pack<T, 4>*>(Y + (long long)c * N + R0 + row);
          }
#pragma unroll
          for (int u = 0; u < PB; ++u) {
            const int c = cg + 4 * (u0 + u);
            if (c < r) {
              const double2 x = sj[c];
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const double2 yv = to_d2(ya[u].v[q]);
                re[q] = fma(yv.x, x.x, re[q]);
                re[q] = fma(-yv.y, x.y, re[q]);
                im[q] = fma(yv.x, x.y, im[q]);
                im[q] = fma(yv.y, x.x, im[q]);
              }
            }
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) part[cg][row + q] = make_double2(re[q], im[q]);
    }
    __syncthreads();
    {
      double2 o = zl[t];
      o.x -= ((part[0][t].x + part[1][t].x) + part[2][t].x) + part[3][t].x;
      o.y -= ((part[0][t].y + part[1][t].y) + part[2][t].y) + part[3][t].y;
      zl[t] = o;
    }
  }
  __syncthreads();
  z[R0 + t] = zl[t];
}

int hodlr_subtree_rows(long long N, int lp, int Lb, const int* ranks) {
  const int sf = kSubtreeRows, nlev = sf == 512 ? 3 : 2;
  if (lp != 64 || Lb - nlev < 1 || N != (64LL << Lb)) return 0;
  for (int l = Lb - nlev; l < Lb; ++l)
    if (ranks[l] < 0 || ranks[l] > 64) return 0;
  return sf;
}

template <typename T>
static void subtree_launch(int sf, const double2* Dinv, const unsigned char* ident, const double2* b,
                           const int* jdev, long long bldj, double2* z, long long N, int Lb, int F,
                           const SubtreeLevels& lv, const unsigned char* nodeact, hipStream_t s) {
  const unsigned grid = (unsigned)(N / sf);
  if (sf == 512) {
    auto kern = k_hodlr_subtree<T, 512>;
    LSK_LAUNCH(kern, grid, 512, 0, s, Dinv, ident, b, jdev, bldj, z, N, Lb, F, lv, nodeact);
  } else {
    auto kern = k_hodlr_subtree<T, 256>;
    LSK_LAUNCH(kern, grid, 256, 0, s, Dinv, ident, b, jdev, bldj, z, N, Lb, F, lv, nodeact);
  }
}

void launch_hodlr_subtree(int fmt, int sf, const double2* Dinv, const unsigned char* ident, const double2* b,
                          const int* jdev, long long bldj, double2* z, long long N, int Lb,
                          const SubtreeLevels& lv, const unsigned char* nodeact, hipStream_t s) {
  const int nlev = sf == 512 ? 3 : (sf == 256 ? 2 : 0);
  const int F = Lb - nlev;
  if (nlev == 0 || F < 1 || N != (64LL << Lb))
    throw std::runtime_error("hodlr subtree: needs 64-row leaves, N = 64 * 2^Lb and 256 or 512 rows per subtree");
  for (int i = 0; i < nlev; ++i)
    if (lv.r[i] < 0 || lv.r[i] > 64 || (lv.r[i] > 0 && (!lv.W[i] || !lv.Y[i] || !lv.K[i])))
      throw std::runtime_error("hodlr subtree: ranks of at most 64 with their factors");
  if (fmt == 2)
    subtree_launch<bf16>(sf, Dinv, ident, b, jdev, bldj, z, N, Lb, F, lv, nodeact, s);
  else if (fmt == 1)
    subtree_launch<float>(sf, Dinv, ident, b, jdev, bldj, z, N, Lb, F, lv, nodeact, s);
  else
    subtree_launch<double>(sf, Dinv, ident, b, jdev, bldj, z, N, Lb, F, lv, nodeact, s);
}

bool launch_hodlr_update(int fmt, const void* Y, const double2* sv, double2* z, long long ldz, long long N, int r,
                         long long nodesize, int nodes, int nrhs, hipStream_t s, double2* z2, long long z2ldr,
                         const int* jdev, long long z2ldj, const unsigned char* ract) {
  if (fmt != 0 && N % 64 == 0 && nodesize % 128 == 0) {
    const int R = fmt == 2 ? 4 : 2;
    const unsigned nbx = (unsigned)((N / R + 255) / 256);
    const int nrf = nrhs > 1 ? nrhs : 0;
    dim3 gridw(nrf ? nbx * nrhs : nbx, nrf ? 1 : nrhs);
    if (fmt == 2) {
      auto kern = k_hodlr_update_wide<bf16>;
      LSK_LAUNCH(kern, gridw, 256, 0, s, (const BF2*)Y, sv, z, ldz, N, r, nodesize, nodes, nrf, z2, z2ldr, jdev,
                 z2ldj, ract);
    } else {
      auto kern = k_hodlr_update_wide<float>;
      LSK_LAUNCH(kern, gridw, 256, 0, s, (const float2*)Y, sv, z, ldz, N, r, nodesize, nodes, nrf, z2, z2ldr, jdev,
                 z2ldj, ract);
    }
    return z2 != nullptr;
  }
  dim3 grid((unsigned)((N + 255) / 256), nrhs);
  if (fmt == 2) {
    auto kern = k_hodlr_update<bf16>;
    LSK_LAUNCH(kern, grid, 256, 0, s, (const BF2*)Y, sv, z, ldz, N, r, nodesize, nodes);
  } else if (fmt == 1) {
    auto kern = k_hodlr_update<float>;
    LSK_LAUNCH(kern, grid, 256, 0, s, (const float2*)Y, sv, z, ldz, N, r, nodesize, nodes);
  } else if (nrhs >= 16 && nodesize % 128 == 0) {
    constexpr int RB = 16;
    dim3 gridb((unsigned)((N + 255) / 256), (unsigned)((nrhs + RB - 1) / RB));
    auto kern = k_hodlr_update_rb<RB>;
    LSK_LAUNCH(kern, gridb, 256, 0, s, (const double2*)Y, sv, z, ldz, N, r, nodesize, nodes, nrhs);
  } else {
    auto kern = k_hodlr_update<double>;
    LSK_LAUNCH(kern, grid, 256, 0, s, (const double2*)Y, sv, z, ldz, N, r, nodesize, nodes);
  }
  return false;
}

// =====================================================================================
// Krylov (Arnoldi) kernels: classical Gram-Schmidt dot products and updates.
// =====================================================================================
// partial[(rhs*nchunks + chunk)*maxv + v] = sum_{i in chunk} conj(Q_v[i]) w[i]
void launch_gs_dot(const double2* Q, long long ldq_vec, long long ldq_rhs, int nv, const double2* w, long long ldw,
                   double2* partial, long long N, int nchunks, int maxv, int nrhs, hipStream_t s) {
  const long long chunk = (N + nchunks - 1) / nchunks;  // the last chunk is clipped at N
  tsdot(0, true, Q, ldq_vec, ldq_rhs, nv, w, ldw, partial, maxv, chunk, nchunks, N, nrhs, s);
}

// h[rhs*maxv + v] (+)= sum_c partial[(rhs*nchunks + c)*maxv + v]; one wave per value
__global__ __launch_bounds__(256) void k_gs_finish(const double2* __restrict__ partial, int nchunks, int nv, int maxv,
                                                   double2* h, int accumulate) {
  const int rhs = blockIdx.y;
  const int v = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (v >= nv) return;
  double re = 0, im = 0;
  for (int c = lane; c < nchunks; c += 64) {
    const double2 p = partial[((long long)rhs * nchunks + c) * maxv + v];
    re += p.x;
    im += p.y;
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (lane == 0) {
    double2* o = h + (long long)rhs * maxv + v;
    if (accumulate) {
      re += o->x;
      im += o->y;
    }
    *o = make_double2(re, im);
  }
}

void launch_gs_finish(const double2* partial, int nchunks, int nv, int maxv, double2* h, int accumulate, int nrhs,
                      hipStream_t s) {
  dim3 grid((nv + 3) / 4, nrhs);
  k_gs_finish<<<grid, 256, 0, s>>>(partial, nchunks, nv, maxv, h, accumulate);
}

// w[i] += sign * sum_v Q_v[i] h[v]
// Device-driven form (jdev != NULL): nv = *jdev + 1 and h advanced by *jdev * h_ldj; rhs with
// skip[rhs] != 0 untouched.
__global__ __launch_bounds__(256) void k_gs_axpy(const double2* __restrict__ Q, long long ldq_vec, long long ldq_rhs,
                                                 int nv, const double2* __restrict__ h, long long h_ldr, double sign,
                                                 double2* __restrict__ w, long long ldw, long long N,
                                                 const int* __restrict__ jdev, long long h_ldj,
                                                 const int* __restrict__ skip) {
  __shared__ double2 hs[256];
  const int rhs = blockIdx.y;
  if (skip && skip[rhs] != 0) return;  // uniform per block
  if (jdev) {
    const int j = *jdev;
    nv = j + 1;
    h += (long long)j * h_ldj;
  }
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double re = 0, im = 0;
  for (int v0 = 0; v0 < nv; v0 += 256) {
    const int cnt = nv - v0 < 256 ? nv - v0 : 256;
    __syncthreads();
    if ((int)threadIdx.x < cnt) hs[threadIdx.x] = h[(long long)rhs * h_ldr + v0 + threadIdx.x];
    __syncthreads();
    if (i < N) {
      const double2* q = Q + rhs * ldq_rhs + (long long)v0 * ldq_vec + i;
      for (int v = 0; v < cnt; ++v) {
        const double2 a = q[(long long)v * ldq_vec];
        const double2 b = hs[v];
        re += a.x * b.x - a.y * b.y;
        im += a.x * b.y + a.y * b.x;
      }
    }
  }
  if (i < N) {
    double2 o = w[rhs * ldw + i];
    o.x += sign * re;
    o.y += sign * im;
    w[rhs * ldw + i] = o;
  }
}

void launch_gs_axpy(const double2* Q, long long ldq_vec, long long ldq_rhs, int nv, const double2* h, int maxv,
                    double sign, double2* w, long long ldw, long long N, int nrhs, hipStream_t s) {
  dim3 grid((unsigned)((N + 255) / 256), nrhs);
  k_gs_axpy<<<grid, 256, 0, s>>>(Q, ldq_vec, ldq_rhs, nv, h, maxv, sign, w, ldw, N, nullptr, 0, nullptr);
}

__global__ __launch_bounds__(256) void k_norm2(const double2* __restrict__ w, long long ldw, double* partial,
                                               long long N, int nchunks) {
  __shared__ double red[32];
  const int ch = blockIdx.x, rhs = blockIdx.y;
  const long long per = (N + nchunks - 1) / nchunks;
  const long long i0 = (long long)ch * per;
  const long long i1 = i0 + per < N ? i0 + per : N;
  double acc = 0;
  for (long long i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const double2 a = w[rhs * ldw + i];
    acc += a.x * a.x + a.y * a.y;
  }
  const double2 sum = block_sum2(acc, 0.0, red);
  if (threadIdx.x == 0) partial[(long long)rhs * nchunks + ch] = sum.x;
}

void launch_norm2(const double2* w, long long ldw, double* partial, long long N, int nchunks, int nrhs,
                  hipStream_t s) {
  dim3 grid(nchunks, nrhs);
  k_norm2<<<grid, 256, 0, s>>>(w, ldw, partial, N, nchunks);
}

__global__ void k_norm2_finish(const double* partial, int nchunks, double* out) {
  const int rhs = blockIdx.x;
  if (threadIdx.x != 0) return;
  double s = 0;
  for (int c = 0; c < nchunks; ++c) s += partial[(long long)rhs * nchunks + c];
  out[rhs] = s;
}

void launch_norm2_finish(const double* partial, int nchunks, double* out, int nrhs, hipStream_t s) {
  k_norm2_finish<<<nrhs, 64, 0, s>>>(partial, nchunks, out);
}

__global__ void k_scale(const double2* __restrict__ w, long long ldw, const double* __restrict__ alpha,
                        double2* __restrict__ out, long long ldo, long long N) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (i >= N) return;
  const double a = alpha[rhs];
  const double2 v = w[rhs * ldw + i];
  out[rhs * ldo + i] = make_double2(a * v.x, a * v.y);
}

void launch_scale(const double2* w, long long ldw, const double* alpha, double2* out, long long ldo, long long N,
                  int nrhs, hipStream_t s) {
  dim3 grid((unsigned)((N + 255) / 256), nrhs);
  k_scale<<<grid, 256, 0, s>>>(w, ldw, alpha, out, ldo, N);
}

__global__ void k_axpby(double a, const double2* x, long long ldx, double b, const double2* y, long long ldy,
                        double2* out, long long ldo, long long N) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (i >= N) return;
  const double2 xv = x[rhs * ldx + i];
  double2 o = make_double2(a * xv.x, a * xv.y);
  if (b != 0.0) {
    const double2 yv = y[rhs * ldy + i];
    o.x += b * yv.x;
    o.y += b * yv.y;
  }
  out[rhs * ldo + i] = o;
}

void launch_axpby(double a, const double2* x, long long ldx, double b, const double2* y, long long ldy, double2* out,
                  long long ldo, long long N, int nrhs, hipStream_t s) {
  dim3 grid((unsigned)((N + 255) / 256), nrhs);
  k_axpby<<<grid, 256, 0, s>>>(a, x, ldx, b, y, ldy, out, ldo, N);
}

__global__ void k_cast(int to_fp32, const void* in, void* out, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (to_fp32) {
    const double2 v = reinterpret_cast<const double2*>(in)[i];
    reinterpret_cast<float2*>(out)[i] = make_float2((float)v.x, (float)v.y);
  } else {
    const float2 v = reinterpret_cast<const float2*>(in)[i];
    reinterpret_cast<double2*>(out)[i] = make_double2((double)v.x, (double)v.y);
  }
}

void launch_cast(bool to_fp32, const void* in, void* out, long long n, hipStream_t s) {
  if (n <= 0) return;
  k_cast<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(to_fp32 ? 1 : 0, in, out, n);
}

// complex128 -> complex bfloat16, rounding the FP32 value to nearest even in its top 16 bits
__device__ inline unsigned short bf16_rne(double d) {
  const unsigned u = __float_as_uint((float)d);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__global__ void k_cast_bf16(const double2* __restrict__ in, BF2* __restrict__ out, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 v = in[i];
  BF2 o;
  o.x = bf16_rne(v.x);
  o.y = bf16_rne(v.y);
  out[i] = o;
}

void launch_cast_bf16(const void* in, void* out, long long n, hipStream_t s) {
  if (n <= 0) return;
  k_cast_bf16<<<(unsigned)((n + 255) / 256), 256, 0, s>>>((const double2*)in, (BF2*)out, n);
}


// =====================================================================================
// Device-driven Arnoldi step.  The Arnoldi index j of the current cycle lives in device
// memory (*jdev), so one step is a fixed launch sequence that a HIP graph can capture and
// replay.  Per right-hand side, state[rhs] = 0 while the cycle runs, 1 once it has ended
// (kfin[rhs] columns), 2 when the column is idle (converged or stopped); kernels leave
// non-active columns untouched.  Layouts: Q and Z column j of rhs at rhs*ld_rhs + j*ld_vec;
// Hessenberg H[rhs][j][0..maxv) (column j contiguous), cs[rhs][m], sn[rhs][m], g[rhs][maxv].
// =====================================================================================
__global__ void k_kd_copy(const double2* __restrict__ src, long long src_ldr, long long src_ldj,
                          double2* __restrict__ dst, long long dst_ldr, long long dst_ldj, long long N,
                          const int* __restrict__ jdev, const int* __restrict__ state) {
  const int rhs = blockIdx.y;
  if (state && state[rhs] != 0) return;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const long long j = *jdev;
  dst[rhs * dst_ldr + j * dst_ldj + i] = src[rhs * src_ldr + j * src_ldj + i];
}

void launch_kd_copy(const double2* src, long long src_ldr, long long src_ldj, double2* dst, long long dst_ldr,
                    long long dst_ldj, long long N, const int* jdev, const int* state, int nrhs, hipStream_t s) {
  dim3 grid((unsigned)((N + 255) / 256), nrhs);
  k_kd_copy<<<grid, 256, 0, s>>>(src, src_ldr, src_ldj, dst, dst_ldr, dst_ldj, N, jdev, state);
}

void launch_kd_dot(const double2* Q, long long ldq_vec, long long ldq_rhs, int maxv, const double2* w, long long ldw,
                   double2* partial, long long N, int nchunks, const int* jdev, const int* state, int nrhs,
                   hipStream_t s) {
  const long long chunk = (N + nchunks - 1) / nchunks;
  tsdot(0, true, Q, ldq_vec, ldq_rhs, maxv, w, ldw, partial, maxv, chunk, nchunks, N, nrhs, s, jdev, state);
}

// out[rhs*out_ldr + j*out_ldj + v] (+)= sum_c partial[(rhs*nchunks + c)*maxv + v], v <= j
__global__ __launch_bounds__(256) void k_kd_finish(const double2* __restrict__ partial, int nchunks, int maxv,
                                                   double2* out, long long out_ldr, long long out_ldj, int accumulate,
                                                   const int* __restrict__ jdev, const int* __restrict__ state) {
  const int rhs = blockIdx.y;
  if (state[rhs] != 0) return;
  const int j = *jdev;
  const int v = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (v > j) return;
  double re = 0, im = 0;
  for (int c = lane; c < nchunks; c += 64) {
    const double2 p = partial[((long long)rhs * nchunks + c) * maxv + v];
    re += p.x;
    im += p.y;
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (lane == 0) {
    double2* o = out + rhs * out_ldr + (long long)j * out_ldj + v;
    if (accumulate) {
      re += o->x;
      im += o->y;
    }
    *o = make_double2(re, im);
  }
}

void launch_kd_finish(const double2* partial, int nchunks, int maxv, double2* out, long long out_ldr,
                      long long out_ldj, int accumulate, const int* jdev, const int* state, int nrhs, hipStream_t s) {
  dim3 grid((maxv + 3) / 4, nrhs);
  k_kd_finish<<<grid, 256, 0, s>>>(partial, nchunks, maxv, out, out_ldr, out_ldj, accumulate, jdev, state);
}

void launch_kd_axpy(const double2* Q, long long ldq_vec, long long ldq_rhs, const double2* h, long long h_ldr,
                    long long h_ldj, double sign, double2* w, long long ldw, long long N, const int* jdev,
                    const int* state, int nrhs, hipStream_t s) {
  dim3 grid((unsigned)((N + 255) / 256), nrhs);
  k_gs_axpy<<<grid, 256, 0, s>>>(Q, ldq_vec, ldq_rhs, 0, h, h_ldr, sign, w, ldw, N, jdev, h_ldj, state);
}

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline double cabs2(double2 a) { return hypot(a.x, a.y); }

// One wave per rhs: ||w|| from the norm partials, H[j+1][j] = ||w||, the previous Givens
// rotations applied to column j, a new rotation annihilating H[j+1][j], g updated, the
// residual estimate |g[j+1]| / fnorm, and the stop decision (estimate <= tol, maxit, restart
// length, breakdown or a non-finite value).  alpha[rhs] = 1/||w|| for a column that goes on.
__global__ __launch_bounds__(64) void k_kd_givens(const double* __restrict__ npart, int nchunks, double2* H, int m,
                                                  int maxv, double* cs, double2* sn, double2* g,
                                                  const int* __restrict__ jdev, int* state, int* its, int* kfin,
                                                  double* est, const double* __restrict__ fnorm,
                                                  const double* __restrict__ tol, int maxit, double* alpha) {
  const int rhs = blockIdx.x, lane = threadIdx.x;
  if (state[rhs] != 0) {
    if (lane == 0) alpha[rhs] = 0.0;
    return;
  }
  double ssq = 0;
  for (int c = lane; c < nchunks; c += 64) ssq += npart[(long long)rhs * nchunks + c];
  ssq = wave_sum(ssq);
  if (lane != 0) return;
  const int j = *jdev;
  const double hn = sqrt(ssq);
  double2* h = H + ((long long)rhs * m + j) * maxv;
  double* c_ = cs + (long long)rhs * m;
  double2* s_ = sn + (long long)rhs * m;
  double2* gg = g + (long long)rhs * maxv;
  // rotation i maps (h[i], h[i+1]) to new values; the new h[i+1] is the next rotation's first
  // entry, so it is carried in registers and only the untouched h[i+1], c_i, s_i are loaded
  // (independent of the carry, so the loads run ahead of the chain)
  double2 carry = h[0];
#pragma unroll 4
  for (int i = 0; i < j; ++i) {
    const double2 a = carry, b = h[i + 1];
    const double ci = c_[i];
    const double2 si = s_[i];
    const double2 sb = cmul(si, b), sa = cmul(cconj(si), a);
    h[i] = make_double2(ci * a.x + sb.x, ci * a.y + sb.y);
    carry = make_double2(ci * b.x - sa.x, ci * b.y - sa.y);
  }
  const double2 a = carry, b = make_double2(hn, 0.0);
  const double aa = cabs2(a), ab = cabs2(b);
  double cc;
  double2 ss;
  if (ab == 0.0) {
    cc = 1.0;
    ss = make_double2(0.0, 0.0);
  } else if (aa == 0.0) {
    cc = 0.0;
    ss = make_double2(b.x / ab, -b.y / ab);
  } else {
    const double t = hypot(aa, ab);
    cc = aa / t;
    const double2 ph = make_double2(a.x / aa, a.y / aa);
    const double2 q = cmul(ph, cconj(b));
    ss = make_double2(q.x / t, q.y / t);
  }
  c_[j] = cc;
  s_[j] = ss;
  const double2 sb = cmul(ss, b);
  h[j] = make_double2(cc * a.x + sb.x, cc * a.y + sb.y);
  h[j + 1] = make_double2(0.0, 0.0);
  const double2 gj = gg[j];
  const double2 t1 = cmul(cconj(ss), gj);
  gg[j + 1] = make_double2(-t1.x, -t1.y);
  gg[j] = make_double2(cc * gj.x, cc * gj.y);
  const int it = its[rhs] + 1;
  its[rhs] = it;
  const double e = cabs2(gg[j + 1]) / fnorm[rhs];
  est[rhs] = e;
  const bool stop = e <= tol[rhs] || it >= maxit || j + 1 >= m || hn == 0.0 || !isfinite(e);
  if (stop) {
    state[rhs] = 1;
    kfin[rhs] = j + 1;
    alpha[rhs] = 0.0;
  } else {
    alpha[rhs] = 1.0 / hn;
  }
}

void launch_kd_givens(const double* npart, int nchunks, double2* H, int m, int maxv, double* cs, double2* sn,
                      double2* g, const int* jdev, int* state, int* its, int* kfin, double* est, const double* fnorm,
                      const double* tol, int maxit, double* alpha, int nrhs, hipStream_t s) {
  k_kd_givens<<<nrhs, 64, 0, s>>>(npart, nchunks, H, m, maxv, cs, sn, g, jdev, state, its, kfin, est, fnorm, tol,
                                  maxit, alpha);
}

// Q_{j+1} = alpha w for columns still active after the rotation
__global__ void k_kd_next(const double2* __restrict__ w, long long ldw, const double* __restrict__ alpha,
                          double2* __restrict__ Q, long long ldq_vec, long long ldq_rhs, long long N,
                          const int* __restrict__ jdev, const int* __restrict__ state) {
  const int rhs = blockIdx.y;
  if (state[rhs] != 0) return;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double a = alpha[rhs];
  const double2 v = w[rhs * ldw + i];
  Q[rhs * ldq_rhs + (long long)(*jdev + 1) * ldq_vec + i] = make_double2(a * v.x, a * v.y);
}

// j += 1 when any column is still active (one thread)
__global__ void k_kd_advance(int* jdev, const int* __restrict__ state, int nrhs) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  bool any = false;
  for (int r = 0; r < nrhs; ++r) any |= state[r] == 0;
  if (any) *jdev += 1;
}

void launch_kd_next(const double2* w, long long ldw, const double* alpha, double2* Q, long long ldq_vec,
                    long long ldq_rhs, long long N, int* jdev, const int* state, int nrhs, hipStream_t s) {
  dim3 grid((unsigned)((N + 255) / 256), nrhs);
  k_kd_next<<<grid, 256, 0, s>>>(w, ldw, alpha, Q, ldq_vec, ldq_rhs, N, jdev, state);
  k_kd_advance<<<1, 64, 0, s>>>(jdev, state, nrhs);
}


// ---- delayed CGS2: one reduction and one update pass over the basis per step ----
// Slot j of Q holds u_j, the new direction after one Gram-Schmidt pass, not yet normalised.
// One pass over Q_0..Q_j gives every inner product the step needs (Q_j = u_j itself gives
// u_j^H u_j and u_j^H w):  partial[((rhs*nblk + b)*2 + x)*maxv + v] = sum over the rows of
// block b of conj(Q_v) y_x, y_0 = u_j, y_1 = w, v <= j.
template <int G>
__global__ __launch_bounds__(256) void k_kd_dot2(const double2* __restrict__ Q, long long ldq_vec, long long ldq_rhs,
                                                 const double2* __restrict__ w, long long ldw,
                                                 double2* __restrict__ partial, int maxv, long long N, int rpb,
                                                 int nblk, const int* __restrict__ jdev,
                                                 const int* __restrict__ state) {
  __shared__ double lds[4][4 * G];
  const int rhs = blockIdx.z;
  if (state[rhs] != 0) return;  // uniform per block
  const int j = *jdev;
  const int c0 = blockIdx.y * G;
  if (c0 > j) return;
  const int ng = j + 1 - c0 < G ? j + 1 - c0 : G;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const double2* Qb = Q + rhs * ldq_rhs;
  const double2* u = Qb + (long long)j * ldq_vec;
  const double2* wb = w + rhs * ldw;
  const long long i0 = (long long)blockIdx.x * rpb;
  const long long i1 = i0 + rpb < N ? i0 + rpb : N;
  double acc[4 * G];
#pragma unroll
  for (int c = 0; c < 4 * G; ++c) acc[c] = 0;
  // columns past j re-read column j (loads stay unconditional); their sums are not stored
  long long coff[G];
#pragma unroll
  for (int c = 0; c < G; ++c) coff[c] = (long long)(c0 + (c < ng ? c : ng - 1)) * ldq_vec;
  for (long long i = i0 + threadIdx.x; i < i1; i += 256) {
    const double2 uv = u[i], xv = wb[i];
    double2 a[G];
#pragma unroll
    for (int c = 0; c < G; ++c) a[c] = Qb[coff[c] + i];
#pragma unroll
    for (int c = 0; c < G; ++c) {
      acc[4 * c] = fma(a[c].x, uv.x, fma(a[c].y, uv.y, acc[4 * c]));
      acc[4 * c + 1] = fma(a[c].x, uv.y, fma(-a[c].y, uv.x, acc[4 * c + 1]));
      acc[4 * c + 2] = fma(a[c].x, xv.x, fma(a[c].y, xv.y, acc[4 * c + 2]));
      acc[4 * c + 3] = fma(a[c].x, xv.y, fma(-a[c].y, xv.x, acc[4 * c + 3]));
    }
    __builtin_amdgcn_sched_group_barrier(0x0020, G + 2, 0);
    __builtin_amdgcn_sched_group_barrier(0x0002, 16 * G, 0);
  }
#pragma unroll
  for (int c = 0; c < 4 * G; ++c) acc[c] = wave_sum(acc[c]);
  if (lane == 0)
#pragma unroll
    for (int c = 0; c < 4 * G; ++c) lds[wv][c] = acc[c];
  __syncthreads();
  const int t = threadIdx.x;
  if (t >= 4 * G) return;
  const int c = t >> 2, x = (t >> 1) & 1, comp = t & 1;
  if (c >= ng) return;
  const double v = lds[0][t] + lds[1][t] + lds[2][t] + lds[3][t];
  double* out = reinterpret_cast<double*>(partial + (((long long)rhs * nblk + blockIdx.x) * 2 + x) * maxv + c0 + c);
  out[comp] = v;
}

// cd[(rhs*2 + x)*maxv + v] = sum_b partial[((rhs*nblk + b)*2 + x)*maxv + v] for v <= j
__global__ __launch_bounds__(256) void k_kd_finish2(const double2* __restrict__ partial, int nblk, int maxv,
                                                    double2* __restrict__ cd, const int* __restrict__ jdev,
                                                    const int* __restrict__ state) {
  const int rhs = blockIdx.y;
  if (state[rhs] != 0) return;
  const int j = *jdev;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int x = k & 1, v = k >> 1;
  if (v > j) return;
  double re = 0, im = 0;
  for (int b = lane; b < nblk; b += 64) {
    const double2 p = partial[(((long long)rhs * nblk + b) * 2 + x) * maxv + v];
    re += p.x;
    im += p.y;
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (lane == 0) cd[((long long)rhs * 2 + x) * maxv + v] = make_double2(re, im);
}

// Step j of delayed CGS2 from cd = (c, d), where c_v = q_v^H u_j and d_v = q_v^H w for v < j,
// c_j = u_j^H u_j and d_j = u_j^H w.  First kernel, one block per right-hand side:
//  * beta = sqrt(c_j - |c|^2) is the norm of q_j' = u_j - Q c (second Gram-Schmidt pass), so
//    column j-1 of the Hessenberg matrix becomes final: Hr[j-1][v] += c_v, Hr[j-1][j] = beta.
//    Its copy in H is rotated (previous Givens rotations, then a new one), g is updated and the
//    column stops on the estimate |g_j| / ||f|| <= tol, maxit, the restart length or breakdown
//    (kfin = j columns).  A column that goes on gets T[j] = (c, beta), which relates the stored
//    z~ to z, and alpha = 1 / beta.
__global__ __launch_bounds__(256) void k_kd_dcgs2(const double2* __restrict__ cd, double2* Hr, double2* H, int m,
                                                  int maxv, double* cs, double2* sn, double2* g, double2* T,
                                                  const int* __restrict__ jdev, int* state, int* its, int* kfin,
                                                  double* est, const double* __restrict__ fnorm,
                                                  const double* __restrict__ tol, int maxit, double* alpha) {
  constexpr int TILE = 512;
  __shared__ double red[32];
  __shared__ int stop_s;
  __shared__ double2 hb_s[TILE], sn_s[TILE];
  __shared__ double cs_s[TILE];
  const int rhs = blockIdx.x, t = threadIdx.x;
  if (state[rhs] != 0) {
    if (t == 0) alpha[rhs] = 0.0;
    return;
  }
  const int j = *jdev;
  const double2* c = cd + (long long)rhs * 2 * maxv;
  double2* hr = Hr + (long long)rhs * (m + 1) * maxv;  // column k at hr + k * maxv
  double ss = 0;
  for (int v = t; v < j; v += 256) ss += c[v].x * c[v].x + c[v].y * c[v].y;
  const double ssq = block_sum2(ss, 0.0, red).x;
  const double b2 = c[j].x - ssq;
  const double beta = b2 > 0 ? sqrt(b2) : 0.0;
  const int jc = j - 1;
  double2* hcol = H + ((long long)rhs * m + (j > 0 ? jc : 0)) * maxv;
  if (j >= 1)
    for (int v = t; v <= j; v += 256) {
      double2 hv = hr[(long long)jc * maxv + v];
      if (v < j) {
        hv.x += c[v].x;
        hv.y += c[v].y;
      } else {
        hv = make_double2(beta, 0.0);
      }
      hr[(long long)jc * maxv + v] = hv;
      hcol[v] = hv;
    }
  __syncthreads();
  // previous rotations on column j-1: the entries, cosines and sines are staged through LDS
  // a tile at a time, so the serial chain of thread 0 waits on LDS rather than on memory
  double* c_ = cs + (long long)rhs * m;
  double2* s_ = sn + (long long)rhs * m;
  double2 carry = make_double2(0.0, 0.0);
  if (j >= 1 && t == 0) carry = hcol[0];
  for (int i0 = 0; i0 < jc; i0 += TILE) {
    const int cnt = jc - i0 < TILE ? jc - i0 : TILE;
    for (int k = t; k < cnt; k += 256) {
      hb_s[k] = hcol[i0 + k + 1];
      cs_s[k] = c_[i0 + k];
      sn_s[k] = s_[i0 + k];
    }
    __syncthreads();
    if (t == 0)
      for (int k = 0; k < cnt; ++k) {
        const double2 a = carry, b = hb_s[k];
        const double ci = cs_s[k];
        const double2 si = sn_s[k];
        const double2 sb = cmul(si, b), sa = cmul(cconj(si), a);
        hcol[i0 + k] = make_double2(ci * a.x + sb.x, ci * a.y + sb.y);
        carry = make_double2(ci * b.x - sa.x, ci * b.y - sa.y);
      }
    __syncthreads();
  }
  if (t == 0) {
    bool stop = !(beta > 0) || !isfinite(beta);
    if (j >= 1) {
      double2* gg = g + (long long)rhs * maxv;
      const double2 a = carry, b = make_double2(beta, 0.0);
      const double aa = cabs2(a), ab = cabs2(b);
      double cc;
      double2 sg;
      if (ab == 0.0) {
        cc = 1.0;
        sg = make_double2(0.0, 0.0);
      } else if (aa == 0.0) {
        cc = 0.0;
        sg = make_double2(b.x / ab, -b.y / ab);
      } else {
        const double tt = hypot(aa, ab);
        cc = aa / tt;
        const double2 ph = make_double2(a.x / aa, a.y / aa);
        const double2 q = cmul(ph, cconj(b));
        sg = make_double2(q.x / tt, q.y / tt);
      }
      c_[jc] = cc;
      s_[jc] = sg;
      const double2 sb = cmul(sg, b);
      hcol[jc] = make_double2(cc * a.x + sb.x, cc * a.y + sb.y);
      hcol[jc + 1] = make_double2(0.0, 0.0);
      const double2 gj = gg[jc];
      const double2 t1 = cmul(cconj(sg), gj);
      gg[jc + 1] = make_double2(-t1.x, -t1.y);
      gg[jc] = make_double2(cc * gj.x, cc * gj.y);
      const int it = its[rhs] + 1;
      its[rhs] = it;
      const double e = cabs2(gg[jc + 1]) / fnorm[rhs];
      est[rhs] = e;
      stop = stop || e <= tol[rhs] || it >= maxit || j >= m || !isfinite(e);
    }
    if (stop) {
      state[rhs] = 1;
      kfin[rhs] = j;
      alpha[rhs] = 0.0;
    } else {
      alpha[rhs] = 1.0 / beta;
    }
    stop_s = stop ? 1 : 0;
  }
  __syncthreads();
  if (stop_s) return;
  double2* tc = T + ((long long)rhs * (m + 1) + j) * maxv;
  for (int v = t; v <= j; v += 256) tc[v] = v < j ? c[v] : make_double2(beta, 0.0);
}

// Second kernel, one wave per entry v <= j of a column that goes on: q_j = q_j' / beta and
// z_j = (z~_j - Z c) / beta give A z_j = (w - Q_j Hbar c) / beta (Hbar = columns 0..j-1 of Hr),
// so the first-pass coefficients h = Q_j^H A z_j follow from c and d without touching the basis:
// h_v = (d_v - (Hbar c)_v) / beta for v < j, h_j = ((d_j - c^H d) / beta - (Hbar c)_j) / beta.
// h is stored as Hr[j] (the next step adds its own second-pass part), and the update pass gets
// coef = (c, e), e = Hbar c / beta + h.
__global__ __launch_bounds__(256) void k_kd_dcgs2_h(const double2* __restrict__ cd, double2* Hr, int m, int maxv,
                                                    double2* __restrict__ coef, const int* __restrict__ jdev,
                                                    const int* __restrict__ state, const double* __restrict__ alpha) {
  const int rhs = blockIdx.y;
  if (state[rhs] != 0) return;
  const int j = *jdev;
  const int v = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (v > j) return;
  const double ib = alpha[rhs];
  const double2* c = cd + (long long)rhs * 2 * maxv;
  const double2* d = c + maxv;
  const double2* hr = Hr + (long long)rhs * (m + 1) * maxv;
  // (Hbar c)_v: column k of Hbar is zero below row k + 1
  double hx = 0, hy = 0;
  for (int k = (v > 0 ? v - 1 : 0) + lane; k < j; k += 64) {
    const double2 a = hr[(long long)k * maxv + v], b = c[k];
    hx += a.x * b.x - a.y * b.y;
    hy += a.x * b.y + a.y * b.x;
  }
  hx = wave_sum(hx);
  hy = wave_sum(hy);
  double2 h;
  if (v < j) {
    h = make_double2((d[v].x - hx) * ib, (d[v].y - hy) * ib);
  } else {
    double sr = 0, si = 0;  // c^H d
    for (int k = lane; k < j; k += 64) {
      sr += c[k].x * d[k].x + c[k].y * d[k].y;
      si += c[k].x * d[k].y - c[k].y * d[k].x;
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    h = make_double2(((d[j].x - sr) * ib - hx) * ib, ((d[j].y - si) * ib - hy) * ib);
  }
  if (lane != 0) return;
  Hr[(long long)rhs * (m + 1) * maxv + (long long)j * maxv + v] = h;
  double2* cf = coef + (long long)rhs * 2 * maxv;
  cf[v] = v < j ? c[v] : make_double2(0.0, 0.0);
  cf[maxv + v] = make_double2(hx * ib + h.x, hy * ib + h.y);
}

// slot j := q_j = (u_j - sum_{v<j} Q_v c_v) / beta and slot j+1 := u_{j+1} = w / beta -
// sum_{v<j} Q_v e_v - q_j e_j in one pass over Q_0..Q_{j-1} (coef = (c, e), alpha = 1/beta)
__global__ __launch_bounds__(256) void k_kd_dcgs2_axpy(double2* __restrict__ Q, long long ldq_vec, long long ldq_rhs,
                                                       const double2* __restrict__ w, long long ldw,
                                                       const double2* __restrict__ coef, int maxv,
                                                       const double* __restrict__ alpha, long long N,
                                                       const int* __restrict__ jdev, const int* __restrict__ state) {
  __shared__ double2 cs_[256], es_[256];
  const int rhs = blockIdx.y;
  if (state[rhs] != 0) return;  // uniform per block
  const int j = *jdev;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const double2* cf = coef + (long long)rhs * 2 * maxv;
  double2* Qb = Q + rhs * ldq_rhs;
  double ax = 0, ay = 0, bx = 0, by = 0;
  for (int v0 = 0; v0 < j; v0 += 256) {
    const int cnt = j - v0 < 256 ? j - v0 : 256;
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
      cs_[threadIdx.x] = cf[v0 + threadIdx.x];
      es_[threadIdx.x] = cf[maxv + v0 + threadIdx.x];
    }
    __syncthreads();
    if (i < N) {
      const double2* q = Qb + (long long)v0 * ldq_vec + i;
#pragma unroll 4
      for (int v = 0; v < cnt; ++v) {
        const double2 a = q[(long long)v * ldq_vec];
        const double2 p = cs_[v], e = es_[v];
        ax += a.x * p.x - a.y * p.y;
        ay += a.x * p.y + a.y * p.x;
        bx += a.x * e.x - a.y * e.y;
        by += a.x * e.y + a.y * e.x;
      }
    }
  }
  if (i >= N) return;
  const double ib = alpha[rhs];
  const double2 u = Qb[(long long)j * ldq_vec + i];
  const double2 x = w[rhs * ldw + i];
  const double2 ej = cf[maxv + j];
  const double2 qj = make_double2((u.x - ax) * ib, (u.y - ay) * ib);
  const double2 un = make_double2(x.x * ib - bx - (qj.x * ej.x - qj.y * ej.y),
                                  x.y * ib - by - (qj.x * ej.y + qj.y * ej.x));
  Qb[(long long)j * ldq_vec + i] = qj;
  Qb[(long long)(j + 1) * ldq_vec + i] = un;
}

constexpr int kDot2Cols = 4;

void launch_kd_dot2(const double2* Q, long long ldq_vec, long long ldq_rhs, int maxv, const double2* w, long long ldw,
                    double2* partial, long long N, int rpb, const int* jdev, const int* state, int nrhs,
                    hipStream_t s) {
  const int nblk = (int)((N + rpb - 1) / rpb);
  dim3 grid(nblk, (maxv + kDot2Cols - 1) / kDot2Cols, nrhs);
  auto kern = k_kd_dot2<kDot2Cols>;
  LSK_LAUNCH(kern, grid, 256, 0, s, Q, ldq_vec, ldq_rhs, w, ldw, partial, maxv, N, rpb, nblk, jdev, state);
  dim3 g2((2 * maxv + 3) / 4, nrhs);
  k_kd_finish2<<<g2, 256, 0, s>>>(partial, nblk, maxv, partial + (long long)nrhs * nblk * 2 * maxv, jdev, state);
}

void launch_kd_dcgs2(const double2* cd, double2* Hr, double2* H, int m, int maxv, double* cs, double2* sn, double2* g,
                     double2* T, double2* coef, const int* jdev, int* state, int* its, int* kfin, double* est,
                     const double* fnorm, const double* tol, int maxit, double* alpha, int nrhs, hipStream_t s) {
  k_kd_dcgs2<<<nrhs, 256, 0, s>>>(cd, Hr, H, m, maxv, cs, sn, g, T, jdev, state, its, kfin, est, fnorm, tol, maxit,
                                  alpha);
  dim3 grid((maxv + 3) / 4, nrhs);
  k_kd_dcgs2_h<<<grid, 256, 0, s>>>(cd, Hr, m, maxv, coef, jdev, state, alpha);
}

void launch_kd_dcgs2_axpy(double2* Q, long long ldq_vec, long long ldq_rhs, const double2* w, long long ldw,
                          const double2* coef, int maxv, const double* alpha, long long N, int* jdev,
                          const int* state, int nrhs, hipStream_t s) {
  dim3 grid((unsigned)((N + 255) / 256), nrhs);
  k_kd_dcgs2_axpy<<<grid, 256, 0, s>>>(Q, ldq_vec, ldq_rhs, w, ldw, coef, maxv, alpha, N, jdev, state);
  k_kd_advance<<<1, 64, 0, s>>>(jdev, state, nrhs);
}

}  // namespace lsk
