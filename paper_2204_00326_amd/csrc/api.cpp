// C ABI of libls: setup, DAFMM matvec, HODLR preconditioner, GMRES solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <map>
#include <queue>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ls.h"
#include "h0.h"
#include "field.h"
#include "hodlr_setup.h"
#include "kernels.h"
#include "plan.h"

using ls::LsError;
using ls::Off;
using ls::zd;

namespace {

thread_local std::string g_last_error;

}  // namespace

namespace ls {
void set_last_error(const std::string& msg) { g_last_error = msg; }
}  // namespace ls

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw LsError(LS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void alloc(size_t b) {
    release();
    if (b == 0) b = 16;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      throw LsError(LS_ENOMEM, std::string("hipMalloc(") + std::to_string(b) + "): " + hipGetErrorString(e));
    }
    bytes = b;
  }
  void ensure(size_t b) {
    if (bytes < b) alloc(b);
  }
  template <class T>
  T* as() const {
    return reinterpret_cast<T*>(p);
  }
  template <class T>
  void upload(const std::vector<T>& v) {
    alloc(v.size() * sizeof(T));
    if (!v.empty()) hip_check(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "upload");
  }
};

template <class F>
void parallel_for(int n, F f) {
  int nt = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  nt = std::min(nt, std::max(1, n));
  std::atomic<int> next(0);
  std::vector<std::thread> th;
  std::vector<std::string> errs(nt);
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, t]() {
      try {
        for (;;) {
          int i = next.fetch_add(1);
          if (i >= n) break;
          f(i);
        }
      } catch (const std::exception& e) {
        errs[t] = e.what();
      }
    });
  for (auto& x : th) x.join();
  for (auto& e : errs)
    if (!e.empty()) throw LsError(LS_EINVAL, e);
}

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// ---------------------------------------------------------------------------------------
// Device-side DAFMM operator for one precision.
// ---------------------------------------------------------------------------------------
struct Phase {
  DevBuf tasks, terms, blk;
  DevBuf part, sk;    // split-K partial planes and the tasks' reduction descriptors
  int nsk = 0;
  long long sk_elems = 0;
  DevBuf kbl;         // matrix-core form: k-block descriptors of every task
  int nblocks = 0;
  int ntasks = 0;
  int tag = 0;        // 0 near+M2L, 1 P2M, 2 M2M, 3 L2L, 4 L2P
  bool mfma = false;  // matrix-core form of the stencil
};

struct FmmDev {
  bool fp32 = false;
  int esz = 16;  // bytes per complex element
  DevBuf ops;    // packed operator matrices
  // per-level multipole / local arrays (levels top..leaf), sized for nrhs_cap
  DevBuf mult, loc, xs, ys;
  std::vector<long long> lvl_off;    // element offset of level nu inside mult/loc (rhs 0)
  std::vector<long long> lvl_size;   // elements per rhs of level nu
  long long ml_rhs = 0;              // rhs stride of mult/loc
  int nrhs_cap = 0;
  Phase p2m, nearm2l, l2p;
  std::vector<Phase> up;    // M2M, deepest parent first
  std::vector<Phase> down;  // L2L, top parent first
  // every pass in one persistent launch (matrix-core form): all tasks and terms, the queue of
  // (task, block) pairs, stage sizes, and the counters (ticket, one per stage, error flag)
  Phase fused;
  DevBuf fneed, fctr;
  int nstages = 0;
  int fused_wg = 0;
  // host copies of per-level ranks
  std::vector<std::vector<int>> rank;
  std::vector<int> kmax;
  int kleaf = 0;
  // operator locations (element offsets in ops) for descriptor building
  long long off_U = 0, off_Ut = 0;
  long long off_near[9] = {0};
  std::vector<std::vector<std::vector<long long>>> off_C;    // [nu][dir][c]: M2M op = C (k_child x Mpad(k))
  std::vector<std::vector<std::vector<long long>>> off_Ct;   // [nu][dir][c]: L2L op = C^T (k x Mpad(k_child))
  std::vector<std::vector<std::vector<long long>>> off_K;    // [nu][dir][term]: M2L op = K^T
  int64_t entries_far = 0;
  int64_t entries_m2l = 0;
  double entries_mid = 0;  // complex multiply-adds of the middle launch (one right-hand side)
  // P2M reads the product's input through the tree-order map (and stores the tree-order copy
  // for the near field) and L2P finishes the output: no separate gather and epilogue launches
  bool io_fold = false;
  int64_t stored_bytes = 0;
};

struct HodlrDev {
  int r = 0, Lb = 0, nleaves = 0, lp = 0;
  int64_t dense_leaves = 0;
  std::vector<int> rank;  // per binary level
  long long N = 0;
  DevBuf Dinv, ident;
  DevBuf Dinv32, Dinv16;  // leaf inverses in complex64 / complex bfloat16
  std::vector<DevBuf> Y64, W64, Y32, W32, Y16, W16;  // 16: complex bfloat16
  std::vector<DevBuf> coreinv, core32, core16;      // SMW core inverses per node, 16-row blocks
  bool have16 = false;
  int64_t used_rank_sum = 0, blocks = 0;  // ACA ranks reached, over all off-diagonal blocks
  int used_rank_max = 0;
  double t_aca_ms = 0, t_apply_ms = 0, t_cores_ms = 0;  // setup phases
  // one byte per 256 Morton rows: 0 where no point of the block has contrast (Y's rows are zero)
  DevBuf ract;
  int64_t rows_active = 0;
  DevBuf alist;          // indices of the 256-row blocks with contrast
  int nact = 0;
  bool sparse = false;   // few enough such blocks that updates run over the list alone
  // one byte per tree node (node j of depth d at (1 << d) + j, depth Lb = the leaves): nonzero
  // where the node holds a point with contrast.  Set after the factors are built; the applies
  // then skip the W^T z chunks and K^-1 products that meet a zero Y.
  DevBuf nodeact;
  DevBuf dlist;                   // per level: the children whose sibling has contrast (W^T z chunks formed)
  std::vector<long long> doff;    // offset of each level's list in dlist
  std::vector<int> dcnt;          // its length
  std::vector<int64_t> dot_rows;  // per level: rows whose W^T z the masked apply forms
  std::vector<int> core_nodes;    // per level: nodes whose two children both hold contrast
  DevBuf partial, svec;
  std::vector<long long> chunk;  // per level
  std::vector<int> nchunks, cpc;
  int64_t bytes = 0;
};

// Device-driven GMRES of one problem: control words, Hessenberg and rotations in device
// memory, and the captured graphs of graph_iters Arnoldi steps (FP64 / FP32 operator).
struct KrylovDev {
  DevBuf ictl;    // int: [0] = j, then state[nrhs], its[nrhs], kfin[nrhs]
  DevBuf dctl;    // double: fnorm[nrhs], tol[nrhs], est[nrhs], alpha[nrhs]
  DevBuf H, cs, sn, g, vin, tmp;
  DevBuf Hr, T, coef;   // delayed CGS2: unrotated Hessenberg, basis change of Z, update coefficients
  int* host = nullptr;  // pinned mirror of ictl (plus est as doubles after it)
  size_t host_bytes = 0;
  hipStream_t cap = nullptr;
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  std::vector<uintptr_t> key[2];
  KrylovDev() = default;
  KrylovDev(const KrylovDev&) = delete;
  KrylovDev& operator=(const KrylovDev&) = delete;
  void drop(int v) {
    if (exec[v]) (void)hipGraphExecDestroy(exec[v]);
    exec[v] = nullptr;
    key[v].clear();
  }
  ~KrylovDev() {
    drop(0);
    drop(1);
    if (host) (void)hipHostFree(host);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

// kernel classes 0..9 time one launch each; 10..19 time a span of launches of the unfused DAFMM
// product (gather, upward pass, near field + M2L, downward pass, epilogue; FP64 then FP32)
constexpr int kProfClasses = 20;
constexpr int kProfSpan = 10;

struct ProfileClass {
  bool enabled = false;
  int every = 1;       // time every `every`-th launch
  int64_t count = 0;   // launches of the class since enabling
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  std::vector<int> tag;  // per timed launch: the caller's tag (a HODLR level; -1 none)
  size_t used = 0;     // timed launches
};

}  // namespace

struct ls_problem {
  ls_options opt;
  int device = 0;            // HIP device current at ls_setup (every vector call runs there)

  void* scratch = nullptr;   // that device's address of the allocation-free entry point's array
  ls::Plan plan;
  ls::NCA nca64, nca32;
  long long N = 0;
  int n = 0;
  double kappa = 0, tol = 0, coef = 0;
  // index maps (device): s2c/c2s caller <-> S, s2m/m2s Morton <-> S, m2c Morton -> caller
  DevBuf s2c, c2s, s2m, m2s, m2c;
  DevBuf q_c, q_m, px, py;
  DevBuf g2c;                    // grid index a*n + b -> caller index
  double gx0 = 0, gy0 = 0, gh = 0;  // centre of cell (0, 0) and the cell side
  FmmDev f64, f32;
  bool have32 = false;
  HodlrDev hod;
  bool have_hodlr = false;
  // workspaces
  DevBuf w_x, w_y, w_t;  // Morton-order vectors (nrhs_cap)
  int ws_cap = 0;
  ls_stats_t stats{};
  ProfileClass prof[kProfClasses];
  // Krylov workspace
  DevBuf kQ, kZ, kw, kz, kr, kh, kpart, knp, kno, kalpha, ky, kx, kf, kdx;
  size_t kcap_key = 0;
  KrylovDev kd;
  bool capturing = false;  // launches are being recorded into a graph (no event timers)
  struct {
    int gs_rows = 1024;    // rows per chunk of the Arnoldi reductions
    int hodlr_rows = 1024;  // max rows per chunk of the HODLR level reductions
    int dot2_rows = 1024;  // rows per workgroup of the delayed-CGS2 inner products
    bool done = false;
  } tune;
};

namespace {

// ---------------------------------------------------------------------------------------
// profiling
// ---------------------------------------------------------------------------------------
struct ProfScope {
  ProfileClass* pc;
  hipStream_t s;
  ProfScope(ls_problem* P, int cls, hipStream_t st, bool on = true, int tag = -1) : pc(&P->prof[cls]), s(st) {
    if (!on || !pc->enabled || P->capturing || (pc->count++ % pc->every) != 0) {
      pc = nullptr;
      return;
    }
    if (pc->used == pc->ev.size()) {
      hipEvent_t a, b;
      hip_check(hipEventCreate(&a), "hipEventCreate");
      hip_check(hipEventCreate(&b), "hipEventCreate");
      pc->ev.push_back({a, b});
      pc->tag.push_back(-1);
    }
    pc->tag[pc->used] = tag;
    auto& pr = pc->ev[pc->used++];
    lsk::set_next_launch_events(pr.first, pr.second);
  }
  ~ProfScope() {
    // the wrapped code made no timed launch: drop the pair
    if (pc && lsk::next_launch_events_pending()) {
      lsk::clear_next_launch_events();
      pc->used--;
    }
  }
};

// a span of launches between two event records on the stream (launch gaps included)
struct SpanScope {
  std::pair<hipEvent_t, hipEvent_t>* pr = nullptr;
  hipStream_t s;
  SpanScope(ls_problem* P, int cls, hipStream_t st) : s(st) {
    ProfileClass* pc = &P->prof[cls];
    if (!pc->enabled || P->capturing || (pc->count++ % pc->every) != 0) return;
    if (pc->used == pc->ev.size()) {
      hipEvent_t a, b;
      hip_check(hipEventCreate(&a), "hipEventCreate");
      hip_check(hipEventCreate(&b), "hipEventCreate");
      pc->ev.push_back({a, b});
    }
    if (pc->tag.size() < pc->ev.size()) pc->tag.resize(pc->ev.size(), -1);
    pc->tag[pc->used] = -1;
    pr = &pc->ev[pc->used++];
    hip_check(hipEventRecord(pr->first, s), "hipEventRecord");
  }
  ~SpanScope() {
    if (pr) (void)hipEventRecord(pr->second, s);
  }
};

// ---------------------------------------------------------------------------------------
// operator upload and descriptor construction
// ---------------------------------------------------------------------------------------
struct OpPacker {
  std::vector<zd> data;
  // store X^T for X (M x K row-major): op[k][m], rows padded to Mpad
  long long add_transposed(const std::vector<zd>& X, int M, int K) {
    int Mpad = round_up(std::max(M, 1), lsk::kRowBlock);
    long long off = (long long)data.size();
    data.resize(data.size() + (size_t)K * Mpad, zd(0));
    for (int m = 0; m < M; ++m)
      for (int k = 0; k < K; ++k) data[off + (size_t)k * Mpad + m] = X[(size_t)m * K + k];
    return off;
  }
  // store X (K x M row-major) directly as op[k][m] with padding
  long long add_direct(const std::vector<zd>& X, int K, int M) {
    int Mpad = round_up(std::max(M, 1), lsk::kRowBlock);
    long long off = (long long)data.size();
    data.resize(data.size() + (size_t)K * Mpad, zd(0));
    for (int k = 0; k < K; ++k)
      for (int m = 0; m < M; ++m) data[off + (size_t)k * Mpad + m] = X[(size_t)k * M + m];
    return off;
  }
};

void build_fmm_ops(ls_problem* P, const ls::NCA& nca, FmmDev& F, bool fp32) {
  const ls::Plan& p = P->plan;
  F.fp32 = fp32;
  F.esz = fp32 ? 8 : 16;
  const int leaf = p.leaf, s = p.leaf_side, s2 = s * s;
  OpPacker pk;
  for (int t = 0; t < 9; ++t) F.off_near[t] = pk.add_transposed(nca.near[t], s2, s2);
  F.rank.assign(leaf + 1, {});
  F.kmax.assign(leaf + 1, 0);
  F.off_C.assign(leaf + 1, {});
  F.off_Ct.assign(leaf + 1, {});
  F.off_K.assign(leaf + 1, {});
  F.entries_far = 0;
  if (p.top <= leaf) {
    F.kleaf = nca.kleaf;
    // P2M op = U as [pt][rank]; L2P op = U^T as [rank][pt]
    F.off_U = pk.add_direct(nca.U, s2, nca.kleaf);
    F.off_Ut = pk.add_transposed(nca.U, s2, nca.kleaf);
    F.entries_far += 2LL * (int64_t)p.lv[leaf].nb * p.lv[leaf].nb * s2 * nca.kleaf;
    for (int nu = p.top; nu <= leaf; ++nu) {
      const ls::LevelNCA& L = nca.lv[nu];
      const ls::Level& l = p.lv[nu];
      F.rank[nu] = L.rank;
      F.kmax[nu] = L.kmax;
      F.off_K[nu].assign(l.ndir, {});
      for (int dir = 0; dir < l.ndir; ++dir) {
        int ad = ls::antipodal(dir, l.ndir);
        for (size_t t = 0; t < L.K[dir].size(); ++t)
          F.off_K[nu][dir].push_back(pk.add_transposed(L.K[dir][t], L.rank[dir], L.rank[ad]));
      }
      if (nu < leaf) {
        const ls::Level& cl = p.lv[nu + 1];
        F.off_C[nu].assign(l.ndir, std::vector<long long>(4, 0));
        F.off_Ct[nu].assign(l.ndir, std::vector<long long>(4, 0));
        for (int dir = 0; dir < l.ndir; ++dir) {
          int cd = cl.hf ? dir / 2 : 0;
          int kc = nca.lv[nu + 1].rank[cd];
          int k = L.rank[dir];
          for (int c = 0; c < 4; ++c) {
            const std::vector<zd>& C = L.C[dir][c];  // kc x k
            F.off_C[nu][dir][c] = pk.add_direct(C, kc, k);
            F.off_Ct[nu][dir][c] = pk.add_transposed(C, kc, k);
            F.entries_far += 2LL * (int64_t)l.nb * l.nb * kc * k;  // M2M + L2L over all parent boxes
          }
        }
      }
      // M2L entries over in-domain pairs
      int nh = l.nb / 2;
      for (int c = 0; c < 4; ++c)
        for (int dir = 0; dir < l.ndir; ++dir) {
          int ad = ls::antipodal(dir, l.ndir);
          for (const Off& d : l.terms[c * l.ndir + dir]) {
            int ca = c >> 1, cb = c & 1, cnt_a = 0, cnt_b = 0;
            for (int h = 0; h < nh; ++h) {
              int sa = 2 * h + ca + d.a, sb = 2 * h + cb + d.b;
              if (sa >= 0 && sa < l.nb) ++cnt_a;
              if (sb >= 0 && sb < l.nb) ++cnt_b;
            }
            F.entries_far += (int64_t)cnt_a * cnt_b * L.rank[dir] * L.rank[ad];
            F.entries_m2l += (int64_t)cnt_a * cnt_b * L.rank[dir] * L.rank[ad];
          }
        }
    }
  }
  if (fp32) {
    std::vector<float> f(pk.data.size() * 2);
    for (size_t i = 0; i < pk.data.size(); ++i) {
      f[2 * i] = (float)pk.data[i].real();
      f[2 * i + 1] = (float)pk.data[i].imag();
    }
    F.ops.upload(f);
  } else {
    F.ops.upload(pk.data);
  }
  F.stored_bytes = (int64_t)pk.data.size() * F.esz;
}

// Term/task descriptors for all phases, for the current mult/loc/xs/ys allocations.
void build_phases(ls_problem* P, FmmDev& F) {
  const ls::Plan& p = P->plan;
  const int leaf = p.leaf, s2 = p.leaf_side * p.leaf_side;
  const char* ops = F.ops.as<char>();
  char* mult = F.mult.as<char>();
  char* loc = F.loc.as<char>();
  const long long es = F.esz;
  auto opp = [&](long long off) { return (const void*)(ops + off * es); };
  auto lvl_ptr = [&](char* base, int nu, int dir) {
    const ls::Level& l = p.lv[nu];
    long long nh = l.nb / 2;
    return (void*)(base + (F.lvl_off[nu] + (long long)dir * F.kmax[nu] * 4 * nh * nh) * es);
  };
  const long long N = P->N;
  // longest chain of k-blocks one wave of the matrix-core form should carry (longer tasks split
  // over more waves, then over more workgroups), so that no block forms a long tail
  const int kMaxChain = F.fp32 ? 144 : 72;
  // stages of the fused launch: P2M, near field, M2M per parent level, M2L per level, L2L per
  // parent level, L2P; a task's stage and prerequisites are set where the task is made
  const int nup = p.top <= leaf ? leaf - p.top : 0;
  const int S_P2M = 0, S_NEAR = 1;
  auto S_UP = [&](int nu) { return 2 + (nu - p.top); };
  auto S_M2L = [&](int nu) { return 2 + nup + (nu - p.top); };
  auto S_DOWN = [&](int nu) { return 2 + nup + (nup + 1) + (nu - p.top); };
  const int S_L2P = 2 + 3 * nup + 1;
  const int nst = p.top <= leaf ? S_L2P + 1 : 2;
  auto set_stage = [](lsk::DTask& tk, int st, int d0, int d1, int d2, int coh_out) {
    tk.stage = st;
    tk.dep[0] = d0;
    tk.dep[1] = d1;
    tk.dep[2] = d2;
    tk.coh_out = coh_out;
  };
  struct HostPhase {
    std::vector<lsk::DTask> tasks;
    std::vector<lsk::DTerm> terms;
    std::vector<int> pairs;
  };
  std::vector<HostPhase> hps;
  auto make_phase = [&](Phase& ph, std::vector<lsk::DTask>& tasks, std::vector<lsk::DTerm>& terms) {
    std::vector<int> blk;
    for (size_t t = 0; t < tasks.size(); ++t) {
      lsk::DTask& tk = tasks[t];
      int kb = 0;
      for (int q = tk.t0; q < tk.t1; ++q) {
        terms[q].kbase = kb;
        kb += terms[q].K;
      }
      tk.ktot = kb;
      tk.Mpad = round_up(std::max(tk.M, 1), lsk::kRowBlock);
      tk.nrb = tk.Mpad / lsk::kRowBlock;
      tk.blk0 = (int)blk.size();
      int nbb = (tk.nh * tk.nh + lsk::kBoxBlock - 1) / lsk::kBoxBlock;
      for (int i = 0; i < nbb * tk.nrb; ++i) blk.push_back((int)t);
    }
    ph.tasks.upload(tasks);
    ph.terms.upload(terms);
    ph.blk.upload(blk);
    ph.nblocks = (int)blk.size();
    ph.ntasks = (int)tasks.size();
  };
  // matrix-core form: 16-row tiles, k in 4-deep blocks, kps waves per box sub-tile split the
  // blocks (more splitting for long tasks and for levels with at most 16 boxes per class)
  // rpg: row tiles a wave multiplies each input tile into (more reuse of the inputs, fewer and
  // longer blocks: 4 for the big near-field + M2L launch, 1 for the short dependent passes)
  // prio (per task, may be empty): tasks of higher priority are dispatched first (the dependent
  // chain of a launch ahead of the independent work packed into it); only their blocks decide
  // whether the launch splits every k-range over all 4 waves.  acc (may be null): split-K
  // reduction descriptors collected over several passes; with flush = false this pass adds its
  // own to them (no reduction after it), with flush = true its reduction launch covers them all.
  // A task's rpg set before the call overrides the phase's.
  // chunk (may be empty): per task (index, count) — the task covers that share of its level's
  // box blocks (count > 1: no split K, its partial planes would cover the whole level).
  auto make_phase_mfma = [&](Phase& ph, std::vector<lsk::DTask>& tasks, std::vector<lsk::DTerm>& terms, int rpg,
                             const std::vector<int>& prio = {}, std::vector<lsk::SplitK>* acc = nullptr,
                             long long* acc_elems = nullptr, bool flush = false,
                             const std::vector<std::array<int, 2>>& chunk = {}) {
    std::vector<int> blk;
    std::vector<int> want(tasks.size());
    const int top_prio = prio.empty() ? 0 : *std::max_element(prio.begin(), prio.end());
    auto lead = [&](size_t t) { return prio.empty() || prio[t] == top_prio; };
    for (size_t t = 0; t < tasks.size(); ++t) want[t] = tasks[t].io ? 1 : (tasks[t].rpg > 0 ? tasks[t].rpg : rpg);
    // a pass whose leading tasks would fill fewer than two workgroups per CU splits their
    // k-ranges over all 4 waves (4x the workgroups, shorter dependent chains)
    for (int pass = 0; pass < 2; ++pass) {
      blk.clear();
      size_t nlead = 0;
      for (size_t t = 0; t < tasks.size(); ++t) {
        lsk::DTask& tk = tasks[t];
        int kb = 0;
        for (int q = tk.t0; q < tk.t1; ++q) {
          terms[q].kbase = kb;
          kb += (terms[q].K + 3) / 4;
        }
        tk.ktot = kb;
        tk.Mpad = round_up(std::max(tk.M, 1), lsk::kRowBlock);
        const int mt = std::min(want[t], (tk.M + 15) / 16);
        tk.rpg = std::max(mt, 1);
        tk.nrb = ((tk.M + 15) / 16 + tk.rpg - 1) / tk.rpg;  // row groups of rpg tiles
        const int nbox = tk.nh * tk.nh;
        // waves that split the k-blocks of a tile: enough that one wave chains at most kMaxChain
        // tile-k-blocks (k-blocks times row tiles)
        const long long chain = (long long)kb * mt;
        // a chunk is filler work next to a dependent chain: short blocks, every k-range split
        // over the 4 waves
        const bool chunked = !chunk.empty() && chunk[t][1] > 1;
        tk.kps = ((pass == 1 && lead(t)) || chunked || nbox <= 16 || chain > 2 * kMaxChain)
                     ? 4
                     : (chain > kMaxChain ? 2 : 1);
        const int per = 16 * (4 / tk.kps);
        tk.nbb = (nbox + per - 1) / per;
        tk.bb0 = 0;
        if (chunked) {
          const int nb = tk.nbb, ci = chunk[t][0], nc = chunk[t][1];
          tk.bb0 = (int)((long long)nb * ci / nc);
          tk.nbb = (int)((long long)nb * (ci + 1) / nc) - tk.bb0;
        }
        // beyond that, workgroups split K (one launch per pass only; the fused launch keeps 1,
        // and so does a chain task whose reduction would be deferred past the next pass)
        tk.kgroups = 1;
        const bool deferred_chain = acc && !flush && !prio.empty() && prio[t] > 0;
        if (!P->opt.fmm_fused && !deferred_chain && !chunked && !tk.io && chain > 4 * kMaxChain)
          tk.kgroups = (int)std::min<long long>(kb, (chain + 4 * kMaxChain - 1) / (4 * kMaxChain));
        tk.blk0 = (int)blk.size();
        for (int i = 0; i < tk.nbb * tk.nrb * tk.kgroups; ++i) blk.push_back((int)t);
        if (lead(t)) nlead += (size_t)tk.nbb * tk.nrb * tk.kgroups;
      }
      if (nlead >= 512) break;
    }
    // k-block descriptors: per task, its terms' 4-deep k-blocks in term order, each with the
    // address of its operator rows and of its inputs (class plane of the term included), the
    // term's box shift and its real depth
    {
      std::vector<lsk::KBlk> kbl;
      std::vector<long long> kb0(tasks.size(), 0);
      for (size_t t = 0; t < tasks.size(); ++t) {
        lsk::DTask& tk = tasks[t];
        kb0[t] = (long long)kbl.size();
        tk.mode = tk.t1 > tk.t0 ? terms[tk.t0].mode : lsk::MODE_SAME;
        tk.nh_in = tk.t1 > tk.t0 ? terms[tk.t0].nh_in : tk.nh;
        tk.in_rhs = tk.t1 > tk.t0 ? terms[tk.t0].in_rhs : 0;
        tk.pks = 4LL * tk.nh_in * tk.nh_in;
        tk.coh_in = tk.t1 > tk.t0 ? terms[tk.t0].coh : 0;
        for (int q = tk.t0; q < tk.t1; ++q) {
          const lsk::DTerm& tm = terms[q];
          if (tm.mode != tk.mode || tm.nh_in != tk.nh_in || tm.in_rhs != tk.in_rhs || tm.coh != tk.coh_in)
            throw LsError(LS_EINVAL, "internal: the terms of a task differ in mode or input level");
          const long long plane = (long long)tm.nh_in * tm.nh_in;
          const long long cin = (tm.mode == lsk::MODE_SHIFT || tm.mode == lsk::MODE_CHILD) ? tm.cin : 0;
          for (int kk = 0; kk < (tm.K + 3) / 4; ++kk) {
            lsk::KBlk d{};
            d.op = (unsigned long long)((const char*)tm.op + (long long)4 * kk * tk.Mpad * F.esz);
            d.in = (unsigned long long)((const char*)tm.in + (4LL * kk * tk.pks + cin * plane) * F.esz);
            // the box shift of a shifted term; zero for every other mode (the kernel adds it
            // unconditionally)
            d.sha = tm.mode == lsk::MODE_SHIFT ? tm.sha : 0;
            d.shb = tm.mode == lsk::MODE_SHIFT ? tm.shb : 0;
            d.klim = std::min(4, tm.K - 4 * kk);
            kbl.push_back(d);
          }
        }
        if ((long long)kbl.size() - kb0[t] != tk.ktot) throw LsError(LS_EINVAL, "internal: k-block count");
      }
      ph.kbl.upload(kbl);
      for (size_t t = 0; t < tasks.size(); ++t) tasks[t].kb = ph.kbl.as<lsk::KBlk>() + kb0[t];
    }
    // split-K partial planes [rhs][g][m][box] per task, and the descriptors of their reduction
    {
      long long pe = 0;
      for (auto& tk : tasks)
        if (tk.kgroups > 1) {
          tk.part_rhs = (long long)tk.kgroups * tk.M * tk.nh * tk.nh;
          pe += tk.part_rhs * F.nrhs_cap;
        }
      ph.part.alloc((size_t)std::max(pe, 1LL) * F.esz);
      long long po = 0;
      std::vector<lsk::SplitK> sk;
      ph.sk_elems = 0;
      long long elems = 0;
      for (auto& tk : tasks)
        if (tk.kgroups > 1) {
          tk.part = ph.part.as<char>() + po * F.esz;
          po += tk.part_rhs * F.nrhs_cap;
          lsk::SplitK d{};
          d.part = tk.part;
          d.out = tk.out;
          d.part_rhs = tk.part_rhs;
          d.out_rhs = tk.out_rhs;
          d.M = tk.M;
          d.nbox = tk.nh * tk.nh;
          d.cout = tk.cout;
          d.G = tk.kgroups;
          d.beta = tk.beta;
          sk.push_back(d);
          elems = std::max(elems, (long long)tk.M * tk.nh * tk.nh);
        }
      if (acc) {
        acc->insert(acc->end(), sk.begin(), sk.end());
        *acc_elems = std::max(*acc_elems, elems);
        if (flush) {
          sk = *acc;
          elems = *acc_elems;
        }
      }
      if (!acc || flush) {
        ph.sk_elems = elems;
        ph.sk.upload(sk);
        ph.nsk = (int)sk.size();
      }
    }
    // dispatch order: blocks with the most k-blocks per wave first (the long ones start early
    // instead of forming the tail); entries are (task, block within the task) pairs
    std::vector<std::array<int, 4>> order;  // priority, work, task, local
    for (size_t q = 0; q < blk.size(); ++q) {
      const lsk::DTask& tk = tasks[blk[q]];
      const int per_wave = (tk.ktot * tk.rpg + tk.kgroups * tk.kps - 1) / (tk.kgroups * tk.kps);
      order.push_back({prio.empty() ? 0 : prio[blk[q]], per_wave, blk[q], (int)q - tk.blk0});
    }
    std::stable_sort(order.begin(), order.end(),
                     [](const auto& a, const auto& b) { return a[0] != b[0] ? a[0] > b[0] : a[1] > b[1]; });
    std::vector<int> pairs;
    for (const auto& o : order) {
      pairs.push_back(o[2]);
      pairs.push_back(o[3]);
    }
    ph.tasks.upload(tasks);
    ph.terms.upload(terms);
    ph.blk.upload(pairs);
    ph.nblocks = (int)blk.size();
    ph.ntasks = (int)tasks.size();
    ph.mfma = true;
    hps.push_back({tasks, terms, pairs});
  };
  auto mk_phase = [&](Phase& ph, std::vector<lsk::DTask>& tasks, std::vector<lsk::DTerm>& terms, int rpg = 1) {
    if (P->opt.stencil_mfma)
      make_phase_mfma(ph, tasks, terms, rpg);
    else
      make_phase(ph, tasks, terms);
  };
  auto shift_term = [&](int c, Off d, int nh_in) {
    lsk::DTerm tm{};
    int ca = c >> 1, cb = c & 1;
    int xa = ca + d.a, xb = cb + d.b;
    tm.mode = lsk::MODE_SHIFT;
    tm.cin = ((xa & 1) << 1) | (xb & 1);
    tm.sha = (xa >= 0) ? xa / 2 : -((-xa + 1) / 2);
    tm.shb = (xb >= 0) ? xb / 2 : -((-xb + 1) / 2);
    tm.nh_in = nh_in;
    return tm;
  };
  const int nhL = p.lv[leaf].nb / 2;
  // A group of tasks of one kind (near field of one class, M2L of one level, P2M, M2M of one
  // level) and the complex multiply-adds it applies per product and right-hand side.
  struct Group {
    std::vector<lsk::DTask> tasks;
    std::vector<lsk::DTerm> terms;
    double work = 0;
  };
  // in-domain (box, term) pairs of a term times its operator size
  auto term_work = [](const lsk::DTask& tk, const lsk::DTerm& tm) {
    long long ca = tk.nh, cb = tk.nh;
    if (tm.mode == lsk::MODE_SHIFT) {
      ca = cb = 0;
      for (int h = 0; h < tk.nh; ++h) {
        ca += (h + tm.sha >= 0 && h + tm.sha < tm.nh_in);
        cb += (h + tm.shb >= 0 && h + tm.shb < tm.nh_in);
      }
    }
    return (double)ca * cb * tk.M * tm.K;
  };
  auto finish = [&](Group& g) {
    g.work = 0;
    for (const lsk::DTask& tk : g.tasks)
      for (int q = tk.t0; q < tk.t1; ++q) g.work += term_work(tk, g.terms[q]);
  };
  // appends a group's tasks (term ranges shifted) with dispatch priority pr, as chunk ci of nc
  // of their box blocks (rpg > 0: row tiles per row group)
  auto append = [](std::vector<lsk::DTask>& tasks, std::vector<lsk::DTerm>& terms, std::vector<int>& prio,
                   std::vector<std::array<int, 2>>& chunk, const Group& g, int pr, int ci = 0, int nc = 1,
                   int rpg = 0) {
    const int off = (int)terms.size();
    for (lsk::DTask tk : g.tasks) {
      tk.t0 += off;
      tk.t1 += off;
      if (rpg > 0) tk.rpg = rpg;
      tasks.push_back(tk);
      prio.push_back(pr);
      chunk.push_back({ci, nc});
    }
    terms.insert(terms.end(), g.terms.begin(), g.terms.end());
  };
  // ---- near field: one group per class (depends only on the gathered input) ----
  std::vector<Group> near_g(4);
  for (int c = 0; c < 4; ++c) {
    Group& g = near_g[c];
    lsk::DTask tk{};
    tk.out = F.ys.p;
    tk.out_rhs = N;
    tk.M = s2;
    tk.nh = nhL;
    tk.cout = c;
    tk.beta = 0;
    tk.rpg = 4;
    set_stage(tk, S_NEAR, -1, -1, -1, p.top <= leaf ? 1 : 0);
    tk.t0 = 0;
    for (int da = -1; da <= 1; ++da)
      for (int db = -1; db <= 1; ++db) {
        lsk::DTerm tm = shift_term(c, {da, db}, nhL);
        tm.op = opp(F.off_near[(da + 1) * 3 + (db + 1)]);
        tm.in = F.xs.p;
        tm.in_rhs = N;
        tm.K = s2;
        g.terms.push_back(tm);
      }
    tk.t1 = (int)g.terms.size();
    g.tasks.push_back(tk);
    finish(g);
  }
  // ---- M2L: one group per level (depends on the multipoles of that level) ----
  std::vector<Group> m2l_g(leaf + 1);
  for (int nu = p.top; nu <= leaf; ++nu) {
    Group& g = m2l_g[nu];
    const ls::Level& l = p.lv[nu];
    int nh = l.nb / 2;
    for (int dir = 0; dir < l.ndir; ++dir) {
      int ad = ls::antipodal(dir, l.ndir);
      // term index lookup for this direction's operator list
      const auto& kofs = (F.fp32 ? P->nca32 : P->nca64).lv[nu].kofs[dir];
      for (int c = 0; c < 4; ++c) {
        lsk::DTask tk{};
        tk.out = lvl_ptr(loc, nu, dir);
        tk.out_rhs = F.ml_rhs;
        tk.M = F.rank[nu][dir];
        tk.nh = nh;
        tk.cout = c;
        tk.beta = 0;
        tk.rpg = 4;
        set_stage(tk, S_M2L(nu), nu == leaf ? S_P2M : S_UP(nu), -1, -1, 1);
        tk.t0 = (int)g.terms.size();
        if (F.rank[nu][ad] > 0)
          for (const Off& d : l.terms[c * l.ndir + dir]) {
            size_t ti = 0;
            while (ti < kofs.size() && !(kofs[ti].a == d.a && kofs[ti].b == d.b)) ++ti;
            if (ti == kofs.size()) throw LsError(LS_EINVAL, "internal: M2L offset missing");
            lsk::DTerm tm = shift_term(c, d, nh);
            tm.op = opp(F.off_K[nu][dir][ti]);
            tm.in = lvl_ptr(mult, nu, ad);
            tm.in_rhs = F.ml_rhs;
            tm.K = F.rank[nu][ad];
            tm.coh = 1;
            g.terms.push_back(tm);
          }
        tk.t1 = (int)g.terms.size();
        if (tk.M > 0) g.tasks.push_back(tk);
      }
    }
    finish(g);
  }
  // ---- the fused launch: every task and term of the phases above, and the queue ----
  auto build_fused = [&]() {
    F.fused = Phase();
    F.nstages = 0;
    // one flag bit per stage (bit 31 marks a wait that ran out): at most 31 stages
    if (!P->opt.stencil_mfma || nst > 31) return;
    std::vector<lsk::DTask> ft;
    std::vector<lsk::DTerm> fm;
    struct Item {
      int task, local, stage;
      double cost;
    };
    std::vector<Item> items;
    for (auto& hp : hps) {
      const int toff = (int)ft.size(), moff = (int)fm.size();
      for (lsk::DTask tk : hp.tasks) {
        tk.t0 += moff;
        tk.t1 += moff;
        ft.push_back(tk);
      }
      fm.insert(fm.end(), hp.terms.begin(), hp.terms.end());
      for (size_t q = 0; q + 1 < hp.pairs.size(); q += 2) {
        const lsk::DTask& tk = hp.tasks[hp.pairs[q]];
        // cost in k-blocks per wave plus a fixed part (waits, term set-up, stores)
        items.push_back({hp.pairs[q] + toff, hp.pairs[q + 1], tk.stage, (double)((tk.ktot + tk.kps - 1) / tk.kps) + 8.0});
      }
    }
    if (items.empty()) return;
    std::vector<std::vector<int>> sitems(nst);
    std::vector<std::array<int, 3>> sdep(nst, std::array<int, 3>{-1, -1, -1});
    for (size_t i = 0; i < items.size(); ++i) sitems[items[i].stage].push_back((int)i);
    for (const lsk::DTask& tk : ft) sdep[tk.stage] = {tk.dep[0], tk.dep[1], tk.dep[2]};
    // list scheduling on W resident workgroups: whenever a workgroup frees up, it takes the next
    // block of the ready stage with the longest remaining chain (a stage is ready once every
    // block of its prerequisites is placed and finished); with none ready, the stage that gets
    // ready first.  Every block thus follows all blocks of its prerequisite stages in the queue.
    const int W = std::max(1, lsk::dafmm_fused_workgroups(F.fp32));
    std::vector<double> span(nst, 0.0), blev(nst, -1.0);
    for (int st = 0; st < nst; ++st) {
      double tot = 0, mx = 0;
      for (int i : sitems[st]) {
        tot += items[i].cost;
        mx = std::max(mx, items[i].cost);
      }
      span[st] = tot / W + mx;
    }
    std::function<double(int)> bl = [&](int st) -> double {
      if (blev[st] >= 0) return blev[st];
      double best = 0;
      for (int u = 0; u < nst; ++u)
        for (int d : sdep[u])
          if (d == st) best = std::max(best, bl(u));
      return blev[st] = span[st] + best;
    };
    for (int st = 0; st < nst; ++st) bl(st);
    std::priority_queue<double, std::vector<double>, std::greater<double>> slots;
    for (int w = 0; w < W; ++w) slots.push(0.0);
    std::vector<size_t> next(nst, 0);
    std::vector<double> done(nst, 0.0);
    auto full = [&](int st) { return next[st] == sitems[st].size(); };
    std::vector<int> order;
    order.reserve(2 * items.size());
    for (size_t placed = 0; placed < items.size(); ++placed) {
      const double t = slots.top();
      slots.pop();
      int pick = -1, wait = -1;
      double wait_t = 0;
      for (int st = 0; st < nst; ++st) {
        if (full(st)) continue;
        bool ok = true;
        double rt = 0;
        for (int d : sdep[st])
          if (d >= 0) {
            if (!full(d)) ok = false;
            rt = std::max(rt, done[d]);
          }
        if (!ok) continue;
        if (rt <= t) {
          if (pick < 0 || blev[st] > blev[pick]) pick = st;
        } else if (wait < 0 || rt < wait_t || (rt == wait_t && blev[st] > blev[wait])) {
          wait = st;
          wait_t = rt;
        }
      }
      if (pick < 0) pick = wait;
      if (pick < 0) throw LsError(LS_EINVAL, "internal: fused DAFMM schedule has no eligible stage");
      double rt = 0;
      for (int d : sdep[pick])
        if (d >= 0) rt = std::max(rt, done[d]);
      const Item& it = items[sitems[pick][next[pick]++]];
      const double fin = std::max(t, rt) + it.cost;
      done[pick] = std::max(done[pick], fin);
      slots.push(fin);
      order.push_back(it.task);
      order.push_back(it.local);
    }
    std::vector<unsigned> need(nst, 0);
    for (int st = 0; st < nst; ++st) need[st] = (unsigned)sitems[st].size();
    // the property every wait relies on: all blocks of a block's prerequisite stages come earlier
    {
      std::vector<unsigned> seen(nst, 0);
      for (size_t q = 0; q < order.size(); q += 2) {
        const lsk::DTask& tk = ft[order[q]];
        for (int d : tk.dep)
          if (d >= 0 && (d >= nst || seen[d] != need[d]))
            throw LsError(LS_EINVAL, "internal: fused DAFMM queue is not in dependency order");
        seen[tk.stage]++;
      }
    }
    F.fused.tasks.upload(ft);
    F.fused.terms.upload(fm);
    F.fused.blk.upload(order);
    F.fused.nblocks = (int)items.size();
    F.fused.ntasks = (int)ft.size();
    F.fused.mfma = true;
    F.fneed.upload(need);
    const size_t cbytes = (size_t)lsk::dafmm_fused_counter_lines(nst) * 128;
    F.fctr.alloc(cbytes);
    hip_check(hipMemset(F.fctr.p, 0, cbytes), "memset");
    F.nstages = nst;
    F.fused_wg = W;
  };
  if (p.top > leaf) {
    // no far field: the near field is the whole product
    F.io_fold = false;
    std::vector<lsk::DTask> tasks;
    std::vector<lsk::DTerm> terms;
    std::vector<int> prio;
    std::vector<std::array<int, 2>> chunk;
    for (const Group& g : near_g) append(tasks, terms, prio, chunk, g, 0);
    mk_phase(F.nearm2l, tasks, terms, 4);
    F.nearm2l.tag = 0;
    F.entries_mid = 0;
    for (const Group& g : near_g) F.entries_mid += g.work;
    build_fused();
    return;
  }
  // ---- P2M ----
  F.io_fold = P->opt.stencil_mfma && !P->opt.fmm_fused;
  Group p2m_g;
  for (int c = 0; c < 4; ++c) {
    lsk::DTask tk{};
    tk.io = F.io_fold ? lsk::IO_GATHER : 0;
    tk.out = lvl_ptr(mult, leaf, 0);
    tk.out_rhs = F.ml_rhs;
    tk.M = F.kleaf;
    tk.nh = nhL;
    tk.cout = c;
    tk.beta = 0;
    set_stage(tk, S_P2M, -1, -1, -1, 1);
    tk.t0 = (int)p2m_g.terms.size();
    lsk::DTerm tm{};
    tm.mode = lsk::MODE_SAME;
    tm.op = opp(F.off_U);
    tm.in = F.xs.p;
    tm.in_rhs = N;
    tm.K = s2;
    tm.nh_in = nhL;
    p2m_g.terms.push_back(tm);
    tk.t1 = (int)p2m_g.terms.size();
    p2m_g.tasks.push_back(tk);
  }
  // ---- M2M (parent nu from children nu+1) ----
  std::vector<Group> m2m_g(leaf + 1);
  for (int nu = leaf - 1; nu >= p.top; --nu) {
    Group& g = m2m_g[nu];
    const ls::Level& l = p.lv[nu];
    const ls::Level& cl = p.lv[nu + 1];
    int nh = l.nb / 2;
    for (int dir = 0; dir < l.ndir; ++dir) {
      int cd = cl.hf ? dir / 2 : 0;
      for (int c = 0; c < 4; ++c) {
        lsk::DTask tk{};
        tk.out = lvl_ptr(mult, nu, dir);
        tk.out_rhs = F.ml_rhs;
        tk.M = F.rank[nu][dir];
        tk.nh = nh;
        tk.cout = c;
        tk.beta = 0;
        set_stage(tk, S_UP(nu), nu == leaf - 1 ? S_P2M : S_UP(nu + 1), -1, -1, 1);
        tk.t0 = (int)g.terms.size();
        for (int cc = 0; cc < 4; ++cc) {
          lsk::DTerm tm{};
          tm.mode = lsk::MODE_CHILD;
          tm.cin = cc;
          tm.op = opp(F.off_C[nu][dir][cc]);
          tm.in = lvl_ptr(mult, nu + 1, cd);
          tm.in_rhs = F.ml_rhs;
          tm.coh = 1;
          tm.K = F.rank[nu + 1][cd];
          tm.nh_in = cl.nb / 2;
          if (tm.K > 0) g.terms.push_back(tm);
        }
        tk.t1 = (int)g.terms.size();
        if (tk.M > 0) g.tasks.push_back(tk);
      }
    }
  }
  // ---- launches up to the middle one: U_0 = P2M, U_j = M2M of level leaf - j (j = 1..nup),
  // U_{nup+1} = the middle launch.  Independent work is packed into the upward launches, whose
  // own dependent chain leaves most of the chip idle: the near field (it needs only the
  // gathered input) in kNearChunks chunks of box blocks per class, spread over U_0..U_nup, in
  // short blocks (one row tile each, no split K); with kPackM2L also the M2L of level nu, which
  // needs the multipoles of nu, in the launch after the one that completes them.  What is not
  // packed forms the middle launch (M2L of the top level at least).  The chain's blocks are
  // dispatched first, and the split-K reductions of all packed work run once, after the middle
  // launch (nothing reads those outputs before the downward pass).  Without the matrix-core form
  // (or in the fused launch) the near field and every M2L form the middle launch.
  F.up.clear();
  F.up.resize(leaf - p.top);
  {
    // measured on the 512^2 disc at kappa 80: packing the near field (4, 8 or 16 chunks per
    // class, one or four row tiles per block) or also the M2L made the FP64 product 7-40% and
    // the FP32 one 15-50% slower than one middle launch with all of it, so both are off
    constexpr int kNearChunks = 0;
    constexpr bool kPackM2L = false;
    constexpr int kFillRpg = 1;
    const bool pack = P->opt.stencil_mfma && !P->opt.fmm_fused;
    const int nU = nup + 1;
    struct Fill {
      const Group* g;
      int ci, nc, rpg;
    };
    std::vector<std::vector<Fill>> fill(nU + 1);
    std::vector<double> load(nU + 1, 0.0);
    for (int nu = p.top; nu <= leaf; ++nu) {
      const int u = (pack && kPackM2L) ? leaf - nu + 1 : nU;
      fill[u].push_back({&m2l_g[nu], 0, 1, 0});
      load[u] += m2l_g[nu].work;
    }
    for (int c = 0; c < 4; ++c) {
      if (pack && kNearChunks > 0) {
        for (int k = 0; k < kNearChunks; ++k) {
          const int u = (int)((long long)k * nU / kNearChunks);
          fill[u].push_back({&near_g[c], k, kNearChunks, kFillRpg});
          load[u] += near_g[c].work / kNearChunks;
        }
      } else {
        fill[nU].push_back({&near_g[c], 0, 1, 0});
        load[nU] += near_g[c].work;
      }
    }
    std::vector<lsk::SplitK> acc;
    long long acc_elems = 0;
    for (int u = 0; u <= nU; ++u) {
      std::vector<lsk::DTask> tasks;
      std::vector<lsk::DTerm> terms;
      std::vector<int> prio;
      std::vector<std::array<int, 2>> chunk;
      if (u == 0) append(tasks, terms, prio, chunk, p2m_g, 1);
      if (u >= 1 && u < nU) append(tasks, terms, prio, chunk, m2m_g[leaf - u], 1);
      for (const Fill& f : fill[u]) append(tasks, terms, prio, chunk, *f.g, 0, f.ci, f.nc, f.rpg);
      Phase& ph = u == 0 ? F.p2m : (u < nU ? F.up[u - 1] : F.nearm2l);
      if (P->opt.stencil_mfma)
        make_phase_mfma(ph, tasks, terms, u == nU ? 4 : 1, prio, &acc, &acc_elems, u == nU, chunk);
      else
        make_phase(ph, tasks, terms);
      ph.tag = u == 0 ? 1 : (u < nU ? 2 : 0);
    }
    // middle-launch work: chunk shares of a class are counted by box blocks, near enough for a
    // rate (the classes have equal box counts up to the domain edge)
    F.entries_mid = load[nU];
  }
  // ---- L2P (accumulates onto the near field) ----
  {
    std::vector<lsk::DTask> tasks;
    std::vector<lsk::DTerm> terms;
    for (int c = 0; c < 4; ++c) {
      lsk::DTask tk{};
      tk.out = F.ys.p;
      tk.out_rhs = N;
      tk.M = s2;
      tk.nh = nhL;
      tk.cout = c;
      tk.beta = 1;
      tk.io = F.io_fold ? lsk::IO_EPILOGUE : 0;
      set_stage(tk, S_L2P, nup > 0 ? S_DOWN(leaf - 1) : -1, S_M2L(leaf), S_NEAR, 0);
      tk.t0 = (int)terms.size();
      lsk::DTerm tm{};
      tm.mode = lsk::MODE_SAME;
      tm.op = opp(F.off_Ut);
      tm.in = lvl_ptr(loc, leaf, 0);
      tm.in_rhs = F.ml_rhs;
      tm.K = F.kleaf;
      tm.coh = 1;
      tm.nh_in = nhL;
      terms.push_back(tm);
      tk.t1 = (int)terms.size();
      tasks.push_back(tk);
    }
    mk_phase(F.l2p, tasks, terms);
    F.l2p.tag = 4;
  }
  // ---- L2L (parent nu -> children nu+1), top first ----
  F.down.clear();
  F.down.resize(leaf - p.top);
  for (int nu = p.top; nu < leaf; ++nu) {
    const ls::Level& l = p.lv[nu];
    const ls::Level& cl = p.lv[nu + 1];
    std::vector<lsk::DTask> tasks;
    std::vector<lsk::DTerm> terms;
    int nhc = cl.nb / 2;
    for (int cdir = 0; cdir < cl.ndir; ++cdir) {
      for (int c = 0; c < 4; ++c) {
        lsk::DTask tk{};
        tk.out = lvl_ptr(loc, nu + 1, cdir);
        tk.out_rhs = F.ml_rhs;
        tk.M = F.rank[nu + 1][cdir];
        tk.nh = nhc;
        tk.cout = c;
        tk.beta = 1;
        set_stage(tk, S_DOWN(nu), S_M2L(nu), S_M2L(nu + 1), nu > p.top ? S_DOWN(nu - 1) : -1, 1);
        tk.t0 = (int)terms.size();
        for (int dir = 0; dir < l.ndir; ++dir) {
          int cd = cl.hf ? dir / 2 : 0;
          if (cd != cdir) continue;
          lsk::DTerm tm{};
          tm.mode = lsk::MODE_PARENT;
          tm.op = opp(F.off_Ct[nu][dir][c]);
          tm.in = lvl_ptr(loc, nu, dir);
          tm.in_rhs = F.ml_rhs;
          tm.coh = 1;
          tm.K = F.rank[nu][dir];
          tm.nh_in = l.nb / 2;
          if (tm.K > 0) terms.push_back(tm);
        }
        tk.t1 = (int)terms.size();
        if (tk.M > 0) tasks.push_back(tk);
      }
    }
    mk_phase(F.down[nu - p.top], tasks, terms);
    F.down[nu - p.top].tag = 3;
  }
  build_fused();
}

void ensure_fmm_capacity(ls_problem* P, FmmDev& F, int nrhs) {
  if (F.nrhs_cap >= nrhs) return;
  const ls::Plan& p = P->plan;
  int cap = std::max(nrhs, 1);
  F.lvl_off.assign(p.leaf + 1, 0);
  F.lvl_size.assign(p.leaf + 1, 0);
  long long tot = 0;
  if (p.top <= p.leaf)
    for (int nu = p.top; nu <= p.leaf; ++nu) {
      long long nh = p.lv[nu].nb / 2;
      F.lvl_off[nu] = tot;
      F.lvl_size[nu] = (long long)p.lv[nu].ndir * F.kmax[nu] * 4 * nh * nh;
      tot += F.lvl_size[nu];
    }
  F.ml_rhs = std::max(tot, 1LL);
  F.mult.alloc((size_t)F.ml_rhs * cap * F.esz);
  F.loc.alloc((size_t)F.ml_rhs * cap * F.esz);
  F.xs.alloc((size_t)P->N * cap * F.esz);
  F.ys.alloc((size_t)P->N * cap * F.esz);
  F.nrhs_cap = cap;
  build_phases(P, F);
}

void run_phase(ls_problem* P, FmmDev& F, Phase& ph, int nrhs, hipStream_t s, int prof_cls = -1,
               const lsk::IoArgs* io = nullptr) {
  if (ph.nblocks == 0 && ph.nsk == 0) return;
  if (ph.mfma) {
    if (prof_cls >= 0) {
      ProfScope ps(P, prof_cls, s);
      lsk::launch_stencil_mfma(F.fp32, ph.tasks.as<lsk::DTask>(), ph.terms.as<lsk::DTerm>(), ph.blk.as<int>(),
                               ph.nblocks, nrhs, s, io);
    } else {
      lsk::launch_stencil_mfma(F.fp32, ph.tasks.as<lsk::DTask>(), ph.terms.as<lsk::DTerm>(), ph.blk.as<int>(),
                               ph.nblocks, nrhs, s, io);
    }
    lsk::launch_splitk_reduce(F.fp32, ph.sk.as<lsk::SplitK>(), ph.nsk, ph.sk_elems, nrhs, s);
    return;
  }
  if (prof_cls >= 0) {
    ProfScope ps(P, prof_cls, s);
    lsk::launch_stencil(ph.tag, F.fp32, ph.tasks.as<lsk::DTask>(), ph.terms.as<lsk::DTerm>(), ph.blk.as<int>(),
                        ph.nblocks, nrhs, s);
  } else {
    lsk::launch_stencil(ph.tag, F.fp32, ph.tasks.as<lsk::DTask>(), ph.terms.as<lsk::DTerm>(), ph.blk.as<int>(),
                        ph.nblocks, nrhs, s);
  }
}

// y = alpha x + coef diag(q) (V x) in Morton (mode 0) or caller (mode 1) order.
// y = alpha x + coef diag(q) (V x) in Morton (mode 0) or caller (mode 1) order; with_q = false:
// y = alpha x + coef (V x).
void fmm_apply(ls_problem* P, bool fp32, const double2* x, long long ldx, double2* y, long long ldy, int nrhs,
               double alpha, double coef, bool caller_order, hipStream_t s, bool with_q = true) {
  FmmDev& F = fp32 ? P->f32 : P->f64;
  if (fp32 && !P->have32) throw LsError(LS_ENOTSUP, "FP32 operator was not built (build_fp32 = 0)");
  ensure_fmm_capacity(P, F, nrhs);
  const long long N = P->N;
  const int* gidx = caller_order ? P->s2c.as<int>() : P->s2m.as<int>();
  const int* eidx = caller_order ? P->c2s.as<int>() : P->m2s.as<int>();
  const double* q = !with_q ? nullptr : (caller_order ? P->q_c.as<double>() : P->q_m.as<double>());
  if (P->opt.fmm_fused && F.fused.nblocks > 0) {
    // every pass in one persistent launch between the gather (which also zeroes its counters)
    // and the epilogue
    unsigned* ctr = F.fctr.as<unsigned>();
    const int lines = lsk::dafmm_fused_counter_lines(F.nstages);
    const unsigned* err = ctr + 32 * (1 + F.nstages);  // first group flag word (bit 31: a wait ran out)
    lsk::launch_gather_zero(fp32, x, ldx, F.xs.p, gidx, N, nrhs, ctr, lines, s);
    {
      ProfScope ps(P, fp32 ? 9 : 8, s);
      lsk::launch_dafmm_fused(fp32, F.fused.tasks.as<lsk::DTask>(), F.fused.terms.as<lsk::DTerm>(),
                              F.fused.blk.as<int>(), F.fused.nblocks, nrhs, F.nstages, ctr, F.fneed.as<unsigned>(),
                              F.fused_wg, s);
    }
    lsk::launch_epilogue_checked(fp32, x, ldx, F.ys.p, eidx, q, alpha, coef, y, ldy, N, nrhs, err, s);
    hip_check(hipGetLastError(), "fused fmm kernels");
    return;
  }
  const int span = kProfSpan + (fp32 ? 5 : 0);
  const ls::Plan& p = P->plan;
  // with io_fold the gather is P2M's and the epilogue L2P's (their spans stay empty)
  const bool fold = F.io_fold && p.top <= p.leaf;
  lsk::IoArgs io{x, ldx, y, ldy, gidx, q, alpha, coef, F.xs.p, F.ys.p};
  {
    SpanScope sp(P, span + 0, s);
    if (!fold) lsk::launch_gather(fp32, x, ldx, F.xs.p, gidx, N, nrhs, s);
  }
  if (p.top <= p.leaf) {
    SpanScope sp(P, span + 1, s);
    run_phase(P, F, F.p2m, nrhs, s, -1, fold ? &io : nullptr);
    for (auto& ph : F.up) run_phase(P, F, ph, nrhs, s);
  }
  {
    SpanScope sp(P, span + 2, s);
    run_phase(P, F, F.nearm2l, nrhs, s, fp32 ? 4 : 0);
  }
  if (p.top <= p.leaf) {
    SpanScope sp(P, span + 3, s);
    for (auto& ph : F.down) run_phase(P, F, ph, nrhs, s);
    run_phase(P, F, F.l2p, nrhs, s, -1, fold ? &io : nullptr);
  }
  {
    SpanScope sp(P, span + 4, s);
    if (!fold) lsk::launch_epilogue(fp32, x, ldx, F.ys.p, eidx, q, alpha, coef, y, ldy, N, nrhs, s);
  }
  hip_check(hipGetLastError(), "fmm kernels");
}

// ---------------------------------------------------------------------------------------
// HODLR
// ---------------------------------------------------------------------------------------
void hodlr_ws_elems(const HodlrDev& H, size_t* np, size_t* ns);

void hodlr_ensure_ws(ls_problem* P, int nrhs) {
  HodlrDev& H = P->hod;
  size_t needp = 0, needs = 0;
  hodlr_ws_elems(H, &needp, &needs);
  H.partial.ensure(needp * nrhs * 16);
  H.svec.ensure(needs * nrhs * 16);
}

// z = (partial) HODLR inverse applied to b (Morton order): leaf solves, then levels
// Lb-1 .. lstop.  b and z may be the same buffer.
// jdev != NULL: b is column *jdev of a basis (b + *jdev * bldj); zcopy != NULL: the result is
// also stored in column *jdev of zcopy (ld per right-hand side zldr, per column zldj)
// Workspaces of one apply: the chunk partials of W^T z and the s vectors of the SMW cores.
struct HodlrWs {
  double2* partial = nullptr;
  double2* svec = nullptr;
  bool timers = true;  // sampled kernel timers may create events
};

// complex entries of the chunk partials and of the s vectors one right-hand side needs
void hodlr_ws_elems(const HodlrDev& H, size_t* np, size_t* ns) {
  size_t needp = 0, needs = 0;
  for (int l = 0; l < H.Lb; ++l) {
    needp = std::max(needp, (size_t)H.nchunks[l] * H.rank[l]);
    needs = std::max(needs, (size_t)(1LL << l) * 2 * H.rank[l]);
  }
  *np = std::max<size_t>(needp, 1);
  *ns = std::max<size_t>(needs, 1);
}

void hodlr_apply(ls_problem* P, int fmt, const double2* b, long long ldb, double2* z, long long ldz, int nrhs,
                 int lstop, hipStream_t s, const int* jdev = nullptr, long long bldj = 0, double2* zcopy = nullptr,
                 long long zldr = 0, long long zldj = 0, const HodlrWs* ws = nullptr) {
  HodlrDev& H = P->hod;
  if (!ws) hodlr_ensure_ws(P, nrhs);
  double2* const partial = ws ? ws->partial : H.partial.as<double2>();
  double2* const svec = ws ? ws->svec : H.svec.as<double2>();
  const bool tm = ws ? ws->timers : true;
  {
    ProfScope ps(P, 2, s, tm);
    // leaf inverses in complex128, or in the factors' precision on request
    const int lf = P->opt.pc_lowp_solves ? fmt : 0;
    const void* D = lf == 2 && H.Dinv16.p ? H.Dinv16.p : (lf >= 1 && H.Dinv32.p ? H.Dinv32.p : H.Dinv.p);
    const int df = D == H.Dinv16.p ? 2 : (D == H.Dinv32.p ? 1 : 0);
    lsk::launch_leaf_apply(df, D, H.ident.as<unsigned char>(), b, ldb, z, ldz, H.lp, H.nleaves, nrhs, s, jdev,
                           bldj);
  }
  // level by level: dot (W^T z), core solve, update (z -= Y s).  With complex bfloat16
  // factors and one right-hand side, an update and the next level's dot share one launch
  // where the next level's chunks are 1024 rows.
  int pend = -1;  // level whose update is still to be applied
  bool copied = false;
  auto update = [&](int a, bool last) {
    const void* Y = fmt == 2 ? H.Y16[a].p : (fmt == 1 ? H.Y32[a].p : H.Y64[a].p);
    ProfScope ps(P, 1, s, tm, a);
    // the listed update also for the last level when z~ is stored: the copy follows in its own
    // launch (the wide kernel's one-wave-per-SIMD column loop is the slower of the two there)
    if (H.sparse && nrhs == 1 && fmt >= 1) {
      lsk::launch_hodlr_update_list(fmt, Y, svec, z, H.N, H.rank[a], H.N >> a, H.alist.as<int>(),
                                    H.nact, s);
      copied = false;
      return;
    }
    copied = lsk::launch_hodlr_update(fmt, Y, svec, z, ldz, H.N, H.rank[a], H.N >> a, 1 << a, nrhs,
                                      s, last ? zcopy : nullptr, zldr, jdev, zldj, H.ract.as<unsigned char>());
  };
  for (int l = H.Lb - 1; l >= lstop; --l) {
    const void* W = fmt == 2 ? H.W16[l].p : (fmt == 1 ? H.W32[l].p : H.W64[l].p);
    int nodes = 1 << l;
    const int rl = H.rank[l];
    if (rl == 0) continue;
    // activity of the level's children (after setup): chunks and core rows that meet a zero Y are skipped
    const unsigned char* cact = H.nodeact.p ? H.nodeact.as<unsigned char>() + (2LL << l) : nullptr;
    if (pend >= 0 && fmt == 2 && nrhs == 1 && !H.sparse && lsk::hodlr_upd_dot_ok(H.N, H.N >> pend, H.chunk[l])) {
      ProfScope pf(P, 6, s, tm, l);
      lsk::launch_hodlr_upd_dot(H.Y16[pend].p, H.rank[pend], svec, H.N >> pend, 1 << pend, W, rl, z,
                                H.N, partial, H.chunk[l], s, H.ract.as<unsigned char>());
    } else {
      if (pend >= 0) update(pend, false);
      ProfScope pd(P, 5, s, tm, l);
      lsk::launch_hodlr_dot(fmt, W, z, ldz, partial, H.N, rl, H.chunk[l], H.nchunks[l], nrhs, s,
                            cact ? H.dlist.as<int>() + H.doff[l] : nullptr, cact ? H.dcnt[l] : 0, H.cpc[l]);
    }
    pend = -1;
    // core inverses in complex128, or in the factors' precision on request
    const int cf = P->opt.pc_lowp_solves ? fmt : 0;
    const void* C = cf == 2 ? H.core16[l].p : (cf == 1 ? H.core32[l].p : H.coreinv[l].p);
    {
      ProfScope pc(P, 7, s, tm, l);
      lsk::launch_hodlr_core(cf, C, partial, svec, rl, nodes, H.cpc[l], H.nchunks[l],
                             true, nrhs, s, cact);
    }
    pend = l;
  }
  if (pend >= 0) update(pend, true);
  if (zcopy && !copied) lsk::launch_kd_copy(z, ldz, 0, zcopy, zldr, zldj, H.N, jdev, nullptr, nrhs, s);
  hip_check(hipGetLastError(), "hodlr kernels");
}

// chunking of the binary levels for the W^T z reductions: chunks tile every child block
// exactly and hold at most max_rows rows where the block size allows
void hodlr_chunks(HodlrDev& H, long long max_rows) {
  const long long N = H.N;
  H.chunk.assign(H.Lb, 0);
  H.nchunks.assign(H.Lb, 0);
  H.cpc.assign(H.Lb, 0);
  for (int l = 0; l < H.Lb; ++l) {
    long long cs = N >> (l + 1);
    long long ch = cs;
    while (ch > max_rows && ch % 2 == 0) ch /= 2;
    H.chunk[l] = ch;
    H.nchunks[l] = (int)(N / ch);
    H.cpc[l] = (int)(cs / ch);
  }
}

void build_hodlr(ls_problem* P, const ls::WTable& W, const std::vector<int>& mort_a, const std::vector<int>& mort_b,
                 const std::vector<double>& qm) {
  HodlrDev& H = P->hod;
  const ls::Plan& p = P->plan;
  const long long N = P->N;
  const int r = P->opt.hodlr_rank;
  H.r = r;
  H.lp = p.leaf_side * p.leaf_side;
  H.nleaves = (int)(N / H.lp);
  H.Lb = 2 * p.leaf;
  H.N = N;
  const double coef = P->coef;
  // leaf inverses (column-major per leaf), on the device: dense leaves by Gauss-Jordan, leaves
  // without contrast the identity
  const int lp = H.lp;
  DevBuf wdev, mad, mbd;
  wdev.upload(W.w);
  mad.upload(mort_a);
  mbd.upload(mort_b);
  {
    std::vector<int> dense, idl;
    for (int leafi = 0; leafi < H.nleaves; ++leafi) {
      bool allzero = true;
      for (int m = 0; m < lp; ++m)
        if (qm[(size_t)leafi * lp + m] != 0.0) allzero = false;
      (allzero ? idl : dense).push_back(leafi);
    }
    std::vector<unsigned char> ident(H.nleaves, 0);
    for (int leafi : idl) ident[leafi] = 1;
    H.Dinv.alloc((size_t)H.nleaves * lp * lp * 16);
    DevBuf dl, il, lA, lB, lbad;
    dl.upload(dense);
    il.upload(idl);
    lsk::launch_leaf_identity(il.as<int>(), (int)idl.size(), lp, H.Dinv.as<double2>(), nullptr);
    const int batch = (int)std::min<size_t>(std::max<size_t>(dense.size(), 1), 1024);
    lA.alloc((size_t)batch * lp * lp * 16);
    lB.alloc((size_t)batch * lp * lp * 16);
    lbad.alloc((size_t)batch * 4);
    std::vector<int> bad(batch);
    for (size_t k0 = 0; k0 < dense.size(); k0 += batch) {
      const int nk = (int)std::min<size_t>(batch, dense.size() - k0);
      hip_check(hipMemsetAsync(lbad.p, 0, (size_t)nk * 4, nullptr), "memset");
      lsk::launch_leaf_invert(wdev.as<double2>(), P->n, mad.as<int>(), mbd.as<int>(), P->q_m.as<double>(), coef, lp,
                              dl.as<int>() + k0, nk, lA.as<double2>(), lB.as<double2>(), H.Dinv.as<double2>(),
                              lbad.as<int>(), nullptr);
      hip_check(hipGetLastError(), "leaf inversion");
      hip_check(hipMemcpy(bad.data(), lbad.p, (size_t)nk * 4, hipMemcpyDeviceToHost), "leaf status");
      for (int k = 0; k < nk; ++k)
        if (bad[k]) throw LsError(LS_EINVAL, "singular HODLR leaf block");
    }
    H.ident.upload(ident);
    H.dense_leaves = (int64_t)dense.size();
    // rows without contrast are identity rows of A, so the same rows of every Y = D^-1 U are zero
    std::vector<unsigned char> ract((size_t)((N + 255) / 256), 0);
    for (long long i = 0; i < N; ++i)
      if (qm[i] != 0.0) ract[(size_t)(i >> 8)] = 1;
    H.rows_active = 0;
    std::vector<int> alist;
    for (size_t b = 0; b < ract.size(); ++b)
      if (ract[b]) {
        H.rows_active += std::min<long long>(256, N - (long long)b * 256);
        alist.push_back((int)b);
      }
    H.ract.upload(ract);
    H.alist.upload(alist);
    H.nact = (int)alist.size();
    // below three quarters of the rows, single-column updates run over the listed blocks (all
    // threads on rows that change) instead of inside the fused update + W^T z launch
    // the listed kernel takes 4 (bf16) or 2 (complex64) consecutive rows per lane with one s,
    // so every node half must hold a multiple of 4 rows (not so for odd leaf sides, e.g. 25- or
    // 49-point leaves)
    bool halves4 = true;
    for (int l = 0; l < H.Lb; ++l)
      if (N % (2LL << l) != 0 || (N >> (l + 1)) % 4 != 0) halves4 = false;
    H.sparse = N % 256 == 0 && halves4 && H.rows_active * 4 < N * 3;
    H.bytes = (int64_t)H.nleaves * lp * lp * 16;
  }
  hodlr_chunks(H, P->tune.hodlr_rows);
  // off-diagonal ACA at fixed rank (rows with q = 0 are known zero)
  H.rank.assign(H.Lb, r);
  if (P->opt.hodlr_rank_div > 0)
    for (int l = 0; l < H.Lb; ++l)
      H.rank[l] = (int)std::max<long long>(1, std::min<long long>(r, (N >> (l + 1)) / P->opt.hodlr_rank_div));
  H.Y64.resize(H.Lb);
  H.W64.resize(H.Lb);
  H.coreinv.resize(H.Lb);
  std::vector<int> used_rank;  // ranks the ACA reached, per block
  const double t_aca0 = now_ms();
  if (P->opt.hodlr_tol <= 0.0) {
    // fixed rank: batched ACA on the device, the factors written in place
    DevBuf rowu, colu, rbuf, pmax, ib, jb, state, kcur, retry;
    std::vector<unsigned char> rz((size_t)N);
    for (long long i = 0; i < N; ++i) rz[i] = qm[i] == 0.0 ? 1 : 0;
    rowu.alloc((size_t)N);
    colu.alloc((size_t)N);
    rbuf.alloc((size_t)N * 16);
    pmax.alloc((size_t)(N / 256 + (1LL << H.Lb) + 1) * 8);  // >= nb * ceil(S / 256) on every level
    const int nbmax = 1 << H.Lb;
    for (DevBuf* d : {&ib, &jb, &state, &kcur, &retry}) d->alloc((size_t)nbmax * 4);
    std::vector<int> hbuf(nbmax);
    hipStream_t s0 = nullptr;
    for (int l = 0; l < H.Lb; ++l) {
      const int rl = H.rank[l];
      H.Y64[l].alloc((size_t)N * rl * 16);
      H.W64[l].alloc((size_t)N * rl * 16);
      hip_check(hipMemsetAsync(H.Y64[l].p, 0, (size_t)N * rl * 16, s0), "memset");
      hip_check(hipMemsetAsync(H.W64[l].p, 0, (size_t)N * rl * 16, s0), "memset");
      hip_check(hipMemcpyAsync(rowu.p, rz.data(), (size_t)N, hipMemcpyHostToDevice, s0), "rows h2d");
      hip_check(hipMemsetAsync(colu.p, 0, (size_t)N, s0), "memset");
      lsk::AcaLevel L{};
      L.W = wdev.as<double2>();
      L.ma = mad.as<int>();
      L.mb = mbd.as<int>();
      L.q = P->q_m.as<double>();
      L.coef = coef;
      L.n = P->n;
      L.N = N;
      L.S = N >> (l + 1);
      L.nb = 1 << (l + 1);
      L.U = H.Y64[l].as<double2>();
      L.V = H.W64[l].as<double2>();
      L.row_used = rowu.as<unsigned char>();
      L.col_used = colu.as<unsigned char>();
      L.rbuf = rbuf.as<double2>();
      L.pmax = pmax.as<double>();
      L.ib = ib.as<int>();
      L.jb = jb.as<int>();
      L.state = state.as<int>();
      L.kcur = kcur.as<int>();
      L.retry = retry.as<int>();
      lsk::launch_aca_start(L, s0);
      const int kmax = (int)std::min<long long>(rl, L.S);
      // kmax steps without a host round trip; blocks that met exactly zero rows (a step that
      // only moved them to their next row) need more, until every block has stopped
      for (int steps = kmax;;) {
        for (int k = 0; k < steps; ++k) {
          lsk::launch_aca_row(L, s0);
          lsk::launch_aca_col(L, kmax, s0);
        }
        hip_check(hipMemcpyAsync(hbuf.data(), state.p, (size_t)L.nb * 4, hipMemcpyDeviceToHost, s0), "state d2h");
        hip_check(hipStreamSynchronize(s0), "aca");
        bool any = false;
        for (int b = 0; b < L.nb; ++b) any |= hbuf[b] == 0;
        if (!any) break;
        steps = 16;
      }
      hip_check(hipMemcpyAsync(hbuf.data(), kcur.p, (size_t)L.nb * 4, hipMemcpyDeviceToHost, s0), "ranks d2h");
      hip_check(hipStreamSynchronize(s0), "aca");
      used_rank.insert(used_rank.end(), hbuf.begin(), hbuf.begin() + L.nb);
      H.bytes += (int64_t)2 * N * rl * 16;
    }
    hip_check(hipGetLastError(), "aca kernels");
  } else {
    // blocks to a tolerance (rank capped): the host ACA with Rjasanow's stopping test
    std::vector<std::vector<zd>> Uh(H.Lb), Wh(H.Lb);
    for (int l = 0; l < H.Lb; ++l) {
      Uh[l].assign((size_t)N * H.rank[l], zd(0));
      Wh[l].assign((size_t)N * H.rank[l], zd(0));
    }
    std::vector<std::pair<int, int>> work;  // (level, node)
    for (int l = 0; l < H.Lb; ++l)
      for (int nd = 0; nd < (1 << l); ++nd) work.push_back({l, nd});
    used_rank.assign(work.size() * 2, 0);
    parallel_for((int)work.size() * 2, [&](int wi) {
      int l = work[wi / 2].first, nd = work[wi / 2].second, which = wi % 2;
      long long ns = N >> l, lo = (long long)nd * ns, mid = lo + ns / 2;
      // which = 0: A[I1, I2] ~ P Q^T ; which = 1: A[I2, I1] ~ R S^T
      long long r0 = which ? mid : lo, c0 = which ? lo : mid;
      int m = (int)(ns / 2), n = (int)(ns / 2);
      std::vector<char> rz(m);
      for (int i = 0; i < m; ++i) rz[i] = qm[r0 + i] == 0.0;
      auto rowfn = [&](int i, zd* out) {
        long long gi = r0 + i;
        double cq = coef * qm[gi];
        int ai = mort_a[gi], bi = mort_b[gi];
        for (int j = 0; j < n; ++j) out[j] = cq * W(ai - mort_a[c0 + j], bi - mort_b[c0 + j]);
      };
      auto colfn = [&](int j, zd* out) {
        long long gj = c0 + j;
        int aj = mort_a[gj], bj = mort_b[gj];
        for (int i = 0; i < m; ++i) out[i] = coef * qm[r0 + i] * W(mort_a[r0 + i] - aj, mort_b[r0 + i] - bj);
      };
      ls::ACAResult R = ls::aca(m, n, H.rank[l], P->opt.hodlr_tol, &rz, rowfn, colfn);
      int k = (int)R.u.size();
      used_rank[wi] = k;
      for (int c = 0; c < k; ++c) {
        for (int i = 0; i < m; ++i) Uh[l][(size_t)c * N + r0 + i] = R.u[c][i];
        for (int j = 0; j < n; ++j) Wh[l][(size_t)c * N + c0 + j] = R.v[c][j];
      }
    });
    for (int l = 0; l < H.Lb; ++l) {
      H.Y64[l].upload(Uh[l]);
      H.W64[l].upload(Wh[l]);
      H.bytes += (int64_t)2 * N * H.rank[l] * 16;
      Uh[l].clear();
      Uh[l].shrink_to_fit();
      Wh[l].clear();
      Wh[l].shrink_to_fit();
    }
  }
  H.t_aca_ms = now_ms() - t_aca0;
  H.used_rank_sum = 0;
  H.used_rank_max = 0;
  for (int k : used_rank) {
    H.used_rank_sum += k;
    H.used_rank_max = std::max(H.used_rank_max, k);
  }
  H.blocks = (int64_t)used_rank.size();
  // Y_l = D_l^{-1} U_l (U becomes Y in place) and the SMW cores, inverted on the device
  hipStream_t s = nullptr;
  int rmax = 0;
  size_t kmax_elems = 1;
  for (int l = 0; l < H.Lb; ++l) {
    rmax = std::max(rmax, H.rank[l]);
    kmax_elems = std::max(kmax_elems, (size_t)(1LL << l) * 4 * H.rank[l] * H.rank[l]);
  }
  hodlr_ensure_ws(P, std::max(rmax, 1));
  DevBuf kA, kB, kbad;
  kA.alloc(kmax_elems * 16);
  kB.alloc(kmax_elems * 16);
  kbad.alloc((size_t)(1LL << H.Lb) * 4);
  std::vector<int> bad((size_t)1 << H.Lb);
  for (int l = H.Lb - 1; l >= 0; --l) {
    const int r = H.rank[l];
    double2* Y = H.Y64[l].as<double2>();
    const double ta = now_ms();
    hodlr_apply(P, 0, Y, N, Y, N, r, l + 1, s);
    // exact zeros where the point has no contrast (the apply kernels skip those rows)
    lsk::launch_zero_rows(Y, N, r, P->q_m.as<double>(), s);
    int nodes = 1 << l;
    lsk::launch_hodlr_dot(0, H.W64[l].p, Y, N, H.partial.as<double2>(), N, r, H.chunk[l], H.nchunks[l], r, s);
    lsk::launch_hodlr_core(0, nullptr, H.partial.as<double2>(), H.svec.as<double2>(), r, nodes, H.cpc[l],
                           H.nchunks[l], false, r, s);
    hip_check(hipStreamSynchronize(s), "hodlr factors");
    const double tc = now_ms();
    H.t_apply_ms += tc - ta;
    const long long ce = lsk::hodlr_core_elems(r);
    H.coreinv[l].alloc((size_t)nodes * ce * 16);
    hip_check(hipMemsetAsync(kbad.p, 0, (size_t)nodes * 4, s), "memset");
    lsk::launch_core_invert(H.svec.as<double2>(), r, nodes, kA.as<double2>(), kB.as<double2>(),
                            H.coreinv[l].as<double2>(), kbad.as<int>(), s);
    hip_check(hipGetLastError(), "core inversion");
    hip_check(hipMemcpyAsync(bad.data(), kbad.p, (size_t)nodes * 4, hipMemcpyDeviceToHost, s), "core status");
    hip_check(hipStreamSynchronize(s), "core inversion");
    for (int nd = 0; nd < nodes; ++nd)
      if (bad[nd]) throw LsError(LS_EINVAL, "singular HODLR core");
    H.bytes += (int64_t)nodes * ce * 16;
    H.t_cores_ms += now_ms() - tc;
  }
  hip_check(hipDeviceSynchronize(), "hodlr setup");
  // node activity for the applies (the factor construction above ran unmasked)
  if (N % (1LL << H.Lb) == 0) {
    std::vector<unsigned char> act((size_t)2 << H.Lb, 0);
    const long long leaf = N >> H.Lb;
    for (long long i = 0; i < N; ++i)
      if (qm[i] != 0.0) act[(size_t)((1LL << H.Lb) + i / leaf)] = 1;
    for (int d = H.Lb - 1; d >= 0; --d)
      for (long long j = 0; j < (1LL << d); ++j)
        act[(size_t)((1LL << d) + j)] = act[(size_t)((2LL << d) + 2 * j)] | act[(size_t)((2LL << d) + 2 * j + 1)];
    H.dot_rows.assign(H.Lb, 0);
    H.core_nodes.assign(H.Lb, 0);
    H.doff.assign(H.Lb, 0);
    H.dcnt.assign(H.Lb, 0);
    std::vector<int> dl;
    for (int l = 0; l < H.Lb; ++l) {
      const unsigned char* c = act.data() + (2LL << l);
      H.doff[l] = (long long)dl.size();
      for (long long j = 0; j < (2LL << l); ++j)
        if (c[j ^ 1]) dl.push_back((int)j);
      H.dcnt[l] = (int)((long long)dl.size() - H.doff[l]);
      for (long long j = 0; j < (1LL << l); ++j) {
        if (c[2 * j] && c[2 * j + 1]) H.core_nodes[l] += 1;
        if (H.chunk[l] < 16)
          H.dot_rows[l] += N >> l;  // the tall-skinny reduction forms every chunk
        else
          H.dot_rows[l] += ((c[2 * j] ? 1 : 0) + (c[2 * j + 1] ? 1 : 0)) * (N >> (l + 1));
      }
    }
    H.nodeact.upload(act);
    if (dl.empty()) dl.push_back(0);
    H.dlist.upload(dl);
  }
  // FP32 copies of the leaf inverses, the off-diagonal factors and the core inverses
  const long long nd = (long long)H.nleaves * H.lp * H.lp;
  H.Dinv32.alloc((size_t)nd * 8);
  lsk::launch_cast(true, H.Dinv.p, H.Dinv32.p, nd, s);
  H.bytes += nd * 8;
  H.Y32.resize(H.Lb);
  H.W32.resize(H.Lb);
  H.core32.resize(H.Lb);
  for (int l = 0; l < H.Lb; ++l) {
    const int r = H.rank[l];
    const long long nc = (1LL << l) * lsk::hodlr_core_elems(r);
    H.Y32[l].alloc((size_t)N * r * 8);
    H.W32[l].alloc((size_t)N * r * 8);
    H.core32[l].alloc((size_t)nc * 8);
    lsk::launch_cast(true, H.Y64[l].p, H.Y32[l].p, (long long)N * r, s);
    lsk::launch_cast(true, H.W64[l].p, H.W32[l].p, (long long)N * r, s);
    lsk::launch_cast(true, H.coreinv[l].p, H.core32[l].p, nc, s);
    H.bytes += (int64_t)2 * N * r * 8 + nc * 8;
  }
  if (P->opt.pc_bf16) {
    H.Dinv16.alloc((size_t)nd * 4);
    lsk::launch_cast_bf16(H.Dinv.p, H.Dinv16.p, nd, s);
    H.bytes += nd * 4;
    H.Y16.resize(H.Lb);
    H.W16.resize(H.Lb);
    H.core16.resize(H.Lb);
    for (int l = 0; l < H.Lb; ++l) {
      const int r = H.rank[l];
      const long long nc = (1LL << l) * lsk::hodlr_core_elems(r);
      H.Y16[l].alloc((size_t)N * r * 4);
      H.W16[l].alloc((size_t)N * r * 4);
      H.core16[l].alloc((size_t)nc * 4);
      lsk::launch_cast_bf16(H.Y64[l].p, H.Y16[l].p, (long long)N * r, s);
      lsk::launch_cast_bf16(H.W64[l].p, H.W16[l].p, (long long)N * r, s);
      lsk::launch_cast_bf16(H.coreinv[l].p, H.core16[l].p, nc, s);
      H.bytes += (int64_t)2 * N * r * 4 + nc * 4;
    }
    H.have16 = true;
  }
  hip_check(hipDeviceSynchronize(), "hodlr cast");
}

// ---------------------------------------------------------------------------------------
// GMRES (Section 6): restarted, right-preconditioned, classical Gram-Schmidt with one
// reorthogonalisation, Givens rotations on the host.  All vectors in Morton order.
// ---------------------------------------------------------------------------------------
struct GmresCfg {
  bool flexible = false;        // keep z_j = M^{-1} q_j and update x += Z y (variable preconditioner / operator)
  double relax = 0.0;           // > 0: use the FP32 operator once every active residual estimate is <= relax
  bool trust_estimate = false;  // inner solves: stop on the Arnoldi residual estimate
  bool x_zero = false;          // the initial guess is zero (skip the first product)
  bool op32 = false;     // FP32 operator
  bool pc = false;       // use the HODLR preconditioner
  int pcf = 0;           // HODLR off-diagonal factors: 0 complex128, 1 complex64, 2 complex bfloat16
  bool dcgs2 = false;    // device-driven steps: delayed CGS2 (one reduction, one update pass)
  int restart = 200;
  int maxit = 2000;
  int max_refine = 1 << 30;  // relax > 0: Krylov cycles that may use FP32 products
};

struct ColState {
  double fnorm = 0, tol = 0;
  int its = 0, status = LS_MAXIT;
  bool done = false;
  bool est_converged = false;
  double last_est = 1.0;
  int cycles = 0;            // Krylov cycles started, each after an FP64 true residual
  double prev_true = 1e300;  // true residual at the previous cycle start
  bool fell_back = false;    // relaxed (FP32) products stagnated; finished with FP64 products
  double relres = 0;
};

void op_apply(ls_problem* P, bool op32, const double2* x, double2* y, int nrhs, hipStream_t s) {
  fmm_apply(P, op32, x, P->N, y, P->N, nrhs, 1.0, P->coef, false, s);
}

// z (ld N) = M^{-1} x (ld ldx)
void pc_apply(ls_problem* P, const GmresCfg& cfg, const double2* x, long long ldx, double2* z, int nrhs,
              hipStream_t s) {
  if (cfg.pc)
    hodlr_apply(P, cfg.pcf, x, ldx, z, P->N, nrhs, 0, s);
  else
    lsk::launch_axpby(1.0, x, ldx, 0.0, x, ldx, z, P->N, P->N, nrhs, s);
}

// row chunks of the Arnoldi reductions (rows per chunk chosen by ls_autotune, default 1024)
int nchunks_for(const ls_problem* P) {
  const long long rows = std::max(1, P->tune.gs_rows);
  return (int)std::max<long long>(1, std::min<long long>(1024, (P->N + rows - 1) / rows));
}

void norms(ls_problem* P, const double2* v, int nrhs, std::vector<double>& out, hipStream_t s) {
  const long long N = P->N;
  int nch = nchunks_for(P);
  P->knp.ensure((size_t)nch * nrhs * 8);
  P->kno.ensure((size_t)nrhs * 8);
  lsk::launch_norm2(v, N, P->knp.as<double>(), N, nch, nrhs, s);
  lsk::launch_norm2_finish(P->knp.as<double>(), nch, P->kno.as<double>(), nrhs, s);
  out.resize(nrhs);
  hip_check(hipMemcpyAsync(out.data(), P->kno.p, nrhs * 8, hipMemcpyDeviceToHost, s), "norm d2h");
  hip_check(hipStreamSynchronize(s), "sync");
  for (auto& x : out) x = std::sqrt(x);
}

// Solve op(A) x = f (Morton order, ld = N) from the x given; per-column tolerances.
void gmres(ls_problem* P, const GmresCfg& cfg, const double2* f, double2* x, int nrhs, std::vector<ColState>& st,
           hipStream_t s) {
  const long long N = P->N;
  const int m = std::max(1, cfg.restart);
  const int maxv = m + 1;
  const int nch = nchunks_for(P);
  P->kQ.ensure((size_t)nrhs * maxv * N * 16);
  P->kw.ensure((size_t)nrhs * N * 16);
  P->kz.ensure((size_t)nrhs * N * 16);
  P->kr.ensure((size_t)nrhs * N * 16);
  P->kh.ensure((size_t)nrhs * maxv * 16);
  P->kpart.ensure((size_t)nrhs * nch * maxv * 16);
  P->kalpha.ensure((size_t)nrhs * 8);
  P->ky.ensure((size_t)nrhs * maxv * 16);
  if (cfg.flexible) P->kZ.ensure((size_t)nrhs * m * N * 16);
  double2* Q = P->kQ.as<double2>();
  double2* Zb = cfg.flexible ? P->kZ.as<double2>() : nullptr;
  const long long ldzr = (long long)m * N;
  double2* w = P->kw.as<double2>();
  double2* z = P->kz.as<double2>();
  double2* r = P->kr.as<double2>();
  double2* hd = P->kh.as<double2>();
  double2* part = P->kpart.as<double2>();
  const long long ldqv = N, ldqr = (long long)maxv * N;
  std::vector<std::vector<zd>> H(nrhs), g(nrhs), sn(nrhs);
  std::vector<std::vector<double>> cs(nrhs);
  std::vector<double> beta, alpha(nrhs), hnorm;
  std::vector<zd> hh((size_t)nrhs * maxv);
  std::vector<int> kcol(nrhs);
  bool first = true;
  bool relax_enabled = cfg.relax > 0;
  for (;;) {
    bool all_done = true;
    for (int c = 0; c < nrhs; ++c) all_done &= st[c].done;
    if (all_done) return;
    // true residual r = f - A x
    if (first && cfg.x_zero) {
      lsk::launch_axpby(1.0, f, N, 0.0, f, N, r, N, N, nrhs, s);
    } else {
      op_apply(P, cfg.op32, x, w, nrhs, s);
      lsk::launch_axpby(1.0, f, N, -1.0, w, N, r, N, N, nrhs, s);
    }
    first = false;
    norms(P, r, nrhs, beta, s);
    bool any = false;
    for (int c = 0; c < nrhs; ++c) {
      if (st[c].done) continue;
      st[c].relres = beta[c] / st[c].fnorm;
      if (!std::isfinite(beta[c])) {
        st[c].done = true;
        st[c].status = LS_NAN;
      } else if (st[c].relres <= st[c].tol) {
        st[c].done = true;
        st[c].status = LS_CONVERGED;
      } else if (st[c].its >= cfg.maxit) {
        st[c].done = true;
        st[c].status = LS_MAXIT;
      } else {
        any = true;
        st[c].cycles++;
        // FP32 products stopped reducing the true residual, or the refinement budget is spent
        if (relax_enabled && st[c].cycles > 1 &&
            (beta[c] > 0.9 * st[c].prev_true || st[c].cycles > cfg.max_refine)) {
          relax_enabled = false;
          st[c].fell_back = true;
        }
        st[c].prev_true = beta[c];
      }
    }
    if (!any) return;
    std::vector<char> active(nrhs, 0);
    for (int c = 0; c < nrhs; ++c) {
      active[c] = !st[c].done;
      alpha[c] = active[c] ? 1.0 / beta[c] : 0.0;
      H[c].assign((size_t)maxv * m, zd(0));
      g[c].assign(maxv, zd(0));
      g[c][0] = active[c] ? beta[c] : 0.0;
      cs[c].assign(m, 0.0);
      sn[c].assign(m, zd(0));
      kcol[c] = 0;
    }
    hip_check(hipMemcpyAsync(P->kalpha.p, alpha.data(), nrhs * 8, hipMemcpyHostToDevice, s), "alpha");
    lsk::launch_scale(r, N, P->kalpha.as<double>(), Q, ldqr, N, nrhs, s);
    bool relaxed = false;
    for (int j = 0; j < m; ++j) {
      // w = A M^{-1} q_j  (flexible: z_j kept for the update)
      if (cfg.flexible) {
        double2* zj = Zb + (long long)j * N;
        if (cfg.pc)
          hodlr_apply(P, cfg.pcf, Q + (long long)j * ldqv, ldqr, zj, ldzr, nrhs, 0, s);
        else
          lsk::launch_axpby(1.0, Q + (long long)j * ldqv, ldqr, 0.0, Q, ldqr, zj, ldzr, N, nrhs, s);
        fmm_apply(P, cfg.op32 || relaxed, zj, ldzr, w, N, nrhs, 1.0, P->coef, false, s);
      } else {
        pc_apply(P, cfg, Q + (long long)j * ldqv, ldqr, z, nrhs, s);
        op_apply(P, cfg.op32 || relaxed, z, w, nrhs, s);
      }
      // CGS2
      {
        ProfScope ps(P, 3, s);
        lsk::launch_gs_dot(Q, ldqv, ldqr, j + 1, w, N, part, N, nch, maxv, nrhs, s);
      }
      lsk::launch_gs_finish(part, nch, j + 1, maxv, hd, 0, nrhs, s);
      lsk::launch_gs_axpy(Q, ldqv, ldqr, j + 1, hd, maxv, -1.0, w, N, N, nrhs, s);
      lsk::launch_gs_dot(Q, ldqv, ldqr, j + 1, w, N, part, N, nch, maxv, nrhs, s);
      // second pass: store correction in the y buffer, then accumulate into hd
      lsk::launch_gs_finish(part, nch, j + 1, maxv, P->ky.as<double2>(), 0, nrhs, s);
      lsk::launch_gs_axpy(Q, ldqv, ldqr, j + 1, P->ky.as<double2>(), maxv, -1.0, w, N, N, nrhs, s);
      lsk::launch_axpby(1.0, hd, maxv, 1.0, P->ky.as<double2>(), maxv, hd, maxv, j + 1, nrhs, s);
      hip_check(hipMemcpyAsync(hh.data(), hd, (size_t)nrhs * maxv * 16, hipMemcpyDeviceToHost, s), "h d2h");
      norms(P, w, nrhs, hnorm, s);
      bool any_active = false;
      for (int c = 0; c < nrhs; ++c) {
        if (!active[c]) {
          alpha[c] = 0.0;
          continue;
        }
        zd* Hc = H[c].data();
        for (int i = 0; i <= j; ++i) Hc[(size_t)i * m + j] = hh[(size_t)c * maxv + i];
        Hc[(size_t)(j + 1) * m + j] = hnorm[c];
        for (int i = 0; i < j; ++i) {
          zd a = Hc[(size_t)i * m + j], b = Hc[(size_t)(i + 1) * m + j];
          Hc[(size_t)i * m + j] = cs[c][i] * a + sn[c][i] * b;
          Hc[(size_t)(i + 1) * m + j] = -std::conj(sn[c][i]) * a + cs[c][i] * b;
        }
        zd a = Hc[(size_t)j * m + j], b = Hc[(size_t)(j + 1) * m + j];
        double cc;
        zd ss;
        if (b == zd(0)) {
          cc = 1.0;
          ss = 0.0;
        } else if (a == zd(0)) {
          cc = 0.0;
          ss = std::conj(b) / std::abs(b);
        } else {
          double t = std::hypot(std::abs(a), std::abs(b));
          cc = std::abs(a) / t;
          ss = (a / std::abs(a)) * std::conj(b) / t;
        }
        cs[c][j] = cc;
        sn[c][j] = ss;
        Hc[(size_t)j * m + j] = cc * a + ss * b;
        Hc[(size_t)(j + 1) * m + j] = 0.0;
        g[c][j + 1] = -std::conj(ss) * g[c][j];
        g[c][j] = cc * g[c][j];
        st[c].its++;
        kcol[c] = j + 1;
        double est = std::abs(g[c][j + 1]) / st[c].fnorm;
        bool stop = est <= st[c].tol || st[c].its >= cfg.maxit || hnorm[c] == 0.0 || !std::isfinite(est);
        if (est <= st[c].tol) st[c].est_converged = true;
        st[c].last_est = est;
        if (stop) {
          active[c] = 0;
          alpha[c] = 0.0;
        } else {
          alpha[c] = 1.0 / hnorm[c];
          any_active = true;
        }
      }
      if (!any_active || j + 1 == m) break;
      if (relax_enabled && !relaxed) {
        bool all_small = true;
        for (int c = 0; c < nrhs; ++c)
          if (active[c] && st[c].last_est > cfg.relax) all_small = false;
        relaxed = all_small;
      }
      hip_check(hipMemcpyAsync(P->kalpha.p, alpha.data(), nrhs * 8, hipMemcpyHostToDevice, s), "alpha");
      lsk::launch_scale(w, N, P->kalpha.as<double>(), Q + (long long)(j + 1) * ldqv, ldqr, N, nrhs, s);
    }
    // y = R^{-1} g per column, x += M^{-1} (Q y)
    std::vector<zd> y((size_t)nrhs * maxv, zd(0));
    for (int c = 0; c < nrhs; ++c) {
      int k = kcol[c];
      const zd* Hc = H[c].data();
      for (int i = k - 1; i >= 0; --i) {
        zd acc = g[c][i];
        for (int jj = i + 1; jj < k; ++jj) acc -= Hc[(size_t)i * m + jj] * y[(size_t)c * maxv + jj];
        y[(size_t)c * maxv + i] = acc / Hc[(size_t)i * m + i];
      }
    }
    hip_check(hipMemcpyAsync(P->ky.p, y.data(), y.size() * 16, hipMemcpyHostToDevice, s), "y h2d");
    int kmaxc = 0;
    for (int c = 0; c < nrhs; ++c) kmaxc = std::max(kmaxc, kcol[c]);
    if (cfg.flexible) {
      lsk::launch_gs_axpy(Zb, N, ldzr, kmaxc, P->ky.as<double2>(), maxv, 1.0, x, N, N, nrhs, s);
    } else {
      hip_check(hipMemsetAsync(w, 0, (size_t)nrhs * N * 16, s), "memset");
      lsk::launch_gs_axpy(Q, ldqv, ldqr, kmaxc, P->ky.as<double2>(), maxv, 1.0, w, N, N, nrhs, s);
      pc_apply(P, cfg, w, N, z, nrhs, s);
      lsk::launch_axpby(1.0, x, N, 1.0, z, N, x, N, N, nrhs, s);
    }
    hip_check(hipStreamSynchronize(s), "gmres cycle");
    if (cfg.trust_estimate)
      for (int c = 0; c < nrhs; ++c)
        if (!st[c].done && st[c].est_converged) {
          st[c].done = true;
          st[c].status = LS_CONVERGED;
        }
  }
}

// ---------------------------------------------------------------------------------------
// GMRES with device-driven Arnoldi steps, graph_iters of them captured into one HIP graph.
// Same method as gmres() above (right preconditioning, CGS2, Givens, restarts from the true
// residual, flexible variant with precision relaxation); the Arnoldi index, the rotations and
// the stop test live on the device, so the host synchronises once per replay instead of
// once per iteration.  Steps replayed after a column has stopped leave it untouched.
// ---------------------------------------------------------------------------------------
struct KdView {
  long long N;
  int nrhs, m, maxv, nch;
  int *jd, *state, *its, *kfin;
  double *fnorm, *tol, *est, *alpha;
};

KdView kd_view(ls_problem* P, int nrhs, int m) {
  KdView v;
  v.N = P->N;
  v.nrhs = nrhs;
  v.m = m;
  v.maxv = m + 1;
  v.nch = nchunks_for(P);
  int* ic = P->kd.ictl.as<int>();
  v.jd = ic;
  v.state = ic + 1;
  v.its = ic + 1 + nrhs;
  v.kfin = ic + 1 + 2 * nrhs;
  double* dc = P->kd.dctl.as<double>();
  v.fnorm = dc;
  v.tol = dc + nrhs;
  v.est = dc + 2 * nrhs;
  v.alpha = dc + 3 * nrhs;
  return v;
}

void kd_ensure(ls_problem* P, const GmresCfg& cfg, int nrhs) {
  const long long N = P->N;
  const int m = std::max(1, cfg.restart), maxv = m + 1, nch = nchunks_for(P);
  P->kQ.ensure((size_t)nrhs * maxv * N * 16);
  if (cfg.flexible) P->kZ.ensure((size_t)nrhs * (cfg.dcgs2 ? maxv : m) * N * 16);
  P->kw.ensure((size_t)nrhs * N * 16);
  P->kz.ensure((size_t)nrhs * N * 16);
  P->kr.ensure((size_t)nrhs * N * 16);
  P->kpart.ensure((size_t)nrhs * nch * maxv * 16);
  if (cfg.dcgs2) {
    const long long nblk = (N + P->tune.dot2_rows - 1) / P->tune.dot2_rows;
    P->kpart.ensure((size_t)nrhs * (nblk + 1) * 2 * maxv * 16);
    P->kd.Hr.ensure((size_t)nrhs * maxv * maxv * 16);
    P->kd.T.ensure((size_t)nrhs * maxv * maxv * 16);
    P->kd.coef.ensure((size_t)nrhs * 2 * maxv * 16);
  }
  P->knp.ensure((size_t)nch * nrhs * 8);
  P->ky.ensure((size_t)nrhs * maxv * 16);
  P->kalpha.ensure((size_t)nrhs * 8);
  KrylovDev& K = P->kd;
  K.ictl.ensure((size_t)(1 + 3 * nrhs) * 4);
  K.dctl.ensure((size_t)4 * nrhs * 8);
  K.H.ensure((size_t)nrhs * m * maxv * 16);
  K.cs.ensure((size_t)nrhs * m * 8);
  K.sn.ensure((size_t)nrhs * m * 16);
  K.g.ensure((size_t)nrhs * maxv * 16);
  K.vin.ensure((size_t)nrhs * N * 16);
  K.tmp.ensure((size_t)nrhs * maxv * 16);
  const size_t hb = (size_t)(1 + 3 * nrhs) * 4 + 8 + (size_t)nrhs * 8;
  if (K.host_bytes < hb) {
    if (K.host) hip_check(hipHostFree(K.host), "hipHostFree");
    K.host = nullptr;
    K.host_bytes = 0;
    hip_check(hipHostMalloc((void**)&K.host, hb, hipHostMallocDefault), "hipHostMalloc");
    K.host_bytes = hb;
  }
  ensure_fmm_capacity(P, P->f64, nrhs);
  if (P->have32) ensure_fmm_capacity(P, P->f32, nrhs);
  if (P->have_hodlr) hodlr_ensure_ws(P, nrhs);
  if (!K.cap) hip_check(hipStreamCreateWithFlags(&K.cap, hipStreamNonBlocking), "hipStreamCreate");
}

void kd_key_phase(std::vector<uintptr_t>& k, const Phase& ph) {
  k.push_back((uintptr_t)ph.tasks.p);
  k.push_back((uintptr_t)ph.terms.p);
  k.push_back((uintptr_t)ph.blk.p);
  k.push_back((uintptr_t)ph.sk.p);
  k.push_back((uintptr_t)ph.nsk);
}

void kd_key_fmm(std::vector<uintptr_t>& k, const FmmDev& F) {
  for (const DevBuf* b : {&F.ops, &F.mult, &F.loc, &F.xs, &F.ys}) k.push_back((uintptr_t)b->p);
  k.push_back((uintptr_t)F.nrhs_cap);
  kd_key_phase(k, F.p2m);
  kd_key_phase(k, F.nearm2l);
  kd_key_phase(k, F.l2p);
  for (const Phase& ph : F.up) kd_key_phase(k, ph);
  for (const Phase& ph : F.down) kd_key_phase(k, ph);
  kd_key_phase(k, F.fused);
  for (const DevBuf* b : {&F.fneed, &F.fctr}) k.push_back((uintptr_t)b->p);
  k.push_back((uintptr_t)F.fused_wg);
}

// everything a captured step depends on: sizes, modes and every device address it touches
std::vector<uintptr_t> kd_key(ls_problem* P, const GmresCfg& cfg, bool op32, int nrhs, int steps) {
  std::vector<uintptr_t> k = {(uintptr_t)nrhs, (uintptr_t)cfg.restart, (uintptr_t)steps, (uintptr_t)cfg.flexible,
                              (uintptr_t)cfg.pc, (uintptr_t)cfg.pcf, (uintptr_t)op32, (uintptr_t)cfg.maxit,
                              (uintptr_t)cfg.dcgs2, (uintptr_t)P->tune.gs_rows, (uintptr_t)P->tune.hodlr_rows,
                              (uintptr_t)P->tune.dot2_rows};
  for (const DevBuf* b : {&P->kQ, &P->kZ, &P->kw, &P->kz, &P->kpart, &P->knp, &P->kd.ictl, &P->kd.dctl, &P->kd.H,
                          &P->kd.cs, &P->kd.sn, &P->kd.g, &P->kd.vin, &P->kd.tmp, &P->kd.Hr, &P->kd.T, &P->kd.coef})
    k.push_back((uintptr_t)b->p);
  kd_key_fmm(k, op32 ? P->f32 : P->f64);
  if (P->have_hodlr) {
    k.push_back((uintptr_t)P->hod.partial.p);
    k.push_back((uintptr_t)P->hod.svec.p);
  }
  return k;
}

// one Arnoldi step: q_j -> (z_j) -> w = A M^{-1} q_j, CGS2, Givens, q_{j+1}
void kd_step(ls_problem* P, const GmresCfg& cfg, bool op32, const KdView& v, hipStream_t s) {
  const long long N = v.N;
  const int nrhs = v.nrhs, m = v.m, maxv = v.maxv, nch = v.nch;
  double2* Q = P->kQ.as<double2>();
  const long long ldqv = N, ldqr = (long long)maxv * N;
  double2* w = P->kw.as<double2>();
  double2* z = P->kz.as<double2>();
  double2* vin = P->kd.vin.as<double2>();
  double2* H = P->kd.H.as<double2>();
  double2* part = P->kpart.as<double2>();
  const long long hr = (long long)m * maxv;
  if (cfg.pc) {
    // the leaf solves read q_j straight from the basis (column index on the device)
    // and the last level's update also stores z~_j into Z (flexible)
    hodlr_apply(P, cfg.pcf, Q, ldqr, z, N, nrhs, 0, s, v.jd, ldqv, cfg.flexible ? P->kZ.as<double2>() : nullptr,
                (long long)(cfg.dcgs2 ? maxv : m) * N, N);
  } else {
    lsk::launch_kd_copy(Q, ldqr, ldqv, vin, N, 0, N, v.jd, v.state, nrhs, s);
    lsk::launch_axpby(1.0, vin, N, 0.0, vin, N, z, N, N, nrhs, s);
    if (cfg.flexible)
      lsk::launch_kd_copy(z, N, 0, P->kZ.as<double2>(), (long long)(cfg.dcgs2 ? maxv : m) * N, N, N, v.jd, v.state,
                          nrhs, s);
  }
  fmm_apply(P, op32, z, N, w, N, nrhs, 1.0, P->coef, false, s);
  if (cfg.dcgs2) {
    // delayed CGS2: slot j holds u_j; one pass of inner products, the small O(j^2) update of
    // the Hessenberg column, one pass writing q_j and u_{j+1}
    {
      ProfScope ps(P, 3, s);
      lsk::launch_kd_dot2(Q, ldqv, ldqr, maxv, w, N, part, N, P->tune.dot2_rows, v.jd, v.state, nrhs, s);
    }
    const long long nblk = (N + P->tune.dot2_rows - 1) / P->tune.dot2_rows;
    const double2* cd = part + (long long)nrhs * nblk * 2 * maxv;
    lsk::launch_kd_dcgs2(cd, P->kd.Hr.as<double2>(), H, m, maxv, P->kd.cs.as<double>(), P->kd.sn.as<double2>(),
                         P->kd.g.as<double2>(), P->kd.T.as<double2>(), P->kd.coef.as<double2>(), v.jd, v.state,
                         v.its, v.kfin, v.est, v.fnorm, v.tol, cfg.maxit, v.alpha, nrhs, s);
    lsk::launch_kd_dcgs2_axpy(Q, ldqv, ldqr, w, N, P->kd.coef.as<double2>(), maxv, v.alpha, N, v.jd, v.state, nrhs,
                              s);
    return;
  }
  {
    ProfScope ps(P, 3, s);
    lsk::launch_kd_dot(Q, ldqv, ldqr, maxv, w, N, part, N, nch, v.jd, v.state, nrhs, s);
  }
  lsk::launch_kd_finish(part, nch, maxv, H, hr, maxv, 0, v.jd, v.state, nrhs, s);
  lsk::launch_kd_axpy(Q, ldqv, ldqr, H, hr, maxv, -1.0, w, N, N, v.jd, v.state, nrhs, s);
  lsk::launch_kd_dot(Q, ldqv, ldqr, maxv, w, N, part, N, nch, v.jd, v.state, nrhs, s);
  double2* t = P->kd.tmp.as<double2>();
  lsk::launch_kd_finish(part, nch, maxv, t, maxv, 0, 0, v.jd, v.state, nrhs, s);
  lsk::launch_kd_axpy(Q, ldqv, ldqr, t, maxv, 0, -1.0, w, N, N, v.jd, v.state, nrhs, s);
  lsk::launch_kd_finish(part, nch, maxv, H, hr, maxv, 1, v.jd, v.state, nrhs, s);
  lsk::launch_norm2(w, N, P->knp.as<double>(), N, nch, nrhs, s);
  lsk::launch_kd_givens(P->knp.as<double>(), nch, H, m, maxv, P->kd.cs.as<double>(), P->kd.sn.as<double2>(),
                        P->kd.g.as<double2>(), v.jd, v.state, v.its, v.kfin, v.est, v.fnorm, v.tol, cfg.maxit,
                        v.alpha, nrhs, s);
  lsk::launch_kd_next(w, N, v.alpha, Q, ldqv, ldqr, N, v.jd, v.state, nrhs, s);
}

hipGraphExec_t kd_graph(ls_problem* P, const GmresCfg& cfg, bool op32, const KdView& v, int steps) {
  KrylovDev& K = P->kd;
  const int slot = op32 ? 1 : 0;
  std::vector<uintptr_t> key = kd_key(P, cfg, op32, v.nrhs, steps);
  if (K.exec[slot] && K.key[slot] == key) return K.exec[slot];
  K.drop(slot);
  hipGraph_t g = nullptr;
  hip_check(hipStreamBeginCapture(K.cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  P->capturing = true;
  try {
    for (int i = 0; i < steps; ++i) kd_step(P, cfg, op32, v, K.cap);
  } catch (...) {
    P->capturing = false;
    (void)hipStreamEndCapture(K.cap, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  P->capturing = false;
  hip_check(hipStreamEndCapture(K.cap, &g), "hipStreamEndCapture");
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  hip_check(e, "hipGraphInstantiate");
  K.exec[slot] = ex;
  K.key[slot] = std::move(key);
  return ex;
}

void gmres_graph(ls_problem* P, const GmresCfg& cfg, const double2* f, double2* x, int nrhs,
                 std::vector<ColState>& st, int steps_in, hipStream_t s) {
  const long long N = P->N;
  const int m = std::max(1, cfg.restart);
  const int maxv = m + 1;
  const int steps = std::max(1, steps_in);
  kd_ensure(P, cfg, nrhs);
  const KdView v = kd_view(P, nrhs, m);
  KrylovDev& K = P->kd;
  double2* w = P->kw.as<double2>();
  double2* z = P->kz.as<double2>();
  double2* r = P->kr.as<double2>();
  double2* Q = P->kQ.as<double2>();
  const long long ldqr = (long long)maxv * N;
  std::vector<double> beta;
  std::vector<int> hi(1 + 3 * nrhs);
  std::vector<double> hd(4 * nrhs);
  bool first = true;
  bool timed = false;
  for (const ProfileClass& pc : P->prof) timed |= pc.enabled;
  bool relax_enabled = cfg.relax > 0;
  for (;;) {
    bool all_done = true;
    for (int c = 0; c < nrhs; ++c) all_done &= st[c].done;
    if (all_done) return;
    if (first && cfg.x_zero) {
      lsk::launch_axpby(1.0, f, N, 0.0, f, N, r, N, N, nrhs, s);
    } else {
      op_apply(P, cfg.op32, x, w, nrhs, s);
      lsk::launch_axpby(1.0, f, N, -1.0, w, N, r, N, N, nrhs, s);
    }
    first = false;
    norms(P, r, nrhs, beta, s);
    bool any = false;
    for (int c = 0; c < nrhs; ++c) {
      if (st[c].done) continue;
      st[c].relres = beta[c] / st[c].fnorm;
      if (!std::isfinite(beta[c])) {
        st[c].done = true;
        st[c].status = LS_NAN;
      } else if (st[c].relres <= st[c].tol) {
        st[c].done = true;
        st[c].status = LS_CONVERGED;
      } else if (st[c].its >= cfg.maxit) {
        st[c].done = true;
        st[c].status = LS_MAXIT;
      } else {
        any = true;
        st[c].cycles++;
        // FP32 products stopped reducing the true residual, or the refinement budget is spent
        if (relax_enabled && st[c].cycles > 1 &&
            (beta[c] > 0.9 * st[c].prev_true || st[c].cycles > cfg.max_refine)) {
          relax_enabled = false;
          st[c].fell_back = true;
        }
        st[c].prev_true = beta[c];
      }
    }
    if (!any) return;
    // cycle start on the device: j = 0, g = (beta, 0, ...), q_0 = r / beta
    hi.assign(1 + 3 * nrhs, 0);
    std::vector<zd> g0((size_t)nrhs * maxv, zd(0));
    for (int c = 0; c < nrhs; ++c) {
      const bool act = !st[c].done;
      hi[1 + c] = act ? 0 : 2;
      hi[1 + nrhs + c] = st[c].its;
      hd[c] = st[c].fnorm;
      hd[nrhs + c] = st[c].tol;
      hd[2 * nrhs + c] = 1.0;
      hd[3 * nrhs + c] = act ? 1.0 / beta[c] : 0.0;
      g0[(size_t)c * maxv] = act ? beta[c] : 0.0;
    }
    hip_check(hipMemcpyAsync(K.ictl.p, hi.data(), hi.size() * 4, hipMemcpyHostToDevice, s), "ctl h2d");
    hip_check(hipMemcpyAsync(K.dctl.p, hd.data(), hd.size() * 8, hipMemcpyHostToDevice, s), "ctl h2d");
    hip_check(hipMemcpyAsync(K.g.p, g0.data(), g0.size() * 16, hipMemcpyHostToDevice, s), "g h2d");
    lsk::launch_scale(r, N, v.alpha, Q, ldqr, N, nrhs, s);
    bool relaxed = false;
    std::vector<double> est(nrhs, 1.0);
    for (;;) {
      const bool use32 = cfg.op32 || relaxed;
      if (timed) {
        // kernel timers are on: the same steps enqueued eagerly, so every launch has its events
        for (int i = 0; i < steps; ++i) kd_step(P, cfg, use32, v, s);
      } else {
        hip_check(hipGraphLaunch(kd_graph(P, cfg, use32, v, steps), s), "hipGraphLaunch");
      }
      hip_check(hipMemcpyAsync(K.host, K.ictl.p, (size_t)(1 + 3 * nrhs) * 4, hipMemcpyDeviceToHost, s), "ctl d2h");
      hip_check(hipMemcpyAsync(est.data(), v.est, (size_t)nrhs * 8, hipMemcpyDeviceToHost, s), "est d2h");
      hip_check(hipStreamSynchronize(s), "gmres steps");
      bool active = false;
      for (int c = 0; c < nrhs; ++c) active |= K.host[1 + c] == 0;
      if (!active) break;
      if (relax_enabled && !relaxed) {
        bool all_small = true;
        for (int c = 0; c < nrhs; ++c)
          if (K.host[1 + c] == 0 && est[c] > cfg.relax) all_small = false;
        relaxed = all_small;
      }
    }
    // y = R^{-1} g per column (host), x += Z y (flexible) or x += M^{-1} (Q y)
    std::vector<zd> y((size_t)nrhs * maxv, zd(0));
    int kmaxc = 0;
    std::vector<zd> R, gh(maxv);
    for (int c = 0; c < nrhs; ++c) {
      st[c].its = K.host[1 + nrhs + c];
      st[c].last_est = est[c];
      if (st[c].done) continue;
      const int k = K.host[1 + 2 * nrhs + c];
      if (est[c] <= st[c].tol) st[c].est_converged = true;
      if (k <= 0) continue;
      kmaxc = std::max(kmaxc, k);
      R.resize((size_t)k * maxv);
      hip_check(hipMemcpyAsync(R.data(), K.H.as<double2>() + (size_t)c * m * maxv, (size_t)k * maxv * 16,
                               hipMemcpyDeviceToHost, s),
                "R d2h");
      hip_check(hipMemcpyAsync(gh.data(), K.g.as<double2>() + (size_t)c * maxv, (size_t)maxv * 16,
                               hipMemcpyDeviceToHost, s),
                "g d2h");
      hip_check(hipStreamSynchronize(s), "sync");
      // R column jj holds rows 0..jj at R[jj*maxv + i]
      for (int i = k - 1; i >= 0; --i) {
        zd acc = gh[i];
        for (int jj = i + 1; jj < k; ++jj) acc -= R[(size_t)jj * maxv + i] * y[(size_t)c * maxv + jj];
        y[(size_t)c * maxv + i] = acc / R[(size_t)i * maxv + i];
      }
      if (cfg.dcgs2 && cfg.flexible) {
        // the stored z~ are Z T (T upper triangular, column jj = (c, beta) of step jj):
        // x += Z y = Z~ (T^{-1} y)
        std::vector<zd> Tc((size_t)k * maxv);
        hip_check(hipMemcpyAsync(Tc.data(), P->kd.T.as<double2>() + (size_t)c * maxv * maxv, Tc.size() * 16,
                                 hipMemcpyDeviceToHost, s),
                  "T d2h");
        hip_check(hipStreamSynchronize(s), "sync");
        zd* yc = &y[(size_t)c * maxv];
        for (int i = k - 1; i >= 0; --i) {
          zd acc = yc[i];
          for (int jj = i + 1; jj < k; ++jj) acc -= Tc[(size_t)jj * maxv + i] * yc[jj];
          yc[i] = acc / Tc[(size_t)i * maxv + i];
        }
      }
    }
    if (kmaxc > 0) {
      hip_check(hipMemcpyAsync(P->ky.p, y.data(), y.size() * 16, hipMemcpyHostToDevice, s), "y h2d");
      if (cfg.flexible) {
        lsk::launch_gs_axpy(P->kZ.as<double2>(), N, (long long)(cfg.dcgs2 ? maxv : m) * N, kmaxc,
                            P->ky.as<double2>(), maxv, 1.0, x, N, N, nrhs, s);
      } else {
        hip_check(hipMemsetAsync(w, 0, (size_t)nrhs * N * 16, s), "memset");
        lsk::launch_gs_axpy(Q, N, ldqr, kmaxc, P->ky.as<double2>(), maxv, 1.0, w, N, N, nrhs, s);
        pc_apply(P, cfg, w, N, z, nrhs, s);
        lsk::launch_axpby(1.0, x, N, 1.0, z, N, x, N, N, nrhs, s);
      }
    }
    hip_check(hipStreamSynchronize(s), "gmres cycle");
    if (cfg.trust_estimate)
      for (int c = 0; c < nrhs; ++c)
        if (!st[c].done && st[c].est_converged) {
          st[c].done = true;
          st[c].status = LS_CONVERGED;
        }
  }
}

// Exact integral of G = (i/4) H0(kappa |y|) over the square cell [-h/2, h/2]^2 (the diagonal
// entry of Eq. (eq:13) at p = 1):  8 int_0^{pi/4} (i/4) [R H1(kappa R)/kappa + 2i/(pi kappa^2)] dtheta,
// R = h / (2 cos theta), by 64-point Gauss-Legendre quadrature in theta.
zd self_cell(double h, double kappa) {
  const int nq = 64;
  std::vector<double> xg(nq), wg(nq);
  for (int i = 0; i < nq; ++i) {  // Gauss-Legendre nodes by Newton iteration on P_nq
    double x = std::cos(lsk::kPi * (i + 0.75) / (nq + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1, p1 = x;
      for (int k = 2; k <= nq; ++k) {
        double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = nq * (x * p1 - p0) / (x * x - 1);
      double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double p0 = 1, p1 = x;
    for (int k = 2; k <= nq; ++k) {
      double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = nq * (x * p1 - p0) / (x * x - 1);
    xg[i] = x;
    wg[i] = 2.0 / ((1 - x * x) * dp * dp);
  }
  zd acc(0);
  for (int i = 0; i < nq; ++i) {
    double th = (xg[i] + 1.0) * (lsk::kPi / 8.0);
    double R = 0.5 * h / std::cos(th);
    lsk::cplx H1 = lsk::hankel1_small(kappa * R);
    zd radial = R * zd(H1.re, H1.im) / kappa + zd(0, 2.0 / (lsk::kPi * kappa * kappa));
    acc += wg[i] * (lsk::kPi / 8.0) * zd(0, 0.25) * radial;
  }
  return 8.0 * acc;
}

// ---------------------------------------------------------------------------------------
// Device scratch of the allocation-free preconditioner apply: a fixed array in the code object
// (one copy per GPU, allocated when the library's code is loaded there, kept until the process
// ends).  Host code never passes the array's name to a kernel: its device address is looked up
// once per device with hipGetSymbolAddress and only that address is used.
// ---------------------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(64) << 20;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_dev;  // per device ordinal: device address of `scratch`, or null

// device address of the scratch array on the current device (looked up once per device)
void* scratch_address(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_dev.size() <= device) g_scratch_dev.resize(device + 1, nullptr);
  if (!g_scratch_dev[device]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      throw LsError(LS_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[device] = ptr;
  }
  return g_scratch_dev[device];
}

inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }

ls_status fail(const LsError& e) {
  g_last_error = e.what();
  return (ls_status)e.code;
}

}  // namespace

// =========================================================================================
// C ABI
// =========================================================================================
extern "C" {

void ls_default_options(ls_options* o) {
  if (!o) return;
  o->leaf_max = 64;
  o->T = 16.0;
  o->sign = -1;
  o->hodlr_rank = 15;
  o->eps_inner = 1e-7;
  o->restart = 200;
  o->maxit = 2000;
  o->prec = LS_FP64;
  o->inner_tol = 1e-5;
  o->max_refine = 10;
  o->build_fp32 = 1;
  o->hodlr_rank_div = 0;
  o->graph_iters = 0;
  o->stencil_mfma = 1;
  o->fmm_fused = 0;
  o->pc_bf16 = 1;
  o->pc_lowp_solves = 0;
  o->hodlr_tol = 0.0;
  o->dcgs2 = 1;
}

const char* ls_last_error(void) { return g_last_error.c_str(); }

static void validate_options(const ls_options& o) {
  if (o.leaf_max < 1) throw LsError(LS_EINVAL, "leaf_max must be >= 1");
  if (!(o.T > 0) || !std::isfinite(o.T)) throw LsError(LS_EINVAL, "T must be positive");
  if (o.sign != -1 && o.sign != 1) throw LsError(LS_EINVAL, "sign must be -1 or +1");
  if (o.hodlr_rank < 0 || o.hodlr_rank > 256) throw LsError(LS_EINVAL, "hodlr_rank must be in [0, 256]");
  if (o.restart < 1) throw LsError(LS_EINVAL, "restart must be >= 1");
  if (o.maxit < 0) throw LsError(LS_EINVAL, "maxit must be >= 0");
  if (o.prec < 0 || o.prec > 2) throw LsError(LS_EINVAL, "prec must be LS_FP64, LS_FP32 or LS_MIXED");
  if (!(o.inner_tol > 0) || o.inner_tol >= 1) throw LsError(LS_EINVAL, "inner_tol must be in (0, 1)");
  if (o.max_refine < 1) throw LsError(LS_EINVAL, "max_refine must be >= 1");
  if (o.hodlr_rank_div < 0) throw LsError(LS_EINVAL, "hodlr_rank_div must be >= 0");
  if (o.graph_iters < 0 || o.graph_iters > 64) throw LsError(LS_EINVAL, "graph_iters must be in [0, 64]");
  if (o.stencil_mfma != 0 && o.stencil_mfma != 1) throw LsError(LS_EINVAL, "stencil_mfma must be 0 or 1");
  if (o.fmm_fused != 0 && o.fmm_fused != 1) throw LsError(LS_EINVAL, "fmm_fused must be 0 or 1");
  if (o.pc_bf16 != 0 && o.pc_bf16 != 1) throw LsError(LS_EINVAL, "pc_bf16 must be 0 or 1");
  if (o.pc_lowp_solves != 0 && o.pc_lowp_solves != 1) throw LsError(LS_EINVAL, "pc_lowp_solves must be 0 or 1");
  if (!(o.hodlr_tol >= 0 && o.hodlr_tol < 1)) throw LsError(LS_EINVAL, "hodlr_tol must be in [0, 1)");
  if (o.dcgs2 != 0 && o.dcgs2 != 1) throw LsError(LS_EINVAL, "dcgs2 must be 0 or 1");
}

ls_status ls_plan_describe(int n, double L, double kappa, const ls_options* opt, ls_plan_info* out) {
  try {
    if (!out) throw LsError(LS_EINVAL, "out is NULL");
    ls_options o;
    ls_default_options(&o);
    if (opt) o = *opt;
    validate_options(o);
    if (!(L > 0) || !std::isfinite(L)) throw LsError(LS_EINVAL, "L must be positive");
    ls::PlanOptions po;
    po.leaf_max = o.leaf_max;
    po.T = o.T;
    ls::Plan p = ls::make_plan(n, L, kappa, po);
    if (p.leaf >= 32) throw LsError(LS_ENOTSUP, "too many levels");
    std::memset(out, 0, sizeof(*out));
    out->levels = p.leaf;
    out->leaf_side = p.leaf_side;
    out->top_level = p.top;
    for (int nu = 0; nu <= p.leaf; ++nu) {
      out->hf[nu] = p.lv[nu].hf;
      out->ndir[nu] = p.lv[nu].ndir;
      out->il_pairs[nu] = p.lv[nu].il_pairs;
      out->max_il[nu] = p.lv[nu].max_il;
    }
    out->near_pairs = p.near_pairs;
    ls::plan_coverage(p, out->coverage_min, out->coverage_max);
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return LS_EINVAL;
  }
}

ls_status ls_setup(const double* points, int64_t N, const double* q, double kappa, double tol, const ls_options* opt,
                   ls_problem** out) {
  if (out) *out = nullptr;
  std::unique_ptr<ls_problem> P;
  try {
    double t0 = now_ms();
    if (!out) throw LsError(LS_EINVAL, "out is NULL");
    if (!points || !q) throw LsError(LS_EINVAL, "points and q must not be NULL");
    if (N <= 0) throw LsError(LS_EINVAL, "N must be positive");
    if (!(kappa > 0) || !std::isfinite(kappa)) throw LsError(LS_EINVAL, "kappa must be positive and finite");
    if (!(tol > 0 && tol < 1)) throw LsError(LS_EINVAL, "tol must be in (0, 1)");
    P.reset(new ls_problem());
    ls_default_options(&P->opt);
    if (opt) P->opt = *opt;
    validate_options(P->opt);
    for (int64_t i = 0; i < 2 * N; ++i)
      if (!std::isfinite(points[i])) throw LsError(LS_EINVAL, "non-finite point coordinate");
    for (int64_t i = 0; i < N; ++i)
      if (!std::isfinite(q[i])) throw LsError(LS_EINVAL, "non-finite contrast value");
    // ---- recognise the uniform cell-centred grid ----
    int n = (int)std::llround(std::sqrt((double)N));
    if ((int64_t)n * n != N) throw LsError(LS_ENOTSUP, "points do not form a square n x n grid (N not a square)");
    double xmin = points[0], xmax = points[0], ymin = points[1], ymax = points[1];
    for (int64_t i = 0; i < N; ++i) {
      xmin = std::min(xmin, points[2 * i]);
      xmax = std::max(xmax, points[2 * i]);
      ymin = std::min(ymin, points[2 * i + 1]);
      ymax = std::max(ymax, points[2 * i + 1]);
    }
    if (n < 2) throw LsError(LS_ENOTSUP, "grid side must be at least 2");
    double h = (xmax - xmin) / (n - 1);
    if (!(h > 0) || std::fabs((ymax - ymin) / (n - 1) - h) > 1e-9 * h)
      throw LsError(LS_ENOTSUP, "points do not form a square grid with equal spacing");
    std::vector<int> ca(N), cb(N), grid2caller((size_t)N, -1);
    for (int64_t i = 0; i < N; ++i) {
      double fa = (points[2 * i] - xmin) / h, fb = (points[2 * i + 1] - ymin) / h;
      long a = std::lround(fa), b = std::lround(fb);
      if (std::fabs(fa - a) > 1e-6 || std::fabs(fb - b) > 1e-6 || a < 0 || a >= n || b < 0 || b >= n)
        throw LsError(LS_ENOTSUP, "points do not lie on a uniform grid");
      int64_t g = (int64_t)a * n + b;
      if (grid2caller[g] >= 0) throw LsError(LS_EINVAL, "duplicate points");
      grid2caller[g] = (int)i;
      ca[i] = (int)a;
      cb[i] = (int)b;
    }
    P->N = N;
    P->n = n;
    P->gx0 = xmin;
    P->gy0 = ymin;
    P->gh = h;
    // the inputs are valid: from here on the setup works on the current device
    hip_check(hipGetDevice(&P->device), "hipGetDevice");
    P->scratch = scratch_address(P->device);
    P->g2c.upload(grid2caller);
    P->kappa = kappa;
    P->tol = tol;
    P->coef = P->opt.sign * kappa * kappa;
    const double L = 0.5 * n * h;
    ls::PlanOptions po;
    po.leaf_max = P->opt.leaf_max;
    po.T = P->opt.T;
    P->plan = ls::make_plan(n, L, kappa, po);
    const ls::Plan& p = P->plan;
    if (P->opt.hodlr_rank > 0 && p.leaf_side * p.leaf_side > 64)
      throw LsError(LS_ENOTSUP, "the HODLR preconditioner needs quadtree leaves of at most 64 points (leaf_max)");
    double t_plan = now_ms();
    // ---- orders: Morton (solver) and S (DAFMM leaf arrays) ----
    const int side = p.leaf_side, nbL = p.lv[p.leaf].nb, nhL = nbL / 2;
    std::vector<int> mort_a(N), mort_b(N), m2c(N), c2m(N);
    {
      std::vector<std::pair<uint64_t, int>> leaves;
      for (int la = 0; la < nbL; ++la)
        for (int lb = 0; lb < nbL; ++lb) {
          uint64_t code = 0;
          for (int bit = 0; bit < 16; ++bit) {
            code |= (uint64_t)((lb >> bit) & 1) << (2 * bit);
            code |= (uint64_t)((la >> bit) & 1) << (2 * bit + 1);
          }
          leaves.push_back({code, la * nbL + lb});
        }
      std::sort(leaves.begin(), leaves.end());
      int64_t t = 0;
      for (auto& lf : leaves) {
        int la = lf.second / nbL, lb = lf.second % nbL;
        for (int a = 0; a < side; ++a)
          for (int b = 0; b < side; ++b) {
            int ga = la * side + a, gb = lb * side + b;
            mort_a[t] = ga;
            mort_b[t] = gb;
            m2c[t] = grid2caller[(int64_t)ga * n + gb];
            c2m[m2c[t]] = (int)t;
            ++t;
          }
      }
    }
    std::vector<int> s2c(N), c2s(N), s2m(N), m2s(N);
    {
      const long long plane = (long long)nhL * nhL;
      for (int ba = 0; ba < nbL; ++ba)
        for (int bb = 0; bb < nbL; ++bb) {
          int c = (ba & 1) * 2 + (bb & 1);
          int ha = ba >> 1, hb = bb >> 1;
          for (int pa = 0; pa < side; ++pa)
            for (int pb = 0; pb < side; ++pb) {
              long long sidx = (long long)(pa * side + pb) * 4 * plane + c * plane + (long long)ha * nhL + hb;
              int ga = ba * side + pa, gb = bb * side + pb;
              int ci = grid2caller[(int64_t)ga * n + gb];
              s2c[sidx] = ci;
              c2s[ci] = (int)sidx;
              s2m[sidx] = c2m[ci];
              m2s[c2m[ci]] = (int)sidx;
            }
        }
    }
    P->s2c.upload(s2c);
    P->c2s.upload(c2s);
    P->s2m.upload(s2m);
    P->m2s.upload(m2s);
    P->m2c.upload(m2c);
    std::vector<double> qc(q, q + N), qm(N), pxv(N), pyv(N);
    for (int64_t t = 0; t < N; ++t) qm[t] = q[m2c[t]];
    for (int64_t i = 0; i < N; ++i) {
      pxv[i] = points[2 * i];
      pyv[i] = points[2 * i + 1];
    }
    P->q_c.upload(qc);
    P->q_m.upload(qm);
    P->px.upload(pxv);
    P->py.upload(pyv);
    // ---- W table on the device (H0 evaluator), self-cell term on the host ----
    ls::WTable W;
    W.n = n;
    {
      DevBuf wt;
      size_t cnt = (size_t)(2 * n - 1) * (2 * n - 1);
      wt.alloc(cnt * 16);
      lsk::launch_wtable(wt.as<double2>(), n, h, kappa, nullptr);
      hip_check(hipGetLastError(), "wtable");
      W.w.resize(cnt);
      hip_check(hipMemcpy(W.w.data(), wt.p, cnt * 16, hipMemcpyDeviceToHost), "wtable d2h");
      W.w[(size_t)(n - 1) * (2 * n - 1) + (n - 1)] = self_cell(h, kappa);
    }
    // ---- NCA factors and device operators ----
    double t_w = now_ms();
    P->nca64 = ls::build_nca(p, W, tol);
    build_fmm_ops(P.get(), P->nca64, P->f64, false);
    if (P->opt.build_fp32) {
      if (P->opt.eps_inner > 0 && P->opt.eps_inner > tol)
        P->nca32 = ls::build_nca(p, W, P->opt.eps_inner);
      else
        P->nca32 = P->nca64;
      build_fmm_ops(P.get(), P->nca32, P->f32, true);
      P->have32 = true;
    }
    ensure_fmm_capacity(P.get(), P->f64, 1);
    if (P->have32) ensure_fmm_capacity(P.get(), P->f32, 1);
    double t_nca = now_ms();
    // ---- HODLR preconditioner ----
    if (P->opt.hodlr_rank > 0) {
      build_hodlr(P.get(), W, mort_a, mort_b, qm);
      P->have_hodlr = true;
    }
    double t_h = now_ms();
    hip_check(hipDeviceSynchronize(), "setup");
    // ---- stats ----
    ls_stats_t& S = P->stats;
    std::memset(&S, 0, sizeof(S));
    S.N = N;
    S.n = n;
    S.levels = p.leaf;
    S.leaf_side = side;
    S.top_level = p.top;
    for (int nu = p.top; nu <= p.leaf; ++nu)
      if (p.lv[nu].hf) S.nlevels_hf++;
    for (int nu = p.top; nu <= p.leaf; ++nu) {
      S.rank_max64 = std::max(S.rank_max64, P->f64.kmax.empty() ? 0 : P->f64.kmax[nu]);
      if (P->have32) S.rank_max32 = std::max(S.rank_max32, P->f32.kmax[nu]);
      S.m2l_pairs += p.lv[nu].il_pairs;
    }
    S.entries_near = p.near_pairs * (int64_t)side * side * side * side;
    S.entries_far64 = P->f64.entries_far;
    S.entries_far32 = P->have32 ? P->f32.entries_far : 0;
    S.entries_m2l64 = P->f64.entries_m2l;
    S.entries_m2l32 = P->have32 ? P->f32.entries_m2l : 0;
    S.entries_mid64 = (int64_t)P->f64.entries_mid;
    S.entries_mid32 = P->have32 ? (int64_t)P->f32.entries_mid : 0;
    S.stored_bytes64 = P->f64.stored_bytes;
    S.stored_bytes32 = P->have32 ? P->f32.stored_bytes : 0;
    S.hodlr_bytes = P->hod.bytes;
    S.hodlr_levels = P->have_hodlr ? P->hod.Lb : 0;
    for (int l = 0; P->have_hodlr && l < P->hod.Lb; ++l) S.hodlr_rank_sum += P->hod.rank[l];
    S.hodlr_dense_leaves = P->have_hodlr ? P->hod.dense_leaves : 0;
    S.hodlr_rank_used_sum = P->have_hodlr ? P->hod.used_rank_sum : 0;
    S.hodlr_blocks = P->have_hodlr ? P->hod.blocks : 0;
    S.hodlr_rank_used_max = P->have_hodlr ? P->hod.used_rank_max : 0;
    S.hodlr_rows_active = P->have_hodlr ? P->hod.rows_active : 0;
    for (int l = 0; P->have_hodlr && l < P->hod.Lb && l < 32; ++l) {
      S.hodlr_dot_rows[l] = l < (int)P->hod.dot_rows.size() ? P->hod.dot_rows[l] : P->N;
      S.hodlr_core_nodes[l] = l < (int)P->hod.core_nodes.size() ? P->hod.core_nodes[l] : (1 << l);
    }
    S.t_hodlr_aca_ms = P->hod.t_aca_ms;
    S.t_hodlr_apply_ms = P->hod.t_apply_ms;
    S.t_hodlr_cores_ms = P->hod.t_cores_ms;
    S.t_plan_ms = t_plan - t0;
    S.t_nca_ms = t_nca - t_w;
    S.t_hodlr_ms = t_h - t_nca;
    S.t_setup_ms = now_ms() - t0;
    *out = P.release();
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return LS_EINVAL;
  }
}

static void check_vec_args(ls_problem* P, const void* x, const void* y, int nrhs, int64_t ld) {
  if (!P) throw LsError(LS_EINVAL, "problem is NULL");
  if (!x || !y) throw LsError(LS_EINVAL, "vector pointer is NULL");
  if (nrhs <= 0) throw LsError(LS_EINVAL, "nrhs must be positive");
  if (ld < P->N) throw LsError(LS_EINVAL, "ld must be >= N");
}

ls_status ls_matvec(ls_problem* P, const void* x, void* y, int nrhs, int64_t ld, int prec, void* stream) {
  try {
    check_vec_args(P, x, y, nrhs, ld);
    if (prec != LS_FP64 && prec != LS_FP32 && prec != LS_MIXED)
      throw LsError(LS_EINVAL, "prec must be LS_FP64, LS_FP32 or LS_MIXED");
    if (x == y) throw LsError(LS_EINVAL, "x and y must not overlap");
    fmm_apply(P, prec == LS_FP32, (const double2*)x, ld, (double2*)y, ld, nrhs, 1.0, P->coef, true,
              (hipStream_t)stream);
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}

ls_status ls_apply_V(ls_problem* P, const void* x, void* y, int nrhs, int64_t ld, int prec, void* stream) {
  try {
    check_vec_args(P, x, y, nrhs, ld);
    if (prec != LS_FP64 && prec != LS_FP32 && prec != LS_MIXED)
      throw LsError(LS_EINVAL, "prec must be LS_FP64, LS_FP32 or LS_MIXED");
    if (x == y) throw LsError(LS_EINVAL, "x and y must not overlap");
    // y = V x: the epilogue with alpha = 0, coef = 1 and no contrast
    fmm_apply(P, prec == LS_FP32, (const double2*)x, ld, (double2*)y, ld, nrhs, 0.0, 1.0, true, (hipStream_t)stream,
              false);
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}

static void ensure_ws(ls_problem* P, int nrhs) {
  if (P->ws_cap >= nrhs) return;
  P->w_x.alloc((size_t)P->N * nrhs * 16);
  P->w_y.alloc((size_t)P->N * nrhs * 16);
  P->w_t.alloc((size_t)P->N * nrhs * 16);
  P->ws_cap = nrhs;
}

ls_status ls_precond_apply(ls_problem* P, const void* r, void* z, int nrhs, int64_t ld, int prec, void* stream) {
  try {
    check_vec_args(P, r, z, nrhs, ld);
    if (prec != LS_FP64 && prec != LS_FP32 && prec != LS_MIXED)
      throw LsError(LS_EINVAL, "prec must be LS_FP64, LS_FP32 or LS_MIXED");
    if (!P->have_hodlr) throw LsError(LS_ENOTSUP, "no HODLR preconditioner (hodlr_rank = 0)");
    hipStream_t s = (hipStream_t)stream;
    ensure_ws(P, nrhs);
    const long long N = P->N;
    double2* a = P->w_x.as<double2>();
    lsk::launch_permute((const double2*)r, ld, a, N, P->m2c.as<int>(), N, nrhs, false, s);
    const int fmt = prec == LS_FP64 ? 0 : (prec == LS_MIXED && P->hod.have16 ? 2 : 1);
    hodlr_apply(P, fmt, a, N, a, N, nrhs, 0, s);
    lsk::launch_permute(a, N, (double2*)z, ld, P->m2c.as<int>(), N, nrhs, true, s);
    hip_check(hipGetLastError(), "precond");
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}

ls_status ls_precond_apply_noalloc(ls_problem* P, const void* r, void* z, int nrhs, int64_t ld, int prec,
                                   void* stream) {
  try {
    check_vec_args(P, r, z, nrhs, ld);
    if (prec != LS_FP64 && prec != LS_FP32 && prec != LS_MIXED)
      throw LsError(LS_EINVAL, "prec must be LS_FP64, LS_FP32 or LS_MIXED");
    if (!P->have_hodlr) throw LsError(LS_ENOTSUP, "no HODLR preconditioner (hodlr_rank = 0)");
    int dev = -1;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (dev != P->device) throw LsError(LS_EINVAL, "the current device is not the problem's device");
    const HodlrDev& H = P->hod;
    const long long N = P->N;
    size_t np = 0, ns = 0;
    hodlr_ws_elems(H, &np, &ns);
    // layout: Morton copy of r (N x nrhs), chunk partials, s vectors; each 256-byte aligned
    const size_t b_vec = align256((size_t)N * nrhs * 16), b_part = align256(np * nrhs * 16),
                 b_svec = align256(ns * nrhs * 16);
    const size_t need = b_vec + b_part + b_svec;
    if (need > kScratchBytes)
      throw LsError(LS_EINVAL, "ls_precond_apply_noalloc: needs " + std::to_string(need) + " bytes of scratch for N = " +
                                   std::to_string(N) + ", nrhs = " + std::to_string(nrhs) + "; the maximum is " +
                                   std::to_string(kScratchBytes));
    char* base = (char*)P->scratch;
    double2* a = (double2*)base;
    HodlrWs ws;
    ws.partial = (double2*)(base + b_vec);
    ws.svec = (double2*)(base + b_vec + b_part);
    ws.timers = false;
    hipStream_t s = (hipStream_t)stream;
    lsk::launch_permute((const double2*)r, ld, a, N, P->m2c.as<int>(), N, nrhs, false, s);
    const int fmt = prec == LS_FP64 ? 0 : (prec == LS_MIXED && H.have16 ? 2 : 1);
    hodlr_apply(P, fmt, a, N, a, N, nrhs, 0, s, nullptr, 0, nullptr, 0, 0, &ws);
    lsk::launch_permute(a, N, (double2*)z, ld, P->m2c.as<int>(), N, nrhs, true, s);
    hip_check(hipGetLastError(), "precond (no allocation)");
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}

ls_status ls_direct_solve(ls_problem* P, const void* f, void* psi, int nrhs, int64_t ld, double tol, int max_refine,
                          ls_solve_info* info, void* stream) {
  try {
    const double t0 = now_ms();
    check_vec_args(P, f, psi, nrhs, ld);
    if (!P->have_hodlr) throw LsError(LS_ENOTSUP, "no HODLR factorisation (hodlr_rank = 0)");
    if (!(tol >= 0 && tol < 1)) throw LsError(LS_EINVAL, "tol must be in [0, 1)");
    if (max_refine < 0) throw LsError(LS_EINVAL, "max_refine must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    const long long N = P->N;
    P->kf.ensure((size_t)N * nrhs * 16);
    P->kx.ensure((size_t)N * nrhs * 16);
    P->kdx.ensure((size_t)N * nrhs * 16);
    ensure_ws(P, nrhs);
    double2* fm = P->kf.as<double2>();
    double2* xm = P->kx.as<double2>();
    double2* dm = P->kdx.as<double2>();
    double2* w = P->w_y.as<double2>();
    lsk::launch_permute((const double2*)f, ld, fm, N, P->m2c.as<int>(), N, nrhs, false, s);
    std::vector<double> fn, rn;
    norms(P, fm, nrhs, fn, s);
    // x = A~^{-1} f, then refinement x += A~^{-1} (f - A x) with FP64 DAFMM products
    hodlr_apply(P, 0, fm, N, xm, N, nrhs, 0, s);
    int steps = 0;
    for (;;) {
      op_apply(P, false, xm, w, nrhs, s);
      lsk::launch_axpby(1.0, fm, N, -1.0, w, N, w, N, N, nrhs, s);
      norms(P, w, nrhs, rn, s);
      bool ok = true;
      for (int c = 0; c < nrhs; ++c) ok &= !(rn[c] > tol * (fn[c] > 0 ? fn[c] : 1.0));
      if (ok || steps >= max_refine) break;
      hodlr_apply(P, 0, w, N, dm, N, nrhs, 0, s);
      lsk::launch_axpby(1.0, xm, N, 1.0, dm, N, xm, N, N, nrhs, s);
      ++steps;
    }
    lsk::launch_permute(xm, N, (double2*)psi, ld, P->m2c.as<int>(), N, nrhs, true, s);
    hip_check(hipStreamSynchronize(s), "direct solve");
    const double t1 = now_ms();
    if (info)
      for (int c = 0; c < nrhs; ++c) {
        const double rel = fn[c] > 0 ? rn[c] / fn[c] : 0.0;
        info[c].iters = steps;
        info[c].relres = rel;
        info[c].status = !std::isfinite(rel) ? LS_NAN : (rel <= tol ? LS_CONVERGED : LS_MAXIT);
        info[c].n_refine = steps;
        info[c].t_solve_ms = t1 - t0;
        info[c].relres0 = 1.0;
      }
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}

ls_status ls_rhs_planewave(ls_problem* P, const double* angles, int nrhs, void* f, int64_t ld, void* stream) {
  try {
    if (!P || !angles || !f) throw LsError(LS_EINVAL, "NULL argument");
    if (nrhs <= 0) throw LsError(LS_EINVAL, "nrhs must be positive");
    if (ld < P->N) throw LsError(LS_EINVAL, "ld must be >= N");
    for (int i = 0; i < nrhs; ++i)
      if (!std::isfinite(angles[i])) throw LsError(LS_EINVAL, "non-finite angle");
    hipStream_t s = (hipStream_t)stream;
    DevBuf ang;
    ang.upload(std::vector<double>(angles, angles + nrhs));
    lsk::launch_planewave(P->px.as<double>(), P->py.as<double>(), P->q_c.as<double>(), ang.as<double>(), P->kappa,
                          -P->coef, (double2*)f, ld, P->N, nrhs, s);
    hip_check(hipStreamSynchronize(s), "planewave");
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}

// ls_solve's body; graph_iters > 0 selects the graph-captured GMRES driver
static void solve_impl(ls_problem* P, const void* f, void* psi, int nrhs, int64_t ld, double tol, int x0_given,
                       int prec_override, ls_solve_info* info, hipStream_t stream, int graph_iters) {
  {
    double t0 = now_ms();
    check_vec_args(P, f, psi, nrhs, ld);
    if (!(tol > 0 && tol < 1)) throw LsError(LS_EINVAL, "tol must be in (0, 1)");
    hipStream_t s = (hipStream_t)stream;
    const long long N = P->N;
    if (prec_override < -1 || prec_override > 2) throw LsError(LS_EINVAL, "prec must be -1, LS_FP64, LS_FP32 or LS_MIXED");
    const int prec = prec_override >= 0 ? prec_override : P->opt.prec;
    if ((prec == LS_FP32 || prec == LS_MIXED) && !P->have32) throw LsError(LS_ENOTSUP, "FP32 operator not built");
    P->kf.ensure((size_t)N * nrhs * 16);
    P->kx.ensure((size_t)N * nrhs * 16);
    P->kdx.ensure((size_t)N * nrhs * 16);
    double2* fm = P->kf.as<double2>();
    double2* xm = P->kx.as<double2>();
    double2* dm = P->kdx.as<double2>();
    lsk::launch_permute((const double2*)f, ld, fm, N, P->m2c.as<int>(), N, nrhs, false, s);
    std::vector<double> fn;
    norms(P, fm, nrhs, fn, s);
    std::vector<ColState> st(nrhs);
    std::vector<int> warm_rejected(nrhs, 0);
    for (int c = 0; c < nrhs; ++c) {
      st[c].fnorm = fn[c] > 0 ? fn[c] : 1.0;
      st[c].tol = tol;
    }
    std::vector<double> rel0(nrhs, 1.0);
    if (x0_given) {
      lsk::launch_permute((const double2*)psi, ld, xm, N, P->m2c.as<int>(), N, nrhs, false, s);
      // minimal-residual scaling of the guess g: x0 = xi g, xi = (A g)^H f / ||A g||^2, which
      // leaves ||f - A x0||^2 = ||f||^2 - |(A g)^H f|^2 / ||A g||^2
      ensure_ws(P, nrhs);
      double2* w = P->w_y.as<double2>();
      op_apply(P, false, xm, w, nrhs, s);
      std::vector<double> an;
      norms(P, w, nrhs, an, s);
      const int nch = nchunks_for(P);
      P->kpart.ensure((size_t)nrhs * nch * 16);
      P->kh.ensure((size_t)nrhs * 16);
      double2* part = P->kpart.as<double2>();
      double2* hd = P->kh.as<double2>();
      lsk::launch_gs_dot(w, N, N, 1, fm, N, part, N, nch, 1, nrhs, s);
      lsk::launch_gs_finish(part, nch, 1, 1, hd, 0, nrhs, s);
      std::vector<zd> dot(nrhs);
      hip_check(hipMemcpyAsync(dot.data(), hd, nrhs * 16, hipMemcpyDeviceToHost, s), "dot d2h");
      hip_check(hipStreamSynchronize(s), "sync");
      std::vector<zd> xi(nrhs, zd(0));
      for (int c = 0; c < nrhs; ++c) {
        const double a2 = an[c] * an[c];
        const double drop = a2 > 0 ? std::norm(dot[c]) / a2 : 0.0;
        const bool ok = std::isfinite(a2) && std::isfinite(drop) && a2 > 0 && fn[c] > 0 && drop > 1e-24 * fn[c] * fn[c];
        if (ok) xi[c] = dot[c] / a2;
        warm_rejected[c] = !ok;
      }
      hip_check(hipMemcpyAsync(hd, xi.data(), nrhs * 16, hipMemcpyHostToDevice, s), "xi h2d");
      // starting residual f - xi A g (reported), then x0 = xi g
      lsk::launch_axpby(1.0, fm, N, 0.0, fm, N, dm, N, N, nrhs, s);
      lsk::launch_gs_axpy(w, N, N, 1, hd, 1, -1.0, dm, N, N, nrhs, s);
      std::vector<double> r0;
      norms(P, dm, nrhs, r0, s);
      for (int c = 0; c < nrhs; ++c)
        if (!warm_rejected[c]) rel0[c] = r0[c] / fn[c];
      hip_check(hipMemsetAsync(w, 0, (size_t)N * nrhs * 16, s), "memset");
      lsk::launch_gs_axpy(xm, N, N, 1, hd, 1, 1.0, w, N, N, nrhs, s);
      lsk::launch_axpby(1.0, w, N, 0.0, w, N, xm, N, N, nrhs, s);
      for (int c = 0; c < nrhs; ++c)
        if (warm_rejected[c]) hip_check(hipMemsetAsync(xm + (long long)c * N, 0, N * 16, s), "memset");
    } else {
      hip_check(hipMemsetAsync(xm, 0, (size_t)N * nrhs * 16, s), "memset");
    }
    for (int c = 0; c < nrhs; ++c)
      if (fn[c] == 0) {
        st[c].done = true;
        st[c].status = LS_CONVERGED;
        hip_check(hipMemsetAsync(xm + (long long)c * N, 0, N * 16, s), "memset");
      }
    GmresCfg cfg;
    cfg.restart = P->opt.restart;
    cfg.dcgs2 = P->opt.dcgs2 != 0;
    cfg.maxit = P->opt.maxit;
    cfg.pc = P->have_hodlr;
    std::vector<int> nref(nrhs, 0);
    if (prec == LS_FP64 || prec == LS_FP32) {
      cfg.op32 = prec == LS_FP32;
      cfg.pcf = prec == LS_FP32 ? 1 : 0;
      if (graph_iters > 0)
        gmres_graph(P, cfg, fm, xm, nrhs, st, graph_iters, s);
      else
        gmres(P, cfg, fm, xm, nrhs, st, s);
    } else {
      // mixed: flexible GMRES whose products switch from the FP64 to the FP32 operator once
      // every residual estimate is below tol / delta32 (relaxation of inexact Krylov methods),
      // FP32 off-diagonal HODLR factors throughout; each restart recomputes the true FP64
      // residual f - A x (iterative refinement); after max_refine such cycles, or once a
      // cycle fails to lower the true residual by 10%, the products stay FP64.
      cfg.op32 = false;
      cfg.pcf = P->hod.have16 ? 2 : 1;
      cfg.flexible = true;
      cfg.relax = std::min(0.5, tol / P->opt.inner_tol);
      cfg.max_refine = P->opt.max_refine;
      if (graph_iters > 0)
        gmres_graph(P, cfg, fm, xm, nrhs, st, graph_iters, s);
      else
        gmres(P, cfg, fm, xm, nrhs, st, s);
      for (int c = 0; c < nrhs; ++c) {
        nref[c] = st[c].cycles;
        if (st[c].fell_back && st[c].status == LS_CONVERGED) st[c].status = LS_REFINE_STAGNATED;
      }
    }
    // final true residual with the FP64 operator
    ensure_ws(P, nrhs);
    double2* w = P->w_y.as<double2>();
    op_apply(P, false, xm, w, nrhs, s);
    lsk::launch_axpby(1.0, fm, N, -1.0, w, N, w, N, N, nrhs, s);
    std::vector<double> rn;
    norms(P, w, nrhs, rn, s);
    lsk::launch_permute(xm, N, (double2*)psi, ld, P->m2c.as<int>(), N, nrhs, true, s);
    hip_check(hipStreamSynchronize(s), "solve");
    double t1 = now_ms();
    if (info)
      for (int c = 0; c < nrhs; ++c) {
        info[c].iters = st[c].its;
        info[c].relres = fn[c] > 0 ? rn[c] / fn[c] : 0.0;
        info[c].status = st[c].status;
        if (warm_rejected[c] && st[c].status == LS_CONVERGED) info[c].status = LS_WARMSTART_REJECTED;
        info[c].n_refine = nref[c];
        info[c].t_solve_ms = t1 - t0;
        info[c].relres0 = fn[c] > 0 ? rel0[c] : 0.0;
      }
  }
}

ls_status ls_solve(ls_problem* P, const void* f, void* psi, int nrhs, int64_t ld, double tol, int x0_given,
                   int prec_override, ls_solve_info* info, void* stream) {
  try {
    if (!P) throw LsError(LS_EINVAL, "NULL problem");
    solve_impl(P, f, psi, nrhs, ld, tol, x0_given, prec_override, info, (hipStream_t)stream, P->opt.graph_iters);
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}

// Autotuner: times the launch shapes of the two reduction kernels on this problem's own sizes
// and keeps the fastest (rows per workgroup chunk of the Arnoldi dot products and norms; max
// rows per chunk of the HODLR level reductions).  Small problems want short chunks (more
// workgroups), large ones long chunks (fewer partial sums).
static const int kGsRows[5] = {128, 256, 512, 1024, 2048};
static const int kPcRows[5] = {64, 128, 256, 512, 1024};

static void autotune_impl(ls_problem* P, ls_tune_info* out, hipStream_t s) {
  const long long N = P->N;
  const int ncols = 32, reps = 5;
  DevBuf A, w, w2, part, np, no;
  A.alloc((size_t)ncols * N * 16);
  w.alloc((size_t)N * 16);
  w2.alloc((size_t)N * 16);
  part.alloc((size_t)1025 * ncols * 16);  // partials of up to 1024 chunks, then the sums
  np.alloc((size_t)1024 * 8);
  no.alloc(64);
  hip_check(hipMemsetAsync(A.p, 0, A.bytes, s), "memset");
  hip_check(hipMemsetAsync(w.p, 0, w.bytes, s), "memset");
  hipEvent_t e0, e1;
  hip_check(hipEventCreate(&e0), "hipEventCreate");
  hip_check(hipEventCreate(&e1), "hipEventCreate");
  auto timed = [&](auto&& body) {
    body();  // warm-up
    hip_check(hipEventRecord(e0, s), "hipEventRecord");
    for (int r = 0; r < reps; ++r) body();
    hip_check(hipEventRecord(e1, s), "hipEventRecord");
    hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
    float ms = 0;
    hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    return 1e3 * (double)ms / reps;
  };
  ls_tune_info info{};
  double best = 1e300;
  int best_gs = P->tune.gs_rows;
  for (int i = 0; i < 5; ++i) {
    P->tune.gs_rows = kGsRows[i];
    const int nch = nchunks_for(P);
    info.gs_us[i] = timed([&] {
      lsk::launch_gs_dot(A.as<double2>(), N, 0, ncols, w.as<double2>(), N, part.as<double2>(), N, nch, ncols, 1, s);
      lsk::launch_gs_finish(part.as<double2>(), nch, ncols, ncols, part.as<double2>() + (size_t)1024 * ncols, 0, 1,
                            s);
      lsk::launch_norm2(w.as<double2>(), N, np.as<double>(), N, nch, 1, s);
      lsk::launch_norm2_finish(np.as<double>(), nch, no.as<double>(), 1, s);
    });
    if (info.gs_us[i] < best) {
      best = info.gs_us[i];
      best_gs = kGsRows[i];
    }
  }
  P->tune.gs_rows = best_gs;
  info.gs_rows = best_gs;
  info.hodlr_rows = P->tune.hodlr_rows;
  if (P->have_hodlr) {
    best = 1e300;
    int best_pc = P->tune.hodlr_rows;
    for (int i = 0; i < 5; ++i) {
      hodlr_chunks(P->hod, kPcRows[i]);
      hodlr_ensure_ws(P, 1);
      const int fmt = P->hod.have16 ? 2 : (P->have32 ? 1 : 0);
      info.pc_us[i] = timed([&] { hodlr_apply(P, fmt, w.as<double2>(), N, w2.as<double2>(), N, 1, 0, s); });
      if (info.pc_us[i] < best) {
        best = info.pc_us[i];
        best_pc = kPcRows[i];
      }
    }
    P->tune.hodlr_rows = best_pc;
    hodlr_chunks(P->hod, best_pc);
    info.hodlr_rows = best_pc;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  hip_check(hipStreamSynchronize(s), "autotune");
  P->tune.done = true;
  if (out) *out = info;
}

ls_status ls_autotune(ls_problem* P, ls_tune_info* out, void* stream) {
  try {
    if (!P) throw LsError(LS_EINVAL, "NULL problem");
    autotune_impl(P, out, (hipStream_t)stream);
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}

// Queue of independent problems: largest first, pulled dynamically by worker threads, each
// with its own HIP stream; every solve runs the graph-captured GMRES driver.
ls_status ls_solve_queue(ls_problem* const* probs, int nprob, const void* const* f, void* const* psi, double tol,
                         int prec, int nworkers, int graph_iters, ls_solve_info* info) {
  try {
    if (!probs || !f || !psi || !info || nprob < 1) throw LsError(LS_EINVAL, "NULL argument or nprob < 1");
    if (nworkers < 0 || nworkers > 16) throw LsError(LS_EINVAL, "nworkers must be in [0, 16]");
    if (graph_iters < 0 || graph_iters > 64) throw LsError(LS_EINVAL, "graph_iters must be in [0, 64]");
    if (!(tol > 0 && tol < 1)) throw LsError(LS_EINVAL, "tol must be in (0, 1)");
    if (prec < -1 || prec > 2) throw LsError(LS_EINVAL, "prec must be -1, LS_FP64, LS_FP32 or LS_MIXED");
    for (int i = 0; i < nprob; ++i) {
      if (!probs[i] || !f[i] || !psi[i]) throw LsError(LS_EINVAL, "NULL problem or vector in the queue");
      for (int j = 0; j < i; ++j)
        if (probs[j] == probs[i]) throw LsError(LS_EINVAL, "a problem appears twice in the queue");
    }
    const int nw = std::min(nprob, nworkers == 0 ? 4 : nworkers);
    const int gi = graph_iters == 0 ? 8 : graph_iters;
    std::vector<int> order(nprob);
    for (int i = 0; i < nprob; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return probs[a]->N > probs[b]->N; });
    std::vector<hipStream_t> streams(nw, nullptr);
    for (auto& st : streams) hip_check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
    std::atomic<int> next{0};
    std::mutex mu;
    std::string err;
    ls_status err_code = LS_OK;
    auto worker = [&](int wi) {
      hipStream_t s = streams[wi];
      for (;;) {
        const int k = next.fetch_add(1);
        if (k >= nprob) return;
        const int p = order[k];
        try {
          if (!probs[p]->tune.done) autotune_impl(probs[p], nullptr, s);
          solve_impl(probs[p], f[p], psi[p], 1, probs[p]->N, tol, 0, prec, &info[p], s, gi);
        } catch (const LsError& e) {
          std::lock_guard<std::mutex> lk(mu);
          if (err_code == LS_OK) {
            err_code = (ls_status)e.code;
            err = std::string("queue problem ") + std::to_string(p) + ": " + e.what();
          }
        }
      }
    };
    std::vector<std::thread> th;
    for (int wi = 0; wi < nw; ++wi) th.emplace_back(worker, wi);
    for (auto& t : th) t.join();
    for (auto& st : streams) (void)hipStreamDestroy(st);
    if (err_code != LS_OK) throw LsError(err_code, err);
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}

namespace {

// Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on P_n
void gauss_legendre(int n, double* t, double* w) {
  for (int i = 0; i < n; ++i) {
    double x = std::cos(lsk::kPi * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    t[i] = x;
    w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
}

const lsk::FieldRules& field_rules() {
  static lsk::FieldRules R = [] {
    lsk::FieldRules r{};
    const int orders[lsk::kFieldRules] = {3, 4, 5, 6, 8, 10, 12, 16, 24, 10};
    int off = 0;
    for (int k = 0; k < lsk::kFieldRules; ++k) {
      r.off[k] = off;
      r.n[k] = orders[k];
      gauss_legendre(orders[k], r.t + off, r.w + off);
      off += orders[k];
    }
    return r;
  }();
  return R;
}

void field_impl(ls_problem* P, const double* targets, int64_t M, const void* psi, int mode, const double* q_t,
                double theta, void* u, double* E, void* stream) {
  if (!P) throw LsError(LS_EINVAL, "NULL problem");
  if (M < 0) throw LsError(LS_EINVAL, "M must be >= 0");
  if (M == 0) return;
  if (!targets || !psi || (mode == 0 && !u) || (mode == 1 && (!q_t || !E)))
    throw LsError(LS_EINVAL, "NULL buffer");
  if (!std::isfinite(theta)) throw LsError(LS_EINVAL, "theta must be finite");
  if (M > (int64_t)INT32_MAX) throw LsError(LS_EINVAL, "too many targets");
  lsk::launch_field_eval(targets, M, P->n, P->gx0, P->gy0, P->gh, P->kappa, psi, P->g2c.as<int>(), field_rules(),
                         mode, q_t, theta, (double)P->opt.sign, u, E, (hipStream_t)stream);
  hip_check(hipGetLastError(), "field kernel");
}

}  // namespace

ls_status ls_field_eval(ls_problem* P, const double* targets, int64_t M, const void* psi, void* u, void* stream) {
  try {
    field_impl(P, targets, M, psi, 0, nullptr, 0.0, u, nullptr, stream);
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}

ls_status ls_error_eval(ls_problem* P, const double* targets, int64_t M, const double* q_t, double theta,
                        const void* psi, double* E, void* stream) {
  try {
    field_impl(P, targets, M, psi, 1, q_t, theta, nullptr, E, stream);
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}

ls_status ls_green_table(int n, double h, double kappa, void* out, void* stream) {
  try {
    if (n < 1 || !(h > 0) || !std::isfinite(h)) throw LsError(LS_EINVAL, "n must be >= 1 and h > 0");
    if (!(kappa > 0) || !std::isfinite(kappa)) throw LsError(LS_EINVAL, "kappa must be positive and finite");
    if (!out) throw LsError(LS_EINVAL, "out is NULL");
    if (kappa * h * 0.7072 >= 4.0) throw LsError(LS_ENOTSUP, "kappa * h too large for the self-cell series");
    hipStream_t s = (hipStream_t)stream;
    lsk::launch_wtable((double2*)out, n, h, kappa, s);
    hip_check(hipGetLastError(), "wtable");
    zd w0 = self_cell(h, kappa);
    double2 v = make_double2(w0.real(), w0.imag());
    hip_check(hipMemcpyAsync((double2*)out + (size_t)(n - 1) * (2 * n - 1) + (n - 1), &v, 16, hipMemcpyHostToDevice, s),
              "w0");
    hip_check(hipStreamSynchronize(s), "sync");
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}

ls_status ls_stats(const ls_problem* P, ls_stats_t* out) {
  if (!P || !out) {
    g_last_error = "NULL argument";
    return LS_EINVAL;
  }
  *out = P->stats;
  return LS_OK;
}

void ls_destroy(ls_problem* P) {
  if (!P) return;
  for (auto& pc : P->prof)
    for (auto& e : pc.ev) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  delete P;
}

ls_status ls_profile_enable(ls_problem* P, int cls, int every) {
  if (!P || cls < 0 || cls >= kProfClasses || every < 0) {
    g_last_error = "bad arguments";
    return LS_EINVAL;
  }
  ProfileClass& pc = P->prof[cls];
  pc.enabled = every != 0;
  if (every) {
    pc.every = every;
    pc.used = 0;
    pc.count = 0;
  }
  return LS_OK;
}

ls_status ls_profile_read_each(ls_problem* P, int cls, double* ms, int* tags, int64_t cap, int64_t* n) {
  try {
    if (!P || cls < 0 || cls >= kProfClasses || cap < 0 || (cap > 0 && (!ms || !tags)) || !n)
      throw LsError(LS_EINVAL, "bad arguments");
    ProfileClass& pc = P->prof[cls];
    const size_t m = std::min(pc.used, (size_t)cap);
    for (size_t i = 0; i < m; ++i) {
      hip_check(hipEventSynchronize(pc.ev[i].second), "event sync");
      float t = 0;
      hip_check(hipEventElapsedTime(&t, pc.ev[i].first, pc.ev[i].second), "elapsed");
      ms[i] = t;
      tags[i] = i < pc.tag.size() ? pc.tag[i] : -1;
    }
    *n = (int64_t)pc.used;
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}

ls_status ls_profile_read(ls_problem* P, int cls, double* total_ms, int64_t* launches, int64_t* all_launches) {
  try {
    if (!P || cls < 0 || cls >= kProfClasses || !total_ms || !launches) throw LsError(LS_EINVAL, "bad arguments");
    ProfileClass& pc = P->prof[cls];
    double tot = 0;
    for (size_t i = 0; i < pc.used; ++i) {
      hip_check(hipEventSynchronize(pc.ev[i].second), "event sync");
      float ms = 0;
      hip_check(hipEventElapsedTime(&ms, pc.ev[i].first, pc.ev[i].second), "elapsed");
      tot += ms;
    }
    *total_ms = tot;
    *launches = (int64_t)pc.used;
    if (all_launches) *all_launches = pc.count;
    return LS_OK;
  } catch (const LsError& e) {
    return fail(e);
  }
}

}  // extern "C"
