// Internals shared by the units of libls behind the C ABI (include/ls.h): device buffers, the
// device state of the DAFMM operator, the HODLR preconditioner and the Krylov driver, the problem
// handle, the launch timers, and the functions one unit calls in another.  Not a public header.
#pragma once
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

namespace lsi {

// the calling thread's last error message (ls_last_error)
extern thread_local std::string g_last_error;


inline double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

inline void hip_check(hipError_t e, const char* what) {
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

// The passes of the product in one launch layout (task lists of P2M, M2M, the middle launch,
// L2L, L2P).
struct Passes {
  Phase p2m, nearm2l, l2p;
  std::vector<Phase> up;    // M2M, deepest parent first
  std::vector<Phase> down;  // L2L, top parent first
  // P2M reads the product's input through the tree-order map (and stores the tree-order copy
  // for the near field) and L2P finishes the output: no separate gather and epilogue launches
  bool io_fold = false;
};

// products of at least this many right-hand sides use the wide layout
constexpr int kWideRhs = 8;

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
  // narrow: products of fewer than kWideRhs columns (short chains and blocks, P2M and L2P with the
  // gather and epilogue folded in: latency first); wide: blocks of columns (longer chains, four
  // row tiles per block in every pass, separate gather and epilogue: throughput first)
  Passes narrow, wide;
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
  // rows per level-F node of the one-launch deep-level apply (0: every level in its own launches)
  int sub_rows = 0;
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
constexpr int kProfClasses = 21;
constexpr int kProfSpan = 10;
constexpr int kProfSubtree = 20;  // the one-launch leaf solves and deepest HODLR levels

struct ProfileClass {
  bool enabled = false;
  int every = 1;       // time every `every`-th launch
  int64_t count = 0;   // launches of the class since enabling
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  std::vector<int> tag;  // per timed launch: the caller's tag (a HODLR level; -1 none)
  size_t used = 0;     // timed launches
};


}  // namespace lsi

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
  lsi::DevBuf s2c, c2s, s2m, m2s, m2c;
  lsi::DevBuf q_c, q_m, px, py;
  lsi::DevBuf g2c;                    // grid index a*n + b -> caller index
  double gx0 = 0, gy0 = 0, gh = 0;  // centre of cell (0, 0) and the cell side
  lsi::FmmDev f64, f32;
  bool have32 = false;
  lsi::HodlrDev hod;
  bool have_hodlr = false;
  // workspaces
  lsi::DevBuf w_x, w_y, w_t;  // Morton-order vectors (nrhs_cap)
  int ws_cap = 0;
  ls_stats_t stats{};
  lsi::ProfileClass prof[lsi::kProfClasses];
  // Krylov workspace
  lsi::DevBuf kQ, kZ, kw, kz, kr, kh, kpart, knp, kno, kalpha, ky, kx, kf, kdx;
  size_t kcap_key = 0;
  lsi::KrylovDev kd;
  bool capturing = false;  // launches are being recorded into a graph (no event timers)
  struct {
    int gs_rows = 1024;    // rows per chunk of the Arnoldi reductions
    int hodlr_rows = 1024;  // max rows per chunk of the HODLR level reductions
    int dot2_rows = 1024;  // rows per workgroup of the delayed-CGS2 inner products
    bool done = false;
  } tune;
};

namespace lsi {

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

// Workspaces of one apply: the chunk partials of W^T z and the s vectors of the SMW cores.
struct HodlrWs {
  double2* partial = nullptr;
  double2* svec = nullptr;
  bool timers = true;  // sampled kernel timers may create events
};

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

inline ls_status fail(const LsError& e) {
  g_last_error = e.what();
  return (ls_status)e.code;
}

// ---- DAFMM operator (api_fmm.cpp) ----
void build_fmm_ops(ls_problem* P, const ls::NCA& nca, FmmDev& F, bool fp32);
void build_phases(ls_problem* P, FmmDev& F);
void ensure_fmm_capacity(ls_problem* P, FmmDev& F, int nrhs);
void run_phase(ls_problem* P, FmmDev& F, Phase& ph, int nrhs, hipStream_t s, int prof_cls = -1,
               const lsk::IoArgs* io = nullptr);
// y = alpha x + coef diag(q) (V x) in Morton (caller_order false) or caller order; with_q = false:
// y = alpha x + coef (V x)
void fmm_apply(ls_problem* P, bool fp32, const double2* x, long long ldx, double2* y, long long ldy, int nrhs,
               double alpha, double coef, bool caller_order, hipStream_t s, bool with_q = true);

// ---- HODLR preconditioner (api_hodlr.cpp) ----
void hodlr_ws_elems(const HodlrDev& H, size_t* np, size_t* ns);
void hodlr_ensure_ws(ls_problem* P, int nrhs);
void hodlr_apply(ls_problem* P, int fmt, const double2* b, long long ldb, double2* z, long long ldz, int nrhs,
                 int lstop, hipStream_t s, const int* jdev = nullptr, long long bldj = 0, double2* zcopy = nullptr,
                 long long zldr = 0, long long zldj = 0, const HodlrWs* ws = nullptr);
void hodlr_chunks(HodlrDev& H, long long max_rows);
void build_hodlr(ls_problem* P, const ls::WTable& W, const std::vector<int>& mort_a, const std::vector<int>& mort_b,
                 const std::vector<double>& qm);

// ---- GMRES (api_gmres.cpp) ----
void op_apply(ls_problem* P, bool op32, const double2* x, double2* y, int nrhs, hipStream_t s);
int nchunks_for(const ls_problem* P);
void norms(ls_problem* P, const double2* v, int nrhs, std::vector<double>& out, hipStream_t s);
void gmres(ls_problem* P, const GmresCfg& cfg, const double2* f, double2* x, int nrhs, std::vector<ColState>& st,
           hipStream_t s);
void gmres_graph(ls_problem* P, const GmresCfg& cfg, const double2* f, double2* x, int nrhs,
                 std::vector<ColState>& st, int steps_in, hipStream_t s);

// ---- setup (api_setup.cpp) ----
zd self_cell(double h, double kappa);

// ---- C ABI unit (api.cpp) ----
void* scratch_address(int device);
void solve_impl(ls_problem* P, const void* f, void* psi, int nrhs, int64_t ld, double tol, int x0_given,
                int prec_override, ls_solve_info* info, hipStream_t s, int graph_iters);

}  // namespace lsi
