// Scheduling entry points of libls: the autotuner of the reduction launch shapes and the queue
// of independent problems solved concurrently on worker streams.
#include "api_internal.h"


using namespace lsi;

extern "C" {

// Autotuner: times the launch shapes of the two reduction kernels on this problem's own sizes
// and keeps the fastest (rows per workgroup chunk of the Arnoldi dot products and norms; max
// rows per chunk of the HODLR level reductions).  Small problems want short chunks (more
// workgroups), large ones long chunks (fewer partial sums).
static const int kGsRows[5] = {256, 512, 1024, 2048, 4096};
static const int kPcRows[5] = {128, 256, 512, 1024, 2048};

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

}  // extern "C"
