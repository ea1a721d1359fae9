// HODLR preconditioner of libls (Section 6): factor construction on the device and the apply
// (leaf solves, per-level Sherman-Morrison-Woodbury).
#include "api_internal.h"

namespace lsi {

// ---------------------------------------------------------------------------------------
// HODLR
// ---------------------------------------------------------------------------------------
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
                 int lstop, hipStream_t s, const int* jdev, long long bldj, double2* zcopy, long long zldr,
                 long long zldj, const HodlrWs* ws) {
  HodlrDev& H = P->hod;
  if (!ws) hodlr_ensure_ws(P, nrhs);
  double2* const partial = ws ? ws->partial : H.partial.as<double2>();
  double2* const svec = ws ? ws->svec : H.svec.as<double2>();
  const bool tm = ws ? ws->timers : true;
  // one right-hand side with complex128 leaf and core solves: the leaf solves and the deepest
  // levels (F .. Lb-1, whose nodes lie inside one level-F node) in one launch
  const int sf = nrhs == 1 && !P->opt.pc_lowp_solves ? H.sub_rows : 0;
  const int F = sf ? H.Lb - (sf == 512 ? 3 : 2) : H.Lb;
  const bool sub = sf > 0 && lstop < F;
  if (sub) {
    lsk::SubtreeLevels lv{};
    for (int l = F; l < H.Lb; ++l) {
      const int i = l - F;
      lv.W[i] = fmt == 2 ? H.W16[l].p : (fmt == 1 ? H.W32[l].p : H.W64[l].p);
      lv.Y[i] = fmt == 2 ? H.Y16[l].p : (fmt == 1 ? H.Y32[l].p : H.Y64[l].p);
      lv.K[i] = H.coreinv[l].as<double2>();
      lv.r[i] = H.rank[l];
    }
    ProfScope ps(P, kProfSubtree, s, tm);
    lsk::launch_hodlr_subtree(fmt, sf, H.Dinv.as<double2>(), H.ident.as<unsigned char>(), b, jdev, bldj, z, H.N,
                              H.Lb, lv, H.nodeact.p ? H.nodeact.as<unsigned char>() : nullptr, s);
  } else {
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
  for (int l = (sub ? F : H.Lb) - 1; l >= lstop; --l) {
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
  H.sub_rows = lsk::hodlr_subtree_rows(N, H.lp, H.Lb, H.rank.data());
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

}  // namespace lsi
