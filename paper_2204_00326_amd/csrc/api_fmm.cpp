// DAFMM operator of libls (Section 5): operator upload, the passes as stencil-GEMM task lists
// (matrix-core or VALU form) and the product y = alpha x + coef diag(q) V x.
#include "api_internal.h"

namespace lsi {

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
  // over more waves, then over more workgroups), so that no block forms a long tail; row tiles
  // per block in the chain passes; set per pass layout below
  int kMaxChain = F.fp32 ? 144 : 72;
  int chain_rpg = 1;
  bool record_hps = true;  // the narrow layout's task lists also feed the fused launch
  Passes* S = &F.narrow;
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
    if (record_hps) hps.push_back({tasks, terms, pairs});
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
    // no far field: the near field is the whole product (the same in both layouts)
    for (Passes* T : {&F.narrow, &F.wide}) {
      record_hps = T == &F.narrow;
      T->io_fold = false;
      T->up.clear();
      T->down.clear();
      std::vector<lsk::DTask> tasks;
      std::vector<lsk::DTerm> terms;
      std::vector<int> prio;
      std::vector<std::array<int, 2>> chunk;
      for (const Group& g : near_g) append(tasks, terms, prio, chunk, g, 0);
      mk_phase(T->nearm2l, tasks, terms, 4);
      T->nearm2l.tag = 0;
    }
    F.entries_mid = 0;
    for (const Group& g : near_g) F.entries_mid += g.work;
    build_fused();
    return;
  }
  // two layouts of the same tasks: narrow (latency first) and wide (throughput first, for blocks
  // of at least kWideRhs columns; longer chains, four row tiles per block, separate gather and
  // epilogue), measured best at one and at 64 columns of the 512^2 disc
  for (int wide = 0; wide < 2; ++wide) {
    S = wide ? &F.wide : &F.narrow;
    record_hps = !wide;
    kMaxChain = wide ? 288 : (F.fp32 ? 144 : 72);
    chain_rpg = wide ? 4 : 1;
    // ---- P2M ----
    S->io_fold = !wide && P->opt.stencil_mfma && !P->opt.fmm_fused;
    Group p2m_g;
    for (int c = 0; c < 4; ++c) {
      lsk::DTask tk{};
      tk.io = S->io_fold ? lsk::IO_GATHER : 0;
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
    S->up.clear();
    S->up.resize(leaf - p.top);
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
        Phase& ph = u == 0 ? S->p2m : (u < nU ? S->up[u - 1] : S->nearm2l);
        if (P->opt.stencil_mfma)
          make_phase_mfma(ph, tasks, terms, u == nU ? 4 : chain_rpg, prio, &acc, &acc_elems, u == nU, chunk);
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
        tk.io = S->io_fold ? lsk::IO_EPILOGUE : 0;
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
      mk_phase(S->l2p, tasks, terms, chain_rpg);
      S->l2p.tag = 4;
    }
    // ---- L2L (parent nu -> children nu+1), top first ----
    S->down.clear();
    S->down.resize(leaf - p.top);
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
      mk_phase(S->down[nu - p.top], tasks, terms, chain_rpg);
      S->down[nu - p.top].tag = 3;
    }
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

void run_phase(ls_problem* P, FmmDev& F, Phase& ph, int nrhs, hipStream_t s, int prof_cls, const lsk::IoArgs* io) {
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

// y = alpha x + coef diag(q) (V x) in Morton (mode 0) or caller (mode 1) order; with_q = false:
// y = alpha x + coef (V x).
void fmm_apply(ls_problem* P, bool fp32, const double2* x, long long ldx, double2* y, long long ldy, int nrhs,
               double alpha, double coef, bool caller_order, hipStream_t s, bool with_q) {
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
  // with io_fold the gather is P2M's and the epilogue L2P's (their spans are not opened: an
  // empty span would read the cost of two event records, about 4 us)
  Passes& S = nrhs >= kWideRhs ? F.wide : F.narrow;
  const bool fold = S.io_fold && p.top <= p.leaf;
  lsk::IoArgs io{x, ldx, y, ldy, gidx, q, alpha, coef, F.xs.p, F.ys.p};
  if (!fold) {
    SpanScope sp(P, span + 0, s);
    lsk::launch_gather(fp32, x, ldx, F.xs.p, gidx, N, nrhs, s);
  }
  if (p.top <= p.leaf) {
    SpanScope sp(P, span + 1, s);
    run_phase(P, F, S.p2m, nrhs, s, -1, fold ? &io : nullptr);
    for (auto& ph : S.up) run_phase(P, F, ph, nrhs, s);
  }
  {
    SpanScope sp(P, span + 2, s);
    run_phase(P, F, S.nearm2l, nrhs, s, fp32 ? 4 : 0);
  }
  if (p.top <= p.leaf) {
    SpanScope sp(P, span + 3, s);
    for (auto& ph : S.down) run_phase(P, F, ph, nrhs, s);
    run_phase(P, F, S.l2p, nrhs, s, -1, fold ? &io : nullptr);
  }
  if (!fold) {
    SpanScope sp(P, span + 4, s);
    lsk::launch_epilogue(fp32, x, ldx, F.ys.p, eidx, q, alpha, coef, y, ldy, N, nrhs, s);
  }
  hip_check(hipGetLastError(), "fmm kernels");
}

}  // namespace lsi
