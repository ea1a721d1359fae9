// Launch wrappers for the device kernels (implemented in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lsk {

// Time the next timed kernel launch on this host thread: it is made with AMD's extended
// launch, which stamps `start` and `stop` from the dispatch (no separate event packets).
// Timed launches: stencil (both forms), HODLR leaf solve, HODLR level dot and update,
// Arnoldi dot products.
void set_next_launch_events(hipEvent_t start, hipEvent_t stop);
bool next_launch_events_pending();
void clear_next_launch_events();

// ---- stencil GEMM: out[m][box] (+)= sum_terms sum_k op[k][m] * in[k][src(box, term)] ----
enum TermMode { MODE_SAME = 0, MODE_SHIFT = 1, MODE_CHILD = 2, MODE_PARENT = 3 };

struct DTerm {
  const void* op;   // complex [K][Mpad] (row = inner index k)
  const void* in;   // input base of (level, direction) for rhs 0
  long long in_rhs; // rhs stride of the input, complex elements
  int K;            // inner dimension
  int mode;         // TermMode
  int cin;          // SHIFT: source class; CHILD: child class
  int sha, shb;     // SHIFT: shift in the class half-grid
  int nh_in;        // half-grid side of the input level
  int kbase;        // sum of K over the task's earlier terms
  int coh;          // fused form: the input is written inside the same launch (read it coherently)
};

// One 4-deep k-block of a matrix-core task: where the operator rows of this block start
// (op: address of op[4 kk][0] of its term), where its inputs start for right-hand side 0 and
// box 0 (in: address of in[4 kk][class plane of the term]), the term's box shift (SHIFT
// mode) and how many of the 4 k are real (the last block of a term may be partial).
struct alignas(32) KBlk {
  unsigned long long op;
  unsigned long long in;
  int sha, shb;
  int klim;
  int pad;
};

struct DTask {
  void* out;         // output base of (level, direction) for rhs 0
  long long out_rhs; // rhs stride of the output
  int M, Mpad;       // output rows (exact / padded to the row block)
  int nh;            // half-grid side of the output level
  int cout;          // output class
  int t0, t1;        // term range
  int beta;          // 0: overwrite, 1: accumulate
  int nrb;           // row blocks = Mpad / kRowBlock (MFMA form: 16-row tiles)
  int blk0;          // first workgroup of this task
  int ktot;          // sum of K over the task's terms (MFMA form: of the 4-deep k-blocks)
  int kps;           // MFMA form: waves of a workgroup that split the k-blocks (1, 2 or 4)
  // fused form (one launch for every pass): the stage this task's blocks count into, up to three
  // stages that must be complete before a block starts (-1: none), and whether the output is read
  // inside the same launch (written coherently)
  int stage;
  int dep[3];
  int coh_out;
  int coh_in;        // fused form: the inputs are written inside the same launch
  // split K (MFMA form, one launch per pass): kgroups > 1 workgroups share each output tile, each
  // summing a contiguous share of the k-blocks into its own partial plane part[rhs][g][m][box]
  // (part_rhs complex per right-hand side); launch_splitk_reduce then adds the planes in the
  // order g = 0, 1, ... into the output
  int kgroups;
  int nbb;           // box blocks of the task
  int bb0;           // matrix-core form: first box block (a task may cover a chunk of its level)
  // matrix-core form, one launch per pass: IO_GATHER = the input is the caller's vector read
  // through the tree-order map (and row group 0 stores the tree-order copy for later passes);
  // IO_EPILOGUE = the output, accumulated onto the tree-order result, is finished into the
  // caller's vector (see IoArgs)
  int io;
  int rpg;           // matrix-core form: 16-row tiles per row group (1..4; nrb = row groups)
  // matrix-core form: the task's k-blocks (ktot of them, in term order), the mode shared by all
  // its terms, the input half-grid side and the input stride between k
  const KBlk* kb;
  int mode;
  int nh_in;
  long long in_rhs;
  long long pks;
  void* part;
  long long part_rhs;
};

constexpr int kRowBlock = 8;
constexpr int kBoxBlock = 64;
constexpr int kStencilWaves = 4;
constexpr int kStencilThreads = 64 * kStencilWaves;

constexpr int IO_GATHER = 1;
constexpr int IO_EPILOGUE = 2;
// The vectors of one product for tasks with io set: x (ldx per right-hand side) in the caller's
// (or the solver's) order, the map tree index -> that order (gidx), the tree-order copies xs and
// ys (N per right-hand side), and the epilogue y[e] = alpha x[e] + coef q[e] v[t] for e = gidx[t]
// (q may be null: 1), v the accumulated tree-order result.
struct IoArgs {
  const double2* x;
  long long ldx;
  double2* y;
  long long ldy;
  const int* gidx;
  const double* q;
  double alpha, coef;
  const void* xs;
  const void* ys;
};

// MFMA form of the stencil (any term modes): a workgroup computes 16 rows x (64 / kps)
// boxes; complex products as four real 16x16x4 matrix-core operations per k-block.  io: the
// vectors of tasks with io set (may be null if none is).
void launch_stencil_mfma(bool fp32, const DTask* tasks, const DTerm* terms, const int* blk_task, int nblocks,
                         int nrhs, hipStream_t s, const IoArgs* io = nullptr);
void launch_stencil(int tag, bool fp32, const DTask* tasks, const DTerm* terms, const int* blk_task, int nblocks,
                    int nrhs, hipStream_t s);

// the output of one split-K task: out[rhs][m][cout][box] (+)= sum_g part[rhs][g][m][box]
struct SplitK {
  const void* part;
  void* out;
  long long part_rhs, out_rhs;
  int M, nbox, cout, G, beta;
};
// after a matrix-core pass with split-K tasks: add their partial planes into their outputs
// (max_elems: the largest M * nbox over the tasks)
void launch_splitk_reduce(bool fp32, const SplitK* sk, int ntask, long long max_elems, int nrhs, hipStream_t s);

// Every DAFMM pass in one persistent launch.  queue: (task, block within the task) pairs in
// an order in which every block's prerequisite stages come earlier; workgroups take the pairs
// (times nrhs right-hand sides, right-hand side fastest) by an atomic ticket, wait until the
// stages their task depends on are complete, compute the block and count it into the task's
// stage.  ctr: the counter block of dafmm_fused_counter_lines(nst) lines, zeroed (first word of
// each line); need: blocks per stage for one right-hand side.  If a wait runs out of its bound,
// bit 31 of the group flag words is set and the results are invalid (launch_epilogue_checked,
// given the first flag word, writes NaN).
void launch_dafmm_fused(bool fp32, const DTask* tasks, const DTerm* terms, const int* queue, int nitems, int nrhs,
                        int nst, unsigned* ctr, const unsigned* need, int nwg, hipStream_t s);
// 128-byte lines of the fused launch's counter block for nst stages (ticket, stage counts, 64
// group flag words; the first unsigned of each line is used)
int dafmm_fused_counter_lines(int nst);
// workgroups the fused launch keeps resident (all CUs times its occupancy)
int dafmm_fused_workgroups(bool fp32);
// launch_gather, and zero the first unsigned of `nz` 128-byte lines at `zero` (the fused launch's
// counter block)
void launch_gather_zero(bool to_fp32, const double2* x, long long ldx, void* xs, const int* idx, long long N, int nrhs,
                        unsigned* zero, int nz, hipStream_t s);
// launch_epilogue; if bit 31 of *err is set, y is NaN
void launch_epilogue_checked(bool from_fp32, const double2* x, long long ldx, const void* ys, const int* idx,
                             const double* q, double alpha, double coef, double2* y, long long ldy, long long N,
                             int nrhs, const unsigned* err, hipStream_t s);

// ---- setup ----
void launch_wtable(double2* W, int n, double h, double kappa, hipStream_t s);

// ---- permutations / epilogue ----
// xs[rhs*N + t] = (T) x[rhs*ldx + idx[t]]
void launch_gather(bool to_fp32, const double2* x, long long ldx, void* xs, const int* idx, long long N, int nrhs,
                   hipStream_t s);
// y[rhs*ldy + i] = alpha * x[rhs*ldx + i] + coef * q[i] * ys[rhs*N + idx[i]]
void launch_epilogue(bool from_fp32, const double2* x, long long ldx, const void* ys, const int* idx, const double* q,
                     double alpha, double coef, double2* y, long long ldy, long long N, int nrhs, hipStream_t s);
// y[rhs*ldy + perm[i]] = x[rhs*ldx + i]    (scatter) / y[rhs*ldy + i] = x[rhs*ldx + perm[i]] (gather)
void launch_permute(const double2* x, long long ldx, double2* y, long long ldy, const int* perm, long long N, int nrhs,
                    bool scatter, hipStream_t s);
void launch_planewave(const double* px, const double* py, const double* q, const double* angles, double kappa,
                      double coef, double2* f, long long ldf, long long N, int nrhs, hipStream_t s);

// ---- HODLR ----
// dfmt: storage of the leaf inverses, 0 complex128, 1 complex64, 2 complex bfloat16
// jdev != NULL: b is advanced by *jdev * bldj on the device (column j of a basis)
void launch_leaf_apply(int dfmt, const void* Dinv, const unsigned char* ident, const double2* b, long long ldb,
                       double2* z, long long ldz, int lp, int nleaves, int nrhs, hipStream_t s,
                       const int* jdev = nullptr, long long bldj = 0);
// complex bfloat16 factors, one right-hand side: z -= Y_a s_a (update of level a, node size
// nodesize_a) and the chunk partials of W_b^T z (dot of level b, chunks of 1024 rows) in one
// launch; the same sums as launch_hodlr_update followed by launch_hodlr_dot
bool hodlr_upd_dot_ok(long long N, long long nodesize_a, long long chunk_b);
void launch_hodlr_upd_dot(const void* Y, int ra, const double2* sv, long long nodesize, int nodes, const void* W,
                          int rb, double2* z, long long N, double2* partial, long long chunk, hipStream_t s,
                          const unsigned char* ract = nullptr);
// clist (optional): the nlist children of the level (cpc chunks each) whose chunk partials are
// formed; the segmented kernel (chunks of at least 16 rows, fewer than 8 right-hand sides or
// low-precision factors) leaves the others unwritten.  A child without contrast has Y = 0, so
// the partials of its sibling's chunks feed nothing: the list holds the children whose sibling
// has contrast.
void launch_hodlr_dot(int fmt, const void* W, const double2* z, long long ldz, double2* partial, long long N, int r,
                      long long chunk, int nchunks, int nrhs, hipStream_t s, const int* clist = nullptr,
                      int nlist = 0, int cpc = 0);
// cfmt: storage of the core inverses, 0 complex128, 1 complex64, 2 complex bfloat16 (r <= 256),
// hodlr_core_elems(r) entries per node in 16-row blocks (rows 16b..16b+15 of every column,
// column after column, rows past 2r zero); coreinv unused when !apply (s = t)
long long hodlr_core_elems(int r);
// cact (apply only, optional, as for launch_hodlr_dot): where a child has no contrast its Y is
// zero and K^-1 reduces to the identity on the half of s the other child uses (s_A = t_A when
// only the first child holds contrast, s_B = t_B when only the second does); that half is
// written as t, the unused half as zeros, without reading K^-1; nodes without contrast get s = 0.
// With apply, one right-hand side and chunks_per_child >= 16 the partials are folded in place (each
// child's sum lands in its first partial) before the core products: they are scratch to the caller.
void launch_hodlr_core(int cfmt, const void* coreinv, const double2* partial, double2* sout, int r, int nodes,
                       int chunks_per_child, int nchunks, bool apply, int nrhs, hipStream_t s,
                       const unsigned char* cact = nullptr);
// z -= Y s per level.  z2 != NULL asks for a copy of the result in column *jdev of a basis
// (z2 + rhs*z2ldr + *jdev*z2ldj); returns whether the launch made it (the caller copies otherwise)
// z -= Y s, one right-hand side, complex64 (fmt 1) or complex bfloat16 (fmt 2) factors, only on the
// nact listed 256-row blocks (blist: block indices; the rows of Y outside them are zero)
void launch_hodlr_update_list(int fmt, const void* Y, const double2* sv, double2* z, long long N, int r,
                              long long nodesize, const int* blist, int nact, hipStream_t s);
// ract (may be NULL): one byte per 256 rows, 0 where no row of the block has contrast (Y's rows are
// zero there; the wide kernels then leave those rows of z untouched and read no Y)
bool launch_hodlr_update(int fmt, const void* Y, const double2* sv, double2* z, long long ldz, long long N, int r,
                         long long nodesize, int nodes, int nrhs, hipStream_t s, double2* z2 = nullptr,
                         long long z2ldr = 0, const int* jdev = nullptr, long long z2ldj = 0,
                         const unsigned char* ract = nullptr);

// The leaf solves and the deepest binary levels of one right-hand side in one launch: one
// workgroup per node of level F = Lb - 3 (512 rows) or Lb - 2 (256 rows) runs the leaf solves
// (complex128 inverses) and the levels Lb-1 .. F (fmt: factors as for launch_hodlr_dot;
// complex128 core inverses) with that node's rows of z in LDS.  nodeact as in the level
// launches (NULL: every node active).  b and z may be the same buffer; jdev as for
// launch_leaf_apply.  Needs 64-row leaves, N = 64 * 2^Lb and ranks of at most 64 on those levels.
constexpr int kSubtreeMaxLevels = 3;
constexpr int kSubtreeRows = 512;  // rows per subtree (512: levels Lb-3..Lb-1; 256: Lb-2..Lb-1)
struct SubtreeLevels {
  const void* W[kSubtreeMaxLevels];     // index i: level F + i
  const void* Y[kSubtreeMaxLevels];
  const double2* K[kSubtreeMaxLevels];  // 16-row blocks, as for launch_hodlr_core
  int r[kSubtreeMaxLevels];
};
// rows per subtree the one-launch form takes for this tree (0: not applicable)
int hodlr_subtree_rows(long long N, int lp, int Lb, const int* ranks);
void launch_hodlr_subtree(int fmt, int sf, const double2* Dinv, const unsigned char* ident, const double2* b,
                          const int* jdev, long long bldj, double2* z, long long N, int Lb,
                          const SubtreeLevels& lv, const unsigned char* nodeact, hipStream_t s);

// ---- Krylov vector kernels (complex128) ----
void launch_gs_dot(const double2* Q, long long ldq_vec, long long ldq_rhs, int nv, const double2* w, long long ldw,
                   double2* partial, long long N, int nchunks, int maxv, int nrhs, hipStream_t s);
void launch_gs_finish(const double2* partial, int nchunks, int nv, int maxv, double2* h, int accumulate, int nrhs,
                      hipStream_t s);
void launch_gs_axpy(const double2* Q, long long ldq_vec, long long ldq_rhs, int nv, const double2* h, int maxv,
                    double sign, double2* w, long long ldw, long long N, int nrhs, hipStream_t s);
void launch_norm2(const double2* w, long long ldw, double* partial, long long N, int nchunks, int nrhs, hipStream_t s);
void launch_norm2_finish(const double* partial, int nchunks, double* out, int nrhs, hipStream_t s);
void launch_scale(const double2* w, long long ldw, const double* alpha, double2* out, long long ldo, long long N,
                  int nrhs, hipStream_t s);
void launch_axpby(double a, const double2* x, long long ldx, double b, const double2* y, long long ldy, double2* out,
                  long long ldo, long long N, int nrhs, hipStream_t s);
void launch_cast(bool to_fp32, const void* in, void* out, long long n, hipStream_t s);
// complex128 -> complex bfloat16 (round to nearest even)
void launch_cast_bf16(const void* in, void* out, long long n, hipStream_t s);


// ---- device-driven Arnoldi step (the Arnoldi index j lives in device memory) ----
// dst column j = src column j for active columns (state[rhs] == 0; state NULL: every column)
void launch_kd_copy(const double2* src, long long src_ldr, long long src_ldj, double2* dst, long long dst_ldr,
                    long long dst_ldj, long long N, const int* jdev, const int* state, int nrhs, hipStream_t s);
// partial dot products of Q columns 0..j with w (conjugated Q)
void launch_kd_dot(const double2* Q, long long ldq_vec, long long ldq_rhs, int maxv, const double2* w, long long ldw,
                   double2* partial, long long N, int nchunks, const int* jdev, const int* state, int nrhs,
                   hipStream_t s);
void launch_kd_finish(const double2* partial, int nchunks, int maxv, double2* out, long long out_ldr,
                      long long out_ldj, int accumulate, const int* jdev, const int* state, int nrhs, hipStream_t s);
// w += sign * Q[:, 0..j] h(j), h(j) = h + rhs*h_ldr + j*h_ldj
void launch_kd_axpy(const double2* Q, long long ldq_vec, long long ldq_rhs, const double2* h, long long h_ldr,
                    long long h_ldj, double sign, double2* w, long long ldw, long long N, const int* jdev,
                    const int* state, int nrhs, hipStream_t s);
void launch_kd_givens(const double* npart, int nchunks, double2* H, int m, int maxv, double* cs, double2* sn,
                      double2* g, const int* jdev, int* state, int* its, int* kfin, double* est, const double* fnorm,
                      const double* tol, int maxit, double* alpha, int nrhs, hipStream_t s);
// Q_{j+1} = alpha w (active columns), then j += 1 if any column is active
void launch_kd_next(const double2* w, long long ldw, const double* alpha, double2* Q, long long ldq_vec,
                    long long ldq_rhs, long long N, int* jdev, const int* state, int nrhs, hipStream_t s);

// ---- delayed CGS2 step (slot j of Q holds u_j, not yet reorthogonalised) ----
// inner products of Q_0..Q_j with u_j and w, blocks of rpb rows, reduced into
// cd = partial + nrhs * nblk * 2 * maxv: cd[(rhs*2 + x)*maxv + v] (x = 0: u_j, 1: w)
void launch_kd_dot2(const double2* Q, long long ldq_vec, long long ldq_rhs, int maxv, const double2* w, long long ldw,
                    double2* partial, long long N, int rpb, const int* jdev, const int* state, int nrhs,
                    hipStream_t s);
// completes Hessenberg column j-1 (Hr unrotated, H rotated), the Givens rotation, the stop test,
// T column j and the update coefficients coef[rhs][2][maxv], alpha = 1/beta
void launch_kd_dcgs2(const double2* cd, double2* Hr, double2* H, int m, int maxv, double* cs, double2* sn, double2* g,
                     double2* T, double2* coef, const int* jdev, int* state, int* its, int* kfin, double* est,
                     const double* fnorm, const double* tol, int maxit, double* alpha, int nrhs, hipStream_t s);
// slot j := q_j, slot j+1 := u_{j+1}; then j += 1 if any column is active
void launch_kd_dcgs2_axpy(double2* Q, long long ldq_vec, long long ldq_rhs, const double2* w, long long ldw,
                          const double2* coef, int maxv, const double* alpha, long long N, int* jdev,
                          const int* state, int nrhs, hipStream_t s);

}  // namespace lsk
