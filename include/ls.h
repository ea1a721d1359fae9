/*
 * libls -- MI355X (gfx950) solver for the discretised 2D Lippmann-Schwinger equation
 *
 *     A psi = f,   A = I + s kappa^2 diag(q) V,   f = -s kappa^2 q u_inc
 *
 * (Gujjula & Ambikasaran, "A new Directional Algebraic Fast Multipole Method based
 * iterative solver for the Lippmann-Schwinger equation accelerated with HODLR
 * preconditioner": Section 1, Eqs. (eq:3), (eq:5), (eq:6); Section 2.2, Eqs. (eq:12a),
 * (eq:13)).  V is the volume potential discretised on a uniform cell-centred grid with
 * one collocation point per cell (p = 1): V_ij = h^2 (i/4) H0^(1)(kappa |x_i - x_j|)
 * for i != j and the exact integral of G over the cell for i = j.  The physical sign is
 * s = -1 (so psi = kappa^2 q u); s = +1 reproduces Eq. (eq:6) as printed.
 *
 * Products with V use the Directional Algebraic FMM of Section 5 with Nested Cross
 * Approximation factors (Section 4); solves use GMRES (Section 6), optionally right-
 * preconditioned by a fixed-rank HODLR approximation of A (Section 6, Eq. (eq:hybrid)).
 *
 * Conventions for every call below
 *   - Setup inputs are HOST arrays and are copied.  Vectors passed to vector calls are
 *     DEVICE pointers owned by the caller, complex interleaved (re, im): complex128
 *     (double[2]) unless stated otherwise.  Several right-hand sides are stored
 *     column-major, column j at offset j*ld (in complex elements), ld >= N.
 *   - Vectors are in the caller's point order (the order of `points` given to ls_setup).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Vector calls are
 *     asynchronous on it unless stated otherwise.
 *   - Every call returns an ls_status; on a non-OK status ls_last_error() returns a
 *     message for the calling thread.  A non-converged solve is not an error: it is
 *     reported in ls_solve_info.status.
 *   - A handle is immutable after ls_setup and may be used from one stream at a time.
 */
#ifndef LS_H
#define LS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ls_problem ls_problem; /* opaque, owned by the library */

typedef enum {
  LS_OK = 0,
  LS_EINVAL = -1,  /* invalid argument (message in ls_last_error) */
  LS_ENOMEM = -2,  /* host or device allocation failed */
  LS_EDEVICE = -3, /* a HIP runtime call failed */
  LS_ENOTSUP = -4  /* input valid but outside what the library supports */
} ls_status;

typedef enum {
  LS_FP64 = 0,  /* complex128 operator, complex128 accumulation */
  LS_FP32 = 1,  /* complex64 operator and accumulation (near field, M2L, translations) */
  LS_MIXED = 2  /* ls_solve only: flexible GMRES with FP32 products once the residual is small,
                   FP32 off-diagonal HODLR factors, FP64 Arnoldi and FP64 residual at each restart */
} ls_prec;

enum {
  LS_CONVERGED = 0,
  LS_MAXIT = 1,
  LS_BREAKDOWN = 2,
  LS_NAN = 3,
  LS_REFINE_STAGNATED = 4,
  LS_WARMSTART_REJECTED = 5
};

typedef struct {
  int leaf_max;       /* max points per quadtree leaf (default 64; at most 64 points per leaf
                         when hodlr_rank > 0, else ls_setup returns LS_ENOTSUP) */
  double T;           /* a box of half-width w is high-frequency iff (kappa w)^2 > T (default 16) */
  int sign;           /* s in A = I + s kappa^2 diag(q) V; -1 (default) or +1 */
  int hodlr_rank;     /* fixed off-diagonal rank r of the HODLR preconditioner, 0..256; 0 = none
                         (default 15) */
  double eps_inner;   /* NCA tolerance of the FP32 operator; <= 0: cast of the FP64 operator (default 1e-7) */
  int restart;        /* GMRES restart length m (default 200) */
  int maxit;          /* max GMRES iterations per solve (default 2000) */
  int prec;           /* ls_prec used by ls_solve (default LS_FP64) */
  double inner_tol;   /* LS_MIXED: relative accuracy delta of the FP32 operator; products switch to FP32
                         once every residual estimate is below tol / delta (default 1e-5) */
  int max_refine;     /* LS_MIXED: Krylov cycles (each started from an FP64 residual f - A x) that may
                         use FP32 products; a column still unconverged after them is finished with
                         FP64 products and reports LS_REFINE_STAGNATED (default 10) */
  int build_fp32;     /* build the FP32 operator at setup (default 1) */
  int hodlr_rank_div; /* 0 (default): rank hodlr_rank at every HODLR level, as in the paper;
                         d > 0: rank min(hodlr_rank, child block size / d) per level */
  int graph_iters;    /* > 0: GMRES iterations run as device-driven Arnoldi steps (Arnoldi index,
                         Givens rotations and stop test on the device), captured into a HIP graph of
                         this many iterations and replayed, one host synchronisation per replay
                         (steps of the last replay after the stop test still run the operator and
                         preconditioner launches, so solves of few, expensive iterations want small
                         graphs); 0: one host round trip per iteration (default 0) */
  int stencil_mfma;   /* 1 (default): every DAFMM pass (near field, P2M, M2M, M2L, L2L, L2P) on the
                         matrix cores (16x16x4 MFMA); 0: the same sums on the vector ALUs */
  int pc_bf16;        /* 1 (default): also keep the HODLR off-diagonal factors in complex bfloat16 and
                         use them in LS_MIXED solves and LS_MIXED preconditioner applies (half the
                         traffic of complex64; flexible GMRES absorbs the inexact preconditioner);
                         0: LS_MIXED uses the complex64 factors */
  int dcgs2;          /* device-driven GMRES (graph_iters > 0): 1 (default) delayed classical
                         Gram-Schmidt with reorthogonalisation, the second pass of step j folded
                         into step j+1: one reduction pass and one update pass over the basis per
                         iteration instead of two of each; the stop test then runs one operator
                         application behind (the last application of a cycle is unused);
                         0: CGS2 as in the host-driven loop */
  int pc_lowp_solves; /* 0 (default): the HODLR leaf solves and SMW core solves stay complex128 in
                         every preconditioner apply; 1: LS_MIXED and LS_FP32 applies also keep the
                         leaf and core inverses in the off-diagonal factors' precision (complex
                         bfloat16 or complex64: less traffic, a less exact preconditioner) */
  double hodlr_tol;   /* 0 (default): every off-diagonal HODLR block at the fixed rank (the
                         preconditioner of Section 6); eps > 0: each block's ACA stops at
                         ||u_k|| ||v_k|| <= eps ||S_k||_F (the HODLR factorisation at a fixed
                         tolerance, Section 6), its rank still capped by hodlr_rank; for
                         ls_direct_solve */
  int fmm_fused;      /* with stencil_mfma = 1: 1 every DAFMM pass of a product runs in one persistent
                         launch whose workgroups take the passes' blocks from a queue in dependency
                         order (the near field fills the waits of the upward and downward chains;
                         same sums per block, bit-identical results); 0 (default): one launch per
                         pass, faster on this part (the chain blocks slow down under the filler) */
  int nca_device;     /* 1 (default): the NCA pivots (ACA at eps_NCA, Section 4.2.2 step 2) and the
                         interpolation operators U, C (X = V(candidates, far pivots) B^-1) are formed on
                         the GPU, one workgroup per direction of a level; 0: on the host (same rules,
                         other rounding, so pivots may differ where magnitudes nearly tie) */
} ls_options;

typedef struct {
  int iters;          /* total GMRES (Arnoldi) iterations */
  double relres;      /* final true relative residual ||f - A psi|| / ||f|| (FP64 operator) */
  int status;         /* LS_CONVERGED; LS_MAXIT (maxit reached); LS_NAN (non-finite residual);
                         LS_WARMSTART_REJECTED (converged, but the given x0 was replaced by zero);
                         LS_REFINE_STAGNATED (LS_MIXED: FP32 products stopped reducing the FP64
                         residual, or max_refine cycles were spent; the column was finished with
                         FP64 products and converged) */
  int n_refine;       /* LS_MIXED: Krylov cycles, each started from an FP64 residual f - A x */
  double t_solve_ms;  /* wall time of the call */
  double relres0;     /* ||f - A x0|| / ||f|| of the start GMRES used (1 for a zero start) */
} ls_solve_info;

typedef struct {
  int64_t N;
  int n;              /* grid side */
  int levels;         /* quadtree leaf level L (root = 0) */
  int leaf_side;      /* cells per leaf side */
  int top_level;      /* coarsest level with a non-empty interaction list */
  int nlevels_hf;     /* number of high-frequency levels with interaction lists */
  int rank_max64;     /* largest NCA rank of the FP64 operator */
  int rank_max32;     /* largest NCA rank of the FP32 operator */
  int64_t entries_near;   /* near-field kernel entries applied per matvec (one RHS) */
  int64_t entries_far64;  /* P2M+M2M+M2L+L2L+L2P entries applied per FP64 matvec */
  int64_t entries_far32;  /* same for the FP32 operator */
  int64_t entries_m2l64;  /* M2L part of entries_far64 */
  int64_t entries_m2l32;  /* M2L part of entries_far32 */
  int64_t m2l_pairs;      /* (box[,direction], source) M2L pairs over all levels */
  int64_t stored_bytes64; /* device bytes of the FP64 DAFMM operators */
  int64_t stored_bytes32;
  int64_t hodlr_bytes;    /* device bytes of the HODLR factors */
  int hodlr_levels;       /* binary levels above the HODLR leaves */
  int hodlr_rank_sum;     /* sum over binary levels of the off-diagonal rank */
  int64_t hodlr_dense_leaves; /* leaves whose diagonal block is not the identity */
  double t_plan_ms, t_nca_ms, t_hodlr_ms, t_setup_ms;
  int64_t hodlr_rank_used_sum;  /* sum of the ranks the ACA reached over the off-diagonal blocks */
  int64_t hodlr_blocks;         /* number of off-diagonal blocks */
  int hodlr_rank_used_max;      /* largest of them */
  /* parts of t_hodlr_ms: off-diagonal ACA; the applies of the finer levels that form
   * Y = D^-1 U (device); forming, inverting (host) and uploading the SMW cores */
  double t_hodlr_aca_ms, t_hodlr_apply_ms, t_hodlr_cores_ms;
  /* rows in 256-row blocks (solver order) that hold a point with contrast; the HODLR level
   * updates skip the other blocks (points without contrast are identity rows of A, so the
   * matching rows of the preconditioner factors Y = D^-1 U are zero) */
  int64_t hodlr_rows_active;
  /* per binary level l < hodlr_levels (at most 32): rows whose W^T z a preconditioner apply
   * forms, and nodes whose core product K^-1 t it forms.  A child node without contrast has
   * Y = 0: its sibling's rows feed nothing, and K^-1 is the identity on the half of s the
   * other child uses, so those chunks and core rows are skipped. */
  int64_t hodlr_dot_rows[32];
  int hodlr_core_nodes[32];
  /* complex multiply-adds per product and right-hand side of the middle launch of the product
   * (kernel timing classes 0 and 4): the M2L of the top level and the near-field classes not
   * packed into the upward-pass launches (all of the near field and M2L without the
   * matrix-core form or in the fused launch) */
  int64_t entries_mid64, entries_mid32;
  /* binary level F from which a preconditioner apply of one right-hand side (complex128 leaf
   * and core solves) runs the leaf solves and the levels F..hodlr_levels-1 in one launch, one
   * workgroup per level-F node (kernel timing class 20); -1: every level in its own launches */
  int hodlr_subtree_level;
} ls_stats_t;

/* Plan description for a uniform n x n grid on [-L, L]^2 (host only, no device use).
 * Per level nu (0..levels): hf[nu], ndir[nu] (cones), il_pairs[nu] (in-domain M2L pairs
 * over (box, direction)), max_il[nu]; near_pairs = ordered neighbouring leaf pairs.
 * coverage_min/max: over all ordered leaf pairs, the number of times each pair is
 * handled (near field or exactly one M2L); both must be 1 (Section 5: every
 * interaction is either near field or transferred by one M2L).  Arrays hold 32 levels. */
typedef struct {
  int levels, leaf_side, top_level;
  int hf[32], ndir[32], max_il[32];
  int64_t il_pairs[32];
  int64_t near_pairs;
  int coverage_min, coverage_max;
} ls_plan_info;

void ls_default_options(ls_options* opt);

/* Build the solver for the points of a uniform cell-centred n x n grid (any order).
 *   points : host, N x 2 row-major (x1, x2); must form a uniform cell-centred square grid.
 *   q      : host, N real contrast values q(x_i) in the same order.
 *   kappa  : wavenumber > 0.   tol : NCA tolerance eps_NCA in (0, 1) (Section 4.2.2).
 *   opt    : NULL for defaults.  *out receives the handle (NULL on error).
 * Synchronous.  Uses the current HIP device.  Errors: LS_EINVAL (N <= 0, kappa <= 0,
 * tol outside (0,1), non-finite or duplicate points, non-finite q, bad options);
 * LS_ENOTSUP (points not a uniform square grid, or a grid the quadtree cannot split
 * into leaves of <= leaf_max points). */
ls_status ls_setup(const double* points, int64_t N, const double* q, double kappa, double tol,
                   const ls_options* opt, ls_problem** out);

/* y = A x (Eq. (eq:12a)) with the DAFMM product (Section 5) for V.
 * x, y: device, N x nrhs complex128, leading dimension ld.  prec: LS_FP64 or LS_FP32
 * (FP32 converts x to complex64 for the operator and accumulates the result in
 * complex128).  x and y must not overlap.  Calls on one handle must not overlap in time (the
 * product's workspaces belong to the handle). */
ls_status ls_matvec(ls_problem* P, const void* x, void* y, int nrhs, int64_t ld, int prec, void* stream);

/* u = V psi: the scattered field on the grid (Section 6, last paragraph before 6.1).  Arguments
 * and overlap rules as for ls_matvec. */
ls_status ls_apply_V(ls_problem* P, const void* x, void* y, int nrhs, int64_t ld, int prec, void* stream);

/* HODLR direct solver (Section 6: the factorisation used as the solver, the paper's choice for
 * many right-hand sides): psi = A~^{-1} f, then iterative refinement psi += A~^{-1} (f - A psi)
 * with FP64 DAFMM products until ||f - A psi|| <= tol ||f|| for every column or max_refine steps
 * (tol = 0: exactly max_refine steps).  A~ is the factorisation built at setup; with hodlr_tol > 0
 * it holds each off-diagonal block to that tolerance.  Same vector conventions as ls_solve; info
 * (host, nrhs, may be NULL): iters = n_refine = refinement steps, relres = final FP64 residual,
 * status LS_CONVERGED (<= tol), LS_MAXIT or LS_NAN.  Synchronous.  LS_ENOTSUP when hodlr_rank = 0. */
ls_status ls_direct_solve(ls_problem* P, const void* f, void* psi, int nrhs, int64_t ld, double tol, int max_refine,
                          ls_solve_info* info, void* stream);

/* z = A~^{-1} r with the fixed-rank HODLR approximation A~ of A (Section 6, Eq. (eq:hybrid)).
 * prec LS_FP64: all factors complex128; LS_FP32: off-diagonal factors stored complex64;
 * LS_MIXED: off-diagonal factors complex bfloat16 when pc_bf16 = 1 (else complex64); leaf
 * and SMW core solves complex128 (unless pc_lowp_solves = 1) and all sums in FP64 in every
 * case.  LS_ENOTSUP when hodlr_rank = 0. */
ls_status ls_precond_apply(ls_problem* P, const void* r, void* z, int nrhs, int64_t ld, int prec, void* stream);

/* ls_precond_apply for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels and the same
 * result, with every workspace (the Morton-order copy of r, the W^T z chunk partials and the
 * SMW s vectors) placed in one fixed 64 MiB array that the library's code object holds on each
 * GPU it runs on, from the load of the library until the process ends; the call makes no
 * hipMalloc, hipFree, event creation or other allocating call.  Arguments, layout and prec as
 * ls_precond_apply; r and z are caller-owned device buffers and must not overlap.  The current
 * device must be the one ls_setup ran on (else LS_EINVAL).  The workspace needs, rounded up to
 * 256 bytes each, 16 N nrhs bytes + 16 nrhs max_l(chunks_l r_l) + 16 nrhs max_l(2^(l+1) r_l)
 * bytes (about 6 MiB per right-hand side at N = 512^2, rank 256); a call that would need more
 * than 64 MiB returns LS_EINVAL with the required size in ls_last_error().  Every call on a GPU
 * shares that GPU's array: calls that overlap in time on one GPU (other streams, other threads,
 * other handles) race and give undefined results.  Nothing in the array needs to start at zero
 * (every entry a call reads was written earlier in the same call). */
ls_status ls_precond_apply_noalloc(ls_problem* P, const void* r, void* z, int nrhs, int64_t ld, int prec,
                                   void* stream);

/* f_j = -s kappa^2 q u_inc(theta_j), u_inc = exp(i kappa (cos t x1 + sin t x2)) (Section 6.2).
 * angles: host, nrhs values.  f: device, N x nrhs complex128. */
ls_status ls_rhs_planewave(ls_problem* P, const double* angles, int nrhs, void* f, int64_t ld, void* stream);

/* Solve A psi = f for nrhs columns by restarted GMRES with right HODLR preconditioning
 * (when hodlr_rank > 0), stopping when ||f - A psi|| / ||f|| <= tol per column.
 * prec: LS_FP64, LS_FP32, LS_MIXED, or -1 for the precision given in the options.
 * f, psi: device, N x nrhs complex128.  x0_given != 0: psi holds the initial guess g.
 * GMRES starts from x0 = xi g with the minimal-residual scale xi = (A g)^H f / ||A g||^2
 * (Hegedus' scaling of an initial guess; costs one FP64 operator product), so that
 * ||f - A x0|| <= ||f||.  A guess that cannot lower the residual (A g orthogonal to f,
 * or non-finite) is replaced by zero, and LS_WARMSTART_REJECTED is reported in
 * info[j].status when the column otherwise converged.
 * info: host array of nrhs entries (may be NULL).  Synchronous on `stream`. */
ls_status ls_solve(ls_problem* P, const void* f, void* psi, int nrhs, int64_t ld, double tol,
                   int x0_given, int prec, ls_solve_info* info, void* stream);

/* Queue of independent problems (Section 6's solver applied to each): solves
 * A_p psi_p = f_p for p < nprob, one right-hand side each, from a zero start, to
 * ||f_p - A_p psi_p|| / ||f_p|| <= tol.  Problems are taken largest first by `nworkers` host
 * threads (0 = 4), each driving its own HIP stream (default priority); every solve uses the
 * graph-captured GMRES driver with `graph_iters` Arnoldi steps per graph (0 = 8) and runs
 * ls_autotune on a problem not tuned before.  prec as in ls_solve (-1 = each problem's
 * options).  probs, f, psi, info: host arrays of nprob entries; f[p], psi[p] are device
 * vectors of N_p complex128 in problem p's point order.  A problem may appear once.
 * Synchronous.  Errors: LS_EINVAL for bad arguments; the first error of any problem is
 * returned (the others still run); per-problem results in info[p]. */
ls_status ls_solve_queue(ls_problem* const* probs, int nprob, const void* const* f, void* const* psi, double tol,
                         int prec, int nworkers, int graph_iters, ls_solve_info* info);

/* Launch-shape autotuner: times the Arnoldi reductions (dot products of 32 basis vectors and a
 * norm) for 256/512/1024/2048/4096 rows per workgroup chunk, and the HODLR preconditioner apply
 * for at most 128/256/512/1024/2048 rows per level-reduction chunk, on this problem's sizes, and
 * keeps the fastest of each for all later calls on P.  out (may be NULL) receives the choices
 * and the measured times.  Synchronous on `stream`. */
typedef struct {
  int gs_rows;       /* chosen rows per chunk, Arnoldi reductions */
  int hodlr_rows;    /* chosen max rows per chunk, HODLR level reductions */
  double gs_us[5];   /* microseconds per candidate 256, 512, 1024, 2048, 4096 */
  double pc_us[5];   /* microseconds per candidate 128, 256, 512, 1024, 2048 (0 without HODLR) */
} ls_tune_info;
ls_status ls_autotune(ls_problem* P, ls_tune_info* out, void* stream);

/* Table of V entries for grid offsets (Section 1 Green's function, Eq. (eq:13) at p = 1):
 * out[(da + n-1) * (2n-1) + (db + n-1)] = h^2 (i/4) H0^(1)(kappa h |(da, db)|) for (da, db) != 0 and
 * the exact integral of G over the cell at (0, 0); |da|, |db| <= n-1.  out: device, (2n-1)^2
 * complex128, owned by the caller.  Synchronous on `stream`.  LS_ENOTSUP if kappa h >= 4/0.7072. */
ls_status ls_green_table(int n, double h, double kappa, void* out, void* stream);

/* Off-grid volume potential (Section 6, the paragraph before Section 6.1: u_scat = V[psi] from
 * the discrete density).  At p = 1 the density is constant on each cell, so
 *   u[t] = sum_j psi_j int_{cell j} G(|x_t - y|) dy,   G = (i/4) H0^(1)(kappa r),
 * for any points x_t, inside or outside the grid.  Cells two or more cells away from the one
 * containing x_t use a tensor Gauss-Legendre rule whose order is set by the distance and by
 * kappa h; the 3 x 3 cells around x_t are integrated in polar coordinates about x_t with graded
 * pieces along each edge.  Accuracy about 1e-10 relative per cell for kappa h <= 1.5 (the
 * polar rules), falling slowly beyond.  targets: DEVICE, M x 2 doubles (x1, x2); psi: DEVICE complex128, N, the caller's point
 * order; u: DEVICE complex128, M.  Direct summation over the N cells (O(M N)); asynchronous on
 * `stream`.  LS_EINVAL for M < 0 or NULL buffers (M = 0 does nothing). */
ls_status ls_field_eval(ls_problem* P, const double* targets, int64_t M, const void* psi, void* u, void* stream);

/* The error function of Eq. (eq:error) at p = 1, the residual of the continuous equation at
 * any points x_t:
 *   E[t] = | psi(x_t) + s kappa^2 q_t[t] u(x_t) - f(x_t) | / kappa^2,  f = -s kappa^2 q u_inc,
 * with u as in ls_field_eval, psi(x_t) the density of the cell containing x_t (0 outside the
 * grid), q_t[t] the contrast at x_t itself (DEVICE, M doubles, from the caller's definition of
 * q, so that f does not depend on the grid) and u_inc = exp(i kappa (cos theta x1 + sin theta x2)).
 * E: DEVICE, M doubles.  Same errors as ls_field_eval. */
ls_status ls_error_eval(ls_problem* P, const double* targets, int64_t M, const double* q_t, double theta,
                        const void* psi, double* E, void* stream);

/* Counters of the handle (ranks, entries applied per matvec, bytes, setup timings). */
ls_status ls_stats(const ls_problem* P, ls_stats_t* out);
void ls_destroy(ls_problem* P);
const char* ls_last_error(void);

/* Host-only: plan (quadtree, regimes, cones, lists, coverage) for an n x n grid on [-L,L]^2. */
ls_status ls_plan_describe(int n, double L, double kappa, const ls_options* opt, ls_plan_info* out);

/* Kernel timing: the timed launches of one kernel class are made with AMD's extended launch,
 * whose dispatch stamps a start and a stop event on the launch stream.  Classes: 0 = near
 * field + M2L launch (FP64 operator), 1 = HODLR level update, 2 = HODLR leaf solve,
 * 3 = Arnoldi dot products, 4 = near field + M2L launch (FP32 operator), 5 = HODLR level dot
 * products (W^T z), 6 = HODLR level update fused with the next level's dot products (complex
 * bfloat16 factors, one right-hand side), 7 = HODLR SMW core products s = K^-1 t, 8 = the fused
 * DAFMM launch (every pass, FP64 operator), 9 = the same with the FP32 operator.  Classes
 * 10..14 time spans of the per-pass DAFMM product with the FP64 operator between two events
 * recorded on the stream (launch gaps included): 10 = gather into the tree order, 11 = upward
 * pass (P2M, M2M), 12 = near field + M2L, 13 = downward pass (L2L, L2P), 14 = epilogue
 * (y = alpha x + coef q V x); 15..19 the same with the FP32 operator; 20 = HODLR leaf
 * solves and deepest levels in one launch (ls_stats_t.hodlr_subtree_level).  every > 0
 * starts (and clears) the counters and times every every-th
 * launch of the class (timed dispatches run one at a time, so sparse sampling keeps the
 * timed run close to an untimed one); 0 stops.  ls_profile_read synchronises and returns the
 * summed time and number of the timed launches, and (all_launches, may be NULL) the number
 * of launches of the class since enabling.  While a class is enabled, graph_iters > 0 solves
 * enqueue their device-driven steps eagerly instead of replaying captured graphs (same
 * kernels and launch shapes). */
ls_status ls_profile_enable(ls_problem* P, int kernel_class, int every);
ls_status ls_profile_read(ls_problem* P, int kernel_class, double* total_ms, int64_t* launches,
                          int64_t* all_launches);
/* The timed launches of a class one by one, in launch order: ms[i] and tags[i] (the binary
 * level for the HODLR classes 1, 5, 6, 7 — the level whose factors the launch reads, for an
 * update fused with the next level's dot products the next level; -1 for the others) for
 * i < min(cap, *n); *n = the number of timed launches.  Synchronises like ls_profile_read. */
ls_status ls_profile_read_each(ls_problem* P, int kernel_class, double* ms, int* tags, int64_t cap, int64_t* n);

/* ---------------------------------------------------------------------------------------
 * Learned GMRES warm start (an extension; the paper has no learned component).
 * A small FNO-style neural operator on the n x n grid image (grid order, image[a][b] = point
 * a*n + b): lift 6 -> width, `layers` x (truncated-DFT spectral convolution with `modes`
 * modes per axis + 1x1 convolution + bias, exact GELU except after the last layer),
 * projection width -> 2.  Inputs X: [B][6][n][n] float (q, cos and sin of the WKB phase
 * kappa d.x + phi, kappa/60, x1, x2); output O: [B][2][n][n] float, the complex envelope of
 * the solution relative to the WKB start b = f exp(i phi): psi0 = b (1 + O_re + i O_im).
 * phi(x) = kappa h sum_{k<2n} g(x - (k + 1/2) h d), g = sqrt(max(1 + q, 0)) - 1 bilinear
 * between cell centres and zero outside, d = (cos theta, sin theta): the phase the local
 * wavenumber kappa sqrt(1 + q) adds along the straight incoming ray (midpoint rule).
 * All buffers are DEVICE pointers owned by the caller unless stated; FP32 parameters.
 * Errors: LS_EINVAL on bad sizes or NULL pointers, LS_EDEVICE on a failed launch.
 * --------------------------------------------------------------------------------------- */
typedef struct ls_nop ls_nop;
typedef struct {
  int n;              /* grid side (>= 8) */
  int width;          /* channels (<= 256) */
  int modes;          /* Fourier modes per axis, 2*modes <= n */
  int layers;         /* spectral layers */
  int batch_max;      /* largest batch B passed to forward */
  uint64_t seed;      /* parameter initialisation */
  int bf16;           /* 1: the channel-mixing layers (lift, 1x1 convolutions, projection, their
                         gradients) on the matrix cores with BF16 inputs and FP32 accumulation,
                         weights kept FP32; 0: FP32 throughout */
} ls_nop_config;

ls_status ls_nop_create(const ls_nop_config* cfg, ls_nop** out);
int64_t ls_nop_param_count(const ls_nop* N);
/* host copies of the flat parameter / gradient vectors (count = ls_nop_param_count);
 * set_params also clears the Adam state */
ls_status ls_nop_get_params(const ls_nop* N, float* host, int64_t count);
ls_status ls_nop_set_params(ls_nop* N, const float* host, int64_t count);
ls_status ls_nop_get_grads(const ls_nop* N, float* host, int64_t count);
/* O = NO(X) for B samples; keeps the activations for ls_nop_backward */
ls_status ls_nop_forward(ls_nop* N, const float* X, float* O, int B, void* stream);
/* parameter gradients (overwritten) of sum(dO * O) for the last forward; reads that forward's
 * input X, which must still be valid */
ls_status ls_nop_backward(ls_nop* N, const float* dO, void* stream);
/* per-sample loss_b = |w O_c - t|^2 / snorm2_b and dO = d(mean_b loss_b)/dO; w, t: [B][n][n]
 * complex64 with w = b/kappa^2, t = (psi - b)/kappa^2 (b the WKB start); snorm2: [B] float
 * (|psi/kappa^2|^2) */
ls_status ls_nop_loss(ls_nop* N, const float* O, const void* w, const void* t, const float* snorm2, int B, float* dO,
                      float* loss, void* stream);
/* one Adam update of all parameters with the gradients of the last backward */
ls_status ls_nop_adam_step(ls_nop* N, float lr, float beta1, float beta2, float eps, void* stream);
/* X[6][n][n] from q (device, n*n doubles, grid order) on the cell-centred grid of [-L, L]^2 */
ls_status ls_nop_features(int n, double L, const double* q, double kappa, double theta, float* X, void* stream);
/* psi0 = f exp(i phi) (1 + O_re + i O_im) for one sample; q: device n*n doubles; O: device
 * [2][n][n] float or NULL (then psi0 = f exp(i phi), the WKB start alone); f, psi0: device
 * complex128, grid order */
ls_status ls_nop_warmstart(int n, double L, const double* q, double kappa, double theta, const float* O,
                           const void* f, void* psi0, void* stream);
void ls_nop_destroy(ls_nop* N);

/* ---------------------------------------------------------------------------------------
 * High-order leaf panels (Section 2.2, Eqs. (eq:7)-(eq:13); the moment tables of Section 2.3)
 * on a uniform tree: nside x nside leaf boxes of half-width beta = L / nside tile [-L, L]^2; box
 * k = ix * nside + iy has centre (-L + (2 ix + 1) beta, -L + (2 iy + 1) beta) and carries the
 * p x p tensor Chebyshev points of the first kind, ascending: node a = i * p + j sits at the
 * centre + beta (x_i, x_j).  The density on a box is the interpolant in the N_p = p (p + 1) / 2
 * polynomials T_a(u) T_b(v), a + b < p (ordered by total degree, then by a), through the
 * pseudo-inverse of the interpolation matrix (Eqs. (eq:9)-(eq:10)), and the operator is
 *     A_ij = delta_ij + sign kappa^2 q_i sum_l Qdag[l, j'] M_l(x_i, B(j)),
 *     M_l(x, B) = int_B G(|x - y|) b_l((y - c_B) / beta) dy,   G(r) = (i/4) H0^(1)(kappa r).
 * Unknowns: box-major, node-minor (N = nside^2 p^2).  The moments of a box at a node at least
 * beta away from it take the tensor Gauss-Legendre rule of max(16, ceil(2 kappa beta) + 12)
 * points per direction; nearer nodes (the box's own included) split the box into the four
 * signed triangles with apex at the node, Duffy-mapped (48 Gauss-Legendre points along the ray)
 * and integrated across with 48 points after a sinh map on each side of the perpendicular's
 * foot.  On a uniform tree the moments depend only on the box offset, so the device holds one
 * table row per offset ((2 nside - 1)^2 rows of p^2 x N_p moments, and of p^2 x p^2 operator
 * blocks).  The product is the dense sum over all box pairs (no far-field compression).
 * ---------------------------------------------------------------------------------------*/
typedef struct ls_panels ls_panels;
/* A function the host evaluates at n points (x[k], y[k]): real and imaginary parts into re[k],
 * im[k] (the contrast q: im = 0).  ctx is passed through unchanged. */
typedef void (*ls_point_fn)(int n, const double* x, const double* y, double* re, double* im, void* ctx);
/* The adaptive, level-restricted quadtree of Section 2.1 on [-L, L]^2 (host, synchronous; calls
 * q and uinc on the host).  A box is split below min_level, and below max_level while
 * (kappa w)^2 > T (w its half-width: the high-frequency regime of Section 3) or while q or uinc is
 * not resolved: the p-th order interpolant of the function on the box (Qdag of its p x p node
 * values, Eqs. (eq:9)-(eq:10)), evaluated at the nodes of its four children, differs from the
 * function there by more than eps_grid times the largest magnitude among those values and the
 * box's own.  Then every leaf with a neighbour (a shared boundary segment) more than one level
 * finer is split, pass after pass, until none is.  Output: *nboxes = the number of leaves and,
 * when it is at most max_boxes, boxes[4 k ..] = (centre x, centre y, half-width, level) of leaf
 * k, depth first with the children of a box in the order (-x, -y), (-x, +y), (+x, -y), (+x, +y)
 * (the first three columns are the input of ls_panels_setup_leaves).  Errors: LS_EINVAL (NULL
 * function or count, p outside 1..8, L, kappa, eps_grid or T not positive and finite, levels not
 * 0 <= min_level <= max_level <= 12, a non-finite function value, more leaves than max_boxes:
 * *nboxes still holds the count). */
ls_status ls_panels_build_tree(double L, int p, double kappa, double eps_grid, double T, int min_level, int max_level,
                               ls_point_fn q, ls_point_fn uinc, void* ctx, int max_boxes, double* boxes,
                               int* nboxes);
/* nside in 1..1024, p in 1..8, L > 0, kappa > 0, sign +1 or -1 (see ls_options.sign);
 * q: host, N node values of the contrast (box-major, node-minor), copied.  Forms the tables
 * on the current device (synchronous).  Errors: LS_EINVAL (bad argument, non-finite q),
 * LS_ENOTSUP (tables above 64 GB), LS_ENOMEM / LS_EDEVICE. */
ls_status ls_panels_setup(int nside, double L, int p, double kappa, const double* q, int sign, ls_panels** out);
/* The same discretisation on the leaves of any tree, for instance the adaptive, level-restricted
 * quadtree of Section 2.1: boxes: host, nboxes x 3 (centre x, centre y, half-width), leaves that
 * tile the domain without overlap (not checked); unknowns box-major in that order, node-minor
 * (N = nboxes p^2 <= 20000).  The moments of every box at every node use the rules above (the far
 * rule's point count taken from each box's half-width), and the device keeps the dense V (N^2
 * complex entries).  ls_panels_apply and ls_panels_solve work as for the uniform tree;
 * ls_panels_moments returns LS_ENOTSUP.  Errors as for ls_panels_setup, LS_ENOTSUP above 20000
 * unknowns. */
ls_status ls_panels_setup_leaves(int nboxes, const double* boxes, int p, double kappa, const double* q, int sign,
                                 ls_panels** out);
/* op 0: y = A x; op 1: y = V x (the volume potential of the density x at the nodes).  x, y:
 * device complex128, nrhs columns of leading dimension ld >= N, not overlapping; asynchronous on
 * stream (NULL: the default stream). */
ls_status ls_panels_apply(ls_panels* P, const void* x, void* y, int nrhs, int64_t ld, int op, void* stream);
/* HODLR preconditioner of the panel system (Section 6, on the discretisation of Section 2.2):
 * unknowns reordered by boxes in Morton order (the bits of the box's y index at the even, those
 * of its x index at the odd positions of the code; for the leaves of any tree the code of the
 * box's lower-left corner on the grid of the smallest box width, ties kept in the given order),
 * nodes inside a box unchanged; leaves of whole boxes with at most 64 unknowns (uniform trees:
 * 4^j boxes; any tree: floor(64 / p^2) boxes, then padding unknowns, identity rows and columns,
 * up to a power-of-two number of leaves); a binary tree that halves the index range; every
 * off-diagonal block compressed by partially pivoted ACA at rank min(rank, half the node);
 * Sherman-Morrison-Woodbury per node.  Factors built on the host (ACA, leaf inverses; entries
 * from the operator blocks, or from the dense V copied to the host) and the device (Y, cores);
 * synchronous.  rank <= 0 drops the factors.  Errors: LS_EINVAL (NULL handle, rank > 256, a
 * singular leaf block or core), LS_ENOTSUP (a uniform tree whose side is not a power of two),
 * LS_ENOMEM / LS_EDEVICE.  Once built, ls_panels_solve is right-preconditioned. */
ls_status ls_panels_precond_setup(ls_panels* P, int rank);
/* z = A~^-1 r.  r, z: device complex128, nrhs columns of leading dimension ld >= N, box-major
 * order (r and z may be the same buffer); asynchronous on stream.  LS_EINVAL without factors. */
ls_status ls_panels_precond_apply(ls_panels* P, const void* r, void* z, int nrhs, int64_t ld, void* stream);
/* The preconditioner's rank cap, leaf size, binary levels, the mean and largest rank the ACA
 * reached over the off-diagonal blocks and the setup time (all zero without factors). */
ls_status ls_panels_precond_info(const ls_panels* P, int* rank, int* leaf, int* levels, double* mean_rank,
                                 int* max_rank, double* setup_ms);
/* psi = A^-1 f by restarted GMRES(restart) from psi = 0 (classical Gram-Schmidt with one
 * reorthogonalisation; right-preconditioned by the HODLR factors of ls_panels_precond_setup when
 * they exist, else unpreconditioned), stopping when the true ||f - A psi|| / ||f|| <= tol
 * (recomputed at every restart) or after maxit products.  f, psi: device complex128 (N), not
 * overlapping.  info: host (iters, relres, status LS_CONVERGED / LS_MAXIT / LS_NAN, n_refine =
 * the GMRES cycles, t_solve_ms).  Synchronous. */
ls_status ls_panels_solve(ls_panels* P, const void* f, void* psi, double tol, int restart, int maxit,
                          ls_solve_info* info, void* stream);
/* host copy of the moment table row of box offset (dx, dy) = target box - source box,
 * |dx|, |dy| < nside: out[(a * N_p + l) * 2 + {0, 1}] = M_l(node a of the target box, source
 * box), real and imaginary parts.  Synchronous. */
ls_status ls_panels_moments(const ls_panels* P, int dx, int dy, double* out);
/* number of unknowns, N_p, and the far rule's points per direction */
ls_status ls_panels_info(const ls_panels* P, int64_t* n_unknowns, int* np, int* nfar);
void ls_panels_destroy(ls_panels* P);

#ifdef __cplusplus
}
#endif
#endif /* LS_H */
