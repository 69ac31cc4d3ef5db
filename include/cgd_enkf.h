/*
 * cgd_enkf.h -- C ABI of the MI355X (gfx950) CGD-EnKF analysis library.
 *
 * One analysis step of the ensemble Kalman filter, solved the conjugate-
 * gradient way of the paper "A Conjugate Gradient Formulation of the EnKF
 * Algorithm" (Lee, Liu, Valyou, Zikatanov):
 *
 *   S   = H A,  A = X_f - xbar 1^T            observed anomalies (Sec. 2.3, eq. Zhat_def)
 *   D   = y 1^T + E - H X_f                    innovations, one column per member
 *   Psi = S S^T / (N-1) + diag(r)              innovation matrix (eq. Psi_zz)
 *   Z   = Psi^{-1} D                           by CG, N right-hand sides (Sec. 3.1-3.3)
 *   X_a = X_f + A (S^T Z) / (N-1)              the update of Algorithm 1
 *
 * Notation: n = state dimension, m = number of observations, N = ensemble
 * size, k = entries per observation-operator row.  (The paper writes m for
 * the state dimension and p for the observation dimension.)
 *
 * Memory and layout
 *   Every array argument is a DEVICE pointer owned by the caller, row-major:
 *     X_f, X_a     n x N  (member index fastest: X[i*N + j])
 *     idx          m x k  int32, 0 <= idx < n; duplicates allowed
 *     w            m x k  observation i = sum_t w[i*k+t] * x[idx[i*k+t]];
 *                         a zero weight pads a short row
 *     y, r_diag    m      observation vector and diag(R), r_diag > 0
 *     eps          m x N  member perturbations of y (stochastic EnKF) or NULL
 *                         for the deterministic form (Remark in Sec. 2.3)
 *   Value arrays are double for CGD_FP64 and float for CGD_FP32 and
 *   CGD_MIXED_BF16.  The library never allocates device memory in these
 *   entry points: it carves the caller's workspace (size from
 *   cgd_enkf_workspace_bytes).  X_a may alias X_f.
 *
 * Execution
 *   All launches go to `stream` (a hipStream_t; NULL = the null stream) and
 *   are asynchronous unless `stats` is non-NULL or opt->validate is set,
 *   which synchronise the stream before returning.  Calls on different
 *   streams with different workspaces are independent.
 *
 * Errors
 *   Status codes only.  Scalar arguments are checked on the host before any
 *   launch; the range of idx, r_diag > 0 and finiteness are checked on the
 *   device only when opt->validate is set.  Non-convergence is not an error:
 *   CGD_NOT_CONVERGED is returned (when stats is non-NULL) and X_a is still
 *   written from the last iterate.
 */
#ifndef CGD_ENKF_H
#define CGD_ENKF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CGD_OK = 0,
  CGD_NOT_CONVERGED = 1,   /* X_a written; at least one column hit maxit        */
  CGD_ERR_ARG = -1,        /* bad scalar argument or NULL pointer               */
  CGD_ERR_INDEX = -2,      /* idx out of [0, n) (validate only)                  */
  CGD_ERR_NONPOS_R = -3,   /* some r_diag <= 0 (validate only)                   */
  CGD_ERR_NONFINITE = -4,  /* non-finite input or CG coefficient                 */
  CGD_ERR_WORKSPACE = -5,  /* workspace NULL or smaller than required            */
  CGD_ERR_HIP = -6,        /* a HIP runtime call failed                          */
  CGD_ERR_UNSUPPORTED = -7, /* size or mode outside what this build supports     */
  CGD_ERR_BUSY = -8        /* the per-member or resident solvers' workgroups
                              were not all
                              resident within 1 ms of their start (another
                              kernel held part of the GPU); nothing was
                              written to X_a.  Retry, or set
                              cgd_tuning.cooperative (with stats only)         */
} cgd_status;

typedef enum {
  CGD_FP64 = 0,        /* everything in double                                   */
  CGD_FP32 = 1,        /* float storage and products; per-column CG scalars in
                          double                                                 */
  CGD_MIXED_BF16 = 2,  /* float storage; S-products in bf16 with float
                          accumulation inside restarted iterative refinement
                          whose outer residual is float S with double
                          accumulation                                           */
  CGD_BF16_SPLIT = 3   /* float storage; each S-product as five bf16 products
                          of split factors (Henry, Tang and Heinecke, 2019):
                          S as two bf16 parts (s1 = bf16(s), s2 = bf16(s - s1)),
                          the vector as three (v1, v2, v3 likewise), and
                          s2 v2 + s1 v3 + s2 v1 + s1 v2 + s1 v1 (their bf16x3
                          set plus the two bf16x6 terms that need no third part
                          of S), float accumulation; S is carried to about
                          2^-18 relative.  Plain CG stopped on the recursive
                          residual as in CGD_FP32; W = S^T Z and the reported
                          true residual from the float S with double
                          accumulation.  Full mode on solver 5 only (N <= 128,
                          no z0, no stall fallback, rr_period 0); elsewhere
                          CGD_ERR_UNSUPPORTED                                   */
} cgd_precision;

typedef enum {
  CGD_PRECOND_NONE = 0,    /* plain CG on Psi z = d                               */
  CGD_PRECOND_DIAG_R = 1   /* CG preconditioned by M = diag(r): the system is
                              solved in the variables of the L^{-1} scaling of
                              Algorithm 2 (eqs. LL-0..LL-2), i.e.
                              (R^{-1/2} Psi R^{-1/2}) (R^{1/2} z) = R^{-1/2} d,
                              whose matrix is I + P P^T with P = R^{-1/2} S /
                              sqrt(N-1) of rank <= N-1, so CG ends in at most N
                              steps in exact arithmetic (Section 5.2, Lemma 1).
                              The iterates are those of preconditioned CG with
                              M = diag(r).  The stop rule, the warm-start
                              fallback tests and relres_out then use the
                              R^{-1}-weighted norm ||v||_{R^{-1}} =
                              ||R^{-1/2} v|| in place of the 2-norm; z0 and
                              z_out stay in the original variables.          */
} cgd_precond;

/* Tuning and diagnostics: overrides of automatic choices and profiling hooks.
 * Not part of the method; NULL cgd_options.tuning means all automatic. */
typedef struct {
  int grid;               /* workgroups of the streaming solver, 0 = automatic  */
  int solver;             /* 0 = automatic, 1 = streaming (any N), 2 = resident
                             (N <= 128 FP32 / 64 FP64, rows fit co-resident),
                             3 = per-member columns (N <= 64, m <= 4096 FP32 /
                             2048 FP64), 4 = split per-member (N <= 64, a slice
                             of m/P rows of S fits one workgroup's LDS, N * P
                             workgroups co-resident), 5 = row-block x
                             member-group (FP32, CGD_MIXED_BF16 or
                             CGD_BF16_SPLIT, N <= 128, no z0, no stall fallback,
                             rr_period 0, workgroups co-resident).
                             CGD_MIXED_BF16 runs on solvers 3 and 5 only,
                             CGD_BF16_SPLIT on solver 5 only                    */
  int rows_per_block;     /* resident solver: 16, 32 or 64 (16 only for N > 64),
                             0 = automatic                                      */
  void* prof_events;      /* host array of two hipEvent_t that the library records
                             on `stream` right before and right after the solve
                             (the dominant kernel), or NULL                       */
  unsigned long long* trace; /* device buffer of 256 entries or NULL: the
                             resident and per-member solvers' workgroup 0 stores
                             the 100 MHz real-time counter at phase boundaries  */
  int cooperative;        /* resident, per-member and row-block x member-group
                             solvers (kinds 2-5),
                             whose workgroups wait for each other (the
                             streaming solver, kind 1, is always launched
                             cooperatively): 0 = plain launch with a
                             start-up census that fails with CGD_ERR_BUSY when
                             the grid is not all resident within 1 ms; 1 =
                             cooperative launch (the runtime runs the whole grid
                             at once or refuses the launch; slower per call)   */
  unsigned census_ticks;  /* the census's wait in 100 MHz ticks, 0 = 100000
                             (1 ms); a tiny value forces the CGD_ERR_BUSY path
                             (tests)                                           */
} cgd_tuning;

typedef struct {
  int prec;               /* cgd_precision                                        */
  int precond;            /* cgd_precond (cgd_enkf_analysis and the batched
                             calls; the reduced mode scales by L^{-1} always)   */
  int rr_period;          /* CGD_MIXED_BF16: at most this many inner CG steps per
                             refinement step, 0 = until the inner residual has
                             dropped by 1e-2                                      */
  const void* z0;         /* device m x N warm start for Z, or NULL (zero start)  */
  int fallback_on_stall;  /* 1: restart a warm-started column from zero when its
                             initial residual exceeds ||d_j|| or its residual
                             falls by less than 10% over 5 iterations
                             (CGD_ERR_UNSUPPORTED with CGD_MIXED_BF16 and z0:
                             its refinement loop has no restart rule)             */
  void* z_out;            /* device m x N: the solution Z, or NULL                */
  int* iters_out;         /* device N ints: iterations per member, or NULL        */
  double* relres_out;     /* device N doubles: ||d_j - Psi z_j|| / ||d_j||
                             evaluated with double accumulation, or NULL          */
  int validate;           /* 1: check idx range, r_diag > 0 and finiteness on the
                             device first (synchronises the stream)              */
  const void* r_factor;   /* NULL: R = diag(r_diag).  Otherwise R is not diagonal
                             and is given by its Cholesky factor R = L L^T with L
                             lower bidiagonal (Section 5.1; a tridiagonal R such
                             as Example 2's, from cgd_tridiag_cholesky): device
                             array of 2m-1 values, diag(L) then the subdiagonal
                             (L[i+1][i]).  The analysis then whitens by L: CG on
                             L^{-1} Psi L^{-T} (L^T z) = L^{-1} d, whose matrix is
                             I + P P^T (rank(P) <= N-1), i.e. CG preconditioned
                             by M = R; the stop rule, warm-start tests and
                             relres_out use ||v||_{R^{-1}} = ||L^{-1} v||, z0 and
                             z_out stay in the original variables, and
                             workspace sizes take mode | 2.  r_diag must still
                             be a valid pointer (diag(R)); precond is implied.
                             Not for batched calls (CGD_ERR_UNSUPPORTED).       */
  const cgd_tuning* tuning; /* host pointer or NULL (automatic)                   */
} cgd_options;

typedef struct {          /* host-side summary (filled when stats != NULL)       */
  int iters_max;
  int iters_min;
  int n_converged;
  int n_fallbacks;
  double relres_max;      /* max over members of the true relative residual      */
} cgd_stats;

/* Default options: CGD_FP64, zero start, no outputs beyond X_a. */
void cgd_options_default(cgd_options* opt);

/* Bytes of device workspace for one call.  mode 0 = cgd_enkf_analysis,
 * 1 = cgd_enkf_reduced_analysis, plus 2 when opt->r_factor is set (the
 * whitening pass's buffers).  Returns 0 for invalid sizes. */
size_t cgd_enkf_workspace_bytes(int n, int m, int N, int k, int prec, int mode);

/*
 * CGD-EnKF analysis (Sections 3.1-3.3, Algorithm 1).
 *
 * Solves Psi z_j = d_j for all N members at once: N independent CG
 * recurrences (per-member alpha_j, beta_j) that share every product with S.
 * Column j stops when ||r_j|| <= tol * ||d_j|| on the recursively updated
 * residual, or after maxit iterations; tol = 0 runs exactly maxit iterations
 * (the fixed-r runs of Tables 4-5).  Then X_a = X_f + A (S^T Z)/(N-1).
 * Requires n >= 1, m >= 1, N >= 2, k >= 1, tol >= 0, maxit >= 0.
 */
cgd_status cgd_enkf_analysis(int n, int m, int N, int k,
                             const void* X_f, void* X_a,
                             const int32_t* idx, const void* w,
                             const void* y, const void* r_diag, const void* eps,
                             double tol, int maxit, const cgd_options* opt,
                             void* workspace, size_t ws_bytes,
                             cgd_stats* stats, void* stream);

/*
 * cgd_enkf_analysis without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  The workspace is a static device array
 * of cgd_enkf_static_scratch_bytes() bytes (32 MiB) inside the library, one
 * per GPU, held until the process ends; this call allocates nothing.  Sizes
 * whose workspace (cgd_enkf_workspace_bytes(n, m, N, k, prec, 0)) exceeds it
 * return CGD_ERR_WORKSPACE before any launch.  Every call on one GPU uses
 * that GPU's array and leaves its contents behind (each launch sequence
 * clears what it needs), so calls that overlap on one GPU (different streams
 * or host threads without ordering) race and must not be issued.  Arguments,
 * results and errors are otherwise those of cgd_enkf_analysis.
 */
size_t cgd_enkf_static_scratch_bytes(void);
cgd_status cgd_enkf_analysis_static(int n, int m, int N, int k,
                                    const void* X_f, void* X_a,
                                    const int32_t* idx, const void* w,
                                    const void* y, const void* r_diag, const void* eps,
                                    double tol, int maxit, const cgd_options* opt,
                                    cgd_stats* stats, void* stream);

/*
 * CGD-EnKF-Reduced analysis (Algorithm 2, Section 5.2) for diagonal R:
 *   L = diag(sqrt((N-1) r)),  P = L^{-1} S,  Yhat = (y - zbar) 1^T + E,
 *   G = I + P^T P,  B = I + P^T L^{-1} Yhat,  X_a = X_f G^{-1} B,
 * with G^{-1} B by CG from W = 0, one recurrence per column of B (at most N
 * iterations in exact arithmetic); tol and maxit act on this N x N solve
 * (relative to ||b_j||).  opt->z0, z_out and relres_out are ignored;
 * iters_out receives the N x N solve's iteration counts.
 */
cgd_status cgd_enkf_reduced_analysis(int n, int m, int N, int k,
                                     const void* X_f, void* X_a,
                                     const int32_t* idx, const void* w,
                                     const void* y, const void* r_diag, const void* eps,
                                     double tol, int maxit, const cgd_options* opt,
                                     void* workspace, size_t ws_bytes,
                                     cgd_stats* stats, void* stream);

/*
 * Simultaneous serial EnKF, sEnKF (Section 2.4, Figure 1, Appendix A
 * Algorithm 3): the analysis with the inverse of the innovation matrix
 * replaced by the inverse of its diagonal, so that every observation
 * component j has its own scalar gain,
 *   X_a = X_f + X_f Zhat^T diag(Zhat Zhat^T + (N-1) R)^{-1} (Y - Z),
 * Z = H X_f, Zhat = Z - zbar 1^T, Y = y 1^T + E, all gains taken from the
 * same X_f.  Only diag(R) = r_diag enters (the method neglects the
 * off-diagonal entries of R by construction; opt->r_factor is ignored).
 * No system is solved: no CG, tol or maxit.  opt->prec must be CGD_FP64 or
 * CGD_FP32 (CGD_ERR_UNSUPPORTED for the BF16 modes); opt->validate and
 * tuning->prof_events act as for cgd_enkf_analysis; iters_out (if set)
 * receives zeros; z0, z_out, relres_out and precond are ignored.  The
 * workspace is that of the reduced mode:
 * cgd_enkf_workspace_bytes(n, m, N, k, prec, 1) bytes, 256-byte aligned.
 * stats (synchronises) reports 0 iterations and N members converged;
 * CGD_ERR_INDEX when an observation index is out of range.  X_a may alias
 * X_f.  Same argument layouts as cgd_enkf_analysis.
 */
cgd_status cgd_senkf_analysis(int n, int m, int N, int k,
                              const void* X_f, void* X_a,
                              const int32_t* idx, const void* w,
                              const void* y, const void* r_diag, const void* eps,
                              const cgd_options* opt, void* workspace, size_t ws_bytes,
                              cgd_stats* stats, void* stream);

/*
 * CGD-EnKF in the explicit-gain form of Figure 2 (Section 3.1, eqs. K_KF_T
 * and K_KF_T_rewrite): every column i = 0..n-1 of K^T (m x n) solves
 *   Psi_z (K^T e_i) = Psi_x^T e_i,  Psi_x = A S^T/(N-1),
 * by its own CG recurrence from zero (per-column alpha, beta; column i stops
 * when ||r_i|| <= tol ||b_i|| on the recursively updated residual, or after
 * maxit iterations), then X_a = X_f + K (Y - Z) with K = (K^T)^T.  The
 * result equals cgd_enkf_analysis's at convergence (Proposition 2) for n
 * right-hand sides in place of N, so it costs about n/N times as much: the
 * form for studying the gain and the CG error of Section 4 (Example 1b), not
 * for production analyses.  One workgroup per 16 columns, all m rows, both
 * S-products on the MFMA; no workgroup waits for another.
 *   opt->prec   CGD_FP64 or CGD_FP32 (else CGD_ERR_UNSUPPORTED); N <= 128
 *               (else CGD_ERR_UNSUPPORTED).
 *   opt->iters_out  device n ints (iterations per column of K^T), or NULL;
 *               opt->validate and tuning->prof_events as for
 *               cgd_enkf_analysis; other options are ignored.
 *   kt_out      device m x n row-major array of the prec's type (K^T), or NULL.
 *   hist_out    device maxit x n doubles, or NULL: entry [t][i] =
 *               alpha_t ||r_t||^2 of column i's step t (written for the
 *               steps taken), which by the Hestenes-Stiefel identity is
 *               ||e_t||^2_Psi - ||e_{t+1}||^2_Psi, so the energy-norm error
 *               of every iterate follows from the tail sums once the column
 *               has converged.
 *   workspace   cgd_enkf_gain_workspace_bytes(n, m, N, k, prec) bytes,
 *               256-byte aligned (0 for unsupported sizes).
 *   stats       (synchronises) iteration range and converged count over the
 *               n columns; relres_max is not computed (0).  CGD_NOT_CONVERGED
 *               when a column stopped at maxit, CGD_ERR_INDEX for an index
 *               out of range.
 * Only diagonal R: opt->r_factor set gives CGD_ERR_UNSUPPORTED.  X_a may
 * alias X_f.
 */
size_t cgd_enkf_gain_workspace_bytes(int n, int m, int N, int k, int prec);
cgd_status cgd_enkf_gain_analysis(int n, int m, int N, int k,
                                  const void* X_f, void* X_a,
                                  const int32_t* idx, const void* w,
                                  const void* y, const void* r_diag, const void* eps,
                                  double tol, int maxit, const cgd_options* opt,
                                  void* kt_out, double* hist_out,
                                  void* workspace, size_t ws_bytes,
                                  cgd_stats* stats, void* stream);

/*
 * Batched analyses (no paper source: many filters per call is an extension;
 * each problem is the analysis of Algorithm 1 as cgd_enkf_analysis computes
 * it).  Many independent filters (each its own n, m, 2 <= N <= 64,
 * k), every problem solved as cgd_enkf_analysis solves it with the
 * per-member solver (same recurrence, stop rule and update).  One call is
 * three launches over work tables: the gather of S and D (one workgroup per
 * gather_rows padded observation rows of a problem), the CG (one workgroup
 * per member of a problem, all members of a problem on one XCD so its S stays
 * in that L2, problems in decreasing order of work, the vectors in the
 * workspace so any m fits), and the ensemble update (one workgroup per
 * update_rows state rows).  No workgroup waits for another.  The row counts
 * are per problem (see cgd_problem); invalid ones make the workspace size 0
 * and prepare return CGD_ERR_ARG.  opt->prec must be
 * CGD_FP64 or CGD_FP32; warm starts, z_out and relres_out are not supported
 * for batches.
 *
 *   1. cgd_enkf_batched_workspace_bytes  size of the batch workspace (0 for
 *      invalid sizes);
 *   2. cgd_enkf_batched_prepare          uploads the problem descriptors and
 *      work tables into the workspace and fills *plan (synchronises
 *      `stream`); the arrays the descriptors point to must stay valid while
 *      the plan is used;
 *   3. cgd_enkf_batched_run              launches only (error-word reset,
 *      gather, CG, update), so with stats == NULL it can be captured into a
 *      HIP graph and replayed; `stats` (host array of `count`, caller order)
 *      synchronises.  Returns CGD_ERR_INDEX when an observation index of any
 *      problem is out of range, CGD_NOT_CONVERGED when a member of any
 *      problem stopped at maxit (with stats only).
 */
typedef struct {
  int n, m, N, k;
  const void* X_f;
  void* X_a;               /* may alias X_f                                       */
  const int32_t* idx;
  const void* w;
  const void* y;
  const void* r_diag;
  const void* eps;         /* or NULL                                             */
  int* iters_out;          /* device N ints or NULL                               */
  int gather_rows;         /* padded observation rows per gather workgroup: 0 for */
                           /* 256, else a multiple of 32 in [32, 4096]            */
  int update_rows;         /* state rows per update workgroup: 0 for 256, else a  */
                           /* multiple of 64 in [64, 4096]                        */
} cgd_problem;             /* the two row counts only shape the work tables (an   */
                           /* autotuner's choice); results do not depend on them  */

/* Filled by cgd_enkf_batched_prepare; read by cgd_enkf_batched_run. */
typedef struct {
  int count, prec;
  int n_gather, n_solve, n_update;   /* workgroups of the three launches (n_solve */
                                     /* includes empty padding entries)           */
  size_t off_desc, off_gtab, off_stab, off_utab, off_prefix, off_coli;
                                     /* byte offsets of regions in the workspace */
  size_t ws_bytes;
} cgd_batch_plan;

size_t cgd_enkf_batched_workspace_bytes(int count, const cgd_problem* probs, int prec);
cgd_status cgd_enkf_batched_prepare(int count, const cgd_problem* probs, int prec,
                                    void* workspace, size_t ws_bytes, cgd_batch_plan* plan,
                                    void* stream);
cgd_status cgd_enkf_batched_run(const cgd_batch_plan* plan, void* workspace, double tol,
                                int maxit, const cgd_options* opt, cgd_stats* stats,
                                void* stream);

/* The same batch in one call: cgd_enkf_batched_prepare (with opt->prec, so
 * it synchronises `stream` and cannot be graph-captured), then
 * cgd_enkf_batched_run.  Workspace: cgd_enkf_batched_workspace_bytes. */
cgd_status cgd_enkf_analysis_batched(int count, const cgd_problem* probs, double tol, int maxit,
                                     const cgd_options* opt, void* workspace, size_t ws_bytes,
                                     cgd_stats* per_problem_stats, void* stream);

/* Cholesky factor of a symmetric tridiagonal R (diagonal r_diag, m values;
 * off-diagonal r_offdiag, m-1 values, R[i][i+1] = R[i+1][i]) for
 * cgd_options.r_factor: writes factor (2m-1 values: diag(L), then L[i+1][i])
 * with R = L L^T; the factor of a tridiagonal matrix is bidiagonal
 * (Section 5.3).  Device arrays in the value type of prec.  A setup call: it
 * runs the O(m) recurrence on one device thread and synchronises `stream`.
 * Returns CGD_ERR_NONPOS_R when R is not positive definite (a pivot <= 0),
 * CGD_ERR_ARG for bad arguments. */
cgd_status cgd_tridiag_cholesky(int m, const void* r_diag, const void* r_offdiag, void* factor,
                                int prec, void* stream);

/* Which solver cgd_enkf_analysis would run for these sizes and options
 * (host-only; queries the current device's occupancy, launches nothing).
 *   solver:          1 = streaming cooperative solver, 2 = resident solver,
 *                    3 = per-member column solver, 4 = split per-member solver,
 *                    5 = row-block x member-group solver
 *   rows_per_block:  observation rows per workgroup block (kinds 1, 2, 4, 5)
 *   workgroups:      workgroups of the solver launch
 * Returns CGD_OK, CGD_ERR_ARG for invalid sizes/options or NULL outputs,
 * CGD_ERR_UNSUPPORTED when opt->solver forces a variant that cannot run,
 * CGD_ERR_HIP when the device query fails. */
cgd_status cgd_enkf_solver_info(int n, int m, int N, int k, const cgd_options* opt,
                                int* solver, int* rows_per_block, int* workgroups);

/* Diagnostic: 0 when every solver variant the library could launch for these
 * sizes indexes only inside its own workspace regions, else the number of
 * regions that would be overrun (-1 for invalid sizes).  Host-only, no GPU. */
int cgd_layout_selfcheck(int n, int m, int N, int k, int prec);

/* Human-readable name of a status code (static storage). */
const char* cgd_status_string(int status);

/* Library version, e.g. "0.1.0". */
const char* cgd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CGD_ENKF_H */
