/*
 * cphifi.h -- C ABI of libcphifi.so, an MI355X (gfx950) solver for the
 * unaligned infinite-dimensional (RKHS) mode subproblem of CP-HIFI tensor
 * decompositions (Brust & Kolda, "Fast and Accurate CP-HIFI Tensor
 * Decompositions Exploiting Kronecker Structure", Section 4).
 *
 * The subproblem (Section 4.1, eq. unaligned-infinite-1): given the psd kernel
 * matrix K (n x n) of the RKHS mode, the observed entries Omega of the data
 * tensor (q of them, each with a time index t_l in [0,n), indices i_l, j_l
 * into the two other modes and a value y_l), the other modes' factor rows and
 * the regularisers lambda > 0 and rho > 0, find W (n x r) solving
 *
 *     (F^T F + lambda (I_r kron K) + rho I) vec(W) = vec(K B),
 *
 * where row l of F is Zhat(l,:) kron K(t_l,:) (eq. F), Zhat(l,:) =
 * A(i_l,:) * B(j_l,:) (eq. zhat) and B(s,:) = sum_{l: t_l = s} y_l Zhat(l,:)
 * is the observed MTTKRP.  The time factor used by CP-HIFI is K W.
 *
 * Method (Section 4.4): preconditioned conjugate gradients with the two-step
 * Kronecker product (Section 4.4.1, eqs. vl, yhat1) and the preconditioner
 * M = gamma V kron K^2 + lambda I kron K + rho I applied through the
 * eigendecompositions of K and V = Z^T Z (Section 4.4.2, eqs. precon, fx).
 *
 * Conventions
 *  - Every matrix argument is a DEVICE pointer unless stated otherwise, owned by
 *    the caller, and must stay valid for the plan's lifetime.
 *  - n x r unknowns (W, X, B, ...) are row-major: element (s, c) at [s*r + c].
 *    (The paper's vec is column-major; vec(W)[c*n + s] = W[s*r + c].)
 *  - K and UK are n x n with row stride `ldk` >= n (elements).  UK holds the
 *    eigenvectors of K in LAPACK (column-major) order: eigenvector k occupies
 *    UK[k*ldk + 0 .. k*ldk + n-1], with eigenvalue dK[k].
 *  - All work is enqueued on the plan's HIP stream (`stream`, a hipStream_t;
 *    NULL = the null stream); cphifi_ui_solve_subproblem also forks part of
 *    its setup onto a second stream of the plan and joins it back into the
 *    plan's stream before it returns.  Call a plan's functions with the
 *    device that was current at its creation (its stream's) current.  Functions marked "async" return before
 *    the GPU finishes; those marked "sync" synchronise the stream before
 *    returning.
 *  - Every function returns a status code (CPHIFI_*).  No exception crosses
 *    the ABI.  On failure cphifi_last_error() gives a thread-local message.
 *  - The library never allocates device memory on the solve path: the caller
 *    provides a workspace of cphifi_ui_workspace_bytes() bytes.
 *  - A plan is not thread-safe.  Distinct plans may run on distinct streams.
 */
#ifndef CPHIFI_H
#define CPHIFI_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define CPHIFI_API __attribute__((visibility("default")))
#else
#define CPHIFI_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* ----------------------------------------------------------------- status */
enum cphifi_status {
  CPHIFI_OK = 0,
  CPHIFI_INVALID_ARG = 1,    /* bad size, null pointer, bad parameter, small workspace */
  CPHIFI_HIP_ERROR = 2,      /* a HIP runtime call failed; detail in cphifi_last_error() */
  CPHIFI_UNSUPPORTED = 3,    /* valid request this build does not implement */
  CPHIFI_BREAKDOWN = 4,      /* PCG breakdown: p^T A p <= 0 or r^T z <= 0 */
  CPHIFI_NUMERIC = 5,        /* NaN or Inf met in the iteration */
  CPHIFI_NOT_CONVERGED = 6   /* soft: iteration cap reached; W and info still written */
};

/* ------------------------------------------------------------- precision */
enum cphifi_precision {
  CPHIFI_FP64 = 0,        /* PCG of Section 4.4 entirely in FP64 (paper form) */
  CPHIFI_MIXED_FP32 = 1,  /* FP64 iterative refinement around an FP32-MFMA inner PCG */
  CPHIFI_MIXED_BF16 = 2   /* same, with the eigenvector products in BF16 MFMA */
};

/* ------------------------------------------------------------------ flags */
enum cphifi_flags {
  CPHIFI_FLAG_WARM_START = 1,   /* W holds x0 on entry to solve (else x0 = 0) */
  CPHIFI_FLAG_VALIDATE = 2,     /* accepted for compatibility: plan_create always
                                   range-checks obs_i / obs_j on the host */
  CPHIFI_FLAG_TIME_KERNELS = 4, /* record HIP events around the n x n products of
                                   one kernel: FP64 plans the transposed FP64
                                   product (K X, U_K X), mixed plans the low-
                                   precision one */
  CPHIFI_FLAG_NO_PRECOND = 8,   /* plain CG (identity preconditioner), FP64 only */
  CPHIFI_FLAG_EIGENBASIS = 16,  /* FP64 PCG in the eigenbasis of K (2 n x n passes
                                   per iteration instead of 4); same solution */
  CPHIFI_FLAG_NO_UKT_COPY = 32, /* plans with n >= 4096 keep a transposed copy of
                                   U_K in the workspace (n ldk doubles, made at
                                   plan creation), so U_K^T X runs the faster
                                   transposed FP64 kernel too; this flag drops
                                   the copy (row-major kernel for U_K^T X) */
  CPHIFI_FLAG_TIME_FP64 = 64,   /* with FLAG_TIME_KERNELS: mixed plans time the
                                   transposed FP64 product (the rotations, the
                                   FP64 residuals and the certificate) instead
                                   of the low-precision one */
  CPHIFI_FLAG_PERSISTENT = 128, /* FP64 paper form, n <= 2048, r <= 32, no kernel
                                   timing, no eigenbasis or structured form:
                                   run the whole PCG in one persistent launch
                                   of co-resident workgroups that meet at
                                   grid barriers (no launch or host poll per
                                   iteration).  Plans with r <= 8 and n r <=
                                   2560, or r <= 12 and n <= 256, take it
                                   without the flag (at n = 208, r = 5: 1.25
                                   against 2.20 ms per solve); above that the
                                   multi-kernel loop is as fast or faster.
                                   Should the
                                   workgroups not all be resident (a barrier
                                   wait times out), the solve falls back to the
                                   multi-kernel loop */
  CPHIFI_FLAG_TOEPLITZ_K = 256, /* K is symmetric Toeplitz, K(s,k) = c(|s-k|) (a
                                   translation-invariant kernel on a uniform
                                   grid; Section 4.4.1 notes the structure):
                                   the K products read c = K(0,:) only (n
                                   doubles; 2 n^2 r flops, O(n r) bytes).
                                   plan_create checks every entry of K against
                                   c to within 1e-12 max|c| (INVALID_ARG
                                   otherwise); products then differ from the
                                   dense ones by at most that much.  Not with
                                   the batched solver */
  CPHIFI_FLAG_NO_GRAPH = 1024,  /* FP64 paper form with n < 4096 normally replays
                                   a HIP graph of 8 captured PCG iterations
                                   (made on the plan's first solve; the host
                                   checks convergence between replays); this
                                   flag keeps the launch-by-launch loop */
  CPHIFI_FLAG_NO_PERSISTENT = 2048, /* never take the persistent launch of
                                   CPHIFI_FLAG_PERSISTENT (not even by default) */
  CPHIFI_FLAG_FP64_RESIDUALS = 4096, /* MIXED_BF16 plans with n >= 4096 keep an
                                   FP32 copy of U_K^T (4 n round_up(n, 256)
                                   bytes, made at plan creation) and form the
                                   refinement residual of a step in FP32 when
                                   the step can only bring the residual to
                                   >= 1e-3 of ||b|| (FP32 rounding, ~1e-7 of
                                   ||b||, is then far below what the next step
                                   needs); later residuals and the certificate
                                   stay FP64.  This flag keeps every residual
                                   in FP64 (no copy) */
  CPHIFI_FLAG_FIBER_COLLAPSE = 512 /* every (time, sample) pair that is observed
                                   at all is observed at all J features once:
                                   the gather-scatter of eqs. vl / yhat1 runs
                                   per fiber as A(i,:) had ((Xhat(s,:) had
                                   A(i,:)) B^T B), r^2 work per fiber instead
                                   of 2 J r (same operator up to rounding).
                                   plan_create checks the structure on the
                                   host (INVALID_ARG otherwise); implicit (A, B)
                                   form only; not with the batched solver */
};

/* Problem description (host struct). */
typedef struct cphifi_ui_desc {
  int64_t n;          /* design points of the RKHS mode (rows of K), >= 1 */
  int64_t r;          /* CP rank, 1..64 */
  int64_t q;          /* number of observations, >= 0 */
  int64_t I, J;       /* rows of A and B (implicit factor form); ignored with Zhat */
  int64_t ldk;        /* row stride of K and UK in elements, >= n; 0 means n */
  double lambda;      /* RKHS regulariser, > 0 */
  double rho;         /* shift of Section 4.1, > 0 */
  double gamma;       /* density of the preconditioner; <= 0 means q / (n I J) */
  double tol;         /* relative residual target ||b - A w|| / ||b|| */
  double inner_tol;   /* mixed forms: inner PCG relative tolerance of every refinement
                         step (<= 0: 1e-3 on the step that can reach tol, 3e-3 on the
                         earlier ones, which cannot) */
  int32_t precision;  /* enum cphifi_precision */
  int32_t flags;      /* OR of enum cphifi_flags */
  int32_t maxit;      /* PCG iteration cap (FP64) or inner cap (mixed); <= 0: 500 */
  int32_t max_refine; /* mixed forms: outer refinement steps; <= 0: 30 */
  int32_t check_every;/* host convergence poll period in iterations; <= 0: auto */
  int32_t reserved;
} cphifi_ui_desc;

/* Device inputs (caller-owned; must outlive the plan). */
typedef struct cphifi_ui_inputs {
  const double* K;         /* n x n (stride ldk), symmetric psd */
  const double* UK;        /* n x n (stride ldk), eigenvectors of K, column-major */
  const double* dK;        /* n eigenvalues of K (same order as UK) */
  const int32_t* obs_ptr;  /* n+1, CSR by time: observations of time s are
                              obs_ptr[s] .. obs_ptr[s+1]-1; obs_ptr[0] = 0,
                              obs_ptr[n] = q, nondecreasing */
  const int32_t* obs_i;    /* q, index into A's rows (implicit form) */
  const int32_t* obs_j;    /* q, index into B's rows (implicit form) */
  const double* A;         /* I x r row-major, or NULL with Zhat */
  const double* B;         /* J x r row-major, or NULL with Zhat */
  const double* Zhat;      /* q x r row-major per-observation Khatri-Rao rows
                              (eq. zhat, any tensor order); NULL = implicit form */
  const double* V;         /* r x r Gram Z^T Z; required with Zhat, optional
                              otherwise (NULL: computed as (A^T A) had (B^T B)) */
} cphifi_ui_inputs;

typedef struct cphifi_solve_info {
  int32_t status;          /* CPHIFI_* of the solve */
  int32_t iters;           /* PCG iterations (FP64) / total inner iterations (mixed) */
  int32_t refine_steps;    /* mixed forms: outer steps taken */
  int32_t gemm_launches;   /* with CPHIFI_FLAG_TIME_KERNELS: timed n x n products */
  double relres_true;      /* ||vec(KB) - A w|| / ||vec(KB)||, recomputed in FP64 */
  double relres_recursive; /* last recursively updated residual (FP64 PCG) */
  double gemm_ms;          /* with CPHIFI_FLAG_TIME_KERNELS: summed event time */
  double* history;         /* optional HOST buffer of maxit+1 doubles receiving the
                              recursive relative residual per iteration, or NULL */
} cphifi_solve_info;

typedef struct cphifi_plan cphifi_plan;

/* Bytes of device workspace a plan for `d` needs (host-only; no GPU call). */
CPHIFI_API int cphifi_ui_workspace_bytes(const cphifi_ui_desc* d, size_t* bytes);

/* Validate `d` and `in`, carve `workspace` (device, >= workspace_bytes bytes,
 * 256-byte aligned) and prepare per-K state: observation work lists and, for
 * the mixed forms, the low-precision copies of U_K.  sync.
 * Errors: INVALID_ARG (n, r, q, I, J out of range; r > 64; lambda <= 0; rho <= 0;
 * tol <= 0; missing pointers; both or neither of Zhat / (A,B); Zhat without V;
 * workspace too small or misaligned; an obs_i / obs_j index out of range),
 * HIP_ERROR. */
CPHIFI_API int cphifi_ui_plan_create(cphifi_plan** out, const cphifi_ui_desc* d,
                          const cphifi_ui_inputs* in, void* workspace,
                          size_t workspace_bytes, void* stream);

/* Per-solve setup of Section 4.4.2: V = Z^T Z (unless given), the
 * eigendecomposition V = U_V D_V U_V^T (eq. eigV, one-workgroup Jacobi) and
 * D(s,c) = 1 / (gamma dV_c dK_s^2 + lambda dK_s + rho) with dK clamped at 0.
 * async. */
CPHIFI_API int cphifi_ui_setup(cphifi_plan* p);

/* Right-hand side of eq. unaligned-infinite-1: b = K B with the observed
 * MTTKRP B(s,:) = sum_{l: t_l = s} y_l Zhat(l,:).  y: q doubles (device);
 * b: n x r row-major (device).  async. */
CPHIFI_API int cphifi_ui_rhs(cphifi_plan* p, const double* y, double* b);

/* The observed MTTKRP alone: Bm(s,:) = sum_{l: t_l = s} y_l Zhat(l,:)
 * (Section 4; for a fully observed tensor this is T Z, the right-hand side
 * of the aligned subproblem, eq. aligned-solve).  y: q doubles, Bm: n x r
 * row-major (device).  async. */
CPHIFI_API int cphifi_ui_mttkrp(cphifi_plan* p, const double* y, double* Bm);

/* y = (F^T F + lambda I kron K + rho I) x by the two-step product of Section
 * 4.4.1, in FP64.  x, y: n x r row-major device buffers (distinct).  async. */
CPHIFI_API int cphifi_ui_apply(cphifi_plan* p, const double* x, double* y);

/* z = M^{-1} x by eq. fx in FP64 (requires cphifi_ui_setup).  async. */
CPHIFI_API int cphifi_ui_precond(cphifi_plan* p, const double* x, double* z);

/* Operator in the eigenbasis of K at the plan's precision:
 * ybar = D_K Ut G(Ut^T D_K xbar) + lambda D_K xbar + rho xbar, where Ut is
 * U_K rounded to the plan precision and G is the gather-scatter of eqs. vl and
 * yhat1.  Equals U_K^T A U_K xbar for exact Ut.  async. */
CPHIFI_API int cphifi_ui_apply_lowp(cphifi_plan* p, const double* xbar, double* ybar);

/* Solve A w = b (b: n x r device, e.g. from cphifi_ui_rhs) by the plan's
 * method; W (n x r device) receives the solution (and holds x0 on entry when
 * FLAG_WARM_START is set).  info (host) is filled; its status is also the
 * return value unless an argument or HIP error occurred first.  The mixed
 * forms return OK only when the FP64 residual of the original system (with
 * K, not its eigenpairs) meets tol: relres_true; when a certificate misses,
 * refinement goes on from that residual (so eigenpairs that are not those of
 * K to working accuracy cost steps, not accuracy).  sync. */
CPHIFI_API int cphifi_ui_solve(cphifi_plan* p, const double* b, double* W,
                    cphifi_solve_info* info);

/* Whole subproblem from the observed values: setup, right-hand side, solve
 * and the FP64 true residual.  y: q doubles (device).  In the mixed forms the
 * refinement starts from the observed MTTKRP B itself (right-hand side
 * b = K B, Section 4.4): U_K^T b = D_K U_K^T B takes one pass over U_K and b
 * is never formed; relres_true is ||K (B - Yhat1 - lambda W) - rho W|| /
 * ||b||, the same FP64 paper-form residual, with ||b|| = ||U_K^T b||.  The
 * FP64 form forms b (cphifi_ui_rhs) and calls cphifi_ui_solve.  The setup's
 * r x r eigendecomposition of V runs on a second stream of the plan (made on
 * the first call, default priority) while the plan's stream forms the
 * right-hand side; the plan's stream waits for it before the first
 * preconditioner application, so all of the call's work is ordered before
 * later work on the plan's stream.  sync. */
CPHIFI_API int cphifi_ui_solve_subproblem(cphifi_plan* p, const double* y, double* W,
                               cphifi_solve_info* info);

/* Release host-side plan state (the workspace belongs to the caller). */
CPHIFI_API int cphifi_ui_plan_destroy(cphifi_plan* p);

/* One-time eigendecomposition K = U_K D_K U_K^T (eq. eigK) on the device
 * with rocSOLVER's divide-and-conquer symmetric eigensolver.  K (n x n,
 * stride ldk) is read; UK (n x n, stride ldk, column-major eigenvectors) and
 * dK (n, ascending) are written.  Allocates and frees its own scratch (setup
 * path only).  sync.  Errors: INVALID_ARG, HIP_ERROR, NUMERIC (solver failed
 * to converge). */
CPHIFI_API int cphifi_kernel_eig(int64_t n, const double* K, int64_t ldk, double* UK,
                      double* dK, void* stream);

/* The same decomposition by the cyclic Jacobi method, parallel round-robin
 * ordering (every step rotates m/2 disjoint index pairs, m = n rounded up to
 * even; each rotation is the symmetric 2 x 2 Schur decomposition that
 * annihilates one off-diagonal entry), written for the device: two launches
 * per step, n steps per sweep, O(n^3) work and traffic per sweep.  Stops when
 * the off-diagonal mass ||A - diag(A)||_F falls to tol ||K||_F (tol > 0, e.g.
 * 1e-14) or after max_sweeps sweeps; sweeps_out (host, may be NULL) receives
 * the count.  K is symmetrised ((K + K^T) / 2) on entry.  Output as
 * cphifi_kernel_eig: UK row k = eigenvector k, dK ascending.  n <= 8192.
 * Allocates and frees its own scratch (2 n^2 doubles; setup path only).  sync.
 * Errors: INVALID_ARG, HIP_ERROR, NUMERIC (not converged within max_sweeps). */
CPHIFI_API int cphifi_kernel_eig_jacobi(int64_t n, const double* K, int64_t ldk, double* UK,
                                        double* dK, double tol, int max_sweeps, int* sweeps_out,
                                        void* stream);

/* ------------------------------------------------------ aligned subproblem
 * Section 3: every entry of the data tensor observed (one shared time grid).
 * The RKHS factor then solves eq. aligned-solve,
 *     (V kron K + lambda I) vec(W) = vec(Bm),  V = Z^T Z,  Bm = T Z (MTTKRP),
 * by one of two methods on K = U_K D_K U_K^T (eq. eigK):
 *   CPHIFI_ALIGNED_DECOUPLED: the decoupled direct solve of Section 3.2,
 *     W = U_K ((U_K^T Bm U_V) had D) U_V^T, D = 1 / (dV_c dK_s + lambda)
 *     (eq. W-decoupled; V = U_V D_V U_V^T, eq. eigV, by one-workgroup Jacobi);
 *   CPHIFI_ALIGNED_PCG: PCG on the transformed system of Section 3.3,
 *     (V kron D_K + lambda I) vec(Wbar) = vec(U_K^T Bm), product D_K X V +
 *     lambda X (eq. pcg-matvec-ai), diagonal preconditioner diag(V)_c dK_s +
 *     lambda (eq. precond-ai), x0 = 0, stop at ||r|| <= tol ||U_K^T Bm||;
 *     the iteration loop runs in one single-workgroup kernel; W = U_K Wbar.
 * Eigenvalues dK < 0 (rounding) are taken as 0.  info: iters (PCG),
 * relres_true = ||Bbar - D_K Wbar V - lambda Wbar|| / ||Bbar|| in FP64 (the
 * residual of eq. aligned-solve for an orthogonal U_K), status.
 * Workspace: device, >= cphifi_aligned_workspace_bytes(), 256-byte aligned.
 * sync.  Errors: INVALID_ARG (sizes, lambda <= 0, tol <= 0 for PCG, missing
 * pointers, workspace), HIP_ERROR; PCG also BREAKDOWN, NUMERIC, NOT_CONVERGED
 * (soft: W and info written). */
enum cphifi_aligned_method {
  CPHIFI_ALIGNED_DECOUPLED = 0,
  CPHIFI_ALIGNED_PCG = 1
};

typedef struct cphifi_aligned_desc {
  int64_t n;          /* grid points (rows of K), >= 1 */
  int64_t r;          /* CP rank, 1..64 */
  int64_t ldk;        /* row stride of UK in elements, >= n; 0 means n */
  double lambda;      /* RKHS regulariser, > 0 */
  double tol;         /* PCG: relative residual target of the transformed system */
  int32_t method;     /* enum cphifi_aligned_method */
  int32_t maxit;      /* PCG iteration cap; <= 0: 500 */
} cphifi_aligned_desc;

typedef struct cphifi_aligned_inputs {
  const double* UK;   /* n x n (stride ldk), eigenvectors of K, column-major
                         (eigenvector k in UK[k*ldk .. k*ldk + n-1]) */
  const double* dK;   /* n eigenvalues of K */
  const double* Bm;   /* n x r row-major MTTKRP T Z (e.g. cphifi_ui_mttkrp) */
  const double* V;    /* r x r Gram Z^T Z, or NULL to form (A^T A) had (B^T B) */
  const double* A;    /* I x r, B: J x r row-major factors (used when V is NULL) */
  const double* B;
  int64_t I, J;
} cphifi_aligned_inputs;

CPHIFI_API int cphifi_aligned_workspace_bytes(const cphifi_aligned_desc* d, size_t* bytes);
CPHIFI_API int cphifi_aligned_solve(const cphifi_aligned_desc* d, const cphifi_aligned_inputs* in,
                                    double* W, void* workspace, size_t workspace_bytes,
                                    void* stream, cphifi_solve_info* info);

/* ------------------------------------------------------------------ ALS
 * CP-HIFI alternating optimisation (Section 2, eq. cp-hifi-subproblem) for a
 * 3-way tensor whose three modes are all infinite-dimensional (the setting of
 * the unaligned experiments of Section 5.2).  Mode k's factor is
 * A_k = K_k W_k.  One outer iteration solves, for k = 0, 1, 2 in turn, the
 * unaligned subproblem of eq. unaligned-infinite-1 for W_k (observations
 * grouped by their mode-k index, Khatri-Rao rows from the other two factors,
 * warm-started from the current W_k; method and precision as in
 * cphifi_ui_solve_subproblem) and then sets A_k = K_k W_k.  The run stops
 * when the relative error ||y - model||_Omega / ||y||_Omega changes by less
 * than als_tol between outer iterations, or after max_outer of them (the
 * paper's runs: 50 iterations, 1e-6; subproblems to relres 1e-6 with at most
 * 75 iterations).  A subproblem that stops at its iteration cap counts in
 * `capped` and the run goes on.  Modes flagged finite take the CP-ALS row
 * update instead (see cphifi_als_desc.finite; W[k] then holds A_k). */
typedef struct cphifi_als_desc {
  int64_t n[3];       /* grid points per mode (rows of K_k), >= 1 */
  int64_t q;          /* observed entries, 1 .. 2^31 - 1 */
  int64_t r;          /* CP rank, 1..64 */
  double lambda[3];   /* RKHS regulariser per mode, > 0 */
  double rho;         /* shift of Section 4.1, > 0 */
  double tol;         /* subproblem relative residual target, > 0 */
  double als_tol;     /* stop when the error changes by less than this, >= 0 */
  int32_t precision;  /* enum cphifi_precision of the subproblem solves */
  int32_t flags;      /* subproblem flags (CPHIFI_FLAG_WARM_START is always added) */
  int32_t maxit;      /* subproblem iteration cap (<= 0: 500) */
  int32_t max_outer;  /* outer iterations, >= 1 */
  int32_t finite[3];  /* nonzero: mode k is finite-dimensional (Section 2: no
                         regulariser, so a CP-ALS block with missing data): its
                         factor A_k is the unknown itself, each row solving
                         (sum_l z_l z_l^T + rho I) a_i = sum_l y_l z_l over its
                         observations (rho keeps rows with few observations
                         definite); K, UK, dK and lambda of the mode unused */
  int32_t reserved;
} cphifi_als_desc;

/* Device inputs (caller-owned; must outlive the object). */
typedef struct cphifi_als_inputs {
  const double* K[3];     /* n_k x n_k (stride n_k), symmetric psd (NULL for finite modes) */
  const double* UK[3];    /* eigenvectors of K_k, laid out as cphifi_ui_inputs.UK */
  const double* dK[3];    /* eigenvalues of K_k */
  const int32_t* coords;  /* q x 3 row-major: the indices (i_0, i_1, i_2) of each entry */
  const double* y;        /* q observed values */
} cphifi_als_inputs;

typedef struct cphifi_als_info {
  int32_t outer;          /* outer iterations run */
  int32_t converged;      /* 1 when the error change fell below als_tol */
  int32_t inner_iters;    /* subproblem iterations over the whole run */
  int32_t capped;         /* subproblem solves that stopped at their cap */
  double rel_error;       /* final relative error on the observed entries */
  double* errors;         /* optional HOST buffer of max_outer + 1 doubles: the error
                             before the first and after every outer iteration */
} cphifi_als_info;

typedef struct cphifi_als cphifi_als;

/* Bytes of device workspace for `d` (host-only; no GPU call). */
CPHIFI_API int cphifi_als_workspace_bytes(const cphifi_als_desc* d, size_t* bytes);

/* Validate `d`, copy the entries and values to the host once (range checks;
 * the per-mode CSR lists and permuted values are built there and uploaded
 * into `workspace`: device, >= cphifi_als_workspace_bytes, 256-byte aligned)
 * and create the three subproblem plans inside it.  sync.
 * Errors: INVALID_ARG (sizes or parameters, a coordinate out of range, missing
 * pointers, workspace too small or misaligned), HIP_ERROR, and any
 * plan-creation error. */
CPHIFI_API int cphifi_als_create(cphifi_als** out, const cphifi_als_desc* d,
                                 const cphifi_als_inputs* in, void* workspace,
                                 size_t workspace_bytes, void* stream);

/* Run the alternating optimisation.  W: host array of 3 device pointers
 * (n_k x r row-major each): the starting weights on entry, the result on
 * exit.  F: host array of 3 device pointers that receive A_k = K_k W_k, or
 * NULL.  info (host) is filled.  sync.  Errors: INVALID_ARG, HIP_ERROR, and
 * NUMERIC / BREAKDOWN from a subproblem (outer iteration and mode named in
 * cphifi_last_error). */
CPHIFI_API int cphifi_als_run(cphifi_als* a, double* const* W, double* const* F,
                              cphifi_als_info* info);

/* Release host-side state and the three plans (the workspace is the caller's). */
CPHIFI_API int cphifi_als_destroy(cphifi_als* a);

/* ------------------------------------------------ products (tuning, tests)
 * The n x n by n x r products behind every step above (K X in Section 4.4.1,
 * U_K^T X and U_K X in eq. fx), exposed for tile tuning and per-variant
 * tests:  Y = op(U) diag(xscale) X.
 *   elt:    0 = FP64 U, 1 = FP32 U, 2 = BF16 U (bf16 needs trans = 0, a row
 *           stride ldu that is a multiple of 8 and >= round_up(n, 128), and
 *           zeros in columns n .. ldu-1), 3 = BF16 U in the 16 x 64 tile
 *           layout the solver's BF16 copies of U_K use: element (i, k) at
 *           ((i / 16) (ldu / 64) + k / 64) 1024 + (i % 16) 64 + k % 64, ldu a
 *           multiple of 64 (>= round_up(n, 128)), round_up(n, 16) rows (rows
 *           >= n are never read), zeros in columns n .. ldu-1.  FP32 and BF16
 *           accumulate in FP32; the two BF16 layouts give identical Y.
 *   trans:  0: op(U) = U (row-major, stride ldu);  1: op(U) = U^T.
 *   mw, s:  tile (16-row MFMA blocks per wave, MFMA steps per k chunk); see
 *           cphifi_product_tile_ok().  ksplit <= 0 chooses the split-K depth.
 *   X:      n x r row-major doubles (device), 1 <= r <= 64;  xscale: n doubles
 *           or NULL;  Y: n x r row-major doubles (device).
 *   workspace: device, >= cphifi_product_workspace_bytes(n, r, elt), 256-byte
 *           aligned (split-K partials and the BF16 split of X).
 * async.  Errors: INVALID_ARG (shape, tile, alignment), HIP_ERROR. */
CPHIFI_API int cphifi_product_workspace_bytes(int64_t n, int64_t r, int elt, size_t* bytes);
CPHIFI_API int cphifi_product_tile_ok(int elt, int mw, int s);
CPHIFI_API int cphifi_product(int elt, int trans, int mw, int s, int ksplit, int64_t n,
                              const void* U, int64_t ldu, const double* X, int64_t r,
                              const double* xscale, double* Y, void* workspace,
                              size_t workspace_bytes, void* stream);

/* The product of cphifi_product for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels and results, with the split-K partials
 * and the BF16 split of X in a static device array of the library
 * (cphifi_product_static_max_bytes() = 64 MiB per GPU, held by every GPU the
 * library runs on until the process ends) instead of a caller workspace.
 * Calls no allocating routine.  ksplit <= 0 takes the split cphifi_product
 * would, reduced until its partials fit; an explicit ksplit must fit.  Every
 * call on a GPU shares that GPU's array, so calls that overlap on one GPU
 * (different streams, or several threads) race: serialise them.  Arguments
 * and layouts as cphifi_product.  async.  Errors: INVALID_ARG (as
 * cphifi_product, and a product whose scratch exceeds the array: n (16
 * ceil(r/16)) 8 bytes per split slab, plus 4 (16 ceil(r/16)) round_up(n, 256)
 * bytes for BF16), UNSUPPORTED (device index >= 64), HIP_ERROR. */
CPHIFI_API size_t cphifi_product_static_max_bytes(void);
CPHIFI_API int cphifi_product_static(int elt, int trans, int mw, int s, int ksplit, int64_t n,
                                     const void* U, int64_t ldu, const double* X, int64_t r,
                                     const double* xscale, double* Y, void* stream);

/* Measurement helper: reads `bytes` of device memory at `buf` once (16-byte
 * loads, `blocks` workgroups of 256 threads striding over the buffer) and
 * writes each workgroup's sum of the doubles it read to partial[blockIdx]
 * (device, >= blocks doubles).  Its duration gives the achievable HBM read
 * rate that the products' rates are compared with.  buf 16-byte aligned,
 * bytes > 0 a multiple of 16, 1 <= blocks <= 65536.  async.  Errors:
 * INVALID_ARG, HIP_ERROR. */
CPHIFI_API int cphifi_stream_read(const void* buf, int64_t bytes, int32_t blocks,
                                  double* partial, void* stream);

/* ------------------------------------------------------- batched solver
 * Many independent UI subproblems (Section 4.4) of uneven n and r solved by
 * the mixed-precision method of cphifi_ui_solve_subproblem (precision
 * MIXED_BF16: FP64 iterative refinement of the system of eq.
 * unaligned-infinite-1 around inner PCG solves in the eigenbasis of K with
 * BF16 eigenvectors and the r x r step of eq. fx), all members together in
 * ONE persistent kernel launch that is captured with its reset kernel in a
 * HIP graph.  The launch starts from each member's observed values y: the
 * per-solve setup of Section 4.4.2 (V = Z^T Z unless given, eig(V) by Jacobi,
 * the inverse diagonal D), the observed MTTKRP B of the right-hand side
 * b = K B, the refinement and the FP64 certificate all run inside it.  Members: implicit (A, B)
 * form, n <= 65536, r <= 48, J r <= 8192 (B is read from an LDS copy), up to
 * 256 per batch; each member's desc and
 * inputs follow cphifi_ui_plan_create (tol: FP64 relres target; inner_tol,
 * maxit, max_refine, FLAG_WARM_START honoured per member).
 *
 * Workspace: device, >= cphifi_batch_workspace_bytes(), 256-byte aligned; it
 * holds every member's plan workspace plus the batch's scalars.  Product tiles
 * per member come from the autotuner's table at `tile_table` (NULL: the file
 * named by CPHIFI_TILE_TABLE, else built-in sizes).  create makes the member
 * plans (cphifi_ui_plan_create and cphifi_ui_setup, so each plan also serves
 * the cphifi_ui_* calls) and synchronizes `stream`.
 * Errors: INVALID_ARG, UNSUPPORTED (other precision, explicit Zhat, n too
 * large), HIP_ERROR, and any member's plan-creation error (member named in
 * cphifi_last_error). */
typedef struct cphifi_batch cphifi_batch;

CPHIFI_API int cphifi_batch_workspace_bytes(int count, const cphifi_ui_desc* descs,
                                            size_t* bytes);
CPHIFI_API int cphifi_batch_create(cphifi_batch** out, int count, const cphifi_ui_desc* descs,
                                   const cphifi_ui_inputs* inputs, void* workspace,
                                   size_t workspace_bytes, void* stream,
                                   const char* tile_table);

/* The plan of member `member` (owned by the batch, valid until destroy): every
 * cphifi_ui_* call works on it; it shares device buffers with the batched
 * solve, so do not run both at once. */
CPHIFI_API int cphifi_batch_plan(cphifi_batch* bt, int member, cphifi_plan** out);

/* Right-hand sides b_i = K_i B_i of all members (cphifi_ui_rhs per member;
 * the batched solve does not need them).  y, b: host arrays of `count` device
 * pointers.  async. */
CPHIFI_API int cphifi_batch_rhs(cphifi_batch* bt, const double* const* y, double* const* b);

/* Bind the observed values y_i (q_i doubles, device; may be NULL when
 * q_i = 0) and solutions W_i (n_i x r_i, device; x0 on entry for members with
 * FLAG_WARM_START) that the graph reads and writes.  y, W: host arrays of
 * `count` device pointers.  The sizes cannot be checked through raw pointers:
 * a shorter buffer is read or written past its end.  stream-ordered. */
CPHIFI_API int cphifi_batch_bind(cphifi_batch* bt, const double* const* y, double* const* W);

/* Solve all members: binds y / W when given (else the last binding), launches
 * the graph on the batch's stream.  With infos (host array of `count`) it
 * waits and fills them (iters = total inner iterations, refine_steps,
 * relres_true = FP64 ||b - A w|| / ||b|| with b = K B, status); the return value is then
 * OK, NOT_CONVERGED, NUMERIC or HIP_ERROR (the worst member; HIP_ERROR also
 * when a bounded grid wait timed out).  With infos NULL it returns after the
 * launch (async); read the results with cphifi_batch_info. */
CPHIFI_API int cphifi_batch_solve(cphifi_batch* bt, const double* const* y, double* const* W,
                                  cphifi_solve_info* infos);
CPHIFI_API int cphifi_batch_info(cphifi_batch* bt, cphifi_solve_info* infos);

/* The instantiated graph (hipGraphExec_t) of one batched solve: launching it
 * on any stream solves the bound batch.  Owned by the batch. */
CPHIFI_API int cphifi_batch_graph(cphifi_batch* bt, void** graph_exec);

/* Rounds run by the last launch (one PCG iteration or one refinement stage of
 * every active member per round) and the persistent grid size.  sync. */
CPHIFI_API int cphifi_batch_rounds(cphifi_batch* bt, int* rounds, int* grid);

/* Where the last launch spent its time, from the device real-time clock as
 * seen by one workgroup: ms[0..7] the eight phases of a round (products A and
 * the Gram V, gather-scatter and the MTTKRP, segment rows + split, products B
 * and eig(V), finish and D, x/r update (with the preconditioner in inner
 * iterations), preconditioner (refinement steps), control + p update), each
 * including its closing grid barrier; ms[8] the per-round setup.  ms: host
 * array of 9.  sync. */
CPHIFI_API int cphifi_batch_phase_ms(cphifi_batch* bt, double* ms);

/* Release the batch's host state and member plans (the workspace belongs to
 * the caller).  Waits for the batch's stream. */
CPHIFI_API int cphifi_batch_destroy(cphifi_batch* bt);

/* Human-readable name of a status code (static string). */
CPHIFI_API const char* cphifi_status_string(int status);

/* Detail of the last error on the calling thread ("" if none). */
CPHIFI_API const char* cphifi_last_error(void);

/* Library version string, e.g. "cphifi 0.1.0 gfx950". */
CPHIFI_API const char* cphifi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CPHIFI_H */
