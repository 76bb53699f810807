/*
 * cmtcs.h -- C ABI of the MI355X (gfx950) library for covariance-free EM (CoFEM) on clustered
 * multi-task compressive sensing (Lin & Ba, arXiv 2310.00420).
 *
 * Model (Sec. 2, Eq. (cmtcs)): task t has measurements y_t = Phi_t z_t + noise, Phi_t is
 * N_t x D, the noise precision is beta, and z_t belongs to one of C clusters with prior
 * precisions alpha_c (a C x D array) and prior probabilities pi_c.
 *
 * The library implements the E-step of CoFEM (Alg. 2) on the GPU: for every task t and cluster
 * c it solves, with the conjugate-gradient method of Alg. 1,
 *       A_tc x = b,   A_tc = beta Phi_t^T Phi_t + diag(alpha_c)            (Eq. (lin-sys))
 * for the posterior-mean right-hand side b_t = beta Phi_t^T y_t and K Rademacher probes
 * p_tck (Sec. 3.1), then forms the posterior mean mu_tc, the diagonal estimate s_tc
 * (Eq. (diag-est)), the log-determinant estimate nu_tc from the CG coefficients (Eqs. (tridiag),
 * (hutch-trace), (logdet-est), Sec. 3.2) and the cluster responsibilities q_tc (Eq. (estep));
 * and the M-step of Eq. (mstep).  A is never formed: each CG step applies Phi_t and Phi_t^T to
 * all right-hand sides of a task at once (Sec. 3.3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Array arguments are DEVICE pointers owned by the caller unless marked HOST.  Arrays are
 *    dense, row-major, without padding, in the element type stated at each argument.
 *  - Work is enqueued on the stream given to cmtcs_create and is asynchronous: outputs are
 *    valid once that stream has been synchronised.  The library never allocates device memory
 *    after cmtcs_create returns.  A call does not wait for the stream, with two exceptions: the
 *    first call with a new number of column slots per task (or after a change of tile shapes)
 *    copies the tile tables and, unless the autotuner is off, times candidate kernels, and waits
 *    for that; and cmtcs_profile reads its timings.  A CG loop always enqueues its whole step
 *    budget (max_iters or fixed_iters steps): every kernel of a step whose right-hand sides
 *    have all stopped returns at once on the device, so no host check is needed.
 *  - Every function returns a cmtcs_status_t; on anything but CMTCS_OK, cmtcs_last_error()
 *    returns a message for the calling thread.  Argument errors are detected on the host before
 *    any work is enqueued, and then no output is written.  No C++ exception crosses the ABI.
 *  - Numerical outcomes of individual solves (max iterations reached, breakdown) are not
 *    errors: they are reported per right-hand side through cmtcs_cg_stats_t.
 *  - A handle is not thread-safe; separate handles are independent.
 */
#ifndef CMTCS_H
#define CMTCS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cmtcs_handle_s* cmtcs_handle_t;

typedef enum {
  CMTCS_OK = 0,
  CMTCS_E_INVALID = 1,      /* bad argument: null pointer, bad size, inconsistent options   */
  CMTCS_E_HIP = 2,          /* a HIP runtime call failed (message names the call)           */
  CMTCS_E_NOMEM = 3,        /* workspace allocation failed in cmtcs_create                  */
  CMTCS_E_UNSUPPORTED = 4   /* valid request outside what this library implements           */
} cmtcs_status_t;

/* Storage type of Phi in device memory. */
typedef enum { CMTCS_F32 = 0, CMTCS_BF16 = 1, CMTCS_F16 = 2 } cmtcs_dtype_t;

/* Arithmetic of the operator products and of the CG vectors.
 *  CMTCS_MATH_F64: Phi products on FP64 matrix cores, CG vectors x, r, d, A d in FP64.
 *  CMTCS_MATH_F32: Phi products on FP32 matrix cores, CG vectors in FP32.
 *  CMTCS_MATH_MIXED: the library keeps Phi in 16 bits (phi_dtype BF16 or F16: a rounded copy
 *                    and a transposed rounded copy, built at create from the FP32 phi), rounds
 *                    the CG direction to the same type, and runs both products on 16-bit matrix
 *                    cores with FP32 accumulation; CG vectors are FP32.  Every refine_every
 *                    steps the recursive residual is replaced by the true residual b - A x,
 *                    computed with FP32 products from the FP32 phi.
 *  In every mode the CG scalars (r.r, d.Ad, gamma, xi), the tridiagonal eigenproblems, the
 *  log-determinants and the responsibilities are FP64. */
typedef enum { CMTCS_MATH_F64 = 0, CMTCS_MATH_F32 = 1, CMTCS_MATH_MIXED = 2 } cmtcs_math_t;

/* Per-right-hand-side CG outcome codes (values of cmtcs_cg_stats_t.status). */
enum {
  CMTCS_CG_CONVERGED = 0,   /* tolerance met, the fixed step count done, or r = 0 exactly   */
  CMTCS_CG_MAX_ITER = 1,    /* tolerance mode: max_iters steps without meeting tol          */
  CMTCS_CG_BREAKDOWN = 2,   /* d.Ad <= 0 or a non-finite scalar; the solve stopped before it */
  CMTCS_CG_NONPOS_RITZ = 3  /* cmtcs_estep probe columns only: the probe's tridiagonal
                               (Eq. (tridiag)) was not certified positive definite (or has
                               non-finite entries, or the solve took no step), so the probe was
                               left out of the average of Eq. (logdet-est); replaces the CG
                               outcome of that column                                       */
};

/* Sensing operator of a problem.
 *  CMTCS_OP_DENSE: Phi_t is a dense N_t x D float matrix (the configurations' Gaussian sensing).
 *  CMTCS_OP_PARTIAL_FOURIER: Phi_t = Omega_t F, the sensing of the experiments of Sec. 4: F is
 *      the unitary D x D DFT, F[k][d] = exp(-2 pi i k d / D) / sqrt(D), and Omega_t keeps the
 *      N_t rows (frequencies) listed in freq.  The complex measurements enter the real model
 *      stacked as [Re y_t; Im y_t] against [Re(Omega_t F); Im(Omega_t F)], with noise precision
 *      beta on each part, so that A = beta Re(F^H Omega_t^T Omega_t F) + diag(alpha_c) and
 *      b_t = beta Re(F^H Omega_t^T y_t); A is applied with FFTs in O(D log D) (Sec. 3.3), and
 *      each right-hand side's whole CG solve runs in one workgroup.  Requires MATH_F64 and D a
 *      power of two, 64..4096.  A frequency listed twice counts twice (its row appears twice). */
typedef enum { CMTCS_OP_DENSE = 0, CMTCS_OP_PARTIAL_FOURIER = 1 } cmtcs_operator_t;

/* Problem data: fixed for the lifetime of a handle.  The library reads phi and y in place (it
 * does not copy them), so they must stay valid and unchanged until destroy. */
typedef struct {
  int32_t T;                /* tasks, >= 1                                                  */
  int32_t C;                /* clusters, >= 1                                               */
  int32_t D;                /* signal length, a positive multiple of 16 (of 32 for
                               MATH_MIXED), <= 16384                                        */
  const int64_t* row_off;   /* HOST, T+1 non-decreasing prefix sums of N_t, row_off[0] = 0;
                               N_t = 0 is allowed (then A_tc = diag(alpha_c)).  Each task's
                               blocks are addressed with 32-bit offsets: round16(N_t)*D*4 bytes of Phi,
                               and slots*round16(N_t)*8 and slots*D*8 bytes of workspace
                               (slots = max_rhs rounded up to whole 16-column fragments, or to
                               whole 144-column groups past 144) must each stay below 4 GiB,
                               else CMTCS_E_UNSUPPORTED                                     */
  const void* phi;          /* device [row_off[T]][D] float: the stacked Phi_t (OP_DENSE;
                               ignored for OP_PARTIAL_FOURIER).  With MATH_F64 the workspace
                               also holds Phi_t transposed (round16(N_t)*D*4 bytes per
                               task), rebuilt from phi by every call that applies the
                               operator                                                     */
  cmtcs_dtype_t phi_dtype;  /* F32 for MATH_F64 / MATH_F32; for MATH_MIXED the 16-bit type
                               (BF16 or F16) the library stores Phi in                      */
  const float* phi_resid;   /* MATH_MIXED only: optional device [row_off[T]][D] float Phi
                               for the FP32 true-residual products (opts.refine_every), e.g.
                               a more accurate copy than phi; NULL = phi.  Caller-owned, read
                               by every residual replacement.  Must be NULL for the other
                               math modes and for OP_PARTIAL_FOURIER (CMTCS_E_INVALID)       */
  const float* y;           /* device measurements, stacked like Phi: [row_off[T]] (OP_DENSE)
                               or [row_off[T]][2] (re, im) pairs (OP_PARTIAL_FOURIER)       */
  double beta;              /* noise precision, > 0                                         */
  cmtcs_math_t math;        /* arithmetic, see cmtcs_math_t                                 */
  int32_t max_rhs;          /* largest number of right-hand sides per task any later call
                               uses: >= C*(K+1) for cmtcs_estep, >= R_per_task for
                               cmtcs_solve                                                   */
  int32_t max_iters;        /* largest CG step count any later call uses (1..4096)          */
  int32_t max_K;            /* largest probe count any later cmtcs_estep uses (>= 0)        */
  cmtcs_operator_t op;      /* sensing operator (zero: OP_DENSE)                            */
  const int32_t* freq;      /* OP_PARTIAL_FOURIER: device [row_off[T]] selected frequencies
                               of each task, each in 0..D-1 (checked at create:
                               CMTCS_E_INVALID otherwise); OP_DENSE: ignored               */
} cmtcs_problem_t;

/* Options of one call.  CG stopping (the paper runs CG "until convergence" in Alg. 1 and for
 * U steps in Sec. 3.1): with fixed_iters = U > 0 every right-hand side takes exactly U steps;
 * otherwise a right-hand side stops after the first step u with ||r_{u+1}|| <= tol ||b||
 * (recursive residual) or after max_iters steps.  Either mode stops a right-hand side before a
 * step whose d.Ad is not positive and finite, and after a step whose r.r is 0 or not finite. */
typedef struct {
  int32_t K;                /* probes per (task, cluster) for cmtcs_estep, >= 1             */
  int32_t max_iters;        /* tolerance mode step cap, 1..problem.max_iters                */
  int32_t fixed_iters;      /* > 0: fixed mode with this many steps (<= problem.max_iters)  */
  double tol;               /* tolerance mode threshold, >= 0                               */
  int32_t refine_every;     /* MATH_MIXED: true-residual replacement period m >= 1;
                               ignored in the other modes                                   */
  uint64_t seed;            /* probe generator key (see cmtcs_estep)                        */
  uint64_t em_iter;         /* EM iteration index mixed into the probe key                  */
  const int8_t* probes;     /* optional device [T][C][K][D] of +1/-1 replacing the
                               generated probes; NULL = generated                           */
  double alpha_max;         /* M-step cap on alpha, > 0 (see cmtcs_mstep)                   */
  int32_t graph;            /* cmtcs_estep / cmtcs_solve, MATH_F64 and MATH_F32: 1 = run the
                               CG steps as one HIP graph, recorded on the first call with a
                               given shape, alpha pointer and step policy and replayed after
                               that (all steps are launched; work for right-hand sides that
                               have stopped is skipped inside the kernels, and kernel timing by
                               cmtcs_profile is not available); 0 = launch step by step.
                               cmtcs_em_iter: 1 = record the whole EM iteration (see there) */
  int32_t common_probes;    /* generated probes only (0 or 1): 1 = every cluster c of task t
                               uses the probes of cluster 0, p(t,c,k) = p(t,0,k) (common random
                               numbers across clusters; not in the paper).  The estimators of
                               each (t, c) are unchanged in distribution, and the Monte Carlo
                               errors of ell_tc and ell_tc' become correlated, so that their
                               difference, which decides q_t, varies less.  0 = independent
                               probes per (t, c) as in Alg. 2 */
  int32_t precond;          /* 0: CG as in Alg. 1.  1: Jacobi-preconditioned CG (not in the
                               paper; dense problems, MATH_F64 / MATH_F32), M = diag(A_tc) =
                               beta diag(Phi_t^T Phi_t) + alpha_c: z = M^-1 r, gamma_u =
                               r.z / d.Ad, xi_u = r'.z' / r.z, d = z' + xi d, the stop rule on the
                               plain ||r||.  The iteration is CG on M^-1/2 A M^-1/2, so in
                               cmtcs_estep each probe's right-hand side is M^1/2 p (its Lanczos
                               run then starts at p and Eq. (hutch-trace) estimates
                               p^T log(M^-1/2 A M^-1/2) p), the log-determinant adds
                               -sum_d log M_dd, and s = M^-1/2 (.) (1/K) sum_k p_k (.) x_k, which
                               stays unbiased for diag Sigma.  Fewer steps where alpha spreads
                               over decades (pruned coordinates).  cmtcs_solve returns A^-1 B
                               and the preconditioned gamma_u, xi_u */
} cmtcs_opts_t;

/* Optional per-right-hand-side outputs, device pointers, each may be NULL.  For cmtcs_estep
 * the right-hand sides of task t are indexed j = c*(K+1) + k with k = 0 the mean system and
 * k = 1..K the probes; for cmtcs_solve j is the caller's column.  Arrays are [T][R]. */
typedef struct {
  int32_t* iters;           /* CG steps taken                                               */
  uint8_t* status;          /* CMTCS_CG_* code                                              */
  double* ritz_min;         /* cmtcs_estep only, [T][C][K]: smallest eigenvalue of the
                               probe's tridiagonal (Eq. (tridiag)); NaN if it took 0 steps  */
  double* ritz_max;         /* cmtcs_estep only, [T][C][K]: largest eigenvalue              */
  int32_t* k_eff;           /* cmtcs_estep only, [T][C]: probes that entered nu-bar (K unless
                               some were left out, see CMTCS_CG_NONPOS_RITZ); 0 makes nu-bar,
                               ell and the q of that task NaN                              */
} cmtcs_cg_stats_t;

/* Creates a handle for one problem on `stream` (a hipStream_t; NULL = the null stream) and
 * the current HIP device.  Allocates the whole workspace for the sizes in *prob and computes
 * b_t = beta Phi_t^T y_t once (Eq. (lin-sys)), since b does not depend on alpha.  For
 * OP_PARTIAL_FOURIER problems cmtcs_estep, cmtcs_em_iter (always step by step), cmtcs_solve,
 * cmtcs_apply, cmtcs_rhs and the M-steps are available; cmtcs_grad returns
 * CMTCS_E_UNSUPPORTED.
 * On success *out receives the handle; on failure *out is set to NULL. */
cmtcs_status_t cmtcs_create(cmtcs_handle_t* out, const cmtcs_problem_t* prob, void* stream);

/* Releases the workspace after the handle's stream has drained.  NULL is accepted. */
cmtcs_status_t cmtcs_destroy(cmtcs_handle_t h);

/* One CoFEM E-step (Alg. 2, inner loop over t and c), for all tasks and clusters.
 *   alpha   [C][D] float, > 0: current prior precisions
 *   log_pi  [C] double: log prior cluster probabilities
 *   mu      [T][C][D] float out: CG solution of the mean system of (t, c)
 *   s       [T][C][D] float out: (1/K) sum_k p_k (.) x_k (Eq. (diag-est))
 *   logdet  [T][C] double out: nu-bar, the estimate of log det Sigma_tc (Eq. (logdet-est))
 *   ell     [T][C] double out: nu-bar + sum_d log alpha_cd + b_t . mu_tc (Eq. (estep))
 *   q       [T][C] double out: softmax over c of ell_tc / 2 + log_pi_c (Eq. (estep))
 *   stats   optional outputs (may be NULL)
 * Probes: unless opts->probes is given, entry d of probe k (0-based) of pair (t, c) is
 * +1 or -1 from bit d mod 64 of word floor(d/64) (bit 0 -> +1, 1 -> -1), where word m is the
 * SplitMix64 output mix(key + (i+1) G), i = ((t C + c) K + k) ceil(D/64) + m, the key is
 * mix(seed + (em_iter+1) G), G = 0x9E3779B97F4A7C15, and mix is SplitMix64's finaliser
 * (Steele, Lea & Flood, OOPSLA 2014).  Probes are fresh per EM iteration, task and cluster
 * (Alg. 2); with opts->common_probes = 1, c is taken as 0 in i, so the clusters of a task
 * share their probes.  A probe whose tridiagonal has a non-positive eigenvalue is left out of the
 * average of Eq. (logdet-est).  The tridiagonals are held in LDS up to a budget of 64 KB per
 * block of four probes (runs of up to 4096 CG steps), otherwise in a workspace sized at create
 * from max_iters; the environment variable CMTCS_SLQ_LDS_BYTES at create lowers that budget
 * (0: always the workspace).  The results do not depend on it. */
cmtcs_status_t cmtcs_estep(cmtcs_handle_t h, const float* alpha, const double* log_pi,
                           const cmtcs_opts_t* opts, float* mu, float* s, double* logdet,
                           double* ell, double* q, cmtcs_cg_stats_t* stats);

/* The M-step of Eq. (mstep) with the diagonal of Sigma replaced by s:
 *   alpha_cd = Nq_c / den_cd,  Nq_c = sum_t q_tc,  den_cd = sum_t q_tc (mu_tcd^2 + s_tcd).
 * The paper states no guards; s is a Monte Carlo estimate, so den can be <= 0.  Applied here:
 * a cluster with Nq_c < 1e-300 keeps its alpha; otherwise alpha_cd = Nq_c / den_cd when
 * den_cd > Nq_c / alpha_max, else alpha_max.  Sums are FP64 in task order.  A task whose q_tc
 * is not finite (its E-step had K_eff = 0, see cmtcs_cg_stats_t) is left out of cluster c's
 * sums, and an entry whose den_cd is not finite (a non-finite mu or s) keeps its alpha_cd, so
 * that one failed task cannot overwrite the whole model.
 *   mu, s [T][C][D] float; q [T][C] double; alpha_inout [C][D] float, updated in place. */
cmtcs_status_t cmtcs_mstep(cmtcs_handle_t h, const float* mu, const float* s, const double* q,
                           const cmtcs_opts_t* opts, float* alpha_inout);

/* Learned cluster weights: the model of Eq. (cmtcs) takes pi as known, and Sec. 2 notes that it
 * can instead be learned as in finite-mixture EM.  That M-step is
 *   log_pi_c = log((1/T) sum_t q_tc),
 * the maximiser of sum_tc q_tc log pi_c over the simplex; a cluster whose responsibilities are all
 * zero gets -inf (its q stays 0 in later E-steps).  Sums are FP64 in task order.
 *   q [T][C] double (from cmtcs_estep); log_pi [C] double, written (it may be the log_pi array
 *   that cmtcs_estep and a recorded cmtcs_em_iter read: the next call sees the new weights).
 * Errors: CMTCS_E_INVALID for a NULL handle or array. */
cmtcs_status_t cmtcs_mstep_pi(cmtcs_handle_t h, const double* q, double* log_pi);

/* Estimate of the marginal log-likelihood of Sec. 2 from an E-step's ell (metrics, logging,
 * convergence checks): per task
 *   L_t = log sum_c pi_c N(y_t; 0, beta^-1 I + Phi_t diag(alpha_c)^-1 Phi_t^T)
 *       = log sum_c exp(ell_tc / 2 + log pi_c) + const_t,
 *   const_t = -(n_t / 2) log(2 pi) + (n_t / 2) log beta - (beta / 2) y_t . y_t,
 * over the task's n_t real measurements (N_t; 2 N_t for partial-Fourier problems, whose complex
 * measurements enter as [Re; Im]), computed at create; and Lhat = (1/T) sum_t L_t.  With CoFEM's
 * ell (the Monte Carlo log-determinant of Eq. (logdet-est)) it is an estimate, exact with
 * exact ell.  ell [T][C] and log_pi [C] double, device; L_task [T] and L_mean (one double)
 * device outputs, each may be NULL.  A task with a non-finite ell (K_eff = 0) gives a NaN L_t
 * and Lhat.  The mean is a fixed-order sum.  Asynchronous on the handle's stream. */
cmtcs_status_t cmtcs_log_likelihood(cmtcs_handle_t h, const double* ell, const double* log_pi,
                                    double* L_task, double* L_mean);

/* One EM iteration of Alg. 2: cmtcs_estep from alpha_inout (no stats) followed by cmtcs_mstep
 * into alpha_inout, with the same arguments, outputs and results as those two calls.  With
 * opts->graph = 1 (MATH_F64 and MATH_F32) the device work of the whole iteration -- CG start,
 * all CG steps (as in the graph mode of cmtcs_estep), diagonal estimate, log-determinant,
 * responsibilities and M-step -- is recorded once as a HIP graph and replayed by later calls
 * with the same shape (K), step policy, tol, alpha_max, common_probes and the same eight
 * array pointers (alpha_inout, log_pi, mu, s, logdet, ell, q, opts->probes); opts->seed and
 * opts->em_iter may change between calls (the probe key is a device word set before each replay).  Other calls
 * on the handle between iterations are allowed.  MATH_MIXED, or graph = 0, launches step by
 * step.  Errors as cmtcs_estep and cmtcs_mstep. */
cmtcs_status_t cmtcs_em_iter(cmtcs_handle_t h, float* alpha_inout, const double* log_pi,
                             const cmtcs_opts_t* opts, float* mu, float* s, double* logdet,
                             double* ell, double* q);

/* Batched CG (Alg. 1) on caller-supplied right-hand sides: for task t and column j solves
 * (beta Phi_t^T Phi_t + diag(alpha_{col_cluster[t][j]})) X[t][j] = B[t][j] from x = 0.
 *   alpha        [C][D] float
 *   R_per_task   columns per task, 1..problem.max_rhs
 *   col_cluster  HOST [T][R_per_task] int32, each in 0..C-1
 *   B, X         [T][R_per_task][D], double for MATH_F64, float otherwise
 *   gamma, xi    optional [T][R_per_task][opts->max_iters or fixed_iters] double outputs: the
 *                step sizes gamma_u and xi_u of Alg. 1, zero past the steps taken
 *   stats        optional (iters, status used)
 * opts->K, seed, em_iter, probes and alpha_max are ignored. */
cmtcs_status_t cmtcs_solve(cmtcs_handle_t h, const float* alpha, int32_t R_per_task,
                           const int32_t* col_cluster, const void* B, void* X, double* gamma,
                           double* xi, const cmtcs_opts_t* opts, cmtcs_cg_stats_t* stats);

/* The right-hand side of the posterior-mean system, b_t = beta Phi_t^T y_t (Eq. (lin-sys)),
 * as computed at create.  b: [T][D], double for MATH_F64, float otherwise. */
cmtcs_status_t cmtcs_rhs(cmtcs_handle_t h, void* b);

/* Gradients of a scalar loss through X = A^-1 B (the differentiation form; derived from the
 * operator A of Eq. (lin-sys)).  Given the solutions X and the adjoint solutions
 * Lam = A^-1 (dLoss/dX) -- A is symmetric, so cmtcs_solve computes both -- of the same
 * columns (same col_cluster):
 *   dalpha[c][d] = - sum over (t, j) with col_cluster[t][j] = c of Lam[t][j][d] X[t][j][d]
 *   dphi rows of task t = - beta sum_j [ (Phi_t Lam_tj) X_tj^T + (Phi_t X_tj) Lam_tj^T ]
 *                         + y_coef * beta * y_t (sum_j Lam_tj)^T
 * y_coef = 1 when B = beta Phi^T y (so B itself depends on Phi), 0 for a fixed B (whose own
 * gradient is Lam).  Products with Phi run on the matrix cores; sums are FP64.
 *   R_per_task   1..problem.max_rhs/2 (the 2R columns X, Lam share the workspace slots)
 *   col_cluster  HOST [T][R_per_task] int32 in 0..C-1
 *   X, Lam       [T][R_per_task][D], double for MATH_F64, float otherwise
 *   dalpha       [C][D] float out (may be NULL);  dphi [row_off[T]][D] float out (may be NULL) */
cmtcs_status_t cmtcs_grad(cmtcs_handle_t h, int32_t R_per_task, const int32_t* col_cluster,
                          const void* X, const void* Lam, double y_coef, float* dalpha,
                          float* dphi);

/* The operator alone (Eq. (lin-sys), applied matrix-free as in Sec. 3.3):
 *   AV[t][j] = beta Phi_t^T (Phi_t V[t][j]) + alpha_{col_cluster[j]} (.) V[t][j]
 * with the same matrix-core products a CG step uses.
 *   alpha        [C][D] float
 *   R_per_task   1..problem.max_rhs;  col_cluster HOST [T][R_per_task] int32 in 0..C-1
 *   V, AV        [T][R_per_task][D], double for MATH_F64, float otherwise */
cmtcs_status_t cmtcs_apply(cmtcs_handle_t h, const float* alpha, int32_t R_per_task,
                           const int32_t* col_cluster, const void* V, void* AV);

/* The operator of cmtcs_apply without a handle, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 *   AV[t][j] = beta Phi_t^T (Phi_t V[t][j]) + alpha_{col_cluster[t][j]} (.) V[t][j],
 * the same matrix-core products, with the default tile shapes (no autotuning).  It allocates
 * nothing: its tile tables, padded copies of V and A V and the intermediate Phi V live in one
 * statically sized device array of 64 MiB per GPU (held by each GPU the library runs on until
 * the process ends), and a problem needing more returns CMTCS_E_INVALID (the message gives the
 * bytes needed).  Every call on a GPU uses that GPU's one array: calls that overlap on one GPU
 * (from several threads or streams) race and must be serialised by the caller.  The call copies
 * its small tables to the device and waits for the stream before launching the products, which
 * then run asynchronously on `stream`.
 *   prob        a dense problem (op OP_DENSE, math MATH_F64 or MATH_F32, phi_dtype F32); its
 *               phi, row_off, beta, T, C and D are used, nothing else
 *   alpha       [C][D] float;  R_per_task >= 1;  col_cluster HOST [T][R_per_task] in 0..C-1
 *   V, AV       [T][R_per_task][D], double for MATH_F64, float for MATH_F32
 *   stream      a hipStream_t (NULL = the null stream) */
cmtcs_status_t cmtcs_apply_noalloc(const cmtcs_problem_t* prob, const float* alpha,
                                   int32_t R_per_task, const int32_t* col_cluster, const void* V,
                                   void* AV, void* stream);

/* Kernel timing for measurement: while enabled, each CG step's two operator products and its
 * vector update are bracketed by HIP events on the handle's stream and their durations are
 * summed.  While enabled, the step-by-step CG loop waits for the events every 8 steps and then
 * also stops enqueueing steps once every right-hand side has stopped (the timings then cover
 * the steps that did work).  For OP_PARTIAL_FOURIER problems, whose CG solves are one
 * kernel each, that kernel's duration is summed in the third slot and the first two stay 0.
 * enable = 1 clears the sums and turns timing on; enable = 0 turns it off; any other value
 * leaves the state unchanged.  When non-NULL, the HOST arrays receive the sums so far
 * (after the stream has drained): totals_ms[3] in milliseconds and counts[3] in launches, in
 * the order {Phi V product, Phi^T W product, CG update}. */
cmtcs_status_t cmtcs_profile(cmtcs_handle_t h, int32_t enable, double* totals_ms,
                             int64_t* counts);

/* Tile shapes in use: rows[0] and rows[1] (HOST) receive the output rows per wave tile of the
 * Phi V and the Phi^T W products; a negative value -r means the LDS-staged kernel, whose tile is
 * four waves of r rows sharing one right-hand-side chunk in LDS.  Unless the environment
 * variable CMTCS_AUTOTUNE is "0" when the handle is created, the first call with a new number of
 * column slots per task times every supported shape of each product on the handle's own buffers
 * and keeps the fastest.  CMTCS_TILES="f,a" at create pins the two shapes (each must be one the
 * library supports; otherwise the defaults stay) and turns the autotuner off. */
cmtcs_status_t cmtcs_tiles(cmtcs_handle_t h, int32_t* rows);

/* Message of the last failed call on this thread ("" if none). */
const char* cmtcs_last_error(void);

/* Library version string. */
const char* cmtcs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CMTCS_H */
