/*
 * gmrf.h -- C ABI of the MI355X GMRF posterior library (libgmrf.so).
 *
 * Computes, for a Gaussian Markov random field prior u ~ N(mu, Q^-1) and a linear
 * Gaussian likelihood y | u ~ N(A u + b, Q_eps^-1) with diagonal Q_eps:
 *   posterior precision  Q_post = Q + A^T Q_eps A                 (Sec. 3.1, conditioning)
 *   posterior mean       mu_post = mu + Q_post^-1 A^T Q_eps (y - A mu - b)
 *                                                                   (Sec. 3.1, eq. posterior-mean)
 *   sparse Cholesky      P Q_post P^T = L L^T with a fill-reducing nested-dissection
 *                        order P computed once per pattern          (Sec. 3.2 and 3.3)
 *   mean                 one forward and one backward triangular solve (Sec. 3.2)
 *   samples              x = mu_post + P^T L^-T z, z ~ N(0, I)        (Sec. 3.2, sampling)
 *   marginal variances   diag(Q_post^-1) by the Takahashi recursion   (Sec. 3.2)
 *   log-determinant      log det Q_post = 2 sum_j log L_jj (follows from the factorisation)
 * plus refactorisation with an unchanged pattern for Gauss-Newton (Sec. 3.3).
 *
 * Conventions shared by every call
 *   - Matrices are CSR, 0-based: int64 row pointers, int32 column indices sorted
 *     ascending within each row, float64 values.  Q stores both triangles; its pattern
 *     must be symmetric and contain the diagonal, and A^T Q_eps A must fall inside it
 *     (data rows touching one element; Galerkin PDE rows of the same FEM stencil).
 *   - Array arguments are DEVICE pointers on the context's device unless marked "host".
 *     The caller owns every buffer; the library never keeps a caller pointer past the
 *     call.  The library copies the patterns (to the host, at the first gmrf_assemble)
 *     and the values it needs.  It owns the factor, the selected inverse and all
 *     workspaces until gmrf_destroy.
 *   - Vectors indexed by unknowns are in the caller's (original) numbering, except the
 *     standard-normal input of gmrf_sample, which is consumed in pivot order (z[k]
 *     drives pivot k); gmrf_stats exposes the pivot order.
 *   - Work is enqueued on the stream given to gmrf_create.  Calls that return host
 *     results (gmrf_analyze, gmrf_logdet, gmrf_solve, gmrf_sample, gmrf_selinv,
 *     gmrf_stats) synchronise that stream before returning.
 *   - Call order: assemble -> analyze -> factor -> {logdet, solve, sample, selinv}.
 *     update_values may follow any call after analyze and must be followed by factor.
 *     A violation returns GMRF_ERR_STATE.
 *   - Errors: every call returns a gmrf_status; on failure gmrf_last_error gives a
 *     message.  A non-positive or NaN pivot is detected on the device during
 *     gmrf_factor and reported by the next synchronising call as GMRF_ERR_NOT_SPD, with
 *     the failing unknown (original numbering) in gmrf_stats_t.failed_index.
 */
#ifndef GMRF_H
#define GMRF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gmrf_ctx* gmrf_t;
typedef int32_t gmrf_status;

enum {
  GMRF_OK = 0,
  GMRF_ERR_ARG = -1,           /* invalid argument, size or pattern */
  GMRF_ERR_STATE = -2,         /* call out of order */
  GMRF_ERR_NOT_SPD = -3,       /* factorisation met a non-positive or NaN pivot */
  GMRF_ERR_PATTERN = -4,       /* values given for a pattern other than the analysed one */
  GMRF_ERR_HIP = -5,           /* HIP runtime error */
  GMRF_ERR_OOM = -6,           /* device allocation failed */
  GMRF_ERR_NOT_CONVERGED = -7  /* refinement stopped above tolerance (result still written) */
};

typedef enum {
  GMRF_FP64 = 0,          /* every factor, solve and selected-inverse operation in FP64 */
  GMRF_FP32_REFINE = 1    /* FP32 fronts and updates on MFMA with FP32 accumulation (the
                             long-K products -- outer panel update, trailing SYRK,
                             Sigma[R', K] -- as six bf16 term products of a three-way bf16
                             split of each FP32 operand, with FP32-level error); FP64
                             diagonal-block pivots, log-det sum, residuals and iterative
                             refinement of the mean */
} gmrf_precision;

/* Options of gmrf_analyze (NULL = defaults). */
typedef struct {
  int32_t leaf_size;   /* nested-dissection leaf size (default 64) */
  int32_t relax_small; /* relaxed supernodes: always merge up to this many columns (8) */
  int32_t relax_mid;   /* ... up to this many columns with <= 50% explicit zeros (32) */
  int32_t relax_big;   /* ... up to this many columns with <= 15% explicit zeros (128) */
} gmrf_options;

typedef struct {
  int64_t n;              /* unknowns */
  int64_t nnz_q;          /* stored entries of Q (both triangles) */
  int64_t m;              /* observations */
  int64_t nnz_a;
  int64_t nnz_l;          /* exact nonzeros of L (diagonal included) */
  int64_t stored_l;       /* supernodal storage of L (relaxation zeros included) */
  int64_t n_super;        /* supernodes */
  int64_t tree_depth;     /* depth of the supernodal elimination tree */
  int64_t max_front;      /* largest front size */
  double flops_factor;    /* sum_j c_j^2 over exact column counts c_j */
  double flops_selinv;    /* 2 sum_j c_j^2 */
  double flops_solve;     /* 4 nnz(L) - 2n, per right-hand side */
  double bytes_front_ws;  /* device bytes of the two front workspaces */
  double bytes_factor;    /* device bytes of L */
  int64_t failed_index;   /* original index of the first failing pivot, -1 if none */
  int32_t precision;      /* precision of the last factorisation */
  int32_t refine_iters;   /* refinement iterations of the last gmrf_solve */
  double refine_resid;    /* ||h - Q_post mu|| / ||h|| after the last gmrf_solve */
} gmrf_stats_t;

/* Create a context on HIP device `device`, enqueuing on `hip_stream` (a hipStream_t;
   NULL = the device's null stream).  *h receives the handle. */
gmrf_status gmrf_create(gmrf_t* h, int device, void* hip_stream);

/* Release every device and host resource of the context.  NULL is accepted. */
gmrf_status gmrf_destroy(gmrf_t h);

/* Conditioning, Sec. 3.1: Q_post = Q + A^T diag(q_eps) A on Q's pattern and
   h = A^T diag(q_eps) (y - A mu_prior - b).
   n, m        unknowns, observations (m may be 0; then A arrays may be NULL).
   q_*         CSR of Q (device).   a_*   CSR of A, m x n (device).
   q_eps, y    m entries (device).  b, mu_prior  m / n entries or NULL (= 0).
   n_blocks, block_ptr  optional block-diagonal structure (host, n_blocks+1 entries,
               block_ptr[0] = 0, block_ptr[n_blocks] = n); gmrf_logdet then returns one
               value per block.  n_blocks = 0 or block_ptr = NULL means one block.
   The first call copies and validates both patterns (sorted, in range, symmetric Q
   with diagonal, A^T A inside Q's pattern) and builds the assembly maps; later calls
   must pass the same pattern (same n, m, nnz; else GMRF_ERR_PATTERN). */
gmrf_status gmrf_assemble(gmrf_t h, int64_t n, const int64_t* q_rowptr, const int32_t* q_col,
                          const double* q_val, int64_t m, const int64_t* a_rowptr,
                          const int32_t* a_col, const double* a_val, const double* q_eps,
                          const double* y, const double* b, const double* mu_prior,
                          int64_t n_blocks, const int64_t* block_ptr);

/* New values on the already assembled patterns (Gauss-Newton, Sec. 3.3): any of the
   pointers may be NULL to keep the previous values.  Re-runs the assembly on device
   without host synchronisation.  Must be followed by gmrf_factor. */
gmrf_status gmrf_update_values(gmrf_t h, const double* q_val, const double* a_val,
                               const double* q_eps, const double* y, const double* b);

/* Symbolic analysis on the host (Sec. 3.2: fill-reducing reordering, once per pattern,
   Sec. 3.3): nested dissection (steered by coords when given: host, n x dim row-major,
   dim 1..3; NULL = purely graph-based), elimination tree, exact column counts, relaxed
   supernodes and the device execution plan. */
gmrf_status gmrf_analyze(gmrf_t h, const double* coords, int dim, const gmrf_options* opts);

/* Numeric factorisation P Q_post P^T = L L^T (Sec. 3.2) in the given precision,
   asynchronous.  Repeatable after gmrf_update_values. */
gmrf_status gmrf_factor(gmrf_t h, gmrf_precision p);

/* log det Q_post (host output, one value per block of gmrf_assemble). */
gmrf_status gmrf_logdet(gmrf_t h, double* out);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving
   loops, harnesses that forbid hipMalloc): the log-determinant of gmrf_logdet written to
   DEVICE memory, with no allocation, no host synchronisation and no status check.
   out_dev: n_blocks doubles (device), one per block of gmrf_assemble, bitwise equal to
   gmrf_logdet's values.  The per-block partial sums live in a fixed 4 MiB workspace of
   the library on each device (at most 8192 blocks; more returns GMRF_ERR_ARG before
   anything is enqueued).  Every partial is written before it is read, so nothing needs
   clearing; calls that overlap on one device (several contexts or streams) share that
   workspace and race.  A failed factorisation is reported by the next synchronising call
   (the value is then meaningless).  Asynchronous on the context's stream. */
gmrf_status gmrf_logdet_noalloc(gmrf_t h, double* out_dev);

/* Posterior mean (Sec. 3.1 eq. posterior-mean; Sec. 3.2: one forward and one backward
   solve).  mu_out: n entries (device).  In GMRF_FP32_REFINE (and in GMRF_FP64 when
   max_refine > 0) iterative refinement with FP64 residuals r = h - Q_post x runs until
   ||r||/||h|| <= tol or max_refine corrections; iters_out and resid_out (host, nullable)
   receive the count and the final relative residual.  Returns GMRF_ERR_NOT_CONVERGED if
   the tolerance was not met (mu_out is still written). */
gmrf_status gmrf_solve(gmrf_t h, double* mu_out, int max_refine, double tol, int* iters_out,
                       double* resid_out);

/* Log marginal likelihood of the data and its gradient with respect to k parameters of
   the prior and of the observation model.  With mu_post the posterior mean, mu = 0 the
   prior mean and r = y - b - A mu_post, the Gaussian identity
   log p(y) = log p(y|u) + log p(u) - log p(u|y) at u = mu_post (conditioning, Sec. 3.1)
   gives
     LML = -M/2 log 2 pi + 1/2 log|Q| + 1/2 log|Q_eps| - 1/2 log|Q_post| - 1/2 mu_post^T Q mu_post
           - 1/2 r^T Q_eps r,
   and, the identity holding for every u, its derivative at u = mu_post needs only the
   explicit dependence:
     dLML = 1/2 tr(Q^-1 dQ) + 1/2 sum(dq_eps / q_eps) - 1/2 tr(Q_post^-1 dQ_post)
            - 1/2 mu_post^T dQ mu_post - 1/2 sum(dq_eps r^2) + (Q_eps r)^T dA mu_post,
     dQ_post = dQ + dA^T Q_eps A + A^T Q_eps dA + A^T diag(dq_eps) A,
   where the traces read the selected inverses (Takahashi, Sec. 3.2) on Q's pattern.
   post:  context with the posterior (assemble with A, q_eps, y, b; analyze; factor).
   prior: a second context with the same Q (values and pattern) and no observations,
          factored.  Both single-block.
   k:     number of parameters; dq: k x nnz_q (device, parameter-major, dq + i*nnz_q is
          dQ/dtheta_i in Q's CSR order); da: k x nnz_a (device, nullable = A constant);
          dqeps: k x m (device, nullable = Q_eps constant).
   max_refine, tol: refinement of the posterior mean as in gmrf_solve.
   out:   host, 1 + k doubles: LML, then dLML/dtheta_i.
   mu_out: device, n doubles, nullable: the refined posterior mean used.
   Runs the log-dets, the refined mean, both selected inversions (overwriting what
   gmrf_selinv returned before) and every reduction on the device with fixed orders;
   synchronises both streams.  Returns GMRF_ERR_NOT_CONVERGED (out still written) if the
   mean's refinement stopped above tol. */
gmrf_status gmrf_lml_gradient(gmrf_t post, gmrf_t prior, int k, const double* dq, const double* da,
                              const double* dqeps, int max_refine, double tol, double* out,
                              double* mu_out);

/* x = Q_post^-1 rhs (one forward and one backward solve with the current factor; no
   refinement; rhs and x_out device, n entries, original order).  Used for adjoints. */
gmrf_status gmrf_solve_rhs(gmrf_t h, const double* rhs, double* x_out);

/* Gauss-Newton for the nonlinear Burgers space-time problem (Sec. 3.3).  Unknowns
   u^k_i, slice k = 0..nt-1, interior node i = 0..nx-1 (homogeneous Dirichlet outside),
   index k*nx + i.  The context must hold Q (prior, analysed) and A with m = nx*nt rows in
   this layout: row i (< nx) observes u^0_i (one entry); row nx + (k-1)*nx + i holds the
   Galerkin implicit-Euler residual
     f = mass_i (u^k_i - u^(k-1)_i)/dt + nu (S u^k)_i + (u_{i+1}^2 + u_i u_{i+1} - u_{i-1} u_i
         - u_{i-1}^2)/6
   with entries at columns (k-1)*nx+i, k*nx+i-1, k*nx+i, k*nx+i+1 (those in range); y and
   q_eps as assembled.  mass (nx) and stiff3 (3*nx: S_{i,i-1}, S_{i,i}, S_{i,i+1}) are
   device arrays.  Each iteration linearises f at u (J values and offset b written into the
   assembled A and b), assembles H = Q + J^T Q_eps J on the analysed pattern (the ordering
   is reused), factors in `precision`, solves for the linearised posterior mean with at
   most `refine` FP64 residual corrections, stopped on the device once
   ||h - H x|| <= refine_tol ||h|| (later corrections add nothing), and takes a
   backtracking Armijo step (c = 1e-4, alpha = 1, 1/2, ..., 1/128, the first that passes;
   none: alpha = 0, the iterate is kept, so the objective never increases) chosen on the
   device.  With use_graph != 0 the iterations after the first
   replay one hipGraph captured by this call (and destroyed before it returns).
   decrement_tol > 0: stop after the first iteration whose Newton decrement lambda^2 / 2
   is below decrement_tol or whose line search takes no step (Sec. 5.3: Gauss-Newton until
   the Newton decrement subceeds a tolerance or a maximum number of steps is reached; the
   host reads each iteration's record); 0: run all `iters` iterations.
   u (device, n): start on entry, final iterate on exit.  rec_out (host, 6*iters,
   nullable): per iteration objective at the start, step length, Newton decrement
   lambda^2 = -grad^T d, grad^T d, the final relative residual of the linearised solve
   and the number of corrections applied; NaN for the iterations the stopping rule
   skipped.  On return the context holds the factor of the
   Gauss-Newton Laplace approximation at the final iterate and mu_post = u, so
   gmrf_logdet, gmrf_sample and gmrf_selinv describe N(u*, (Q + J*^T Q_eps J*)^-1). */
gmrf_status gmrf_gn_burgers(gmrf_t h, int64_t nx, int64_t nt, double dt, double nu,
                            const double* mass, const double* stiff3, int iters, int precision,
                            int refine, double refine_tol, double decrement_tol, int use_graph, double* u,
                            double* rec_out);

/* Gauss-Newton (Sec. 3.3) for observation residuals with a pointwise power nonlinearity,
   e.g. the lumped Galerkin rows of -Laplace u + u^3 = f:
     f_r(u) = sum_e lin_val[e] u[col e] + nl_coef[r] * u[nl_col[r]]^power      (row r of A),
   with data y and noise q_eps as assembled (A's pattern must hold each row's nonlinear
   unknown; nl_col[r] = -1 marks a linear row).  lin_val: nnz_a (device, A's CSR order);
   nl_col: m int32 (device); nl_coef: m (device); power: 2..8.  Each iteration writes the
   linearisation J = lin + power * c * u^(power-1) (at the nonlinear unknown) and
   b = (1 - power) c u^power into the assembled A and b, then proceeds exactly as
   gmrf_gn_burgers (H = Q + J^T Q_eps J on the analysed pattern, refined solve, device
   Armijo line search, hipGraph replay after the first iteration, the same stopping rule,
   Laplace approximation at the final iterate); rec_out receives the same 6 values per
   iteration.  Returns
   GMRF_ERR_PATTERN if a nonlinear unknown is not a stored column of its row. */
gmrf_status gmrf_gn_pointwise(gmrf_t h, const double* lin_val, const int32_t* nl_col, const double* nl_coef,
                              int power, int iters, int precision, int refine, double refine_tol,
                              double decrement_tol, int use_graph, double* u, double* rec_out);

/* Conjugate gradients (Sec. 3.2, the alternative to the factorisation when fill is too
   large): preconditioned CG for Q_post x = rhs on the device, FP64 vectors and fixed-order
   reductions; preconditioner precond = 0: the diagonal of Q_post (needs only
   gmrf_assemble and gmrf_analyze), 1: the context's factor (one forward and one backward
   solve per iteration; after gmrf_factor, FP32 or FP64).  k right-hand sides (n x k,
   column-major, device) solved one after the other; rhs = NULL (k = 1) solves for the
   posterior mean (Sec. 3.1: x = mu + Q_post^-1 h).  x0 (device, nullable): starting
   iterate, e.g. the previous Gauss-Newton direction (Sec. 3.3).  Stops when
   ||rhs - Q_post x|| <= tol ||rhs|| or after maxit iterations (with the diagonal
   preconditioner the residual is checked every 8 iterations, so up to 7 iterations may
   follow the one that met the tolerance); iters_out / resid_out
   (host, k, nullable) receive the counts and final relative residuals.  Returns
   GMRF_ERR_NOT_CONVERGED if a column stopped above tol (x_out still written). */
gmrf_status gmrf_pcg(gmrf_t h, int64_t k, const double* rhs, const double* x0, double* x_out, int precond,
                     int maxit, double tol, int* iters_out, double* resid_out);

/* CG sampling (Sec. 3.2): with a left square root R of the prior precision (Q = R R^T;
   n x r CSR, device: int64 row pointers, int32 columns, values) the vector
   b = R w1 + A^T Q_eps^1/2 w2 has covariance Q_post, so x = mu_post + Q_post^-1 b is a
   posterior draw; Q_post^-1 b by gmrf_pcg's iteration.  w1: r x k, w2: m x k (device,
   column-major, standard normal; w2 unused when m = 0); x_out: n x k.  Needs the
   posterior mean of a previous gmrf_solve. */
gmrf_status gmrf_sample_cg(gmrf_t h, int64_t k, int64_t r, const int64_t* r_rowptr, const int32_t* r_col,
                           const double* r_val, const double* w1, const double* w2, double* x_out,
                           int precond, int maxit, double tol, int* iters_out);

/* Rao-Blackwellised Monte Carlo marginal variances (Sec. 3.2, the estimator of Siden et al.
   the paper cites): from k draws x_s of N(0, Q_post^-1) (n x k, device, column-major,
   centred), var_i = 1/Q_ii + (1/k) sum_s ((1/Q_ii) sum_{j != i} (Q_post)_ij x_sj)^2.
   var_out: n (device). */
gmrf_status gmrf_rbmc_variances(gmrf_t h, int64_t k, const double* xs, double* var_out);

/* k posterior samples x = mu_post + P^T L^-T z (Sec. 3.2, sampling) from the mean of the
   last gmrf_solve.  z: n x k float32, column-major, pivot order (device).
   x_out: n x k float64, column-major, original order (device).  1 <= k <= 16. */
gmrf_status gmrf_sample(gmrf_t h, int64_t k, const float* z, double* x_out);

/* Selected inverse by the Takahashi recursion (Sec. 3.2, marginal variances).
   var_out: diag(Q_post^-1), n entries (device).  sigma_q_out (nullable, device): the
   entries of Q_post^-1 at every stored entry of Q, in Q's CSR order.  The factor is kept. */
gmrf_status gmrf_selinv(gmrf_t h, double* var_out, double* sigma_q_out);

/* The same selected inversion started asynchronously: it is queued after the work
   already on the context's stream, runs on a second stream owned by the context, and
   the call returns at once, so that gmrf_solve, gmrf_sample and gmrf_logdet of the same
   factor overlap with it.  var_out and sigma_q_out must stay allocated and unread until
   gmrf_selinv_wait returns.  Every call that writes or reallocates what the inversion
   reads (gmrf_assemble, gmrf_update_values, gmrf_analyze, gmrf_factor, gmrf_gn_burgers,
   another gmrf_selinv*) and gmrf_destroy first wait for it. */
gmrf_status gmrf_selinv_submit(gmrf_t h, double* var_out, double* sigma_q_out);

/* Host wait for the inversion started by gmrf_selinv_submit (no-op if none). */
gmrf_status gmrf_selinv_wait(gmrf_t h);

/* Deterministic sum_e a[e] * b[e] over len entries (device inputs, host output); used
   for traces tr(Q_post^-1 dQ) = sum over Q's pattern of Sigma_e dQ_e. */
gmrf_status gmrf_dot(gmrf_t h, int64_t len, const double* a, const double* b, double* out);

/* Whittle-Matern precision values (Sec. 2.2, eq. sparse-prec-matrix, alpha = 2) on the
   stored pattern of Q: given the lumped mass M~, the stiffness S and S M~^-1 S placed on
   that pattern (device, nnz entries each, zeros where absent), writes
     q_out  = tau^-2 (kappa^4 M~ + 2 kappa^2 S + S M~^-1 S)   (= tau^-2 K M~^-1 K,
                                                                K = kappa^2 M~ + S)
     dq_out = dQ/dlog(kappa) = 4 kappa^2 tau^-2 K             (nullable)
   Enqueued on the context's stream; needs no prior call. */
gmrf_status gmrf_matern_values(gmrf_t h, int64_t nnz, const double* m_on_q, const double* s_on_q,
                               const double* sms_on_q, double kappa, double tau, double* q_out,
                               double* dq_out);

/* y = V x for V given by its values on the stored pattern of Q (device, nnz_q values; x,
   y device, n entries).  After gmrf_assemble.  Asynchronous. */
gmrf_status gmrf_spmv(gmrf_t h, const double* v_val, const double* x, double* y);

/* Data misfit sum_r q_eps[r] (y - b - A x)_r^2 for x (device, n entries); host output. */
gmrf_status gmrf_misfit(gmrf_t h, const double* x, double* out);

/* Counters of the analysed pattern and of the last calls (host output); also reports a
   pending device status (GMRF_ERR_NOT_SPD). */
gmrf_status gmrf_stats(gmrf_t h, gmrf_stats_t* out);

/* Pivot order (host output, n entries): perm[k] = original index of pivot k. */
gmrf_status gmrf_pivot_order(gmrf_t h, int32_t* perm_out);

/* Elapsed device milliseconds of the phases of the last gmrf_factor, gmrf_solve and
   gmrf_selinv calls, measured with events on the context's stream (host output, 3
   entries: factor, solve, selinv). */
gmrf_status gmrf_phase_ms(gmrf_t h, double* out3);

/* Per-kernel-class profile: device time between events recorded around every launch
   of the class while profiling is on, with the algorithmic flops and bytes of those
   launches as counted from the supernodal structure (lower triangles only). */
typedef struct {
  char name[32];
  int64_t launches;
  double ms;
  double flops;
  double bytes;
} gmrf_kernel_stat_t;

/* Reset the per-class counters and switch per-launch events off (enable == 0), on for
   every class (enable == 1), or on for the classes whose bits are set in any other
   value of enable (bit i = i-th record of gmrf_kernel_stats), so that a timed run can
   carry events around one kernel class only. */
gmrf_status gmrf_profile(gmrf_t h, int enable);

/* Copy up to `capacity` class records (host) and the number of classes to *count;
   synchronises the stream. */
gmrf_status gmrf_kernel_stats(gmrf_t h, gmrf_kernel_stat_t* out, int capacity, int* count);

/* One profiled launch: its class (index of the gmrf_kernel_stats record), the
   algorithmic flops and bytes it was charged, and its duration between the events
   recorded around it (ms). */
typedef struct {
  int32_t cls;
  int32_t reserved;
  double flops;
  double bytes;
  double ms;
} gmrf_launch_rec_t;

/* Copy up to `capacity` records (host) of the launches profiled since the last
   gmrf_profile call, in launch order, and their total number to *count (out may be NULL
   to query the count); synchronises the streams. */
gmrf_status gmrf_launch_records(gmrf_t h, gmrf_launch_rec_t* out, int64_t capacity, int64_t* count);

/* Message of the last failing call on this context (never NULL). */
const char* gmrf_last_error(gmrf_t h);

/* Host-only symbolic analysis with no device (for tests and planning): pattern of Q
   (host CSR as in gmrf_assemble), optional coords.  perm_in (host, n entries, nullable):
   a fill-reducing order to analyse instead of the library's nested dissection (perm_in[k]
   = original index of pivot k; it is postordered, which leaves the fill unchanged), e.g.
   to compare the fill of two orderings (Sec. 3.2: the cost depends on the fill).
   perm_out (n entries) and colcount_out (n entries, exact column counts of L in pivot
   order) may be NULL; stats_out receives the pattern counters (device fields zero). */
gmrf_status gmrf_symbolic_host(int64_t n, const int64_t* rowptr, const int32_t* col,
                               const double* coords, int dim, const gmrf_options* opts,
                               const int32_t* perm_in, int32_t* perm_out, int64_t* colcount_out,
                               gmrf_stats_t* stats_out);

#ifdef __cplusplus
}
#endif

#endif /* GMRF_H */
