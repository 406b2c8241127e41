/*
 * rbmc.h -- C ABI of the MI355X (gfx950) overlapping Rao-Blackwellized Monte
 * Carlo (RBMC) library: marginal variances diag(Q^-1) and log-determinant
 * gradients tr(Q^-1 dQ/dtheta_j) of a space-time Gaussian Markov random field
 *
 *     Q(theta) = Q_t (x) Q_s + A^T Q_y A
 *
 * following Zhumekenov, Krainski & Rue, "Parallel Selected Inversion for
 * Space-Time Gaussian Markov Random Fields" (arXiv 2309.05435):
 *   - posterior precision Q = Q_x + A^T Q_y A and marginals diag(Q^-1):
 *     Sec. 2.3, eq:lgm:2 and eq:lgm:3;
 *   - gradients d log|Q| / dtheta_j = tr(Q^-1 dQ_j) = sum_ik (Q^-1)_ik (dQ_j)_ik:
 *     eq:lgm:4, eq:hyperpar:3 and eq:hyperpar:4;
 *   - the estimator: overlapping RBMC, Alg. 3 (blocks) and Alg. 4 (diagonal);
 *   - samples x ~ N(0, Q^-1) by a Krylov solver, Sec. 3.3 (here conjugate
 *     gradients on the perturbed system Q x = F z, Sec. 2.4);
 *   - the posterior mean with fixed effects by the Schur complement, Sec. 3.1
 *     (eq:mean:3-5, eq:var:1), and the gradient of log pi(theta | y), Sec. 3.4
 *     (eq:hyperpar:1-4).
 *
 * Model (the separable case of Sec. 2.2): an mx x my grid on the unit square,
 * h = 1/(max(mx,my)-1), lumped mass C = h^2 I, G = 5-point Neumann graph
 * Laplacian (stiffness), Q_s = tau (kappa^4 C + 2 kappa^2 G + G C^-1 G)
 * (eq:spde:4 with alpha = 2, read linear in tau); Q_t = the precision of a
 * stationary unit-variance AR(1) with correlation rho over T steps; Q_y =
 * sigma^-2 I on the observed space-time nodes.  theta = (log kappa, log tau,
 * rho, log sigma).  Node index i = t*mx*my + iy*mx + ix (space fastest).
 *
 * Conventions for every call:
 *   - return value: rbmc_status; 0 = ok, > 0 = warning (outputs valid),
 *     < 0 = error (outputs undefined); rbmc_last_error() gives a message;
 *   - pointers documented "device" are hipMalloc'd (or torch CUDA/HIP tensor)
 *     memory on the context's device; "host" pointers are ordinary memory;
 *     the caller owns every buffer it passes; the library never frees them
 *     and keeps no pointer to them after the call returns;
 *   - multi-vectors are column-major n x n_rhs: vector k occupies
 *     [k*n, (k+1)*n) (a torch tensor of shape (n_rhs, n));
 *   - work is ordered on the context's HIP stream; calls that produce
 *     outputs synchronize that stream before returning;
 *   - a context and its models are not thread-safe.
 */
#ifndef RBMC_H
#define RBMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RBMC_OK = 0,
  RBMC_W_NOT_CONVERGED = 1, /* PCG hit pcg_maxit for some sample; outputs computed */
  RBMC_E_ARG = -1,          /* invalid argument (message says which) */
  RBMC_E_NOT_SPD = -2,      /* a dense block lost positive definiteness (report says where) */
  RBMC_E_OOM = -3,          /* device allocation failed */
  RBMC_E_DEVICE = -4,       /* HIP runtime error */
  RBMC_E_UNSUPPORTED = -5   /* option not built */
} rbmc_status;

typedef struct rbmc_ctx rbmc_ctx;     /* device id, stream, workspace, kernels */
typedef struct rbmc_model rbmc_model; /* stencil coefficients, plan, factors */

/* The model.  theta enters through log_kappa (kappa = sqrt(8)/range),
 * log_tau, rho (|rho| < 1) and log_sigma.  obs_mask: host, length
 * n = mx*my*T, 1 = observed (copied at creation). */
typedef struct {
  int32_t mx, my, T;
  double h;
  double log_kappa, log_tau, rho, log_sigma;
  const uint8_t* obs_mask;
} rbmc_model_desc;

/* Cores Omega_p = time slabs x spatial boxes (Alg. 4 partitions the graph of
 * Q into non-overlapping parts): T is split into n_tslabs slabs, mx into
 * n_tiles_x and my into n_tiles_y pieces; in each split the first
 * (len mod parts) pieces get one extra element.  Core p =
 * (slab * n_tiles_y + tile_y) * n_tiles_x + tile_x.  Each core is grown by
 * overlap_hops rounds of graph neighbours of Q to Omega_p* (Alg. 4); the
 * separator is S_p = N(Omega_p*) \ Omega_p*.
 * The blocks of the block-Jacobi PCG preconditioner (Sec. 3.3 names block
 * Jacobi as the block form of the split preconditioner) are the cores unless
 * pc_tslabs > 0, in which case they are pc_tslabs time slabs x pc_tiles_x x
 * pc_tiles_y spatial boxes split by the same rule; the choice changes the
 * sampler's iteration count, not the samples it converges to. */
/* separators = 1: the non-overlapping variant (Alg. 2).  The first step of
 * every slab after the first and the first two grid lines (in x, in y) of
 * every tile after the first form the separator S; the cores are the slabs
 * and tiles without them (each slab after the first needs >= 2 steps, each
 * tile after the first >= 3 lines), overlap_hops must be 0.  Q's graph
 * reaches one step in time and L1 distance 2 in space, so S separates the
 * cores: given x_S they are independent.  Core nodes get
 * (Q_pp^-1)_ii + Var(Q_pp^-1 Q_pS x_S)_i, separator nodes Var(x_S)_i from
 * the samples; traces are not defined (grad_mask must be 0). */
typedef struct {
  int32_t n_tslabs, n_tiles_x, n_tiles_y, overlap_hops;
  int32_t pc_tslabs, pc_tiles_x, pc_tiles_y; /* 0 = same as the cores */
  int32_t separators;                        /* 0: Alg. 4 cores; 1: Alg. 2 */
} rbmc_decomp_desc;

/* Precision.  RBMC_FP64: every step in FP64.  RBMC_MIXED: the dense
 * products of the correction solves run on the FP32 matrix cores (operands
 * rounded to FP32, each K chunk of 16 summed in FP32 and accumulated in
 * FP64); the block-tridiagonal factorizations (inversions of the Schur
 * complements), the selected entries, the sampler (its preconditioner
 * included: FP32-rounded solves would cost the exact chain preconditioner
 * extra PCG iterations), the operators and the diagonal/trace accumulation
 * stay FP64. */
enum { RBMC_FP64 = 0, RBMC_MIXED = 1 };
/* Preconditioners of the PCG sampler (Sec. 3.3):
 *   RBMC_PC_BJ          block Jacobi over the blocks of rbmc_decomp_desc (the
 *                       plain method), each block factored block-tridiagonally;
 *   RBMC_PC_BJ_LEARNED  block Jacobi with the learned correction below;
 *   RBMC_PC_SPECTRAL    M = Q_t (x) Q_s + dbar I, dbar = n_obs / (sigma^2 n):
 *                       the prior precision with the observation term spread
 *                       evenly, applied exactly in the basis that diagonalizes
 *                       it (2-D DCT-II in space, which diagonalizes the Neumann
 *                       grid Laplacian and hence Q_s; one tridiagonal solve in
 *                       time per spatial frequency).  Not in the paper. */
enum { RBMC_PC_BJ = 0, RBMC_PC_BJ_LEARNED = 1, RBMC_PC_SPECTRAL = 2 };
/* How the selected entries of Q_AA^-1 and the correction solves of a
 * subdomain A = Omega_p* are computed (the estimator's values are the same
 * up to rounding either way):
 *   RBMC_SEL_BLOCKTRI  two-sided block-tridiagonal inversion of Q_AA over its
 *                      time steps (dense spatial blocks; Alg. 4's subdomain
 *                      solve as a block-tridiagonal factorization);
 *   RBMC_SEL_KRON      Q_AA = Q_t|A (x) Q_s|R + D_A is a Kronecker product plus
 *                      a diagonal of rank n_o (the observed nodes of A), so
 *                      Q_AA^-1 = V (x) S^-1 - Zt Y Zt^T (Woodbury) with S =
 *                      Q_s|R inverted once per spatial region (shared by all
 *                      time slabs), V = (Q_t|A)^-1 and Y the inverse of the
 *                      n_o x n_o capacitance matrix;
 *   RBMC_SEL_AUTO      the one with fewer dense flops for the call's models. */
enum { RBMC_SEL_AUTO = 0, RBMC_SEL_BLOCKTRI = 1, RBMC_SEL_KRON = 2 };
enum { RBMC_GRAD_LOGKAPPA = 1, RBMC_GRAD_LOGTAU = 2, RBMC_GRAD_RHO = 4, RBMC_GRAD_LOGSIGMA = 8 };

typedef struct {
  int32_t n_samples;  /* n_k >= 0 (0: deterministic part only); calls that sample
                         take at most 65535 columns (n_models x n_k when batched) */
  int32_t pcg_maxit;  /* > 0 */
  double pcg_rtol;    /* per-sample ||b - Q x||_2 / ||b||_2 target, > 0 */
  int32_t precision;  /* RBMC_FP64 | RBMC_MIXED */
  int32_t precond;    /* RBMC_PC_BJ | RBMC_PC_BJ_LEARNED | RBMC_PC_SPECTRAL */
  uint32_t grad_mask; /* RBMC_GRAD_* bits; traces are written in bit order */
  int32_t sample_chunk; /* rbmc_estimate with RBMC_SEL_KRON: samples drawn and
                           corrected per pass (0: all at once); the estimator is
                           a sum over samples (Alg. 4), so the passes add up to
                           the same result while the sampler's workspace holds
                           one pass.  Other calls: must be 0 or >= n_samples */
  int32_t method;     /* RBMC_SEL_* */
} rbmc_est_opts;

typedef struct {
  double t_sample, t_factor, t_select, t_correct, t_total; /* seconds; t_select: core steps */
  int32_t pcg_it_max;      /* iterations of the slowest sample */
  double pcg_it_mean;      /* mean iterations over samples */
  double max_rel_residual; /* max_k ||b_k - Q x_k|| / ||b_k|| (recurrence) */
  double err_estimate;     /* plug-in mean relative MC error of diag */
  int64_t peak_bytes;      /* device workspace held by the model */
  int32_t fail_subdomain, fail_block; /* where a dense block lost SPD, else -1 */
} rbmc_report;

/* Create a context on HIP device `device`; hip_stream is a hipStream_t (NULL
 * = the default stream).  The stream is not owned.
 * Scheduling of rbmc_estimate / rbmc_estimate_batched (environment, read
 * here): by default the sampler and the corrections run on one library
 * stream, the subdomain factorization on a second and the core steps
 * (selected inverse entries) on a third (both can be kept off
 * RBMC_RESERVE_CUS compute units, default 0); the factorization and the
 * core steps are enqueued by their own host thread, and the given stream
 * waits for all of it.  RBMC_OVERLAP=0 runs everything one step after the other on
 * the given stream; RBMC_LAUNCH_THREADS=1 enqueues all streams from the
 * calling thread.  The Kronecker method (RBMC_SEL_KRON) runs on the given
 * stream, one batch of subdomains at a time, each batch as large as the free
 * device memory allows (at most RBMC_KRON_BATCH_BYTES bytes of workspace when
 * that variable is set; a single subdomain always forms a batch). */
rbmc_status rbmc_ctx_create(int device, void* hip_stream, rbmc_ctx** out);
void rbmc_ctx_destroy(rbmc_ctx* ctx);

/* Build Q(theta) matrix-free (stencil coefficients on the device) and plan
 * the decomposition: cores, Omega_p* and S_p per Alg. 4, block-Jacobi cores.
 * Errors: RBMC_E_ARG for mx,my < 2, T < 1, mx my T >= 2^31 (node indices
 * of a sample are 32-bit), h <= 0, |rho| >= 1, non-finite theta,
 * decomposition counts outside [1, len], overlap_hops < 0. */
rbmc_status rbmc_model_create(rbmc_ctx* ctx, const rbmc_model_desc* desc,
                              const rbmc_decomp_desc* decomp, rbmc_model** out);
void rbmc_model_destroy(rbmc_model* m);

/* Replace theta; the plan is kept, factors are recomputed on next use. */
rbmc_status rbmc_model_set_theta(rbmc_model* m, double log_kappa, double log_tau, double rho,
                                 double log_sigma);

/* Operators for y = Op x (device x, y; n_rhs columns):
 *   RBMC_OP_Q: Q (n -> n); RBMC_OP_F: the perturbation map F with F F^T = Q,
 *   input [z1 (n) ; z2 (n_obs, ascending observed index)] (n + n_obs -> n);
 *   RBMC_OP_DQ_*: dQ/dtheta_j (n -> n).  n_rhs <= 65535. */
enum {
  RBMC_OP_Q = 0,
  RBMC_OP_DQ_LOGKAPPA = 1,
  RBMC_OP_DQ_LOGTAU = 2,
  RBMC_OP_DQ_RHO = 3,
  RBMC_OP_DQ_LOGSIGMA = 4,
  RBMC_OP_F = 5
};
rbmc_status rbmc_apply_op(rbmc_model* m, int op, const double* x, double* y, int32_t n_rhs);

/* rbmc_apply_op for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops): the same operators and results, with no
 * hipMalloc, hipFree or other allocation.  Its per-column tables and the
 * model view go to a fixed 2 MiB device block of the library (one per device,
 * held until the process ends); the work is enqueued on the context's stream
 * and NOT synchronized (the caller synchronizes before reading y).  n_rhs <=
 * 65535 (RBMC_E_ARG beyond).  Calls that overlap on one device share the
 * block and race; calls ordered on one stream do not. */
rbmc_status rbmc_apply_op_noalloc(rbmc_model* m, int op, const double* x, double* y,
                                  int32_t n_rhs);

/* Samples x_k = Q^-1 F z_k by preconditioned conjugate gradients (Sec. 3.3;
 * perturbation form, Sec. 2.4) with the preconditioner opts->precond, x0 = 0,
 * stopping per sample at ||b - Q x|| <= pcg_rtol ||b||.
 * z: device, (n + n_obs) x n_samples; x: device, n x n_samples.
 * Returns RBMC_W_NOT_CONVERGED if some sample hit pcg_maxit. */
rbmc_status rbmc_sample(rbmc_model* m, const rbmc_est_opts* opts, const double* z, double* x,
                        rbmc_report* rep);

/* Solves Q x_k = b_k (eq:lgm:2's Q) for opts->n_samples right-hand sides by
 * the sampler's preconditioned conjugate gradients (Sec. 3.3): x0 = 0,
 * preconditioner opts->precond, stop per column at ||b - Q x|| <= pcg_rtol
 * ||b||.  b, x: device, n x n_samples (column k at k n), distinct buffers;
 * b is not modified.  With b = e_i, x_i = (Q^-1)_ii exactly up to the
 * tolerance: the reference for the estimator's true error.
 * Returns RBMC_W_NOT_CONVERGED if some column hit pcg_maxit. */
rbmc_status rbmc_solve(rbmc_model* m, const rbmc_est_opts* opts, const double* b, double* x,
                       rbmc_report* rep);

/* Overlap from the posterior correlation range.  Sec. 3.2.2 takes n_l as
 * the lag at which the correlation falls to about zero, with separate time
 * and space values; Sec. 5 proposes probing the posterior range for it.  One
 * solve Q y = e_c (rbmc_solve with opts' preconditioner, tolerance and
 * iteration cap) at the centre node c = (T/2, my/2, mx/2) (integer halves)
 * gives the covariance column; its ratios y_j / y_c stand for the
 * correlations (Sigma_jc / Sigma_cc: the marginal variance near the centre
 * taken as uniform).
 *   lags[0] time lag: the smallest d >= 1 with |y_j| <= eps y_c at every
 *           node j = (t, my/2, mx/2), |t - T/2| >= d (graph hops in time);
 *   lags[1] space lag: the smallest L >= 1 with |y_j| <= eps y_c at every
 *           node j of step T/2 at L1 grid distance >= L from the centre;
 *   lags[2] suggested overlap_hops = max(lags[0], ceil(lags[1] / 2)) (one
 *           hop of Q's graph moves one step in time and up to two grid steps
 *           in space; rbmc_decomp_desc grows both with one count).
 * A lag one past the largest distance in the grid means the correlation did
 * not fall below eps inside the domain.
 * corr_time (host, T values, or NULL): y_j / y_c at (t, my/2, mx/2);
 * corr_space (host, mx my values, or NULL): y_j / y_c at step T/2.
 * Allocates and frees 2 n doubles of device memory.  Errors: RBMC_E_ARG for
 * NULL m, opts or lags, or eps outside (0, 1); the status of the solve
 * (RBMC_W_NOT_CONVERGED is returned with the lags of the last iterate). */
rbmc_status rbmc_probe_overlap(rbmc_model* m, const rbmc_est_opts* opts, double eps,
                               int32_t* lags, double* corr_time, double* corr_space);

/* Posterior mean with fixed effects (Sec. 3.1) and the fixed-effects term
 * of the latent variances (eq:var:1).  The latent field is x = (u, beta):
 * u on the grid with prior precision Q_t (x) Q_s, and n_beta fixed effects
 * with a diagonal prior precision Q_beta.  The observations are
 * y = A_u u + A_beta beta + noise of precision Q_y = sigma^-2 I (eq:lgm:1,
 * eq:mean:3); A_u selects the observed nodes, and Q_uu = Q_t (x) Q_s +
 * A_u^T Q_y A_u is the model's Q.  With the Schur complement
 * S = Q_betabeta - Q_betau Q_uu^-1 Q_ubeta (eq:mean:5):
 *   mu_beta   = S^-1 (A_beta^T Q_y y - Q_betau Q_uu^-1 A_u^T Q_y y),
 *   mu_u      = Q_uu^-1 (A_u^T Q_y y - Q_ubeta mu_beta),
 *   var_beta  = S^-1 = Var(beta),
 *   var_u_add = diag(Q_uu^-1 Q_ubeta S^-1 Q_betau Q_uu^-1): eq:var:1 adds it
 *               to diag(Q_uu^-1) (rbmc_estimate's diagonal) for diag(Var(u)).
 * The n_beta + 1 solves with Q_uu run together on the sampler's conjugate
 * gradients (rbmc_solve with opts' preconditioner, precision, tolerance and
 * iteration cap; opts->n_samples is ignored).  mu_u then follows from them by
 * linearity, as w - W mu_beta with w = Q_uu^-1 A_u^T Q_y y and
 * W = Q_uu^-1 Q_ubeta, in place of a further solve.
 * y: device, n_obs observations in ascending observed-node order (may be
 *    NULL if n_obs = 0).
 * a_beta: device, n_beta x n_obs, covariate j's values at j n_obs in the
 *    order of y (may be NULL if n_beta = 0 or n_obs = 0).
 * q_beta: host, n_beta finite positive prior precisions.
 * mu_u: device, n (distinct from y and a_beta).  mu_beta: host, n_beta.
 * var_beta: host, n_beta x n_beta row-major, or NULL.  var_u_add: device,
 *    n, or NULL.  NULL is allowed for mu_beta and q_beta when n_beta = 0.
 * 0 <= n_beta <= RBMC_MAX_FIXED_EFFECTS.  Allocates and frees
 * 2 (n_beta + 1) n doubles plus at most 2048 n_beta (n_beta + 1) doubles of
 * Gram partials (17 MB at n_beta = 32) of device memory; synchronizes the
 * context stream before returning.  rep: the solve's report, t_total
 * for the whole call.
 * Errors: RBMC_E_ARG (a NULL that is not allowed, n_beta out of range, a
 * q_beta entry not finite and positive); RBMC_E_NOT_SPD if S has a
 * non-positive pivot; RBMC_W_NOT_CONVERGED from the solve is returned with
 * all outputs computed from the last iterates. */
/* Gradient of the log marginal posterior of the hyperparameters (Sec. 3.4,
 * eq:hyperpar:1-4) for the model without fixed effects and a flat prior on
 * theta.  At x = mu(theta) the densities of eq:hyperpar:1 give
 * log pi(theta|y) = 1/2 log|Q_y| + 1/2 log|Q_u| - 1/2 log|Q|
 *                   - 1/2 r^T Q_y r - 1/2 mu^T Q_u mu + const,
 * Q_u = Q_t (x) Q_s, Q_y = sigma^-2 I, mu = Q^-1 A_u^T Q_y y, r = y - A_u mu;
 * mu's own theta-derivative drops out (it makes the joint exponent
 * stationary), so component j (log kappa, log tau, rho, log sigma) is the sum
 * of five terms, returned in this order in row j of terms_out:
 *   1/2 d_j log|Q_y|          -n_obs for log sigma, else 0;
 *   1/2 tr(Q_u^-1 d_j Q_u)    closed form: Q_s = (tau / h^2)(kappa^2 h^2 I + G)^2
 *                             is diagonal in the DCT-II basis (eigenvalues of
 *                             G: l_a + l_b, l_a = 2 - 2 cos(pi a / mx), l_b
 *                             likewise with my) and |Q_t| = (1 - rho^2)^-(T-1):
 *                             1/2 T sum_ab 4 kappa^2 h^2 / (kappa^2 h^2 + l_a + l_b),
 *                             n / 2, n_s (T - 1) rho / (1 - rho^2), 0;
 *   -1/2 tr(Q^-1 d_j Q)       the RBMC estimator (eq:hyperpar:4): from the
 *                             samples x (rbmc_estimate_from_samples) when x
 *                             is given or opts->n_samples = 0, else drawn on
 *                             the device from seed (rbmc_estimate, z = NULL);
 *                             opts->grad_mask is ignored (all four);
 *   -1/2 r^T (d_j Q_y) r      sigma^-2 ||r||^2 for log sigma, else 0;
 *   -1/2 mu^T (d_j Q_u) mu    d_j Q_u = d_j Q for log kappa, log tau, rho
 *                             (rbmc_apply_op), 0 for log sigma.
 * mu comes from rbmc_posterior_mean with n_beta = 0 (opts' preconditioner,
 * tolerance and iteration cap).
 * y: device, n_obs observations (ascending observed node; NULL if n_obs = 0).
 * x: device, n x opts->n_samples samples, or NULL.  grad_out: host, 4.
 * terms_out: host, 4 x 5 row-major, or NULL.  mu_out: device, n, or NULL.
 * Allocates and frees 7 n doubles (plus 64 KB of Gram partials) of device
 * memory besides what the estimator and the solve allocate; synchronizes
 * the context stream.  rep: the estimator's report with the larger PCG iteration count of
 * the two solves and t_total for the whole call.
 * Errors: those of rbmc_posterior_mean and of the estimator call; a warning
 * (RBMC_W_NOT_CONVERGED) of either is returned with the outputs computed. */
rbmc_status rbmc_grad_log_posterior(rbmc_model* m, const rbmc_est_opts* opts, const double* y,
                                    const double* x, uint64_t seed, double* grad_out,
                                    double* terms_out, double* mu_out, rbmc_report* rep);

#define RBMC_MAX_FIXED_EFFECTS 32
rbmc_status rbmc_posterior_mean(rbmc_model* m, const rbmc_est_opts* opts, const double* y,
                                int32_t n_beta, const double* a_beta, const double* q_beta,
                                double* mu_u, double* mu_beta, double* var_beta,
                                double* var_u_add, rbmc_report* rep);

/* The estimator from given samples (Alg. 4 for the diagonal; Alg. 3 rows
 * with eq:hyperpar:4 for the traces): for each core p,
 *   diag_i = (Q_AA^-1)_ii + (1/n_k) sum_k (mu_k)_i^2,  i in Omega_p,
 *   mu_k = Q_AA^-1 Q_AB x_k|B,  A = Omega_p*, B = S_p,
 *   trace_j = sum_p sum_{i in Omega_p, c in A}
 *             [(Q_AA^-1)_ic + (1/n_k) sum_k (mu_k)_i (mu_k)_c] (dQ_j)_ic.
 * x: device n x n_samples (ignored when n_samples = 0); diag_out: device, n;
 * trace_out: host, popcount(grad_mask) values (may be NULL if grad_mask = 0). */
rbmc_status rbmc_estimate_from_samples(rbmc_model* m, const rbmc_est_opts* opts, const double* x,
                                       double* diag_out, double* trace_out, rbmc_report* rep);

/* rbmc_sample followed by rbmc_estimate_from_samples (the full hot path).
 * z: device (n + n_obs) x n_samples standard normals, or NULL: then column k
 * of z is elements [k (n + n_obs), (k + 1)(n + n_obs)) of the device stream
 * of `seed` (rbmc_normals), drawn per sample pass without storing all of z
 * (needs the Kronecker method; RBMC_E_UNSUPPORTED otherwise).  With
 * opts->sample_chunk = c < n_samples (Kronecker method) the samples are drawn
 * and corrected in passes of c columns; the result equals the one-pass
 * estimate up to summation order.  Workspace for x is held by the context. */
rbmc_status rbmc_estimate(rbmc_model* m, const rbmc_est_opts* opts, const double* z, uint64_t seed,
                          double* diag_out, double* trace_out, rbmc_report* rep);

/* Standard normals of the stream of `seed`: out[i] = element offset + i
 * (i < count).  Element e is the first (e even) or second (e odd) value of
 * the Box-Muller transform of pair e / 2, whose two 53-bit uniforms come from
 * the four words of Philox4x32-10 (Salmon et al., SC11) with key = seed and
 * counter = (e / 2, 0, 0): any element depends only on (seed, e).
 * out: device, count doubles; ordered on the context stream (synchronized).
 * RBMC_E_ARG for count < 0. */
rbmc_status rbmc_normals(rbmc_ctx* ctx, uint64_t seed, uint64_t offset, int64_t count,
                         double* out);

/* rbmc_estimate for n_models independent models of one context at once
 * (the estimator of Alg. 3/4 applied to each model; models may differ in
 * grid, time length, decomposition and theta).  Every kernel launch covers
 * the chains and sample columns of all models, so many small problems fill
 * the device together.  Results equal n_models separate rbmc_estimate calls
 * up to floating-point summation order of the sampler's dot products
 * (they are per column, so in practice identical).
 * z[j]: device (n_j + n_obs_j) x n_samples; diag_out[j]: device, n_j;
 * trace_out[j]: host, popcount(grad_mask) (the array may be NULL if
 * grad_mask = 0).  The report aggregates all models (timings, the largest
 * PCG iteration count and residual, the node-averaged error estimate).
 * Errors: RBMC_E_ARG for NULL entries, a model listed twice, or models of
 * another context. */
rbmc_status rbmc_estimate_batched(rbmc_ctx* ctx, int32_t n_models, rbmc_model* const* models,
                                  const rbmc_est_opts* opts, const double* const* z,
                                  double* const* diag_out, double* const* trace_out,
                                  rbmc_report* rep);

/* Launch-shape choices of a context (not part of the method; results differ
 * only by rounding).  Products with K <= small_k, or launches with fewer
 * than small_tiles 128 x 128 tiles, use the 64 x 64-tile FP64 GEMM; batches
 * of at least four blocks, all of order >= wide_from, take rank-512
 * Gauss-Jordan steps (else 256; one to three blocks: 128).  Defaults 256,
 * 768, 2048.  RBMC_E_ARG if small_k or small_tiles < 0 or wide_from < 2048
 * (the sweep workspaces are sized for rank 512 from order 2048). */
typedef struct {
  int32_t small_k, small_tiles, wide_from;
} rbmc_tune;
rbmc_status rbmc_ctx_get_tune(rbmc_ctx* ctx, rbmc_tune* t);
rbmc_status rbmc_ctx_set_tune(rbmc_ctx* ctx, const rbmc_tune* t);

typedef struct {
  rbmc_tune best;        /* the choice now in force on the context */
  double best_ms;        /* its time for one estimate (ms) */
  double default_ms;     /* the defaults' time (ms; -1 when read from the cache) */
  int32_t from_cache;    /* 1: read from the cache, no runs */
  int32_t n_candidates;  /* configurations timed */
  int32_t cache_written; /* 1: a line was appended to the cache */
} rbmc_tune_report;

/* Autotuner: times rbmc_estimate_batched(ctx, n_models, models, opts, z, ...)
 * end to end (factorizations included: every model's factors are redone)
 * for each candidate (small_k in {256, 512} x small_tiles in {768, 1536} x
 * wide_from in {2048, never}), one warm-up and one timed run each, and keeps
 * the fastest on the context.  The end-to-end time is what counts: a faster
 * factorization can slow the overlapped step.  cache_path (may be NULL): a
 * text file with one line per tuned workload (key, small_k, small_tiles,
 * wide_from, ms, signature), the key a hash of the device architecture, the
 * options and every model's grid and decomposition; a matching line is used
 * without any run, a new result is appended.  The models' outputs are left
 * undefined (the runs write to scratch buffers); z as for
 * rbmc_estimate_batched. */
rbmc_status rbmc_autotune(rbmc_ctx* ctx, int32_t n_models, rbmc_model* const* models,
                          const rbmc_est_opts* opts, const double* const* z, const char* cache_path,
                          rbmc_tune_report* out);

/* Learned correction of the block-Jacobi preconditioner (used when
 * opts->precond = RBMC_PC_BJ_LEARNED; not part of the paper's method).  With
 * u = M_BJ^-1 r and v = N_w(r, u), the preconditioned residual becomes
 * z = u + g v, where the per-column step g = (v.r - v.Qu) / v.Qv minimizes
 * the energy error ||z - Q^-1 r||_Q along v (g = 0 when v.Qv <= 0), so the
 * correction never makes one preconditioning step worse than block Jacobi;
 * PCG then uses the flexible (Polak-Ribiere) update.  N_w: four 3-D
 * convolutions 3x3x3 over the (t, y, x) grid of a sample, channels
 * 2 -> 16 -> 16 -> 16 -> 1 (inputs r and u, both divided by ||r||), ReLU
 * between, no bias (so N_w(a r, a u) = a N_w(r, u) for a > 0), zero outside
 * the grid; BF16 weights, FP32 accumulation.  A model whose trained
 * correction did not reduce the held-out energy error falls back to plain
 * block Jacobi.  Weight vector (RBMC_PC_NWEIGHTS floats): layer l's
 * W[co][ci][tap] after layer l-1's, tap = (dt+1)*9 + (dy+1)*3 + (dx+1). */
#define RBMC_PC_NWEIGHTS 15120
typedef struct {
  int32_t n_pairs;  /* training pairs (>= 2), e.g. 2000 */
  int32_t epochs;   /* passes over the pairs (>= 0) */
  int32_t batch;    /* pairs per Adam step (0: 8) */
  float lr;         /* Adam step size (0: 1e-3) */
  uint64_t seed;    /* pair order, initial weights */
} rbmc_train_opts;

/* Train N_w on pairs the sampler generates: a block-Jacobi PCG run on the
 * right-hand sides F z gives x*; an identical second run stops at evenly
 * spaced iterations k; each column there gives one pair (r_k, u_k, e_k) / ||r_k||
 * with e_k = x* - x_k the error (Q e_k = r_k).  Adam minimizes the mean over
 * pairs of the relative energy error ||u + N_w(r, u) - e||_Q^2 / ||e||_Q^2
 * (whole grids, Q applied in FP64).  The pairs of the last max(1, n_train/4)
 * columns are held out (n_train >= 2): the ratio of its energy error with the correction to that without
 * (block Jacobi alone) goes to loss_out[epochs] and to the report's
 * err_estimate; loss_out[e] is the mean training ratio of epoch e (host,
 * epochs + 1 floats, may be NULL).  A correction with a held-out ratio
 * below 1 is then tried: PCG on the held-out right-hand sides at the
 * caller's pcg_rtol, with and without it; it is used only if it needs fewer
 * iterations and less time (a weak correction makes the nonlinear, flexible
 * PCG slower than plain block Jacobi, and each application of N_w costs
 * about 30 kflop per node).  Training continues from the current weights
 * if the model has any (a new model starts from He-scaled normals with the
 * last layer zero, i.e. from plain block Jacobi).
 * z: device (n + n_obs) x n_train standard normals; pcg_opts: pcg_maxit and
 * pcg_rtol of the pair-generating runs.  Pairs are held in FP32 on the
 * device (12 bytes per node per pair); RBMC_E_ARG if they exceed 16 GiB. */
rbmc_status rbmc_precond_train(rbmc_model* m, const rbmc_est_opts* pcg_opts,
                               const rbmc_train_opts* train_opts, const double* z,
                               int32_t n_train, float* loss_out, rbmc_report* rep);
/* y = N_w(r, u) for n_rhs device vectors r, u (n x n_rhs each; no
 * normalization); for testing. */
rbmc_status rbmc_precond_apply(rbmc_model* m, const double* r, const double* u, double* y,
                               int32_t n_rhs);
typedef struct {
  int32_t ready;            /* the model has weights */
  int32_t usable;           /* RBMC_PC_BJ_LEARNED applies them (else plain block Jacobi) */
  double val_ratio;         /* held-out energy-error ratio of the last training (-1: none) */
  int32_t trial_it_bj;      /* PCG iterations of the trial, block Jacobi (-1: no trial) */
  int32_t trial_it_learned; /* and with the correction (-1: no trial) */
  double trial_s_bj;        /* sampler seconds of the trial, block Jacobi (-1: no trial) */
  double trial_s_learned;   /* and with the correction (-1: no trial) */
} rbmc_pc_info;
rbmc_status rbmc_precond_info(rbmc_model* m, rbmc_pc_info* info);
/* Weights (host, RBMC_PC_NWEIGHTS floats); RBMC_E_ARG if the model has none. */
rbmc_status rbmc_precond_get_weights(rbmc_model* m, float* w);
/* Set the weights (host, finite); they are used as given (usable = 1, no
 * held-out ratio, no trial). */
rbmc_status rbmc_precond_set_weights(rbmc_model* m, const float* w);

/* Planner query, host only (no device needed): core label of every node
 * (label_out, length n; -1 on the separator layers of Alg. 2) and, for core
 * p, the node state (state_out, length n: 1 core, 2 overlap, 3 separator,
 * 0 outside). Either output may be NULL. */
rbmc_status rbmc_plan_query(const rbmc_model_desc* desc, const rbmc_decomp_desc* decomp, int32_t p,
                            int32_t* label_out, uint8_t* state_out);

/* Instrumentation (for throughput and roofline reporting, not part of the
 * method).  While enabled, every launch of a kernel family is bracketed by
 * HIP events on the context stream and its algorithmic work is counted:
 *   RBMC_KF_GEMM         dense products on the FP64 matrix cores, 128 x 128
 *                        tiles (also those inside the inversions); flops = 2 M K N
 *                        over the unpadded block sizes (lower-half updates:
 *                        half of that);
 *   RBMC_KF_SPD_INVERSE  one Gauss-Jordan inversion batch, all its kernels
 *                        (its products are also counted under RBMC_KF_GEMM);
 *                        flops = sum n_b^3;
 *   RBMC_KF_SPMM         q = Q p in the sampler; bytes = 16 per node and
 *                        sample (read p, write q);
 *   RBMC_KF_RSTENCIL     restricted-stencil products with dense blocks;
 *                        bytes = 16 per output entry;
 *   RBMC_KF_PANELS       gathers/scatters/right-hand sides; bytes = 16 per
 *                        panel entry;
 *   RBMC_KF_GEMM_MIXED   dense products on the FP32 matrix cores (RBMC_MIXED);
 *                        flops as RBMC_KF_GEMM;
 *   RBMC_KF_GEMM_SMALL   FP64 matrix-core products with 64 x 64 tiles (short
 *                        K or few tiles); flops as RBMC_KF_GEMM;
 *   RBMC_KF_INV_SMALL    register-resident inversions of blocks of order
 *                        w <= 128 (one workgroup each); flops = sum w^3;
 *   RBMC_KF_OFFDIAG      off-diagonal time-block entries on the stencil
 *                        pattern of the core rows (13 dot products per row);
 *                        bytes = 16 n_b^2 per block pair (each read once);
 *   RBMC_KF_DCT          the 2-D DCT-II/III transforms of the spectral
 *                        preconditioner, one axis per launch: by FFT (grid
 *                        sides powers of two; bytes = 16 per entry, read and
 *                        write) or as matrix-core products (flops = 2 m per
 *                        entry);
 *   RBMC_KF_KRON_REDUCE  group sums of the Kronecker form (k_kron_reduce);
 *                        bytes = 24 per entry of X_g (X_g, Z, K_R Z read once);
 *   RBMC_KF_SPEC_SOLVE   per-frequency tridiagonal solves of the spectral
 *                        preconditioner; bytes = 16 per entry (read, write);
 *   RBMC_KF_MC           Monte Carlo sums of the correction panels (k_mc);
 *                        bytes = 8 per entry of mu_t (each panel read once);
 *   RBMC_KF_TMIX         time mixing of stacked panels (k_kron_tmix); bytes =
 *                        16 per entry and step (24 when it adds a panel).
 * rbmc_ctx_profile(ctx, 1) clears and enables, (ctx, 0) disables;
 * rbmc_ctx_profile_read synchronizes the stream and sums the records. */
enum {
  RBMC_KF_GEMM = 0,
  RBMC_KF_SPD_INVERSE = 1,
  RBMC_KF_SPMM = 2,
  RBMC_KF_RSTENCIL = 3,
  RBMC_KF_PANELS = 4,
  RBMC_KF_GEMM_MIXED = 5,
  RBMC_KF_GEMM_SMALL = 6,
  RBMC_KF_INV_SMALL = 7,
  RBMC_KF_OFFDIAG = 8,
  RBMC_KF_DCT = 9,
  RBMC_KF_KRON_REDUCE = 10,
  RBMC_KF_SPEC_SOLVE = 11,
  RBMC_KF_MC = 12,
  RBMC_KF_TMIX = 13,
  RBMC_KF_COUNT = 14
};
typedef struct {
  int64_t launches;
  double total_ms;
  double alg_flops;
  double alg_bytes;
} rbmc_kernel_stats;
rbmc_status rbmc_ctx_profile(rbmc_ctx* ctx, int enable);
rbmc_status rbmc_ctx_profile_read(rbmc_ctx* ctx, int family, rbmc_kernel_stats* out);

/* Thread-local message of the last failing call ("" if none). */
const char* rbmc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RBMC_H */
