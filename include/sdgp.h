/*
 * sdgp.h -- sparsity-discovering exact Gaussian processes on AMD Instinct
 * MI355X (gfx950): C ABI of libsdgp.so.
 *
 * Method: Noack, Krishnan, Risser, Reyes, "Exact Gaussian Processes for
 * Massive Datasets via Non-Stationary Sparsity-Discovering Kernels"
 * (arXiv:2205.09070).  The library assembles the sparse covariance of the
 * compactly supported, non-stationary kernel of Section 2.2 and evaluates the
 * log marginal likelihood of Section 2.1 (eqn:log_likelihood), its gradient
 * and the posterior of eq:pred_distr, entirely on one GPU in FP64.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Points: x is a DEVICE array of n*dim doubles, row-major (point a's
 *   coordinates at x[a*dim .. a*dim+dim-1]), 1 <= dim <= 4, in the caller's
 *   order.  Observations y: DEVICE array of n doubles (prior mean 0: centre y
 *   first).  All device arrays belong to the caller unless stated.
 * - Hyperparameters h: HOST array of sdgp_num_hyper(desc) doubles laid out
 *     [sigma2, r_core, {a_ij, beta_ij, r_ij, c_ij[0..dim-1]} for i<n1, j<n2
 *      (j fastest), noise_var]
 *   sigma2 > 0 scales the core, r_core > 0 is its support radius, (a, beta,
 *   r, c) are the peak height, shape, radius and centre of bump function i's
 *   j-th bump (eq:bump, with the indicator taken as "inside the ball"), and
 *   noise_var >= 0 is the diagonal noise V = noise_var * I.  n1 <= 64.
 * - Kernel (Section 2.2, eq:bump_kernel): with psi the core profile of
 *   u = |x_a - x_b| / r_core and F_i(x) = sum_j f_ij(x),
 *     PRODUCT: k(x_a, x_b) = sigma2 psi(u) * sum_i F_i(x_a) F_i(x_b)
 *     SUM:     k(x_a, x_b) = sigma2 psi(u) + sum_i F_i(x_a) F_i(x_b)
 *   Core KSTAT is eq:kstat; core WENDLAND_C2 is (1-u)^(l+1)((l+1)u+1) with
 *   l = floor(dim/2)+2.
 * - Stored pattern: (a, b) is stored iff a == b, or the core support
 *   (|x_a-x_b|^2 < r_core^2) and/or (PRODUCT: and, SUM: or) a shared bump
 *   support (both points strictly inside some ball of one bump function i).
 *   Stored values may be exactly 0.0 (exp underflow inside a support).
 * - Streams: every call enqueues its work on the stream given to
 *   sdgp_create and returns after that work is complete when it writes host
 *   outputs.  A context is not thread-safe; use one per stream.
 * - Errors: a non-zero sdgp_status means the outputs are unspecified;
 *   sdgp_last_error returns a message.  No C++ exception crosses the ABI.
 *   INVALID_ARG: bad sizes, NULL pointers, non-finite or non-positive radii,
 *   dim outside 1..4, n1 > 64.  OOM: device allocation failed.  NOT_SPD: CG
 *   met p^T A p <= 0.  NOT_CONVERGED: some CG column missed cg_rtol within
 *   cg_max_iter (outputs are then best effort).  HIP: a HIP runtime error.
 *   CAPACITY: a caller buffer is too small (required size is returned).
 */
#ifndef SDGP_H
#define SDGP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sdgp_ctx sdgp_ctx;

typedef enum {
  SDGP_OK = 0,
  SDGP_ERR_INVALID_ARG = 1,
  SDGP_ERR_OOM = 2,
  SDGP_ERR_NOT_SPD = 3,
  SDGP_ERR_NOT_CONVERGED = 4,
  SDGP_ERR_HIP = 5,
  SDGP_ERR_CAPACITY = 6
} sdgp_status;

enum { SDGP_CORE_WENDLAND_C2 = 0, SDGP_CORE_KSTAT = 1 };
enum { SDGP_COMBINE_PRODUCT = 0, SDGP_COMBINE_SUM = 1 };
enum { SDGP_PROBE_RADEMACHER = 0, SDGP_PROBE_IDENTITY = 2 };
enum { SDGP_PRECOND_NONE = 0, SDGP_PRECOND_LOWRANK = 1 };
enum { SDGP_OPERATOR_ASSEMBLED = 0, SDGP_OPERATOR_FACTORED = 1 };

typedef struct {
  int32_t dim;      /* 1..4 */
  int32_t n1;       /* number of bump functions f_i, 0..64 */
  int32_t n2;       /* bumps per function, >= 1 when n1 > 0 */
  int32_t core;     /* SDGP_CORE_* */
  int32_t combine;  /* SDGP_COMBINE_* */
} sdgp_kernel_desc;

/* Estimator options for the log-det (stochastic Lanczos quadrature on the
 * coefficients of the CG solves) and the gradient's trace term (Hutchinson
 * through the same solves).  SDGP_PROBE_RADEMACHER uses `probes` sign
 * vectors from the counter-based SplitMix64 generator keyed by `seed`
 * (probe p, row a of the caller's order: output number p*2^32 + a + 1,
 * sign of bit 63); SDGP_PROBE_IDENTITY uses the n unit vectors, which makes
 * both terms exact up to the CG tolerance (n <= 16384).  lanczos_steps caps
 * the quadrature's tridiagonal size per probe (0: all CG steps).
 *
 * precond = SDGP_PRECOND_LOWRANK (SUM combine, Rademacher probes only):
 * under SUM, A = K_core + F F^T + noise_var I with F[a,i] = F_i(x_a), and
 * the core part plus noise has the constant diagonal c = sigma2 psi(0) +
 * noise_var, so M = c I + F F^T holds the whole (rank <= n1) bump part.  The
 * CG becomes preconditioned CG with M (applied through the n1 x n1 matrix
 * c I + F^T F), probes become b_p = sqrt(c) w_p + F v_p (w_p as above, v_p
 * n1 signs from outputs p*2^32 + 2^32 - 1 - i) with covariance M, and
 *   ln det A = ln det M + tr ln(M^{-1/2} A M^{-1/2}),
 * the second term by Lanczos quadrature from the preconditioned CG
 * coefficients weighted by b_p^T M^{-1} b_p, and the gradient's trace by
 * (A^{-1} b_p)^T dA (M^{-1} b_p).  Estimates stay unbiased; the CG needs far
 * fewer iterations when the bump functions hold many points.
 *
 * operator_form = SDGP_OPERATOR_FACTORED (needs SUM, Rademacher probes and
 * the low-rank preconditioner): the CG and the adjoint use the exact
 * identity K = K_core + F F^T of the SUM combine -- the sparse matrix holds
 * only the core supports (and the diagonal), F (F^T P) is applied in the
 * solver's update pass, and the bump-parameter adjoint is formed from F^T X
 * and F^T V instead of a loop over the bump cliques.  Same results as the
 * assembled operator up to rounding; sdgp_info.nnz then counts the core
 * pattern.  SDGP_OPERATOR_ASSEMBLED (default) stores every entry of K.
 *
 * probe_rtol (0 = cg_rtol): the tolerance of the probe columns' solves,
 * whose only use is the stochastic log-det and trace estimates (Section
 * 4: approximate log-determinants); y's solve keeps cg_rtol.  When every
 * probe column has stopped while y still iterates, a single evaluation
 * finishes y with the column-0 kernels only (a sparse matrix-vector
 * product per iteration).  At the 1M-point workload probe_rtol 1e-6 moves
 * the LML by less than 1e-12 and the gradient by less than 1e-9 (relative,
 * in the runs measured) against 1e-10, far inside the estimators' standard
 * errors.  Batched evaluations apply
 * the tolerance but keep every column in the launches. */
typedef struct {
  int32_t probes;          /* P, 1..64 for Rademacher */
  int32_t lanczos_steps;   /* 0 = use every CG step */
  int32_t kind;            /* SDGP_PROBE_* */
  int32_t cg_max_iter;     /* > 0 */
  uint64_t seed;
  double cg_rtol;          /* y (and identity / caller columns): |r| <= cg_rtol |b| */
  int32_t precond;         /* SDGP_PRECOND_* */
  int32_t operator_form;   /* SDGP_OPERATOR_* */
  double probe_rtol;       /* >= 0; Rademacher probe columns (0 = cg_rtol) */
} sdgp_estimator;

/* Per-call diagnostics (all optional). ms[] phase times when timing is on:
 * [0] ordering, [1] bump precompute, [2] pruning, [3] count+scan, [4] fill,
 * [5] CG, [6] SLQ, [7] adjoint. */
typedef struct {
  int64_t nnz;             /* stored entries of K */
  int64_t candidates;      /* candidate pairs the assembly's count pass tests
                              (each row times the candidate points of its cell) */
  int32_t cg_iters;        /* block-CG iterations run */
  int32_t cg_iters_y;      /* iterations of the y column */
  double cg_relres_max;    /* max final relative residual over columns */
  double yKy;              /* y^T A^{-1} y */
  double logdet;           /* estimate of ln det A */
  double logdet_stderr;    /* standard error over probes (0 for identity) */
  double ritz_min;         /* extreme Ritz values over probes */
  double ritz_max;
  double ms[8];
  int64_t spmm_launches;   /* SpMM launches inside CG */
  double spmm_ms;          /* summed SpMM launch time (timing on) */
} sdgp_info;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t, may be NULL for the null stream).  The context owns its
 * device workspace, freed by sdgp_destroy. */
sdgp_status sdgp_create(sdgp_ctx** out, int device, void* hip_stream);
void sdgp_destroy(sdgp_ctx* ctx);
/* Last error message of ctx (or of the last failed sdgp_create if NULL). */
const char* sdgp_last_error(const sdgp_ctx* ctx);
/* Enable (1) or disable (0) per-phase and per-SpMM-launch HIP-event timing. */
sdgp_status sdgp_set_timing(sdgp_ctx* ctx, int enable);
/* Context options: "timing" (0/1, as sdgp_set_timing); "graph" (0/1):
 * run the CG iterations as a captured hipGraph of 8 iterations replayed
 * until every column (and every population member) has converged; the
 * iteration counters live on the device, so replays past convergence or
 * past cg_max_iter do nothing; "union_spmm" (-1 default: on from
 * 65536 points when the lists fit in half of the free device memory, 0 off,
 * 1 on): the
 * CG SpMM reads, for every 4 consecutive rows of its row order, one sorted
 * list of the 4 rows' distinct columns with 4 values per entry (0 where a
 * row lacks the column), so each neighbour row of P is gathered once for
 * the 4 rows (lists built once per solve); "fw_mfma" (-1 default = 1, 0, 1):
 * the preconditioner / factored-operator products
 * F w of the CG update kernels per 16-row tile on the matrix cores instead
 * of per-row broadcasts; "update_blocks" (0 default: one round of the
 * blocks the GPU holds at once, from the kernels' occupancy; or 1..65535):
 * the grid size of the CG update kernels (at most one block per 16 rows);
 * "spmm_blocks" (0 default = 32768, or a multiple of 8 up to 65535): the
 * grid size of the CG SpMM (blocks are dealt to the 8 XCDs in turn).
 * "autotune" (0 off, 1 default, 2): the CG launch-shape autotuner.  The
 * first solve of a problem class (device architecture, bump-function count
 * class, right-hand-side slabs, single or population, log2 of the rows,
 * entries per row in half-octaves for single solves, operator form,
 * preconditioner) times
 * candidate shapes -- SpMM over union lists or CSR rows, SpMM grid, update
 * grid, F w product form -- in short trial solves of 24 CG iterations on
 * the call's own matrix, keeps the fastest, and stores it (see
 * sdgp_tune_cache_get); later solves of the class read it back.  1: classes
 * from 65536 rows; 2: every solve.  Explicitly set "union_spmm", "fw_mfma",
 * "spmm_blocks" or "update_blocks" switch the tuner off for the context.
 * "workspace_cap" (bytes, 0 default = no cap): the most device workspace
 * the context may hold; a call that would grow it further fails with
 * SDGP_ERR_OOM before allocating (its outputs are then unspecified, the
 * context stays usable).
 * "timing" and "graph" leave the results bitwise unchanged;
 * "union_spmm", "fw_mfma", "update_blocks" and "spmm_blocks" change only the
 * order of floating-point sums
 * (agreement to rounding).  Unknown names or
 * values: INVALID_ARG. */
sdgp_status sdgp_set_option(sdgp_ctx* ctx, const char* name, int64_t value);

/* Reads a context option (the names of sdgp_set_option) or the launch
 * shape of the context's last CG solve: "last_spmm_blocks",
 * "last_update_blocks", "last_union_spmm" (0/1), "last_fw_mfma" (0/1) and
 * "last_tuned" (0: options or defaults, 1: tuned shape read from the store,
 * 2: tuned during that call); "last_y_tail": iterations the last solve ran
 * on y alone after every probe column had stopped (see probe_rtol).
 * value: host.  Unknown name: INVALID_ARG. */
sdgp_status sdgp_get_option(const sdgp_ctx* ctx, const char* name, int64_t* value);

/* Persistent store of the autotuner: a JSON object in the file `path`
 * (NULL: $SDGP_TUNE_CACHE, else $HOME/.cache/sdgp/autotune.json), one entry
 * per problem-class key, values[4] = {spmm_blocks (multiple of 8, 8..65535),
 * update_blocks (1..65535), union_spmm (-1..1), fw_mfma (-1..1)}.  get:
 * INVALID_ARG when the key (or the file) is missing or the entry is
 * malformed; put: INVALID_ARG for out-of-range values, a key holding '"'
 * or a newline, or a file that cannot be written (the entry then still
 * serves this process).  Unparsable lines of the file are ignored; the file
 * is replaced atomically.  Host only. */
sdgp_status sdgp_tune_cache_get(const char* path, const char* key, int64_t* values);
sdgp_status sdgp_tune_cache_put(const char* path, const char* key, const int64_t* values);

/* 2 + n1*n2*(3+dim) + 1, or -1 for an invalid descriptor. */
int64_t sdgp_num_hyper(const sdgp_kernel_desc* desc);

/* Number of stored entries of K for (x, h) (Section 2.3: the sparse
 * covariance, assembled tile by tile); nnz_out is a host pointer. */
sdgp_status sdgp_kernel_nnz(sdgp_ctx* ctx, const sdgp_kernel_desc* desc,
                            const double* x, int64_t n, const double* h,
                            int64_t* nnz_out);

/* Assemble K (+ noise_var on the diagonal when add_noise) as CSR in the
 * caller's point order with ascending columns (Section 2.2 kernel, Section
 * 2.3 sparse assembly).  row_ptr: device int64[n+1]; col: device
 * int32[capacity]; val: device double[capacity].  *nnz_out (host) receives
 * the entry count; if it exceeds capacity the call returns SDGP_ERR_CAPACITY
 * without writing col/val.  Requires nnz < 2^31. */
sdgp_status sdgp_kernel_assemble(sdgp_ctx* ctx, const sdgp_kernel_desc* desc,
                                 const double* x, int64_t n, const double* h,
                                 int add_noise, int64_t* row_ptr, int32_t* col,
                                 double* val, int64_t capacity, int64_t* nnz_out);

/* Same matrix in the library's locality order (points sorted by grid cell):
 * row/column s of the output is caller point perm[s]; perm: device
 * int32[n].  This is the order the solver runs in.  The count's prefix sum
 * and the fill write row_ptr / col / val directly (no staging copy); when
 * nnz exceeds capacity the call returns SDGP_ERR_CAPACITY with row_ptr
 * written (row_ptr[n] = nnz) and col / val / perm untouched. */
sdgp_status sdgp_kernel_assemble_sorted(sdgp_ctx* ctx, const sdgp_kernel_desc* desc,
                                        const double* x, int64_t n, const double* h,
                                        int add_noise, int64_t* row_ptr, int32_t* col,
                                        double* val, int32_t* perm, int64_t capacity,
                                        int64_t* nnz_out);

/* Y = A X for a caller CSR A (device int64 row_ptr[n+1], int32 col, double
 * val) and row-major X, Y: device double[n*R], 1 <= R.  The SpMM of the CG
 * solver (Section 2.5: iterative solves on the sparse covariance). */
sdgp_status sdgp_csr_spmm(sdgp_ctx* ctx, int64_t n, const int64_t* row_ptr,
                          const int32_t* col, const double* val,
                          const double* X, int32_t R, double* Y);

/* Log marginal likelihood (eqn:log_likelihood with V = noise_var I, prior
 * mean 0, additive constant dropped):
 *   ln L = -1/2 y^T A^{-1} y - 1/2 ln det A,  A = K + noise_var I,
 * with A^{-1} y by CG (Section 2.5) and ln det A by stochastic Lanczos
 * quadrature over the probe columns' CG coefficients.  lml_out: host. */
sdgp_status sdgp_lml(sdgp_ctx* ctx, const sdgp_kernel_desc* desc, const double* x,
                     const double* y, int64_t n, const double* h,
                     const sdgp_estimator* est, double* lml_out, sdgp_info* info);

/* ln L of eqn:log_likelihood (Section 2.1, as sdgp_lml) and its gradient
 * with respect to every entry of h -- the derivative of eqn:log_likelihood
 * that Section 4 names as future work (gradient-based training):
 *   d lnL/d theta = 1/2 alpha^T (dA/dtheta) alpha - 1/2 tr(A^{-1} dA/dtheta),
 * alpha = A^{-1} y, the trace by Hutchinson through the probe solves, and
 * dA/dtheta recomputed per stored entry from the kernel of Section 2.2
 * (eq:kstat / Wendland core, eq:bump) -- never stored.  grad_out: host
 * double[sdgp_num_hyper(desc)] in the layout of h; lml_out: host; info:
 * host or NULL.  Errors as sdgp_lml; grad_out NULL: INVALID_ARG. */
sdgp_status sdgp_lml_grad(sdgp_ctx* ctx, const sdgp_kernel_desc* desc, const double* x,
                          const double* y, int64_t n, const double* h,
                          const sdgp_estimator* est, double* lml_out, double* grad_out,
                          sdgp_info* info);

/* For callers that cannot allocate device memory (code under stream or
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * sdgp_lml_grad with no device allocation.  Same arguments, results and
 * errors as sdgp_lml_grad, with these differences:
 *  - every piece of device workspace is carved from a static array of
 *    256 MiB that the library holds on each device it runs on until the
 *    process ends; the call makes no hipMalloc / hipFree and calls no
 *    allocating library routine;
 *  - n > 65535: INVALID_ARG before any device work; an input whose
 *    workspace exceeds 256 MiB (many points with many probes, identity
 *    probes beyond a few thousand points) fails with SDGP_ERR_OOM;
 *  - the context's "timing" and "graph" options are ignored for the call;
 *  - all calls on one device share the array: the library serialises them
 *    (a mutex per device, held until the call's device work has finished),
 *    and each call clears what it needs; work that the caller overlaps with
 *    the call outside the library never touches the array.
 * The context's own workspace (of the other entry points) is untouched. */
sdgp_status sdgp_lml_grad_noalloc(sdgp_ctx* ctx, const sdgp_kernel_desc* desc, const double* x,
                                  const double* y, int64_t n, const double* h,
                                  const sdgp_estimator* est, double* lml_out, double* grad_out,
                                  sdgp_info* info);

/* A population of B hyperparameter vectors on one shared point set
 * (Section 2.4 training repeats eqn:log_likelihood for many h).  The
 * factored operator (operator_form = SDGP_OPERATOR_FACTORED) is rejected
 * with INVALID_ARG before any device work.  The points
 * are ordered once (cell side = the largest core radius), every member is
 * assembled into storage of its own, and all members' block CGs advance
 * together -- every solver kernel is one launch with the member as grid
 * z, so members with uneven entry counts share the GPU -- followed by each
 * member's quadrature and adjoint.  Probes are common to all members.
 * H is a host array B*n_h (member m at H[m*n_h]); lml_out: host double[B];
 * grad_out: host double[B*n_h]; member_status: host int32[B] (per-member
 * sdgp_status; one failing member does not affect the others); info: host
 * array of B sdgp_info or NULL.  Returns SDGP_OK when the batch ran, even if
 * some members failed. */
sdgp_status sdgp_lml_grad_batched(sdgp_ctx* ctx, const sdgp_kernel_desc* desc,
                                  const double* x, const double* y, int64_t n,
                                  const double* H, int32_t B, const sdgp_estimator* est,
                                  double* lml_out, double* grad_out,
                                  int32_t* member_status, sdgp_info* info);

/* Posterior at n0 test points x0 (device n0*dim) per eq:pred_distr with
 * m0 = 0: mean = kappa^T A^{-1} y, var = k(x0,x0) - kappa^T A^{-1} kappa,
 * kappa = k(x, x0).  mean_out, var_out: device double[n0]. */
sdgp_status sdgp_posterior_mean_var(sdgp_ctx* ctx, const sdgp_kernel_desc* desc,
                                    const double* x, const double* y, int64_t n,
                                    const double* h, const double* x0, int64_t n0,
                                    const sdgp_estimator* est, double* mean_out,
                                    double* var_out);

/* Randomised Taylor-series log-det of Boutsidis et al. (2017), the estimator
 * Section 2.5 names: with alpha = max_a sum_b |A_ab| (>= lambda_max) and
 * C = I - A/alpha,
 *   ln det A ~= N ln alpha - sum_{k=1}^{terms} (1/k) (1/P) sum_p z_p^T C^k z_p
 * for A = K + noise_var I and P Rademacher probes z_p (the generator of
 * sdgp_estimator, keyed by seed).  The truncation error is at most
 * N rho^(terms+1) / ((terms+1)(1-rho)), rho = 1 - lambda_min/alpha, so it
 * needs many terms for ill-conditioned A (Stochastic Lanczos quadrature in
 * sdgp_lml is the default).  logdet_out, alpha_out: host. */
sdgp_status sdgp_logdet_taylor(sdgp_ctx* ctx, const sdgp_kernel_desc* desc, const double* x,
                               int64_t n, const double* h, int32_t probes, int32_t terms,
                               uint64_t seed, double* logdet_out, double* alpha_out);

/* Upper bound of the fraction s of stored covariances contributed by the bump
 * part of the kernel (Section 2.2, eq:sparsity_estimate, disjoint-support
 * bound):  s <= sum_i sum_j sum_k Vol(dim, r_ij) Vol(dim, r_ik) / V_X^2 with
 * Vol(dim, r) = pi^(dim/2) / Gamma(dim/2 + 1) r^dim and V_X the volume of the
 * input domain (1 for the unit cube).  h: host array as above.  Host-only
 * (no device work); s_out: host. */
sdgp_status sdgp_sparsity_bound(const sdgp_kernel_desc* desc, const double* h,
                                double domain_volume, double* s_out);

/* Section 2.4 objectives for a likelihood value lml and sparsity s:
 * augmented (eq:augmented) lml + (1 - s) lml; feasible (eq:constrained) is 1
 * when s < requirement.  Host-only; outputs are host pointers. */
sdgp_status sdgp_sparsity_objective(double lml, double s, double requirement,
                                    double* augmented_out, int32_t* feasible_out);

/* ------------------------------------------------------------------------
 * Training driver over the batched path: differential evolution
 * (DE/rand/1/bin of Storn and Price, J. Global Optim. 11, 1997), the
 * derivative-free population search over hyperparameters for which the
 * batched evaluation is built (the paper maximises the LML derivative-free,
 * by MCMC: Sections 2.5 and 3).
 * Random numbers: the SplitMix64 counter generator of sdgp_estimator, with
 * stream keys derived from (seed, generation, member, draw); deterministic.
 * ------------------------------------------------------------------------ */

/* Fitness used by sdgp_train_de. */
typedef enum {
  SDGP_DE_LML = 0,          /* ln L */
  SDGP_DE_AUGMENTED = 1,    /* the augmented objective of sdgp_sparsity_objective */
  SDGP_DE_CONSTRAINED = 2   /* ln L when the sparsity bound s(h) < requirement, else -inf */
} sdgp_de_objective;

typedef struct {
  int32_t generations;      /* >= 0 */
  double F;                 /* differential weight, (0, 2] */
  double CR;                /* crossover probability, [0, 1] */
  uint64_t seed;
  int32_t objective;        /* sdgp_de_objective */
  double requirement;       /* sparsity requirement (objectives 1, 2) */
  double domain_volume;     /* V_X of sdgp_sparsity_bound (objectives 1, 2) */
} sdgp_de_options;

/* Trial vectors of one DE generation: for member m of the population H
 * (host, B x nh, row-major) pick r1, r2, r3 distinct and != m, a forced
 * component jrand, and set T[m][j] = H[r1][j] + F (H[r2][j] - H[r3][j]) where
 * u_j < CR or j == jrand, else H[m][j].  A component outside [lo[j], hi[j]]
 * is redrawn uniformly between the violated bound and H[m][j]; components
 * with lo[j] == hi[j] stay fixed.  Needs B >= 4, lo <= H <= hi.  Host only;
 * T: host, B x nh.  INVALID_ARG on bad sizes, bounds or F / CR. */
sdgp_status sdgp_de_trials(int32_t B, int32_t nh, const double* H, const double* lo,
                           const double* hi, double F, double CR, uint64_t seed,
                           uint64_t generation, double* T);

/* Selection: row m of H and fit[m] take T[m] and ft[m] when ft[m] >= fit[m]
 * (a NaN trial fitness never wins; a NaN incumbent always loses to a
 * number).  replaced_out (host, may be NULL) receives the count.  Host
 * only. */
sdgp_status sdgp_de_select(int32_t B, int32_t nh, double* H, double* fit, const double* T,
                           const double* ft, int32_t* replaced_out);

/* Runs opt->generations DE generations on the device path: the initial
 * population H and every generation's trials are evaluated with one batched
 * evaluation each (sdgp_lml_grad_batched semantics; a member whose
 * evaluation fails gets fitness -inf), then selected.  H (host, B x nh) is
 * updated in place; fit (host, B) receives the final fitness;
 * history (host, generations + 1, may be NULL) the best fitness after the
 * initial evaluation and after each generation.  x, y: device, as in
 * sdgp_lml. */
sdgp_status sdgp_train_de(sdgp_ctx* ctx, const sdgp_kernel_desc* desc, const double* x,
                          const double* y, int64_t n, double* H, int32_t B, const double* lo,
                          const double* hi, const sdgp_estimator* est,
                          const sdgp_de_options* opt, double* fit, double* history);

#ifdef __cplusplus
}
#endif

#endif /* SDGP_H */
