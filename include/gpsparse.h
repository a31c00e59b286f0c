/*
 * gpsparse.h - C ABI of the MI355X (gfx950) sparse-covariance exact-GP library.
 *
 * The library assembles the covariance of the compactly supported,
 * nonstationary kernel of "Compactly-supported nonstationary kernels for
 * computing exact Gaussian processes on big data" (arXiv 2411.05869),
 *
 *     K_pq = s0 f0(x_p, x_q; r0) + sum_{i=1..n1} f_i(x_p) f_i(x_q) + sigma^2 [p = q]
 *
 * (Sec. 2.1, Eq. C_sparse with the Wendland part of Eq. compSupp, the bump
 * sums of Eq. sumOfBumps / bumpFcn; Sec. 3.1 Eq. Zcov for the nugget; unit
 * core kernel), evaluates the Gaussian log-likelihood of Sec. 3.1 Eq. Zmarg
 * (log det K and y^T K^-1 y, the three tasks of Sec. 3.3) and the kriging
 * mean of Sec. 3.2.  All numerical work runs in HIP kernels on one GPU.
 *
 * Conventions shared by every entry point:
 *   - Pointers named *_dev are device pointers on the context's device; all
 *     other pointers are host pointers.  Caller-owned buffers are never
 *     retained past the call.
 *   - All work is issued on the context's HIP stream.  A call returns after
 *     its results are complete unless stated otherwise.
 *   - Every call returns gp_status; no C++ exception crosses the ABI.  On an
 *     error the message is available from gp_last_error(ctx).  Input errors
 *     (GP_EINVAL) are detected on the host before any device work.
 *   - Objects (gp_dataset, gp_matrix, gp_predictor) belong to the context
 *     that created them and are freed through its allocator.  A context is
 *     not thread-safe: use one context per host thread / serving slot.
 *   - Point coordinates are n x d row-major float64 with 1 <= d <= 3.
 */
#ifndef GPSPARSE_H
#define GPSPARSE_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define GP_API __attribute__((visibility("default")))
#else
#define GP_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gp_status {
  GP_OK = 0,
  GP_EINVAL = 1,    /* invalid argument (shape, hyper-parameter, non-finite input) */
  GP_ENOMEM = 2,    /* the allocator failed or a size limit was exceeded */
  GP_ENOTCONV = 3,  /* iteration limit reached; outputs hold the last iterate */
  GP_ENOTPD = 4,    /* non-positive curvature met: matrix not positive definite */
  GP_EDEVICE = 5    /* HIP runtime error or an internal consistency check failed */
} gp_status;

typedef enum gp_precision {
  GP_FP64 = 0,      /* float64 values, vectors and accumulation */
  GP_MIXED = 1      /* float32 stored values; products with float64 vectors and accumulation */
} gp_precision;

typedef enum gp_logdet_mode {
  GP_LOGDET_SLQ = 0,    /* stochastic Lanczos quadrature (Sec. 3.3 Lanczos log-det) */
  GP_LOGDET_EXACT = 1,  /* Lanczos to dimension n with full re-orthogonalisation (n <= 8192) */
  GP_LOGDET_NONE = 2,   /* skip the log-determinant (quadratic form only) */
  GP_LOGDET_SLQ_REORTH = 3  /* the SLQ estimator with every residual re-orthogonalised
                               against all Lanczos vectors (classical Gram-Schmidt,
                               twice): the basis stays orthonormal to rounding, so runs
                               that differ only in rounding agree closely (parity runs);
                               work space n_lanczos x n x 32 float64 */
} gp_logdet_mode;

typedef struct gp_ctx gp_ctx;
typedef struct gp_dataset gp_dataset;
typedef struct gp_matrix gp_matrix;
typedef struct gp_predictor gp_predictor;

/* Device-memory allocator supplied by the caller (e.g. a framework's caching
 * allocator).  alloc returns a device pointer or NULL; free receives the
 * pointer and the size that was requested. */
typedef void* (*gp_alloc_fn)(size_t bytes, void* user);
typedef void (*gp_free_fn)(void* ptr, size_t bytes, void* user);

/* ------------------------------------------------------------------ context
 * gp_ctx_create: binds a context to `device` and the HIP stream `stream`
 * (a hipStream_t; NULL = the null stream).  alloc/free may both be NULL, in
 * which case the library uses the device's stream-ordered memory pool.
 * Errors: GP_EINVAL (bad device, only one of alloc/free given), GP_EDEVICE. */
GP_API gp_status gp_ctx_create(int device, void* stream, gp_alloc_fn alloc, gp_free_fn free_fn,
                        void* user, gp_ctx** out);
/* Releases the context's workspace.  Objects it created must be destroyed first. */
GP_API gp_status gp_ctx_destroy(gp_ctx* ctx);
/* Re-targets later work of the context to another stream. */
GP_API gp_status gp_ctx_set_stream(gp_ctx* ctx, void* stream);
/* Last error message of the context ("" if none).  Valid until the next call. */
GP_API const char* gp_last_error(const gp_ctx* ctx);
/* Bytes currently held by the context's workspace and live objects. */
GP_API gp_status gp_ctx_memory(const gp_ctx* ctx, size_t* bytes_in_use, size_t* peak_bytes);
/* HBM budget of the context: a device allocation that would raise the bytes
 * in use (as gp_ctx_memory counts them: datasets, matrices, predictors and
 * work space of this context) above `bytes` fails with GP_ENOMEM before the
 * allocator is called; the call that needed it returns GP_ENOMEM and frees
 * what it had allocated.  0 = no budget (the default).  Memory already held
 * is kept even if it exceeds a new, smaller budget. */
GP_API gp_status gp_ctx_set_hbm_budget(gp_ctx* ctx, size_t bytes);
/* Concurrency of one likelihood (Sec. 3.3: the log det and the solve are
 * independent tasks): with on = 1 (the default) gp_loglik, gp_loglik_async
 * and gp_loglik_batch enqueue the SLQ log det on a second stream of the
 * context, ordered after the call's earlier work and joined before its
 * result, so its launches run beside the solver's; with on = 0 the log det
 * runs after the solve on the context's stream.  The results are the same
 * bitwise either way (the same kernels in the same order per task). */
GP_API gp_status gp_ctx_set_concurrency(gp_ctx* ctx, int32_t on);

/* Per-kernel timing: while enabled, the library brackets its kernel launches
 * with HIP events on the context's stream.  gp_profile_enable clears the
 * record; gp_profile_read synchronises and returns one entry per kernel name
 * (launch count and total milliseconds); *n_out receives the number of
 * distinct names even when it exceeds max_entries. */
typedef struct gp_profile_entry {
  char name[32];
  int64_t count;
  double total_ms;
} gp_profile_entry;
GP_API gp_status gp_profile_enable(gp_ctx* ctx, int32_t on);
GP_API gp_status gp_profile_read(gp_ctx* ctx, int32_t max_entries, gp_profile_entry* out, int32_t* n_out);
/* Restricts the timing to the names in `names`, a comma-separated list as
 * gp_profile_read reports them (NULL or "" times every name again).  Each
 * timed launch group adds two events to its stream, so a caller timing one
 * product in a measured region can leave the others untimed.  Kept until the
 * next call; GP_EINVAL for a name longer than 31 characters. */
GP_API gp_status gp_profile_only(gp_ctx* ctx, const char* names);

/* ------------------------------------------------------------------ dataset
 * gp_dataset_create: copies and spatially bins n points (x_dev, n x d
 * row-major float64, caller-owned, read during the call).  The points are
 * sorted by a cell key on a regular grid with cell edge cell[k] per
 * coordinate (host array of d positive values; NULL picks about eight
 * points per cell).  Cells never decide membership in the covariance pattern;
 * they only bound the candidate search.  The binned copy stays resident on
 * the device until gp_dataset_destroy.
 * Errors: GP_EINVAL (n < 1, d not in 1..3, non-finite coordinate, cell <= 0),
 * GP_ENOMEM, GP_EDEVICE. */
GP_API gp_status gp_dataset_create(gp_ctx* ctx, int64_t n, int32_t d, const double* x_dev,
                            const double* cell, gp_dataset** out);
GP_API gp_status gp_dataset_destroy(gp_ctx* ctx, gp_dataset* ds);
/* n, d, number of grid cells, and the cell edges used (cell_out: d doubles or NULL). */
GP_API gp_status gp_dataset_info(const gp_dataset* ds, int64_t* n, int32_t* d, int64_t* n_cells,
                          double* cell_out);
/* Binned position -> original index (perm_dev: n int32, caller-owned). */
GP_API gp_status gp_dataset_permutation(gp_ctx* ctx, const gp_dataset* ds, int32_t* perm_dev);

/* ------------------------------------------------------- hyper-parameters
 * theta_sparse of Sec. 2.1 (s0, r0, {h_ij, a_ij, b_ij, r_ij}) plus the error
 * variances of Eq. Zcov, Delta = diag[tau^2(x_1), ..., tau^2(x_N)], given as a
 * constant nugget sigma^2 and optional per-point values tau2; all in host
 * memory and copied by each call, except tau2 (device memory, read during the
 * call only).
 *   r0[k]  coordinate-specific Wendland radii (> 0; Appendix E uses
 *          per-coordinate truncation radii); u = |((x - x') / r0)|.
 *   h      n1*n2*d bump centres, bump (i, j) at h[(i*n2 + j)*d + k]
 *   r      n1*n2*d bump radii per coordinate (> 0; +INF drops the coordinate)
 *   a      n1*n2 amplitudes (>= 0; a = 0 removes the bump)
 *   b      n1*n2 shapes (> 0)
 * Support tests use the float64 expression sum_k ((x_k - c_k) * (1 / r_k))^2
 * < 1 evaluated left to right without fused multiply-add.
 * Limits: 1 <= n1 <= 64, n1*n2 <= 4096, s0 > 0, nugget >= 0.
 * core (optional) multiplies C_sparse, see gp_core.
 * tau2 (optional, NULL for none): n float64 values in device memory, in the
 * dataset's original point order, finite and >= 0 (checked on the device:
 * GP_EINVAL otherwise).  The diagonal entry of row p is
 * C_core C_sparse + sigma^2 + tau2[p], added in that order.  Only gp_assemble
 * reads it: the cross-covariances of gp_predict and gp_predict_var carry no
 * error variances. */
/* Core kernel C_core of C_y = C_core x C_sparse (Sec. 2, Eq. sparseCov; the
 * nugget is added after the product).  The core is strictly positive, so it
 * never changes the sparsity pattern; it only scales the stored values.
 *   GP_CORE_MATERN:   sigma0^2 M_nu(|(x - x') / ell|)             (Sec. 2.2)
 *   GP_CORE_PACIOREK: sigma(x) sigma(x') (Sigma(x) Sigma(x'))^(d/4)
 *                     / ((Sigma(x) + Sigma(x')) / 2)^(d/2) M_nu(sqrt(Q)),
 *                     Q = |(x - x') / ell|^2 / ((Sigma(x) + Sigma(x')) / 2)
 *                     (Appendix B, Eq. PScov, its denominator read as
 *                     Sigma(x) + Sigma(x')), with log-linear fields
 *                     log sigma(x) = log sigma0 + sum_m s_m(x) phi_sigma[m],
 *                     log Sigma(x) = log Sigma0 + sum_m s_m(x) phi_Sigma[m],
 *                     s_m(x) = exp(-|(x - centers[m]) / width|^2 / 2).
 * M_nu is the Matern correlation 2^(1-nu)/Gamma(nu) (sqrt(2 nu) t)^nu
 * K_nu(sqrt(2 nu) t) at nu = nu2 / 2 in {1/2, 3/2, 5/2}, or exp(-t^2/2) for
 * nu2 = 0 (the limit nu -> infinity).  Host memory, copied by each call.
 * Limits: sigma0, ell[k], Sigma0, width[k] finite and > 0; 0 <= n_basis <= 16;
 * centers (n_basis x d), phi_sigma, phi_Sigma (n_basis) finite. */
typedef enum gp_core_kind {
  GP_CORE_NONE = 0,      /* C_core = 1 */
  GP_CORE_MATERN = 1,
  GP_CORE_PACIOREK = 2
} gp_core_kind;

typedef struct gp_core {
  int32_t kind;            /* gp_core_kind */
  int32_t nu2;             /* 2 nu: 1, 3 or 5; 0 for nu = infinity */
  double sigma0;
  double ell[3];
  double Sigma0;           /* PACIOREK only */
  int32_t n_basis;         /* PACIOREK only */
  int32_t reserved;
  const double* centers;   /* n_basis x d, row-major */
  double width[3];
  const double* phi_sigma; /* n_basis */
  const double* phi_Sigma; /* n_basis */
} gp_core;

typedef struct gp_theta {
  int32_t d;
  int32_t n1;
  int32_t n2;
  int32_t wendland_variant;  /* 0: cubic coefficient 35 as printed in Eq. compSupp; 1: 32 */
  double s0;
  double r0[3];
  const double* h;
  const double* r;
  const double* a;
  const double* b;
  double nugget;
  const gp_core* core;       /* NULL: C_core = 1 */
  const double* tau2;        /* device, n values in original order, or NULL */
} gp_theta;

/* ------------------------------------------------------------------ matrix
 * gp_assemble: builds K(theta) + sigma^2 I for the dataset as a CSR matrix
 * owned by the library, rows and columns in binned order, full symmetric
 * storage, every column once per row.  A row of a point with no bump group
 * holds its columns in ascending order.  A row of a point whose bump-group
 * mask is M first holds the columns U_M = {q : mask(q) & M != 0} in ascending
 * order (one list shared by all rows with mask M), then its remaining local
 * columns in ascending order.  The pattern is exactly the set of pairs that
 * pass a support test (local Wendland support, a shared bump group, or the
 * diagonal); entries whose value underflows stay stored.  Values are float64
 * (GP_FP64) or float32 rounded from float64 (GP_MIXED).
 * Errors: GP_EINVAL (theta), GP_ENOMEM, GP_EDEVICE (device error or the
 * count and fill passes disagree). */
GP_API gp_status gp_assemble(gp_ctx* ctx, const gp_dataset* ds, const gp_theta* theta,
                      gp_precision prec, gp_matrix** out);
GP_API gp_status gp_matrix_destroy(gp_ctx* ctx, gp_matrix* m);
/* n, nnz, bytes held by the matrix (CSR arrays, group tables and the caches
 * built on first use: int16 column offsets, block-Jacobi inverses, row
 * quads), precision, longest row. */
GP_API gp_status gp_matrix_info(const gp_matrix* m, int64_t* n, int64_t* nnz, size_t* bytes,
                         int32_t* prec, int64_t* max_row);
/* Storage layout of the matrix, for byte accounting: the entries of the
 * rows' group blocks (stored without column ids: rows with mask M share the
 * list U_M), the other entries (column ids stored, read by the one-column
 * product as int16 offsets when col16 = 1), the U_M entries the group
 * products stage (one pass over U_M per tile of 16 rows for one column, per
 * super-tile of 64 rows for several), and the cache of the 32-column product
 * (0 until the first such product built it): the rows listed in groups of
 * four and the entries of the four-row column unions. */
typedef struct gp_matrix_layout_info {
  int64_t nnz_group;          /* entries in group blocks */
  int64_t nnz_csr;            /* the other entries */
  int64_t group_rows;         /* rows with a group block */
  int64_t group_masks;        /* distinct group masks M */
  int64_t group_list_entries; /* sum of |U_M| */
  int64_t gemv_stage_entries; /* U_M entries read by one one-column product */
  int64_t gemm_stage_entries; /* U_M entries read by one multi-column product */
  int64_t long_rows;          /* rows whose other entries exceed 128 */
  int32_t col16;              /* int16 column offsets built and used */
  int32_t reserved;
  int64_t listed_rows;        /* rows listed for the four-row unions (padded) */
  int64_t quad_entries;       /* entries of the four-row unions */
} gp_matrix_layout_info;
GP_API gp_status gp_matrix_layout(const gp_matrix* m, gp_matrix_layout_info* out);
/* Writes the matrix in ORIGINAL point order with ascending columns into
 * caller device buffers: row_ptr_dev (n+1 int64), col_dev (nnz int32),
 * val_dev (nnz float64; float32 values are widened).  Debug/parity path. */
GP_API gp_status gp_matrix_export_csr(gp_ctx* ctx, const gp_matrix* m, int64_t* row_ptr_dev,
                               int32_t* col_dev, double* val_dev);
/* Y = K X for nrhs right-hand sides, X and Y n x nrhs row-major float64 in
 * ORIGINAL point order (device).  Uses the matrix's value precision with
 * float64 accumulation.  The first one-column product stores the columns of
 * the rows' local parts as int16 offsets from the row (2 bytes per nonzero;
 * kept unless an offset does not fit).  The first product with 32 columns
 * (nrhs = 32 here, and the Lanczos blocks of gp_loglik) builds a cache kept with the matrix
 * until it is destroyed: for every four consecutive binned rows the union of
 * their columns with the four rows' values (about 5 bytes per nonzero in the
 * mixed form, 9 in float64). */
GP_API gp_status gp_matvec(gp_ctx* ctx, const gp_matrix* m, int32_t nrhs, const double* x_dev,
                    double* y_dev);

/* gp_matvec_noalloc: y = K x for one right-hand side, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid allocation).  Same product and result as gp_matvec
 * with nrhs = 1 (x_dev, y_dev: n float64 in ORIGINAL point order, device,
 * caller-owned; they must not overlap), but it allocates nothing: the two
 * n-vectors gp_matvec stages in binned order live in a fixed 64 MiB array of
 * device memory that the library holds on every GPU it has run on until the
 * process ends (its address is looked up when a context is created), so
 * n <= 4,194,304.  It builds no cache (a product reads the int16 column
 * offsets only if an earlier product built them; either form gives bitwise
 * the same y), records no profiling events and does not synchronise: the call
 * returns once the work is enqueued on the context's stream, and y is
 * complete when the stream reaches that point.  Every call on one GPU shares
 * that GPU's array: calls that overlap in time on one GPU (other streams,
 * other contexts, other threads) race and must be ordered by the caller.
 * Errors: GP_EINVAL (NULL argument, n above the limit), GP_EDEVICE. */
GP_API gp_status gp_matvec_noalloc(gp_ctx* ctx, const gp_matrix* m, const double* x_dev, double* y_dev);

/* ------------------------------------------------------------ likelihood */
typedef enum gp_precond {
  GP_PRECOND_JACOBI = 0,        /* diagonal of K */
  GP_PRECOND_BLOCK_JACOBI = 1   /* dense diagonal blocks over the binning cells (<= 32 points) */
} gp_precond;

/* Linear solver for alpha = K^-1 y.  MINRES is the method the paper used
 * (Sec. 3.3; Paige and Saunders): it needs K symmetric only (the
 * preconditioner positive definite); conjugate gradients are cheaper per step
 * on a positive-definite K.  AUTO runs conjugate gradients; if they end with
 * GP_ENOTCONV it continues with MINRES from their last iterate, if they meet
 * non-positive curvature (GP_ENOTPD) it runs MINRES from zero (either way up to
 * max_iter more steps).  MINRES forms its products in float64 arithmetic on
 * the stored values (float32 values for a GP_MIXED matrix). */
typedef enum gp_solver {
  GP_SOLVER_CG = 0,
  GP_SOLVER_MINRES = 1,
  GP_SOLVER_AUTO = 2
} gp_solver;

typedef struct gp_solve_opts {
  double rtol;          /* stop when |y - K alpha|_2 <= rtol |y|_2 (default 1e-10) */
  int32_t max_iter;     /* iteration cap of each solver (default 10000) */
  int32_t n_probes;     /* SLQ probes (default 30, at most 64) */
  int32_t n_lanczos;    /* SLQ Lanczos steps (default 50, at most 128) */
  int32_t logdet_mode;  /* gp_logdet_mode */
  int32_t precond;      /* gp_precond for the solver (default block Jacobi) */
  int32_t solver;       /* gp_solver (default GP_SOLVER_AUTO) */
  uint64_t seed;        /* probe seed */
} gp_solve_opts;

/* Fills opts with the defaults listed above. */
GP_API void gp_solve_opts_default(gp_solve_opts* opts);

typedef struct gp_loglik_result {
  double loglik;        /* -1/2 logdet - 1/2 quad - (n/2) log(2 pi) */
  double logdet;        /* log det K */
  double quad;          /* y^T K^-1 y */
  double logdet_se;     /* standard error of the SLQ estimate (0 in exact mode) */
  double relres;        /* final |y - K alpha| / |y| (float64 true residual) */
  int32_t cg_iters;     /* conjugate-gradient iterations */
  int32_t refreshes;    /* float64 true-residual recomputations */
  int32_t lanczos_steps;/* Lanczos steps taken (max over probes; n in exact mode) */
  int32_t status;       /* gp_status of the solve */
  int32_t minres_iters; /* MINRES iterations (0 when it did not run) */
  int32_t reserved;
} gp_loglik_result;

/* gp_loglik: log p(y | theta) for the residual y = z - W beta (y_dev: n
 * float64 in ORIGINAL point order).  Quadratic form by preconditioned
 * conjugate gradients and/or MINRES on K (gp_solver, gp_precond); log det by
 * stochastic Lanczos quadrature on the Jacobi-scaled matrix (or exact
 * Lanczos, see gp_logdet_mode).  Every product reads the matrix's stored
 * values (float32 for a GP_MIXED matrix) with float64 vectors and float64
 * accumulation; vectors, Lanczos coefficients, quadrature and the quadratic
 * form are float64.  alpha_dev (n float64, original order, may be NULL)
 * receives K^-1 y.  opts may be NULL (defaults).
 * Errors: GP_EINVAL, GP_ENOMEM, GP_ENOTCONV (result and alpha hold the last
 * iterate), GP_ENOTPD, GP_EDEVICE. */
GP_API gp_status gp_loglik(gp_ctx* ctx, const gp_matrix* m, const double* y_dev,
                    const gp_solve_opts* opts, double* alpha_dev, gp_loglik_result* out);

/* gp_loglik_async: the log-likelihood of gp_loglik (Sec. 3.1 Eq. Zmarg; the
 * log-det and solve tasks of Sec. 3.3), enqueued on the context's stream
 * without waiting for it: every decision of the solver (convergence checks,
 * the true-residual pass) is taken on the device, so nothing is read back to
 * the host.  The conjugate gradients are enqueued in blocks of 8 iterations
 * up to opts->max_iter; the iterations after convergence return at once
 * (a few microseconds each), so set max_iter near the expected count, e.g.
 * twice that of an earlier evaluation on the same data (GP_ENOTCONV in
 * out->status when it is not enough).  The last kernel writes the result
 * into *out, which must be pinned host memory (hipHostMalloc) or device
 * memory; if event (a hipEvent_t, or NULL) is given it is recorded on the
 * stream after that kernel: *out and alpha_dev are complete once the event
 * has completed.  Errors found on the device (GP_ENOTCONV, GP_ENOTPD,
 * non-finite y) are reported in out->status only.  Solver: conjugate
 * gradients (GP_SOLVER_AUTO runs them without the MINRES fallback); logdet
 * mode GP_LOGDET_SLQ, GP_LOGDET_SLQ_REORTH or GP_LOGDET_NONE.  The first
 * likelihood of a matrix builds its product and preconditioner caches with
 * host synchronisations, then enqueues the rest.  The context's work space
 * is in use until the event completes: later calls on the same context and
 * stream are ordered after it.
 * Errors (returned): GP_EINVAL (arguments, solver, GP_LOGDET_EXACT, out not
 * reachable by the device), GP_ENOMEM, GP_EDEVICE. */
GP_API gp_status gp_loglik_async(gp_ctx* ctx, const gp_matrix* m, const double* y_dev, const gp_solve_opts* opts,
                                 double* alpha_dev, gp_loglik_result* out, void* event);

/* gp_loglik_batch: the log-likelihoods of nreq problems (Sec. 3.1 Eq. Zmarg),
 * evaluated together: the sampler of Appendix C evaluates many
 * hyper-parameter proposals whose matrices are small (a few thousand to tens
 * of thousands of rows, Sec. 3.3), each too small to fill the device alone.
 * The matrices K[r] (one precision; each of its own dataset and theta) are
 * stacked into one block-diagonal matrix, so every product, vector and
 * reduction launch serves all problems; each problem keeps its own scalars,
 * convergence test and probes, and stops on its own (its vector work ends,
 * the shared products run until every problem has ended).  Each result
 * equals what gp_loglik returns for that problem alone, bitwise.
 * y_dev[r]: n_r float64 in the ORIGINAL order of K[r]'s dataset;
 * alpha_dev (may be NULL, as may alpha_dev[r]) receives K[r]^-1 y[r].
 * out: nreq results in host memory (the call waits for the device; it reads
 * back one flag per 8 iterations to stop once all problems have ended).
 * Solver: GP_SOLVER_CG, or GP_SOLVER_AUTO, where a problem whose conjugate
 * gradients end in GP_ENOTCONV or GP_ENOTPD is evaluated again alone by
 * gp_loglik (MINRES fallback); logdet mode GP_LOGDET_SLQ or GP_LOGDET_NONE.
 * The call builds each matrix's product and preconditioner caches if needed
 * and a stacked copy of the matrices (about their total size) that it frees
 * before it returns.
 * Returns GP_OK when every problem succeeded, else the status of the first
 * that did not (each out[r].status holds its own; a non-finite y[r] gives
 * GP_EINVAL there); GP_EINVAL (arguments, solver, logdet mode, mixed
 * precisions), GP_ENOMEM or GP_EDEVICE for the whole call. */
GP_API gp_status gp_loglik_batch(gp_ctx* ctx, int32_t nreq, const gp_matrix* const* K, const double* const* y_dev,
                                 const gp_solve_opts* opts, double* const* alpha_dev, gp_loglik_result* out);

/* gp_solve: alpha = K^-1 y only (the quadratic-form task of Sec. 3.3). */
GP_API gp_status gp_solve(gp_ctx* ctx, const gp_matrix* m, const double* y_dev,
                   const gp_solve_opts* opts, double* alpha_dev, gp_loglik_result* out);

/* ------------------------------------------------------------- prediction
 * gp_predictor_create: caches what the kriging mean of Sec. 3.2 needs for a
 * fixed theta and alpha = K^-1 y (alpha_dev: n float64 in ORIGINAL order of
 * the training dataset): alpha in binned order and, per bump group i, the
 * coefficient c_i = sum_q f_i(x_q) alpha_q.  The training dataset must
 * outlive the predictor. */
GP_API gp_status gp_predictor_create(gp_ctx* ctx, const gp_dataset* train, const gp_theta* theta,
                              const double* alpha_dev, gp_predictor** out);
GP_API gp_status gp_predictor_destroy(gp_ctx* ctx, gp_predictor* p);

/* gp_predict: posterior mean m(x*) = sum_q C_y(x*, x_q) alpha_q (no nugget)
 * for m test points (xstar_dev: m x d row-major float64) into mean_dev (m
 * float64).  The cross-covariance is evaluated and applied in one pass and
 * never stored.  GP_MIXED evaluates each cross-covariance value in float64
 * (as the matrix's values are), rounds it to float32 and multiplies it by a
 * float32 copy of alpha in float32; the sum is float64.  Test
 * coordinates are device data and are not checked: a non-finite test point
 * passes no support test and gets mean 0.
 * Errors: GP_EINVAL (m < 0, NULL buffers, unknown precision), GP_EDEVICE. */
GP_API gp_status gp_predict(gp_ctx* ctx, const gp_predictor* p, int64_t m, const double* xstar_dev,
                     gp_precision prec, double* mean_dev);

/* gp_predict_batch: the kriging means of Sec. 3.2 for nreq requests in one
 * launch (Sec. 3.3: many prediction requests are served together).  Request
 * r asks for the mean of predictor preds[r] (host array of nreq pointers;
 * requests may share a predictor or use predictors of other hyper-parameters
 * or training datasets) at the rows row_offsets[r] .. row_offsets[r+1] - 1 of
 * xstar_dev (row_offsets: host array of nreq + 1 non-decreasing values,
 * row_offsets[0] = 0; empty requests allowed); xstar_dev (row_offsets[nreq] x d
 * row-major float64, device) and mean_dev (row_offsets[nreq] float64, device)
 * hold all requests' rows back to back.  Every row gets the value gp_predict
 * gives for it with the same predictor and precision.  All predictors must
 * share the dimension d and the core kernel kind.
 * Errors: GP_EINVAL (nreq < 0, NULL arguments, offsets not starting at 0 or
 * decreasing, mixed d or core kinds, unknown precision), GP_EDEVICE. */
GP_API gp_status gp_predict_batch(gp_ctx* ctx, int32_t nreq, const gp_predictor* const* preds,
                                  const int64_t* row_offsets, const double* xstar_dev, gp_precision prec,
                                  double* mean_dev);

/* gp_mean_residual: y = z - W beta, the residual of the prior mean
 * E[z] = W beta of Sec. 3.1 (Eq. Zmarg), the y_dev that gp_loglik and gp_solve
 * take.  W_dev: n x p covariates stored column by column (W[k * n + i] is
 * covariate k of point i, ORIGINAL point order), device; beta: p float64 in
 * host memory, copied by the call; z_dev, y_dev: n float64, device (y may
 * alias z).  p = 0 copies z.
 * Errors: GP_EINVAL (n < 1, p < 0, NULL buffers, non-finite beta), GP_EDEVICE. */
GP_API gp_status gp_mean_residual(gp_ctx* ctx, int64_t n, int32_t p, const double* W_dev, const double* beta,
                           const double* z_dev, double* y_dev);

/* gp_predict_var: posterior variance of the latent process at m test points
 * (Sec. 3.2: the diagonal of C_{y|z} = C_y - C_{y,z} C_z^{-1} C_{z,y}),
 *   var(x*) = C_y(x*, x*) - c^T K^{-1} c,   c = C_{z,y}(., x*)  (no nugget),
 * into var_dev (m float64, device).  K must have been assembled with theta
 * (checked against a fingerprint of every hyper-parameter except tau2, which
 * enters K only and is not read here).  The test points
 * (xstar_dev: m x d row-major float64, device) are taken 32 at a time: their
 * cross-covariance columns are formed on the device and K W = C is solved by
 * 32 preconditioned conjugate-gradient recurrences in lockstep (one sparse
 * product with 32 columns per step, float64 vectors, the matrix's stored
 * values; opts->precond: block Jacobi, the default, or Jacobi), each stopping
 * when |c_s - K w_s| <= opts->rtol |c_s|; a float64 true residual is taken at
 * the end.  opts may be NULL (defaults; rtol, max_iter and precond are used).
 * Work space: seven n x 32 float64 blocks.
 * out (may be NULL) receives iteration counts and the largest final relative
 * residual.
 * Errors: GP_EINVAL (theta differs from K's, m < 0, NULL buffers),
 * GP_ENOTCONV (a column missed rtol within max_iter steps; var holds the
 * last iterate's values), GP_ENOTPD, GP_ENOMEM, GP_EDEVICE. */
typedef struct gp_var_result {
  int64_t iters;            /* iterations summed over the batches */
  int32_t max_batch_iters;  /* most iterations of one batch */
  int32_t status;           /* gp_status */
  double relres;            /* largest final |c - K w| / |c| */
} gp_var_result;

GP_API gp_status gp_predict_var(gp_ctx* ctx, const gp_matrix* K, const gp_theta* theta, int64_t m,
                         const double* xstar_dev, const gp_solve_opts* opts, double* var_dev,
                         gp_var_result* out);

#ifdef __cplusplus
}
#endif
#endif /* GPSPARSE_H */
