/*
 * lsq2l -- two-level additive Schwarz preconditioned CG for sparse linear
 * least squares, min ||A x - b||_2 (A is m x n, m >= n), on one MI355X.
 *
 * The method is that of Al Daas, Jolivet and Scott, "A robust algebraic
 * domain decomposition preconditioner for sparse normal equations":
 *   - the normal equations C x = A^T b, C = A^T A (Section 1, eq. normal);
 *   - overlapping column subdomains Omega_i = [Omega_Ii, Omega_Gamma_i] built
 *     from a given column partition (Section 3, eq. reorderedA; Algorithm 1);
 *   - local matrices C_ii = A(:,Omega_i)^T A(:,Omega_i) and local SPSD
 *     splittings Ct_ii = A(Xi_i,Omega_i)^T A(Xi_i,Omega_i) (eq. spsd_normal_eq);
 *   - a coarse space from the generalized eigenproblems of Lemma 2.4 /
 *     eq. (gevp) thresholded by tau, and the coarse matrix
 *     C_00 = (A R_0^T)^T (A R_0^T) (Algorithm 1);
 *   - the two-level additive preconditioner
 *     M = R_0^T C_00^{-1} R_0 + sum_i R_i^T C_ii^{-1} R_i (eq. two_level_schwarz).
 *
 * Conventions shared by every call:
 *   - All array pointers are DEVICE pointers unless the comment says "host".
 *   - A is CSR, 0-based, int32 indices, strictly increasing columns in a row,
 *     nnz < 2^31.  "Nonzero" means "stored": the sparsity pattern decides the
 *     index sets, whatever the stored values.
 *   - Every device operation is enqueued on the HIP stream given at setup
 *     (NULL = the default stream).  Calls return after the work they launch
 *     has finished, unless stated otherwise.
 *   - Errors are returned as status codes; nothing is thrown across the ABI.
 *     lsq2l_last_error() describes the last failure of the calling thread.
 *   - A handle is not thread-safe: one caller at a time per handle.
 */
#ifndef LSQ2L_H
#define LSQ2L_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lsq2l_ctx* lsq2l_handle;

typedef enum {
  LSQ2L_OK = 0,
  LSQ2L_NOT_CONVERGED = 1,     /* max_it reached: x holds the last iterate, info is valid   */
  LSQ2L_EINVAL = -1,           /* bad argument (sizes, partition, tau, options)             */
  LSQ2L_ENOMEM = -2,           /* a device or host allocation failed                        */
  LSQ2L_EHIP = -3,             /* a HIP runtime call failed                                 */
  LSQ2L_CHOL_BREAKDOWN = -4,   /* a local or coarse Cholesky met a non-positive pivot       */
  LSQ2L_PCG_BREAKDOWN = -5     /* p^T C p <= 0 or a non-finite scalar in the iteration      */
} lsq2l_status;

enum { LSQ2L_FP64 = 0, LSQ2L_MIXED = 1 };           /* lsq2l_options.precision */
/* lsq2l_options.variant.  ADDITIVE: M = M_ASM + Q (eq. two_level_schwarz).
 * ONE_LEVEL: M = M_ASM (eq. one_level_schwarz), no coarse space is computed.
 * BALANCED: M = Q + (I - C Q)^T M_ASM (I - C Q) (eq. balanced), the paper's
 * choice in practice with M_ASM; same setup as ADDITIVE, and each application
 * costs two coarse corrections and two products with C = A^T A more.
 * Q = R_0^T E^{-1} R_0 with E = R_0 C R_0^T in all three. */
enum { LSQ2L_ADDITIVE = 0, LSQ2L_ONE_LEVEL = 1, LSQ2L_BALANCED = 2 };

typedef struct {
  double  tol;        /* stop when ||A^T(b - A x)||_2 <= tol ||A^T b||_2 (default 1e-8)          */
  int32_t max_it;     /* PCG iteration limit (default 10000)                                      */
  int32_t precision;  /* LSQ2L_FP64: everything in double.  LSQ2L_MIXED: the local triangular
                         solves read a float copy of the (double) local factors, and the coarse
                         restriction and prolongation a float copy of the (double) coarse basis
                         (E is built from the double basis); all accumulation, recurrences, dot
                         products, residuals and the coarse solve stay double                   */
  int32_t flexible;   /* 1: flexible PCG, beta = z_{k+1}^T (r_{k+1} - r_k) / (z_k^T r_k)          */
  int32_t variant;    /* LSQ2L_ADDITIVE (two-level, default), LSQ2L_ONE_LEVEL (M_ASM) or
                         LSQ2L_BALANCED (eq. balanced); any other value returns LSQ2L_EINVAL    */
  int32_t nev_max;    /* keep at most this many coarse vectors per subdomain (0 = no cap)         */
  int32_t check_every;/* read the residual norm back every this many iterations (default 1)       */
  int32_t use_graph;  /* 1: capture one PCG iteration (SpMVs, dot products, scalar updates, M r)
                         into a HIP graph per solve call and replay it; results are the same as
                         without (default 0)                                                    */
} lsq2l_options;

typedef struct {
  int32_t iterations;     /* PCG iterations performed                                    */
  int32_t restarts;       /* restarts from the true residual (at most 3)                  */
  double  relres;         /* true relative residual ||A^T(b - A x)|| / ||A^T b|| at exit  */
  double  relres_rec;     /* recurrence residual at exit                                  */
  double  solve_ms;       /* wall time of the call                                        */
} lsq2l_solve_info;

typedef struct {
  int64_t m, n, nnz;
  int32_t nparts;         /* number of subdomains (all instances of a batch)            */
  int32_t ninstances;     /* 1, or the batch size of lsq2l_setup_batched                */
  int64_t n0;             /* coarse dimension sum_i p_i                                  */
  int32_t max_ni;         /* largest overlapping subdomain |Omega_i|                     */
  int32_t max_p;          /* largest p_i                                                 */
  int64_t factor_bytes;   /* device bytes of the local factors (stored tiles)            */
  int64_t factor_dense_bytes; /* what dense lower-triangular local factors would take   */
  int64_t factor_tiles;   /* number of stored 32 x 32 factor tiles                       */
  double  t_plan_ms;      /* index sets, envelopes, transposition (host + device)        */
  double  t_assemble_ms;  /* local matrices C_ii, Ct_GG, equilibration                  */
  double  t_factor_ms;    /* batched local Cholesky                                      */
  double  t_eigen_ms;     /* coarse selection (reduced eigenproblems) and X_i            */
  double  t_coarse_ms;    /* W = A R_0^T, E = W^T W, Cholesky and inverse of E          */
  double  t_total_ms;     /* wall time of setup                                          */
} lsq2l_setup_info;

/* One least-squares instance for lsq2l_setup_batched (device arrays except part). */
typedef struct {
  int32_t m, n, nnz;
  const int32_t* rowptr;  /* device, m + 1 */
  const int32_t* colind;  /* device, nnz   */
  const double*  vals;    /* device, nnz   */
  const int32_t* part;    /* host, n: column partition, values in [0, nparts) */
  int32_t nparts;
} lsq2l_problem;

/* Fill *opt with the defaults listed above. */
void lsq2l_default_options(lsq2l_options* opt);

/*
 * Build the preconditioner (Algorithm 1) for the CSR matrix A and the column
 * partition part[0..n) (host array; every part in [0, nparts) must be
 * non-empty).  overlap must be 1 (the one-layer overlap of Section 3); tau
 * must lie in (0, 1] (coarse vectors are the directions with lambda > 1/tau
 * in eq. gevp).  A's arrays are copied: the caller may free them afterwards.
 * Returns EINVAL on bad sizes or partition, CHOL_BREAKDOWN if a local or the
 * coarse matrix is not numerically positive definite (e.g. A rank deficient).
 * opt may be NULL (defaults).  On success *out owns all derived device data.
 */
lsq2l_status lsq2l_setup(int32_t m, int32_t n, int32_t nnz,
                         const int32_t* rowptr, const int32_t* colind, const double* vals,
                         const int32_t* part, int32_t nparts, int32_t overlap, double tau,
                         const lsq2l_options* opt, void* hip_stream, lsq2l_handle* out);

/*
 * Several independent instances in one handle: their subdomains share the
 * batched local kernels, and one PCG iterates all instances with per-instance
 * scalars and convergence (an instance that has converged stops changing).
 * The instances are laid out back to back: rows of instance k start at
 * sum_{l<k} m_l, columns at sum_{l<k} n_l.
 */
lsq2l_status lsq2l_setup_batched(int32_t count, const lsq2l_problem* probs, double tau,
                                 const lsq2l_options* opt, void* hip_stream, lsq2l_handle* out);

/*
 * Solve min ||A x - b|| with PCG on C x = A^T b, x_0 = 0 (eq. normal, two-level
 * preconditioner).  b: device, m doubles; x: device, n doubles (written).
 * For a batched handle, b and x are the concatenations over the instances and
 * info (if not NULL) points to ninstances entries.  The handle keeps copies of
 * b and x for lsq2l_backward.  Returns NOT_CONVERGED (x = last iterate) when
 * max_it is reached, PCG_BREAKDOWN on a non-positive curvature or NaN.
 */
lsq2l_status lsq2l_solve(lsq2l_handle h, const double* b, double* x, lsq2l_solve_info* info);

/*
 * Adjoint of the last solve for a loss L(x): g = dL/dx (device, n).  Solves
 * C lambda = g with the same preconditioner and writes dL/db = A lambda
 * (device, m) and dL/dvals (device, nnz, in the CSR order of A):
 * dL/dA_ij = r_i lambda_j - (A lambda)_i x_j with r = b - A x.  Either output
 * may be NULL.  info (optional) reports the adjoint PCG.
 */
lsq2l_status lsq2l_backward(lsq2l_handle h, const double* g, double* dLdb, double* dLdvals,
                            lsq2l_solve_info* info);

/* y = A x (trans = 0; x has n, y has m entries) or y = A^T x (trans = 1), device. */
lsq2l_status lsq2l_spmv(lsq2l_handle h, int32_t trans, const double* x, double* y);

/* z = M r with the preconditioner of the handle (device, n entries each).
 * z may be r itself. */
lsq2l_status lsq2l_apply_preconditioner(lsq2l_handle h, const double* r, double* z);

/* Sizes and phase timings of the setup. */
lsq2l_status lsq2l_get_info(lsq2l_handle h, lsq2l_setup_info* out);

/*
 * Index sets of subdomain i (host outputs, each may be NULL): sizes[0..3] =
 * {n_Ii, |Xi_i|, n_Gamma_i, p_i}; interior, xi, gamma receive Omega_Ii, Xi_i,
 * Omega_Gamma_i in ascending order (global 0-based indices; for a batch,
 * indices of the concatenated problem).
 */
lsq2l_status lsq2l_get_subdomain(lsq2l_handle h, int32_t i, int32_t* sizes,
                                 int32_t* interior, int32_t* xi, int32_t* gamma);

/*
 * Coarse basis of subdomain i: X_i (host output, n_Ii x p_i, column-major),
 * the interior block of R_i^T D_i Z_i, normalised so that X_i^T C_I X_i = I.
 */
lsq2l_status lsq2l_get_coarse_basis(lsq2l_handle h, int32_t i, double* X);

/*
 * Profiling hook: launch one hot-path kernel `reps` times on the handle's
 * stream between two HIP events and report the mean duration per launch
 * (*avg_ms) and the algorithmic HBM bytes one launch must move (*bytes).
 * kernel: 0 = y = A x, 1 = x = A^T y (CSR SpMV), 2 = batched local
 * triangular solves of the preconditioner (precision of the handle),
 * 3 = dense coarse solve E^{-1} c.  Buffers are the handle's own work
 * vectors; results are discarded.  EINVAL for an unknown kernel or a kernel
 * the handle does not use (3 without a coarse space).
 */
lsq2l_status lsq2l_time_kernel(lsq2l_handle h, int32_t kernel, int32_t reps, double* avg_ms,
                               double* bytes);

/* Release every resource of the handle (NULL is ignored).  Its device
 * memory goes to a process-wide cache (at most 32 GiB) that later handles on
 * the same device draw from. */
void lsq2l_destroy(lsq2l_handle h);

/* Free the device memory held in that cache, and the pinned host buffers
 * (at most 4 GiB) that setups keep for reading A's pattern back.  Handles
 * that are still alive keep theirs.  Call it with no setup running in
 * another thread. */
void lsq2l_release_cache(void);

/* Message of the last error on the calling thread ("" if none). */
const char* lsq2l_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LSQ2L_H */
