/*
 * lsq2l -- two-level Schwarz preconditioned Krylov solvers for sparse linear
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
 *     M = R_0^T C_00^{-1} R_0 + sum_i R_i^T C_ii^{-1} R_i (eq. two_level_schwarz),
 *     and the variants of Section 2 (eqs. one_level_schwarz, RAS, balanced,
 *     deflated);
 *   - the Krylov methods: CG on the normal equations, left-preconditioned
 *     LSQR and right-preconditioned restarted GMRES (Section 4.1, "Solution
 *     phase").
 *
 * Conventions shared by every call:
 *   - All array pointers are DEVICE pointers unless the comment says "host".
 *   - A is CSR, 0-based: int64 row pointers, int32 column indices (strictly
 *     increasing in a row), double values; m, n and nnz must stay below 2^31.
 *     "Nonzero" means "stored": the sparsity pattern decides the index sets,
 *     whatever the stored values.
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
  LSQ2L_PCG_BREAKDOWN = -5     /* a Krylov breakdown: p^T C p <= 0, a non-finite scalar, or
                                  a zero norm in LSQR's bidiagonalization                    */
} lsq2l_status;

enum { LSQ2L_FP64 = 0, LSQ2L_MIXED = 1 };           /* lsq2l_options.precision */

/* lsq2l_options.variant (Q = R_0^T E^{-1} R_0 with E = R_0 C R_0^T in all):
 *   ADDITIVE:  M = M_ASM + Q (eq. two_level_schwarz), the default.
 *   ONE_LEVEL: M = M_ASM = sum_i R_i^T C_ii^{-1} R_i (eq. one_level_schwarz);
 *              no coarse space is computed.
 *   BALANCED:  M = Q + (I - C Q)^T M_ASM (I - C Q) (eq. balanced), the paper's
 *              pairing with LSQR; two coarse corrections and two products with
 *              C more per application.
 *   RAS:       M = M_RAS = sum_i R_i^T D_i C_ii^{-1} R_i (eq. RAS), one level,
 *              nonsymmetric (GMRES only).
 *   DEFLATED:  M = Q + M_RAS (I - C Q) (eq. deflated), the paper's pairing with
 *              GMRES; nonsymmetric (GMRES only).
 * ADDITIVE, BALANCED and DEFLATED share the setup; ONE_LEVEL and RAS skip the
 * coarse space. */
enum { LSQ2L_ADDITIVE = 0, LSQ2L_ONE_LEVEL = 1, LSQ2L_BALANCED = 2, LSQ2L_RAS = 3,
       LSQ2L_DEFLATED = 4 };

/* lsq2l_options.krylov (Section 4.1, "Solution phase"):
 *   PCG:   preconditioned CG on C x = A^T b, x_0 = 0; stops when the
 *          recurrence residual ||r_k|| <= tol ||A^T b||, then checks the true
 *          residual ||A^T (b - A x)|| <= tol ||A^T b|| and restarts from it
 *          (at most 3 times).  Symmetric variants only.
 *   LSQR:  left-preconditioned LSQR (Golub-Kahan bidiagonalization of
 *          A W^{-1} with M = W^{-1} W^{-T}, carried in the M^{-1} inner product
 *          so that only products with M are needed); stops when LSQR's own
 *          estimate of ||(A W^{-1})^T (A x - b)|| / (||A W^{-1}||_F ||A x - b||)
 *          falls below tol.  Symmetric variants only.
 *   GMRES: right-preconditioned restarted GMRES(restart) on C x = A^T b,
 *          x_0 = 0; stops when the (unpreconditioned) residual
 *          ||A^T b - C x|| <= tol ||A^T b||, checked on the true residual at
 *          every restart and at exit.  Any variant. */
enum { LSQ2L_PCG = 0, LSQ2L_LSQR = 1, LSQ2L_GMRES = 2 };

typedef struct {
  double  tol;        /* stopping tolerance of the Krylov method (default 1e-8)                  */
  int32_t max_it;     /* iteration limit (default 10000)                                          */
  int32_t precision;  /* LSQ2L_FP64: everything in double.  LSQ2L_MIXED: the local factors the
                         triangular solves use are computed in float (FP32 MFMA Cholesky of a
                         float copy of the equilibrated C_ii, FP32 accumulation) and the solves
                         run in float; the coarse restriction and prolongation read a float
                         copy of the (double) coarse basis (E is built from the double basis).
                         The coarse selection (eq. gevp), E, the coarse solve, recurrences, dot
                         products and residuals stay double.  If a float factorization meets a
                         non-positive pivot, every solve factor is computed in double and
                         rounded to float instead (lsq2l_setup_info.mixed_fallback = 1)        */
  int32_t flexible;   /* PCG: 1 = flexible beta = z_{k+1}^T (r_{k+1} - r_k) / (z_k^T r_k)        */
  int32_t variant;    /* LSQ2L_ADDITIVE, ONE_LEVEL, BALANCED, RAS or DEFLATED (above); a
                         nonsymmetric variant with PCG or LSQR returns LSQ2L_EINVAL              */
  int32_t nev_max;    /* keep at most this many coarse vectors per subdomain (0 = no cap)         */
  int32_t check_every;/* PCG: read the residual norm back every this many iterations (default 1) */
  int32_t use_graph;  /* PCG: 1 = capture one iteration (SpMVs, dot products, scalar updates,
                         M r) into a HIP graph per solve call and replay it; results are the
                         same as without (default 0)                                             */
  int32_t krylov;     /* LSQ2L_PCG (default), LSQ2L_LSQR or LSQ2L_GMRES                           */
  int32_t restart;    /* GMRES restart length (default 100, Section 4.2)                          */
  double  diag_shift_rel; /* s = diag_shift_rel * ||C||_F: the preconditioner is built for
                         C + s I (the least-squares matrix [A; sqrt(s) I]) and used on C, as in
                         Section 4.1 "Setup phase" (which uses 1e-10); default 0 = no shift     */
  double  adjoint_tol;/* tolerance of the adjoint solve of lsq2l_backward (0 = tol); see
                         lsq2l_backward for how it is applied                                    */
  int32_t autotune;   /* 1: time the candidate launch shapes of the SpMV on this matrix at setup
                         and keep the fastest (see lsq2l_autotune); 0 (default): the built-in
                         choice                                                                  */
  int32_t solve_order;/* order of Omega_i in the factors the local solves of M use (C_ii^{-1} r
                         does not depend on it): LSQ2L_ORDER_AUTO (default) takes, per
                         subdomain, the global-column order when its tile envelope is at most
                         0.85 of that of [Omega_Ii, Omega_Gamma_i] (the order the coarse
                         selection factors C_ii in); LSQ2L_ORDER_SPLIT keeps [Omega_Ii,
                         Omega_Gamma_i] everywhere, LSQ2L_ORDER_GLOBAL takes the global-column
                         order everywhere                                                      */
  int32_t local_factor;/* LSQ2L_FACTOR_CHOLESKY (default): local factors from the Cholesky
                         factorization of the assembled, equilibrated C_ii.  LSQ2L_FACTOR_QR:
                         C_ii is never formed (Remarks 3.1 and 3.2): every local factor is the
                         R of a thin Householder QR of the equilibrated A(:, Omega_i) (FP64;
                         rounded to float for the solves of LSQ2L_MIXED), and the coarse
                         selection takes the principal angles between range(A(Xi_i, Omega_Ii))
                         and range(A(Xi_i, Omega_Gamma_i)), the numerical range of the latter
                         from a column-pivoted QR of the R of A(Xi_i, Omega_Gamma_i); the
                         condition number of the local blocks is not squared on the way.  Not
                         with diag_shift_rel > 0 (LSQ2L_EINVAL); subdomains of up to 32,768
                         padded positions (else LSQ2L_CHOL_BREAKDOWN with a message)           */
} lsq2l_options;

enum { LSQ2L_ORDER_AUTO = 0, LSQ2L_ORDER_SPLIT = 1, LSQ2L_ORDER_GLOBAL = 2 };
enum { LSQ2L_FACTOR_CHOLESKY = 0, LSQ2L_FACTOR_QR = 1 };

typedef struct {
  int32_t iterations;     /* Krylov iterations performed (per instance for batched handles)  */
  int32_t restarts;       /* PCG: restarts from the true residual; GMRES: restart cycles      */
  double  relres;         /* true relative residual ||A^T(b - A x)|| / ||A^T b|| at exit;
                             for lsq2l_backward, ||g - C lambda|| / ||g||                     */
  double  relres_rec;     /* the method's own residual estimate at exit (PCG: recurrence
                             residual; LSQR: its normal-equation test quantity; GMRES: the
                             Hessenberg least-squares residual)                             */
  double  solve_ms;       /* wall time of the call                                          */
  double  backward_err;   /* lsq2l_backward: ||g - C lambda|| / (||C||_2 ||lambda|| + ||g||),
                             ||C||_2 from a power iteration; 0 for lsq2l_solve               */
} lsq2l_solve_info;

typedef struct {
  int64_t m, n, nnz;
  int32_t nparts;         /* number of subdomains (all instances of a batch)            */
  int32_t ninstances;     /* 1, or the batch size of lsq2l_setup_batched                */
  int64_t n0;             /* coarse dimension sum_i p_i                                  */
  int32_t max_ni;         /* largest overlapping subdomain |Omega_i|                     */
  int32_t max_p;          /* largest p_i                                                 */
  int64_t factor_bytes;   /* device bytes of the factors the local solves read (stored
                             tiles, float in LSQ2L_MIXED)                                */
  int64_t factor_dense_bytes; /* what dense lower-triangular local factors would take   */
  int64_t factor_tiles;   /* stored 32 x 32 tiles of the factors the local solves read   */
  int64_t factor_nnz_min; /* sum_i nnz(L_i): entries of the local Cholesky factors under
                             a fill-reducing order of each Omega_i, the fewest of a
                             nested-dissection order, the global column order and
                             [Omega_Ii, Omega_Gamma_i] (symbolic factorization; the
                             algorithmic minimum the local solves must read); -1 until
                             lsq2l_time_kernel computed it                               */
  double  shift;          /* s = diag_shift_rel ||C||_F actually applied (0 if none)     */
  double  t_plan_ms;      /* index sets, envelopes, transposition (host + device)        */
  double  t_assemble_ms;  /* local matrices C_ii, Ct_GG, equilibration                  */
  double  t_factor_ms;    /* batched local Cholesky                                      */
  double  t_eigen_ms;     /* coarse selection (reduced eigenproblems) and X_i            */
  double  t_coarse_ms;    /* W = A R_0^T, E = W^T W, Cholesky and inverse of E          */
  double  t_total_ms;     /* wall time of setup                                          */
  int32_t spmv_lanes_A;   /* SpMV shape used with A (see lsq2l_autotune)                    */
  int32_t spmv_lanes_AT;  /* the same for A^T                                              */
  double  t_prepare_ms;   /* reading, concatenating and validating the input (before
                             t_total_ms starts)                                         */
  int64_t split_tiles;    /* stored tiles of the factors in [Omega_Ii, Omega_Gamma_i] order
                             (the coarse selection's)                                   */
  int32_t solve_permuted; /* subdomains whose solve factor is in global-column order     */
  int32_t mixed_fallback; /* LSQ2L_MIXED: 1 if the solve factors were computed in double
                             after a float factorization broke down                     */
} lsq2l_setup_info;

/* One least-squares instance for lsq2l_setup_batched. */
typedef struct {
  int64_t m, n, nnz;
  const int64_t* rowptr;  /* device, m + 1 */
  const int32_t* colind;  /* device, nnz   */
  const double*  vals;    /* device, nnz   */
  const int32_t* part;    /* host or device, n: column partition, values in [0, nparts) */
  int32_t nparts;
  int32_t reserved;
} lsq2l_problem;

/* Fill *opt with the defaults listed above. */
void lsq2l_default_options(lsq2l_options* opt);

/*
 * Build the preconditioner (Algorithm 1) for the CSR matrix A and the column
 * partition part[0..n) (host or device array, detected from the pointer;
 * every part in [0, nparts) must be non-empty).  overlap must be 1 (the
 * one-layer overlap of Section 3); tau must lie in (0, 1] (coarse vectors are
 * the directions with lambda > 1/tau in eq. gevp).  A's arrays are copied:
 * the caller may free them afterwards.  Returns EINVAL on bad sizes,
 * partition or options, CHOL_BREAKDOWN if a local or the coarse matrix is not
 * numerically positive definite (e.g. A rank deficient and no shift).
 * opt may be NULL (defaults).  On success *out owns all derived device data.
 */
lsq2l_status lsq2l_setup(int64_t m, int64_t n, int64_t nnz,
                         const int64_t* rowptr, const int32_t* colind, const double* vals,
                         const int32_t* part, int32_t nparts, int32_t overlap, double tau,
                         const lsq2l_options* opt, void* hip_stream, lsq2l_handle* out);

/*
 * Several independent instances in one handle: their subdomains share the
 * batched local kernels, and one Krylov loop iterates all instances with
 * per-instance scalars and convergence (an instance that has converged stops
 * changing).  The instances are laid out back to back: rows of instance k
 * start at sum_{l<k} m_l, columns at sum_{l<k} n_l.
 */
lsq2l_status lsq2l_setup_batched(int32_t count, const lsq2l_problem* probs, double tau,
                                 const lsq2l_options* opt, void* hip_stream, lsq2l_handle* out);

/*
 * Solve min ||A x - b|| with the Krylov method of the options on C x = A^T b
 * (eq. normal) and the preconditioner of the handle.  b: device, m doubles;
 * x: device, n doubles (written).  For a batched handle, b and x are the
 * concatenations over the instances and info (if not NULL) points to
 * ninstances entries.  The handle keeps copies of b and x for
 * lsq2l_backward.  Returns NOT_CONVERGED (x = last iterate) when max_it is
 * reached, PCG_BREAKDOWN on a Krylov breakdown or NaN.
 */
lsq2l_status lsq2l_solve(lsq2l_handle h, const double* b, double* x, lsq2l_solve_info* info);

/*
 * lsq2l_solve for a batched handle with one right-hand side and one solution
 * buffer per instance: b[k] (device, m_k doubles) and x[k] (device, n_k
 * doubles, written) for k < ninstances; b and x are host arrays of device
 * pointers.  info (optional) receives ninstances entries.
 */
lsq2l_status lsq2l_solve_batched(lsq2l_handle h, const double* const* b, double* const* x,
                                 lsq2l_solve_info* info);

/*
 * Adjoint of the last solve for a loss L(x): g = dL/dx (device, n).  Solves
 * C lambda = g with the same preconditioner and Krylov method and writes
 * dL/db = A lambda (device, m) and dL/dvals (device, nnz, in the CSR order of
 * A): dL/dA_ij = r_i lambda_j - (A lambda)_i x_j with r = b - A x.  Either
 * output may be NULL.  The adjoint aims at ||g - C lambda|| <= t ||g||,
 * t = adjoint_tol (or tol); when rounding keeps it from that (CG after its
 * restarts, GMRES when a whole cycle no longer halves the residual, both
 * typical for kappa(C) near 1/(t eps)), it accepts lambda if the normwise
 * backward error ||g - C lambda|| / (||C||_2 ||lambda|| + ||g||) is at most t,
 * and returns NOT_CONVERGED otherwise.  ||C||_2 comes from 30 steps of the
 * power method on the first call.  info (optional) reports the adjoint
 * solve, with backward_err set.
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
 * 3 = dense coarse solve E^{-1} c, 4 = batched local triangular solves priced
 * at the algorithmic minimum (factor_nnz_min entries read per sweep).
 * Buffers are the handle's own work vectors; results are discarded.  EINVAL
 * for an unknown kernel or a kernel the handle does not use (3 without a
 * coarse space).
 */
lsq2l_status lsq2l_time_kernel(lsq2l_handle h, int32_t kernel, int32_t reps, double* avg_ms,
                               double* bytes);

/*
 * Autotuner of the SpMV launch shape (the CSR products of Section 4.1's
 * iteration): for y = A x and x = A^T y on the handle's own matrix, times
 * every candidate shape with HIP events over `reps` launches each and keeps
 * the fastest for all later products of the handle.  Shapes: -1 = row
 * blocks of about 1024 entries staged through LDS, one thread summing each
 * row; -2 = the same with non-temporal (streaming) loads of the matrix;
 * 0 = the built-in choice, -2 when the matrix arrays (12 bytes per entry)
 * exceed the 256 MB last-level cache and -1 otherwise; 1, 2, 4, ..., 64 =
 * that many lanes per row.  The tuner times -2, -1 and the lane counts.
 * lanes (host, 2 entries, for A and A^T) receives the chosen shapes; with
 * reps = 0 nothing is timed and the shapes are set from lanes instead
 * (EINVAL unless both are -2, -1, 0 or a power of two up to 64).  Results
 * depend on the shape only through the summation order inside a row.
 */
lsq2l_status lsq2l_autotune(lsq2l_handle h, int32_t reps, int32_t* lanes);

/*
 * Transpose of a CSR matrix on the device (the A^T of Section 4.1, formed
 * once per setup): the columns of A become the rows of A^T, with the rows of
 * each column in ascending order.  In: m, n, nnz < 2^31; rowptr (m + 1, int32),
 * colind (nnz), vals (nnz, may be NULL).  Out: trowptr (n + 1), trow (nnz,
 * row index of each entry of A^T), tvals (nnz, may be NULL), tperm (nnz, may
 * be NULL: the index in A of each entry of A^T).  Runs a counting sort
 * (column histogram, exclusive scan, scatter, per-column ordering) on
 * `hip_stream`; its work arrays (n + 1 counters and the scan's block sums)
 * are allocated and freed inside the call.  EINVAL on bad sizes or NULL
 * required pointers.  Column indices must lie in [0, n).
 */
lsq2l_status lsq2l_transpose(int32_t m, int32_t n, int32_t nnz, const int32_t* rowptr,
                             const int32_t* colind, const double* vals, int32_t* trowptr,
                             int32_t* trow, double* tvals, int32_t* tperm, void* hip_stream);

/*
 * lsq2l_transpose for callers that cannot allocate device memory (code that
 * must not call hipMalloc, e.g. tight serving loops or harnesses that forbid
 * it): the same arguments, results and errors, but the sort's work space
 * comes from a static per-device array of 104 MiB that the library holds
 * from its load until the process ends, and the call makes no allocation.
 * Limit: the work space must fit, which holds for nnz <= 2^23 and
 * n <= 2^23 (larger inputs return LSQ2L_EINVAL naming the bytes needed).
 * All calls on one device share that array: calls that overlap on one GPU
 * (several host threads or streams at once) race and must be serialized by
 * the caller.  The call synchronizes its stream (it reads back the column
 * check), so it cannot be captured into a HIP graph.
 */
lsq2l_status lsq2l_transpose_noalloc(int32_t m, int32_t n, int32_t nnz, const int32_t* rowptr,
                                     const int32_t* colind, const double* vals, int32_t* trowptr,
                                     int32_t* trow, double* tvals, int32_t* tperm,
                                     void* hip_stream);

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
