// Device-side data of a handle and the host launchers of every kernel.
#pragma once

#include "internal.hpp"

namespace lsq2l {

struct DevMatrix {            // A and its transpose (device copies owned by the handle)
  int32_t m = 0, n = 0;
  int64_t nnz = 0;
  int32_t* rowptr = nullptr;  // m + 1
  int32_t* colind = nullptr;  // nnz
  double* vals = nullptr;     // nnz
  int32_t* trowptr = nullptr; // n + 1
  int32_t* trow = nullptr;    // nnz
  double* tvals = nullptr;    // nnz
  int32_t* tperm = nullptr;   // nnz: A^T entry k is vals[tperm[k]]
  int spmv_group = 0;         // A x: 0 row blocks through LDS, else lanes per row
  int spmvt_group = 0;        // A^T y, the same
  int32_t* blk = nullptr;     // LDS row blocks of A (spmv_blocks(nnz) + 1)
  int32_t* tblk = nullptr;    // the same for A^T
};

struct DevPlan {              // subdomain layout (device copies of HostPlan)
  SubDesc* subs = nullptr;
  int32_t* omega = nullptr;
  int32_t* xi = nullptr;
  int32_t* part = nullptr;
  int32_t* locown = nullptr;
  int32_t* tileF = nullptr;
  int64_t* tileOff = nullptr;
  int32_t* own_ptr = nullptr;
  int32_t* own_pos = nullptr;
  int32_t* solve_order = nullptr;  // subdomains by decreasing stored factor tiles
  SubDesc* subs_ord = nullptr;     // subs in that order: the one-workgroup-per-subdomain
                                   // setup kernels start the largest subdomains first
  int max_np = 0;             // largest padded local size
  int min_nG = 0, max_nG = 0;  // least and largest interface size
  // layout of the solve factor only: where each position lives in the local
  // vectors (loc index, -1 on padding; null: loc_off + position), and
  // scratch local vectors for the subdomains solved in global memory
  int32_t* sperm = nullptr;
  double* yscratch = nullptr;
  const SubDesc* heavy() const { return subs_ord ? subs_ord : subs; }
};

struct DevCoarse {            // coarse space and coarse operator
  PairDesc* pairs = nullptr;
  int32_t* pair_rows = nullptr;   // (pos in Xi_i, pos in Xi_j) per shared row
  SegDesc* segs = nullptr;
  int32_t* eF = nullptr;          // envelope of E (tile rows, global coarse numbering)
  int64_t* eOff = nullptr;
  int32_t* e_seg_of_tile = nullptr;
  int32_t* erows = nullptr;       // per tile column K: tile rows I > K with F(I) <= K
  int64_t* eptr = nullptr;
  int32_t* einv_bin_ptr = nullptr;   // per workgroup of the inverse: its column blocks
  int32_t* einv_bin_cols = nullptr;
  int4* e_items = nullptr;        // (pair, row block, column block) work items of E
  double* e_part = nullptr;       // row partials of the symmetric coarse solve
  double* e_u = nullptr;          // column partials of the symmetric coarse solve, per chunk
  int4* e_chunks = nullptr;       // (tile column, first row tile, row tiles) per chunk
  int32_t* e_chunk_ptr = nullptr; // chunks of each tile column
  int e_nchunks = 0;
};

// row tiles per chunk of the symmetric coarse solve (one row per thread of
// a 256-thread workgroup)
constexpr int ESYM_ROWTILES = 8;

// --- device transpose of A (hand-written radix sort) ------------------------
size_t transpose_temp_bytes(int64_t nnz, int32_t n);
void launch_permute_rows(hipStream_t st, int32_t m, const int32_t* perm, const int32_t* rowptr,
                         const int32_t* colind, const double* vals, const int32_t* prowptr,
                         int32_t* pcolind, double* pvals);
// trowptr (n + 1), trow and tperm (nnz) written; tvals written if not null
// (vals must then be given); temp holds transpose_temp_bytes(nnz, n) bytes
hipError_t launch_transpose(hipStream_t st, int32_t m, int32_t n, int64_t nnz, const int32_t* rowptr,
                            const int32_t* colind, const double* vals, int32_t* trowptr,
                            int32_t* trow, double* tvals, int32_t* tperm, void* temp,
                            size_t temp_bytes);
// one instance of the input of a (batched) setup, with its first row,
// column and entry in the concatenation
struct InstDesc {
  const int64_t* rowptr;
  const int32_t* colind;
  const double* vals;
  int64_t m, n, nnz, r0, c0, e0;
};
enum { CSR_FIRST = 0, CSR_LAST, CSR_MONO, CSR_RANGE, CSR_ORDER, CSR_KINDS };
// the concatenated, checked CSR of all S instances (see k_concat_rows):
// rp (M + 1), ci and vals (NNZ), bad (CSR_KINDS smallest failing rows)
void launch_concat(hipStream_t st, int S, const InstDesc* d, int64_t M, int64_t NNZ, int32_t* rp,
                   int32_t* ci, double* vals, unsigned long long* bad);
// flag (one int32, device) = 1 if a column index lies outside [0, n)
void launch_check_cols(hipStream_t st, int64_t nnz, const int32_t* colind, int32_t n, int32_t* flag);

// --- sparse kernels -------------------------------------------------------
// group 0: row blocks staged through LDS (needs the block table blk of the
// matrix, else one lane per row), their loads streaming if the matrix is
// larger than the last-level cache; SPMV_ROWS_CACHED / SPMV_ROWS_STREAM: row
// blocks with cached / streaming loads; 1 .. 64: lanes per row
enum { SPMV_ROWS_CACHED = -1, SPMV_ROWS_STREAM = -2 };
void launch_spmv(hipStream_t st, int32_t nrows, const int32_t* rowptr, const int32_t* colind,
                 const double* vals, const double* x, double* y, int group, int64_t nnz,
                 const int32_t* blk);
// the LDS row blocks of a CSR matrix: spmv_blocks(nnz) blocks, described by
// a table of spmv_table_len(nnz) int32 (first row and its start, per block)
int64_t spmv_blocks(int64_t nnz);
int64_t spmv_table_len(int64_t nnz);
void launch_row_blocks(hipStream_t st, int32_t nrows, const int32_t* rowptr, int64_t nnz, int32_t* blk);
void launch_grad_vals(hipStream_t st, int32_t m, const int32_t* rowptr, const int32_t* colind,
                      const double* r, const double* lam, const double* Alam, const double* x,
                      double* out);

// --- vector / reduction kernels --------------------------------------------
constexpr int RED_BLOCKS = 256;   // partial sums per segment
void launch_dot(hipStream_t st, int S, const int64_t* seg_ptr, const double* a, const double* b,
                double* partial);
enum ScalarOp { OP_R0 = 0, OP_RHO_INIT = 1, OP_ALPHA = 2, OP_RNORM = 3, OP_BETA = 4 };
struct Scalars {
  double *rho, *alpha, *beta, *rn2, *r0n2, *pq;
  int32_t* done;      // 0 active, 1 converged, 2 breakdown
  int32_t* its;       // iterations of each instance (x updated while active)
};
void launch_scalar(hipStream_t st, int op, int S, const double* partial, const double* partial2,
                   Scalars sc, double tol2, int flexible);
void launch_axpy_xr(hipStream_t st, int64_t n, int S, const int64_t* seg_ptr, const double* alpha,
                    const double* p, const double* q, double* x, double* r);
void launch_xpby(hipStream_t st, int64_t n, int S, const int64_t* seg_ptr, const double* beta,
                 const double* z, double* p);
void launch_sub(hipStream_t st, int64_t n, const double* a, const double* b, double* out);
void launch_add(hipStream_t st, int64_t n, const double* a, const double* b, double* out);
void launch_fill(hipStream_t st, int64_t n, double v, double* out);
void launch_copy(hipStream_t st, int64_t n, const double* a, double* out);
// out_k = a_k * f[segment of k] (per-instance factors on the device)
void launch_scale_seg(hipStream_t st, int64_t n, int S, const int64_t* seg_ptr, const double* f,
                      const double* a, double* out);
void launch_fill_i32(hipStream_t st, int64_t n, int32_t v, int32_t* out);
// a fixed pseudo-random vector in [-1, 1) (start of the power method)
void launch_hash_fill(hipStream_t st, int64_t n, double* out);

// --- LSQR (left-preconditioned, M^{-1} inner product) ------------------------
// per-instance scalars, LSQR_NSC per instance at sc + s * LSQR_NSC
enum LsqrSc { LS_ALPHA = 0, LS_BETA, LS_RHOBAR, LS_PHIBAR, LS_ANORM2, LS_T1, LS_T2, LS_TEST,
              LS_RNORM0, LS_NSC };
constexpr int LSQR_NSC = LS_NSC;
enum LsqrOp { LSQR_INIT_BETA = 0, LSQR_INIT_ALPHA = 1, LSQR_BETA = 2, LSQR_ALPHA = 3 };
void launch_lsqr_scalar(hipStream_t st, int op, int S, const double* partial, double* sc,
                        int32_t* done, int32_t* its, double tol);
// u = a - alpha u (m-space, row segments; active instances only)
void launch_lsqr_u(hipStream_t st, int64_t m, int S, const int64_t* seg_row, const double* sc,
                   const int32_t* done, const double* a, double* u, int first);
// u *= 1 / beta (m-space)
void launch_lsqr_unorm(hipStream_t st, int64_t m, int S, const int64_t* seg_row, const double* sc,
                       const int32_t* done, double* u);
// q = q - beta zh (n-space)
void launch_lsqr_q(hipStream_t st, int64_t n, int S, const int64_t* seg_col, const double* sc,
                   const int32_t* done, const double* zh, double* q, int first);
// zh = q / alpha; v = s / alpha; x += t1 w; w = v + t2 w (first: w = v, x untouched)
void launch_lsqr_update(hipStream_t st, int64_t n, int S, const int64_t* seg_col, const double* sc,
                        const int32_t* done, const double* q, const double* s, double* zh,
                        double* v, double* w, double* x, int first);

// --- GMRES -------------------------------------------------------------------
// partial[(s * RED_BLOCKS + b) * ld + i] = chunk b of segment s of V_i . w, i < k
void launch_multidot(hipStream_t st, int S, const int64_t* seg_ptr, int64_t n, int k,
                     const double* V, const double* w, double* partial, int ld);
// h[s * ld + i] (+)= sum_b partial (fixed order), i < k
void launch_multidot_reduce(hipStream_t st, int S, int k, const double* partial, int ld,
                            double* h, int accumulate);
// w -= sum_{i<k} V_i h[s * ld + i]
void launch_multi_axpy(hipStream_t st, int S, const int64_t* seg_ptr, int64_t n, int k,
                       const double* V, const double* h, int ld, double* w);
// out = sum_{i<k} V_i y[s * ld + i]
void launch_multi_gemv(hipStream_t st, int S, const int64_t* seg_ptr, int64_t n, int k,
                       const double* V, const double* y, int ld, double* out);
// out_k = a_k / sqrt(nrm2[segment]) (0 where the norm is zero or the instance is done)
void launch_normalize_seg(hipStream_t st, int64_t n, int S, const int64_t* seg_ptr,
                          const double* nrm2, const int32_t* done, const double* a, double* out);
// norm2[s] = sum_b partial[s * RED_BLOCKS + b]
void launch_seg_sum(hipStream_t st, int S, const double* partial, double* out);

// --- subdomain kernels -------------------------------------------------------
void launch_gather_values(hipStream_t st, int64_t nnz, const int32_t* perm, const double* src,
                          double* dst);
// with inv (not null), also the tile envelope Fg of the global-order
// layouts gsub (Fg set by launch_solve_env_init first)
// scale non-null: assemble S C_ii S and S Ct_GG S directly (S = scale, from
// launch_col_scale), identity on the padding diagonal
void launch_assemble(hipStream_t st, int nsub, const DevPlan& P, const DevMatrix& M, double* fac,
                     double* ctg, const int32_t* inv = nullptr, const SubDesc* gsub = nullptr,
                     int32_t* Fg = nullptr, const double* scale = nullptr);
void launch_equilibrate(hipStream_t st, int nsub, const DevPlan& P, double* fac, double* ctg,
                        double* scale);
// interior_only: factor the interior tile columns only (L_I and L_GI)
void launch_chol_local(hipStream_t st, int nsub, const DevPlan& P, double* fac, double* dinv,
                       int32_t* status, bool interior_only = false);
// the same in FP32 (FP32 MFMA, FP32 accumulation)
void launch_chol_local_f32(hipStream_t st, int nsub, const DevPlan& P, float* fac, float* dinv,
                           int32_t* status);
// solve factor in the global-column order of each subdomain: inv (indexed
// like loc) maps an [I, Gamma] position to its global-order position;
// gsub describes the global-order layout (np, ntiles, tile_base); Fg,
// initialized here to the diagonal, gets its tile envelope from the assembly
void launch_solve_inv(hipStream_t st, int nsub, const DevPlan& P, int32_t* inv);
void launch_solve_env_init(hipStream_t st, int nsub, const SubDesc* gsub, int32_t* Fg);
// Ps.sperm (filled with -1 first) from the chosen layouts (ssub.spare set:
// global order)
void launch_solve_perm(hipStream_t st, int nsub, const DevPlan& P, const SubDesc* ssub,
                       const int32_t* inv, int32_t* sperm);
// the solve layout's matrix (double) from the assembled, equilibrated C_ii
void launch_gather_solve(hipStream_t st, int nsub, const DevPlan& P, const DevPlan& Ps,
                         const double* fac, double* out);
void launch_to_float(hipStream_t st, int64_t n, const double* src, float* dst);
void launch_gather_local(hipStream_t st, int nsub, const DevPlan& P, const double* scale,
                         const double* r, double* loc);
void launch_local_solve(hipStream_t st, int nsub, const DevPlan& P, const double* fac,
                        const double* dinv, double* loc);
void launch_local_solve_f32(hipStream_t st, int nsub, const DevPlan& P, const float* fac,
                            const float* dinv, double* loc);
// allows the streaming local solve its dynamic LDS (once per process)
hipError_t local_solve_configure();
// restricted: each column takes its owner's interior value only (R_i^T D_i, eq. RAS)
void launch_scatter_local(hipStream_t st, int32_t n, const DevPlan& P, const double* scale,
                          const double* loc, const double* X, const double* dcoarse, double* z,
                          bool restricted = false);
void launch_scatter_local(hipStream_t st, int32_t n, const DevPlan& P, const double* scale,
                          const double* loc, const float* X, const double* dcoarse, double* z,
                          bool restricted = false);
// ||C(Omega_Ii, :)||_F^2 of every subdomain from the assembled (unscaled) C_ii
void launch_frob_interior(hipStream_t st, int nsub, const DevPlan& P, const double* fac,
                          double* out);
// C_ii += s I on the real (non-padding) positions
void launch_add_diag(hipStream_t st, int nsub, const DevPlan& P, double s, double* fac);

// --- local factors from thin QR factorizations (k_qr.hip) --------------------
// QR_SEL: L_I and L_GI of the layout P from the rows Xi_i (out = fac, dinv);
// QR_SOLVE: the whole factor of C_ii in the layout Lay (the solve layout, inv
// the [I, Gamma] -> global-order position map of its permuted subdomains);
// QR_GAMMA: R_G of A(Xi_i, Omega_Gamma_i) into the dense interface matrices
// (out = ctg, zeroed by the caller).  The factor arrays must be zero on
// entry; strip holds 32 * total_loc doubles, zero on entry and on return;
// qscr holds 2 total_loc + nsub int32 (row-stream tables).
// status: first failing subdomain + 1 (zero or non-finite diagonal, or a
// layout beyond the kernel's tables).
enum { QR_SEL = 0, QR_SOLVE = 1, QR_GAMMA = 2 };
constexpr int QR_STRIP_ROWS = 32;
void launch_qr_local(hipStream_t st, int mode, int nsub, const DevPlan& P, const DevPlan& Lay,
                     const DevMatrix& M, const int32_t* inv, const double* scale, double* out,
                     double* dinv, double* strip, int32_t* qscr, int64_t total_loc, int32_t* status);
// scale = 1 / ||A(:, c)|| per position of the layout P (0 on padding)
void launch_col_scale(hipStream_t st, int nsub, const DevPlan& P, const DevMatrix& M, double* scale);

// --- coarse space ------------------------------------------------------------
void launch_gamma_T(hipStream_t st, int nsub, const DevPlan& P, const double* fac, double* Tg);
// ld x ld work matrices per subdomain of the selection (work holds
// SEL_WORK_MATS * total_g doubles; Y, the selected vectors, is the first)
constexpr int SEL_WORK_MATS = 5;
// qr_range: ctg holds the interface factors R_G of the QR route (k_qr.hip)
// instead of Ct_GG, and the range basis comes from a pivoted QR of them
void launch_select(hipStream_t st, int nsub, const DevPlan& P, const double* ctg, const double* Tg,
                   double* work, double tau, int nev_max, int32_t* p_out, double* sig_out,
                   int qr_range = 0);
void launch_coarse_X(hipStream_t st, int nsub, const DevPlan& P, const double* fac,
                     const double* dinv, const double* scale, const double* work,
                     const double* sig, double* X);
void launch_coarse_W(hipStream_t st, int nsub, const DevPlan& P, const DevMatrix& M,
                     const double* X, double* W);
void launch_coarse_E(hipStream_t st, int nitems, const DevPlan& P, const DevCoarse& Cc,
                     const double* W, double* efac);
// diagonal blocks of E += s X_i^T X_i (the rows sqrt(s) e_j of a shifted C)
void launch_coarse_E_shift(hipStream_t st, int nitems, const DevPlan& P, const DevCoarse& Cc,
                           const double* X, double s, double* efac);
// one step of the tile Cholesky of E for a list of independent diagonal
// blocks (jobs of EJOB_INTS ints, see k_echol_step); echol_job_blocks gives
// the workgroups one job takes
constexpr int EJOB_INTS = 6;
int echol_job_blocks(int nr, int npr);
void launch_echol_step(hipStream_t st, const DevCoarse& Cc, const int32_t* jobs, int njobs,
                       int nblocks, double* efac, double* edinv, int32_t* status);
void launch_tile_transpose(hipStream_t st, int64_t ntiles, const double* in, double* out);
void launch_einv(hipStream_t st, int nbins, const DevCoarse& Cc, const double* efac,
                 const double* edinv, const double* efacT, const double* edinvT, double* einv);
void launch_coarse_restrict(hipStream_t st, int nsub, const DevPlan& P, int max_p, const double* X,
                            const double* r, double* c);
void launch_coarse_restrict(hipStream_t st, int nsub, const DevPlan& P, int max_p, const float* X,
                            const double* r, double* c);
void launch_set_values(hipStream_t st, int64_t n, const int64_t* idx, double v, double* out);
void launch_einv_gemv(hipStream_t st, int64_t n0, int S, const DevCoarse& Cc, const double* einv,
                      const double* c, double* d);

}  // namespace lsq2l
