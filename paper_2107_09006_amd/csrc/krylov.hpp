// Krylov drivers on the normal equations C x = A^T b (eq. normal) and the
// operator products they share (defined in api.cpp and krylov.cpp).
#pragma once

#include <vector>

#include "ctx.hpp"

namespace lsq2l {

struct KrylovResult {
  std::vector<int32_t> its;          // iterations per instance
  std::vector<double> relres;        // true ||rhs - C x|| / ||rhs|| per instance
  std::vector<double> relres_rec;    // the method's own residual estimate
  std::vector<double> backward_err;  // adjoint: normwise backward error
  std::vector<int32_t> converged;
  int restarts = 0;
  int total_its = 0;
};

// products (api.cpp)
void spmv_it_A(lsq2l_ctx* c, const double* x, double* y);
void spmv_it_AT(lsq2l_ctx* c, const double* y, double* x);
void spmv_A(lsq2l_ctx* c, const double* x, double* y);
void spmv_AT(lsq2l_ctx* c, const double* y, double* x);
void apply_C(lsq2l_ctx* c, const double* x, double* y, double* tmp);
void apply_M(lsq2l_ctx* c, const double* r, double* z);
void local_solves(lsq2l_ctx* c);
lsq2l_status read_seg_sums(lsq2l_ctx* c, const double* partial, std::vector<double>& out);
lsq2l_status true_residual(lsq2l_ctx* c, const double* x, std::vector<double>& rel,
                           std::vector<double>* x2);
lsq2l_status norm_C(lsq2l_ctx* c);

// CG (api.cpp): x_0 = 0 on C x = c->rhs
lsq2l_status pcg(lsq2l_ctx* c, double* x, bool adjoint, double tol, KrylovResult& res);
// left-preconditioned LSQR on min ||A x - b|| (krylov.cpp); b is m doubles
lsq2l_status lsqr(lsq2l_ctx* c, const double* b, double* x, double tol, KrylovResult& res);
// right-preconditioned GMRES(restart) on C x = c->rhs (krylov.cpp)
lsq2l_status gmres(lsq2l_ctx* c, double* x, bool adjoint, double tol, KrylovResult& res);
// work vectors of the method chosen in c->opt (krylov.cpp)
lsq2l_status krylov_alloc(lsq2l_ctx* c);
// sum_i nnz(L_i) under a fill-reducing order of Omega_i (the best of nested
// dissection, the global column order and [Omega_Ii, Omega_Gamma_i])
// (symbolic factorization on the host, krylov.cpp); cached in c->fac_nnz_min
lsq2l_status factor_nnz_min(lsq2l_ctx* c);

}  // namespace lsq2l
