// Internal deflation interfaces.
#pragma once

#include "common.h"

struct EigResult {
  int iters = 0;
  bool converged = false;
  int64_t degree_sum = 0;      // Chebyshev degrees summed over the outer steps
  double max_residual = 0.0;   // max ||Q x - lambda x|| / ||Q||_bound over the wanted pairs
  std::vector<double> lambda;  // signed eigenvalues, ordered by |lambda| then lambda
};

// k eigenpairs of Q = Gamma5 D_level with the smallest |lambda|; X written to Xout [k][n].
EigResult eig_coarsest(dmlmc_hier* H, int level, int k, double tol, c128* Xout);
// k eigenpairs of J = Q_a^-1 - P_ab Q_b^-1 P_ab^H (P_ab = P_a ... P_{b-1}) with the largest
// |lambda| (ties: lambda descending), by block Davidson with exact residual expansion;
// the solves inside J use solve_level (precision prec, tolerance solve_rtol).  X written
// to Xout [k][n_a].
EigResult eig_difference(dmlmc_hier* H, int a, int b, int k, double tol, double solve_rtol, dmlmc_precision prec,
                         c128* Xout);
// Re sum_i x_i^H Gamma5 (J x_i) for the deflation's vectors, J applied with solves to rtol
// (the small trace term of an inexact deflation).
double difference_trace_term(dmlmc_hier* H, const dmlmc_defl* D, dmlmc_precision prec, double rtol);
// W = J V for nv vectors (device [nv][n_a], FP64)
void apply_J(dmlmc_hier* H, int a, int b, const c128* V, c128* W, int nv, dmlmc_precision prec, double rtol);
// W = Gamma5 X (FP64 and FP32 copies) and the trace term from D->X64 and D->lambda (kind 0:
// sum x^H Gamma5 x / lambda; kind 1: sum lambda x^H Gamma5 x).
void defl_finish(dmlmc_hier* H, dmlmc_defl* D);
// C[r][i] = <w_i, x_r> and X <- X - W C
void defl_coeffs_fp64(dmlmc_ctx* ctx, const dmlmc_defl* D, const c128* X, int b, int64_t ldx, c128* C);
void defl_project_fp64(dmlmc_ctx* ctx, const dmlmc_defl* D, c128* X, int b, int64_t ldx, const c128* C);
void defl_coeffs_mfma(dmlmc_ctx* ctx, const dmlmc_defl* D, const c128* X, int b, int64_t ldx, c128* C,
                      DevBuf& scratch);
void defl_project_mfma(dmlmc_ctx* ctx, const dmlmc_defl* D, const c128* X, c128* Y, int b, int64_t ldx, int64_t ldy,
                       const c128* C);
// Y = X - W (W^H X) for b unpadded RHS ([b][n], X and Y disjoint) on the matrix cores, as
// defl_coeffs_mfma + defl_project_mfma, with the K-chunk partials and C placed in `part`
// (defl_project_scratch_entries complex128 entries, fully overwritten): no allocation and no
// timing events.
size_t defl_project_scratch_entries(const dmlmc_defl* D, int b);
void defl_project_mfma_into(hipStream_t stream, const dmlmc_defl* D, const c128* X, c128* Y, int b, c128* part);
// b -> (r, e0) with C = W^H b, r = b - W C = b - D e0, e0 = X Lambda^-1 C (exact inverse on
// the deflation space), for a deflated coarsest-level solve; FP32 matrix cores for MIXED.
void defl_coarse_split(dmlmc_hier* H, const dmlmc_defl* D, const c128* b, int nrhs, c128* r, c128* e0,
                       dmlmc_precision prec);
// X <- (I - W W^H) X; FP64 kernels for DMLMC_FP64, FP32 matrix-core kernels for DMLMC_MIXED.
void defl_apply(dmlmc_hier* H, const dmlmc_defl* D, c128* X, int b, int64_t ldx, dmlmc_precision prec);
