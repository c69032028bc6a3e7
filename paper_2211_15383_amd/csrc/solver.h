// Internal solver interfaces (V-cycle, Krylov pieces, level solves).
#pragma once

#include "common.h"

struct Workspace {
  std::map<std::string, DevBuf> bufs;
};

// Named scratch buffer of a hierarchy, kept between calls and grown on demand.  A
// pointer stays valid until the same (name, level) is requested with a larger size.
void* hier_buf(dmlmc_hier* H, const char* name, int level, size_t bytes);

DevBuf& hier_devbuf(dmlmc_hier* H, const char* name, int level);
// Largest Krylov basis (vectors) the fused Gram-Schmidt passes accept.
int gs_max_basis();

struct KrylovArrays {
  int m = 0, hld = 0;
  c128* H = nullptr;     // [nrhs][m][m+1] (column-major per RHS)
  double* cs = nullptr;  // [nrhs][m]
  c128* sn = nullptr;    // [nrhs][m]
  c128* g = nullptr;     // [nrhs][m+1]
  c128* h1 = nullptr;    // [nrhs][m+1]
  c128* h2 = nullptr;    // [nrhs][m+1]
  c128* y = nullptr;     // [nrhs][m]
  double* nrm2 = nullptr;
  double* res = nullptr;
  double* invb = nullptr;
};
KrylovArrays krylov_arrays(dmlmc_hier* H, const char* prefix, int level, int m, int nrhs);
void krylov_init(dmlmc_ctx* ctx, const KrylovArrays& k, int nrhs);
template <typename RV>
void arnoldi_step(dmlmc_ctx* ctx, Cx<RV>* V, c128* w, int j, int64_t n, int nrhs, const KrylovArrays& k);
// Single-pass form: unnormalised complex-FP32 basis u_i with scales s_i = 1/||u_i||
// (scale[i][nrhs]); the new vector is wscale[r] * w (wscale NULL: factor 1), w complex
// FP32 or FP64; FP64 arithmetic.
template <typename RW>
void arnoldi_step_cgs1(dmlmc_ctx* ctx, c64* U, double* scale, const Cx<RW>* w, int j, int64_t n, int nrhs,
                       const KrylovArrays& k, const double* wscale = nullptr);
void krylov_solution(dmlmc_ctx* ctx, const KrylovArrays& k, int iters, int nrhs);
// y[r][i] *= scale[i][r] for i < iters
void krylov_scale_y(dmlmc_ctx* ctx, const KrylovArrays& k, const double* scale, int iters, int nrhs);
template <typename RZ, typename RX>
// x = sum_i y_i Z_i, or x += sum_i y_i Z_i (in FP64) when accumulate
void launch_combine(dmlmc_ctx* ctx, const Cx<RZ>* Z, int iters, const KrylovArrays& k, Cx<RX>* x, int64_t n, int nrhs,
                    bool accumulate);
template <typename RV>
void launch_scale_store(dmlmc_ctx* ctx, const c128* w, const double* invb, Cx<RV>* v, int64_t n, int nrhs);

template <typename R>
void vcycle(dmlmc_hier* H, int l, const Cx<R>* b, Cx<R>* x, int nrhs);
template <typename R>
void smooth(dmlmc_hier* H, int l, Cx<R>* x, const Cx<R>* b, int nrhs, int sweeps);

struct SolveResult {
  int iters = 0;
  int ir_steps = 0;
  bool converged = false;
  double relres_max = 0.0;
};
// Solves D_l X = B (device FP64 [nrhs][n_l]); X overwritten.
SolveResult solve_level(dmlmc_hier* H, int l, const c128* B, c128* X, int nrhs, dmlmc_precision prec, double rtol,
                        int maxiter);
