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
// FP32 or FP64; FP64 arithmetic.  U and w hold RHS r at r * ld (ld = 0: n), basis vector
// i at i * nrhs * ld.
// dots_G > 0: the dots were already formed as dots_G block partials per RHS in the buffer
// gs_partials returns (launch_wilson_dots); only their sums and the update remain.
template <typename RW>
void arnoldi_step_cgs1(dmlmc_ctx* ctx, c64* U, double* scale, const Cx<RW>* w, int j, int64_t n, int nrhs,
                       const KrylovArrays& k, const double* wscale = nullptr, int64_t ld = 0, int dots_G = 0);
// The context's Gram-Schmidt partial-sum buffer, large enough for the passes on vectors of
// length n and for extra_G block partials per RHS (its address stays valid for both).
double* gs_partials(dmlmc_ctx* ctx, int64_t n, int nrhs, int extra_G);
// Vectors longer than this take the multi-workgroup Gram-Schmidt passes.
int64_t gs_fused_max_n();
void krylov_solution(dmlmc_ctx* ctx, const KrylovArrays& k, int iters, int nrhs);
// y[r][i] *= scale[i][r] for i < iters
void krylov_scale_y(dmlmc_ctx* ctx, const KrylovArrays& k, const double* scale, int iters, int nrhs);
template <typename RZ, typename RX>
// x = sum_i y_i Z_i, or x += sum_i y_i Z_i (in FP64) when accumulate; Z_i holds RHS r at
// i * nrhs * ldz + r * ldz, x at r * ldx (0: n)
void launch_combine(dmlmc_ctx* ctx, const Cx<RZ>* Z, int iters, const KrylovArrays& k, Cx<RX>* x, int64_t n, int nrhs,
                    bool accumulate, int64_t ldz = 0, int64_t ldx = 0);
// v (stride ldv) = w (stride ldw) * invb[r]
template <typename RV>
void launch_scale_store(dmlmc_ctx* ctx, const c128* w, const double* invb, Cx<RV>* v, int64_t n, int nrhs,
                        int64_t ldw = 0, int64_t ldv = 0);

// Stride of the solver's internal multi-RHS work vectors on level l: the level size plus
// 256 entries below the coarsest level (from 4096 entries on), so that one entry of
// consecutive right-hand sides does not repeat the same HBM channel at power-of-two
// level sizes; the coarsest level keeps its size.
int64_t work_ld(const dmlmc_hier* H, int l);

// b, x: RHS r at r * ld (ld = 0: the level size); the coarser levels' vectors use work_ld
template <typename R>
void vcycle(dmlmc_hier* H, int l, const Cx<R>* b, Cx<R>* x, int nrhs, int64_t ld = 0);
template <typename R>
void smooth(dmlmc_hier* H, int l, Cx<R>* x, const Cx<R>* b, int nrhs, int sweeps, int64_t ld = 0);

struct SolveResult {
  int iters = 0;
  int ir_steps = 0;
  bool converged = false;
  double relres_max = 0.0;
};
// Solves D_l X = B (device FP64 [nrhs][n_l]); X overwritten.
SolveResult solve_level(dmlmc_hier* H, int l, const c128* B, c128* X, int nrhs, dmlmc_precision prec, double rtol,
                        int maxiter);
