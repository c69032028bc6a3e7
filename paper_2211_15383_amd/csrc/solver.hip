// Multigrid-preconditioned Krylov solves (Sec. 3.1, eq. 8 applied recursively):
//   * V-cycle: pre-smoothing, restriction P^H, recursion / coarsest solve, prolongation
//     P, post-smoothing (SAP on the fine level, red/black block Gauss-Seidel on coarse
//     levels);
//   * coarsest solve: fixed-count GMRES (no host synchronisation, graph-capturable);
//   * right-preconditioned FGMRES with per-RHS Krylov spaces, FP64 Arnoldi (classical
//     Gram-Schmidt with one reorthogonalisation, FP64 dots), Givens on the device;
//   * outer FP64 refinement: every restart recomputes r = b - D x in FP64, so the mixed
//     path (complex FP32 operator and preconditioner inside the cycle) converges to the
//     FP64 tolerance.
#include <algorithm>
#include <cmath>

#include "solver.h"

namespace {

// ---------------------------------------------------------------- Krylov bookkeeping kernels
__global__ void init_cycle_kernel(const double* __restrict__ nrm2, c128* __restrict__ g, double* __restrict__ invb,
                                  double* __restrict__ res, int m, int nrhs) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const double beta = sqrt(fmax(nrm2[r], 0.0));
  for (int i = 0; i <= m; ++i) g[r * (m + 1) + i] = cmk(0.0, 0.0);
  g[r * (m + 1)] = cmk(beta, 0.0);
  invb[r] = beta > 0.0 ? 1.0 / beta : 0.0;
  res[r] = beta;
}

// Column j of the Hessenberg matrix from the two Gram-Schmidt passes and ||w||; applies
// the previous Givens rotations, forms the new one, updates g and the residual estimate.
__global__ void arnoldi_finish_kernel(int j, int m, const c128* __restrict__ h1, const c128* __restrict__ h2,
                                      int hld, const double* __restrict__ nrm2, c128* __restrict__ H,
                                      double* __restrict__ cs, c128* __restrict__ sn, c128* __restrict__ g,
                                      double* __restrict__ res, double* __restrict__ invb, int nrhs) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  c128* col = H + (int64_t)r * (m + 1) * m + (int64_t)j * (m + 1);
  for (int i = 0; i <= j; ++i) col[i] = h1[r * hld + i] + h2[r * hld + i];
  const double beta = sqrt(fmax(nrm2[r], 0.0));
  for (int i = 0; i < j; ++i) {
    const double c = cs[r * m + i];
    const c128 s = sn[r * m + i];
    const c128 a = col[i], b = col[i + 1];
    col[i] = c * a + s * b;
    col[i + 1] = c * b - conj(s) * a;
  }
  const c128 a = col[j];
  const double aa = sqrt(cabs2(a));
  const double rho = sqrt(aa * aa + beta * beta);
  double c;
  c128 s;
  if (rho == 0.0) {
    c = 1.0;
    s = cmk(0.0, 0.0);
    col[j] = cmk(0.0, 0.0);
  } else if (aa == 0.0) {
    c = 0.0;
    s = cmk(1.0, 0.0);
    col[j] = cmk(beta, 0.0);
  } else {
    const c128 ph = cmk(a.x / aa, a.y / aa);
    c = aa / rho;
    s = (beta / rho) * ph;
    col[j] = rho * ph;
  }
  cs[r * m + j] = c;
  sn[r * m + j] = s;
  c128* gr = g + (int64_t)r * (m + 1);
  const c128 gj = gr[j];
  gr[j + 1] = cmk(-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x));  // -conj(s) g_j
  gr[j] = c * gj;
  res[r] = sqrt(cabs2(gr[j + 1]));
  invb[r] = beta > 0.0 ? 1.0 / beta : 0.0;
}

// y = R^-1 g over the first k columns (upper triangular, zero pivots give zero).
__global__ void backsub_kernel(int k, int m, const c128* __restrict__ H, const c128* __restrict__ g,
                               c128* __restrict__ y, int nrhs) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const c128* Hr = H + (int64_t)r * (m + 1) * m;
  for (int i = k - 1; i >= 0; --i) {
    c128 acc = g[(int64_t)r * (m + 1) + i];
    for (int l = i + 1; l < k; ++l) acc = acc - Hr[l * (m + 1) + i] * y[r * m + l];
    const c128 d = Hr[i * (m + 1) + i];
    const double dd = cabs2(d);
    y[r * m + i] = dd > 0.0 ? cmk((acc.x * d.x + acc.y * d.y) / dd, (acc.y * d.x - acc.x * d.y) / dd)
                            : cmk(0.0, 0.0);
  }
}

// v_out (RV) = w * invb[r]
template <typename RV>
__global__ void scale_store_kernel(const c128* __restrict__ w, const double* __restrict__ invb, Cx<RV>* __restrict__ v,
                                   int64_t n) {
  const int r = blockIdx.y;
  const double s = invb[r];
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const c128 a = w[r * n + p];
    v[r * n + p] = cmk((RV)(a.x * s), (RV)(a.y * s));
  }
}

// x (RX) = sum_i y[r][i] Z_i (RZ)
template <typename RZ, typename RX>
__global__ void combine_kernel(const Cx<RZ>* __restrict__ Z, int k, const c128* __restrict__ y, int ym,
                               Cx<RX>* __restrict__ x, int64_t n, int64_t vstride) {
  const int r = blockIdx.y;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    double ax = 0.0, ay = 0.0;
    for (int i = 0; i < k; ++i) {
      const c128 yi = y[r * ym + i];
      const Cx<RZ> z = Z[i * vstride + r * n + p];
      ax += yi.x * (double)z.x - yi.y * (double)z.y;
      ay += yi.x * (double)z.y + yi.y * (double)z.x;
    }
    x[r * n + p] = cmk((RX)ax, (RX)ay);
  }
}

inline unsigned gridn(int64_t n) { return (unsigned)std::min<int64_t>(std::max<int64_t>(1, ceil_div(n, 256)), 2048); }

}  // namespace

// ---------------------------------------------------------------- scratch buffers
void* hier_buf(dmlmc_hier* H, const char* name, int level, size_t bytes) {
  if ((int)H->ws.size() < (int)H->lv.size() + 1) H->ws.resize(H->lv.size() + 1);
  if (!H->ws[level]) H->ws[level].reset(new Workspace());
  DevBuf& b = H->ws[level]->bufs[name];
  b.ensure(bytes);
  return b.p;
}

DevBuf& hier_devbuf(dmlmc_hier* H, const char* name, int level) {
  hier_buf(H, name, level, 0);
  return H->ws[level]->bufs[name];
}

dmlmc_hier::~dmlmc_hier() {}

KrylovArrays krylov_arrays(dmlmc_hier* H, const char* prefix, int level, int m, int nrhs) {
  KrylovArrays k;
  std::string p(prefix);
  k.m = m;
  k.hld = m + 1;
  k.H = (c128*)hier_buf(H, (p + "H").c_str(), level, sizeof(c128) * (size_t)nrhs * (m + 1) * m);
  k.cs = (double*)hier_buf(H, (p + "cs").c_str(), level, sizeof(double) * (size_t)nrhs * m);
  k.sn = (c128*)hier_buf(H, (p + "sn").c_str(), level, sizeof(c128) * (size_t)nrhs * m);
  k.g = (c128*)hier_buf(H, (p + "g").c_str(), level, sizeof(c128) * (size_t)nrhs * (m + 1));
  k.h1 = (c128*)hier_buf(H, (p + "h1").c_str(), level, sizeof(c128) * (size_t)nrhs * (m + 1));
  k.h2 = (c128*)hier_buf(H, (p + "h2").c_str(), level, sizeof(c128) * (size_t)nrhs * (m + 1));
  k.y = (c128*)hier_buf(H, (p + "y").c_str(), level, sizeof(c128) * (size_t)nrhs * m);
  k.nrm2 = (double*)hier_buf(H, (p + "n2").c_str(), level, sizeof(double) * nrhs);
  k.res = (double*)hier_buf(H, (p + "res").c_str(), level, sizeof(double) * nrhs);
  k.invb = (double*)hier_buf(H, (p + "ib").c_str(), level, sizeof(double) * nrhs);
  return k;
}

void krylov_init(dmlmc_ctx* ctx, const KrylovArrays& k, int nrhs) {
  hipLaunchKernelGGL(init_cycle_kernel, dim3(ceil_div(nrhs, 64)), dim3(64), 0, ctx->stream, k.nrm2, k.g, k.invb,
                     k.res, k.m, nrhs);
  LAUNCH_CHECK();
}

// One Arnoldi step: orthogonalise w (FP64, [nrhs][n]) against V_0..V_j (RV) by CGS2,
// update the Hessenberg column and rotations, store V_{j+1} = w / ||w||.
template <typename RV>
void arnoldi_step(dmlmc_ctx* ctx, Cx<RV>* V, c128* w, int j, int64_t n, int nrhs, const KrylovArrays& k) {
  const int64_t vstride = (int64_t)nrhs * n;
  launch_multidot<RV>(ctx, V, j + 1, w, n, nrhs, n, vstride, k.h1, k.hld);
  launch_multiaxpy<RV>(ctx, V, j + 1, w, n, nrhs, n, vstride, k.h1, k.hld);
  launch_multidot<RV>(ctx, V, j + 1, w, n, nrhs, n, vstride, k.h2, k.hld);
  launch_multiaxpy<RV>(ctx, V, j + 1, w, n, nrhs, n, vstride, k.h2, k.hld);
  launch_norms2<double>(ctx, w, n, nrhs, n, k.nrm2);
  hipLaunchKernelGGL(arnoldi_finish_kernel, dim3(ceil_div(nrhs, 64)), dim3(64), 0, ctx->stream, j, k.m, k.h1, k.h2,
                     k.hld, k.nrm2, k.H, k.cs, k.sn, k.g, k.res, k.invb, nrhs);
  LAUNCH_CHECK();
  hipLaunchKernelGGL((scale_store_kernel<RV>), dim3(gridn(n), nrhs), dim3(256), 0, ctx->stream, w, k.invb,
                     V + (int64_t)(j + 1) * vstride, n);
  LAUNCH_CHECK();
}

void krylov_solution(dmlmc_ctx* ctx, const KrylovArrays& k, int iters, int nrhs) {
  hipLaunchKernelGGL(backsub_kernel, dim3(ceil_div(nrhs, 64)), dim3(64), 0, ctx->stream, iters, k.m, k.H, k.g, k.y,
                     nrhs);
  LAUNCH_CHECK();
}

template <typename RZ, typename RX>
void launch_combine(dmlmc_ctx* ctx, const Cx<RZ>* Z, int iters, const KrylovArrays& k, Cx<RX>* x, int64_t n,
                    int nrhs) {
  hipLaunchKernelGGL((combine_kernel<RZ, RX>), dim3(gridn(n), nrhs), dim3(256), 0, ctx->stream, Z, iters, k.y, k.m, x,
                     n, (int64_t)nrhs * n);
  LAUNCH_CHECK();
}

template <typename RV>
void launch_scale_store(dmlmc_ctx* ctx, const c128* w, const double* invb, Cx<RV>* v, int64_t n, int nrhs) {
  hipLaunchKernelGGL((scale_store_kernel<RV>), dim3(gridn(n), nrhs), dim3(256), 0, ctx->stream, w, invb, v, n);
  LAUNCH_CHECK();
}

// ---------------------------------------------------------------- coarsest solve
// Fixed-count GMRES from x = 0 on D_L (precision R for the operator and basis, FP64 dots
// and Givens); no host synchronisation.
template <typename R>
void coarsest_gmres(dmlmc_hier* H, int l, const Cx<R>* b, Cx<R>* x, int nrhs) {
  dmlmc_ctx* ctx = H->ctx;
  const Level& L = H->lv[l - 1];
  const int64_t n = L.n();
  const int m = std::max(1, H->coarsest_iters);
  const bool f32 = std::is_same<R, float>::value;
  Cx<R>* V = (Cx<R>*)hier_buf(H, f32 ? "cg_V32" : "cg_V64", l, sizeof(Cx<R>) * (size_t)(m + 1) * nrhs * n);
  c128* w = (c128*)hier_buf(H, "cg_w", l, sizeof(c128) * (size_t)nrhs * n);
  Cx<R>* wr = (Cx<R>*)hier_buf(H, f32 ? "cg_wr32" : "cg_wr64", l, sizeof(Cx<R>) * (size_t)nrhs * n);
  KrylovArrays k = krylov_arrays(H, "cg_", l, m, nrhs);
  launch_norms2<R>(ctx, b, n, nrhs, n, k.nrm2);
  krylov_init(ctx, k, nrhs);
  launch_cast<double, R>(ctx, b, w, n, nrhs, n, n);
  launch_scale_store<R>(ctx, w, k.invb, V, n, nrhs);
  const int64_t vstride = (int64_t)nrhs * n;
  for (int j = 0; j < m; ++j) {
    apply_op<R>(ctx, L, V + j * vstride, wr, nrhs);
    launch_cast<double, R>(ctx, wr, w, n, nrhs, n, n);
    arnoldi_step<R>(ctx, V, w, j, n, nrhs, k);
  }
  krylov_solution(ctx, k, m, nrhs);
  launch_combine<R, R>(ctx, V, m, k, x, n, nrhs);
}

// ---------------------------------------------------------------- V-cycle
template <typename R>
void smooth(dmlmc_hier* H, int l, Cx<R>* x, const Cx<R>* b, int nrhs, int sweeps) {
  const Level& L = H->lv[l - 1];
  for (int s = 0; s < sweeps; ++s) {
    for (int color = 0; color < 2; ++color) {
      if (L.fine)
        launch_sap<R>(H->ctx, L, x, b, nrhs, color, H->sap_mr_iters);
      else
        launch_coarse_gs<R>(H->ctx, L, x, b, nrhs, color);
    }
  }
}

template <typename R>
void vcycle(dmlmc_hier* H, int l, const Cx<R>* b, Cx<R>* x, int nrhs) {
  const int Lmax = (int)H->lv.size();
  if (l == Lmax) {
    coarsest_gmres<R>(H, l, b, x, nrhs);
    return;
  }
  dmlmc_ctx* ctx = H->ctx;
  const Level& L = H->lv[l - 1];
  const Level& C = H->lv[l];
  const bool f32 = std::is_same<R, float>::value;
  const int64_t n = L.n(), nc = C.n();
  Cx<R>* bc = (Cx<R>*)hier_buf(H, f32 ? "vc_b32" : "vc_b64", l + 1, sizeof(Cx<R>) * (size_t)nrhs * nc);
  Cx<R>* xc = (Cx<R>*)hier_buf(H, f32 ? "vc_x32" : "vc_x64", l + 1, sizeof(Cx<R>) * (size_t)nrhs * nc);
  if (H->nu_pre > 0) {
    Cx<R>* r = (Cx<R>*)hier_buf(H, f32 ? "vc_r32" : "vc_r64", l, sizeof(Cx<R>) * (size_t)nrhs * n);
    launch_fill_zero<Cx<R>>(ctx, x, (size_t)nrhs * n);
    smooth<R>(H, l, x, b, nrhs, H->nu_pre);
    apply_op<R>(ctx, L, x, r, nrhs);
    launch_xmy<R>(ctx, b, r, n, nrhs, n, n);
    launch_restrict<R>(ctx, L, r, bc, nrhs);
  } else {
    launch_restrict<R>(ctx, L, b, bc, nrhs);
  }
  vcycle<R>(H, l + 1, bc, xc, nrhs);
  launch_prolong<R>(ctx, L, xc, x, nrhs, H->nu_pre > 0);
  smooth<R>(H, l, x, b, nrhs, H->nu_post);
}

// ---------------------------------------------------------------- FGMRES cycle
// Solves A e = r approximately (one cycle of at most m iterations, stopping when every
// residual estimate is <= target[r]); r, e in FP64.  RP: precision of the operator inside
// the cycle and of the preconditioner.  Returns the number of iterations.
template <typename RP>
int fgmres_cycle(dmlmc_hier* H, int l, const c128* r, c128* e, int nrhs, int m, const std::vector<double>& target,
                 std::vector<double>& res_host) {
  dmlmc_ctx* ctx = H->ctx;
  const Level& L = H->lv[l - 1];
  const int64_t n = L.n();
  const bool f32 = std::is_same<RP, float>::value;
  const int64_t vstride = (int64_t)nrhs * n;
  c128* V = (c128*)hier_buf(H, "fg_V", l, sizeof(c128) * (size_t)(m + 1) * vstride);
  Cx<RP>* Z = (Cx<RP>*)hier_buf(H, f32 ? "fg_Z32" : "fg_Z64", l, sizeof(Cx<RP>) * (size_t)m * vstride);
  c128* w = (c128*)hier_buf(H, "fg_w", l, sizeof(c128) * (size_t)vstride);
  Cx<RP>* vin = nullptr;
  Cx<RP>* wr = nullptr;
  if (f32) {
    vin = (Cx<RP>*)hier_buf(H, "fg_vin32", l, sizeof(Cx<RP>) * (size_t)vstride);
    wr = (Cx<RP>*)hier_buf(H, "fg_wr32", l, sizeof(Cx<RP>) * (size_t)vstride);
  }
  KrylovArrays k = krylov_arrays(H, "fg_", l, m, nrhs);
  launch_norms2<double>(ctx, r, n, nrhs, n, k.nrm2);
  krylov_init(ctx, k, nrhs);
  launch_scale_store<double>(ctx, r, k.invb, V, n, nrhs);
  int it = 0;
  res_host.assign(nrhs, 0.0);
  for (int j = 0; j < m; ++j) {
    Cx<RP>* zj = Z + j * vstride;
    if (f32) {
      launch_cast<float, double>(ctx, V + j * vstride, (c64*)vin, n, nrhs, n, n);
      vcycle<RP>(H, l, vin, zj, nrhs);
      apply_op<RP>(ctx, L, zj, wr, nrhs);
      launch_cast<double, RP>(ctx, wr, w, n, nrhs, n, n);
    } else {
      vcycle<RP>(H, l, (const Cx<RP>*)(V + j * vstride), zj, nrhs);
      apply_op<RP>(ctx, L, zj, (Cx<RP>*)w, nrhs);
    }
    arnoldi_step<double>(ctx, V, w, j, n, nrhs, k);
    it = j + 1;
    HIPCHK(hipMemcpyAsync(res_host.data(), k.res, sizeof(double) * nrhs, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    bool done = true;
    for (int q = 0; q < nrhs; ++q) {
      if (!std::isfinite(res_host[q])) throw DmlmcError(DMLMC_ENUMERIC, "NaN/Inf in the Krylov residual estimate");
      if (res_host[q] > target[q]) done = false;
    }
    if (done) break;
  }
  krylov_solution(ctx, k, it, nrhs);
  launch_combine<RP, double>(ctx, Z, it, k, e, n, nrhs);
  return it;
}

// ---------------------------------------------------------------- solve with FP64 refinement
SolveResult solve_level(dmlmc_hier* H, int l, const c128* B, c128* X, int nrhs, dmlmc_precision prec, double rtol,
                        int maxiter) {
  dmlmc_ctx* ctx = H->ctx;
  const Level& L = H->lv[l - 1];
  const int64_t n = L.n();
  c128* Rr = (c128*)hier_buf(H, "sv_R", l, sizeof(c128) * (size_t)nrhs * n);
  c128* E = (c128*)hier_buf(H, "sv_E", l, sizeof(c128) * (size_t)nrhs * n);
  double* nrm = (double*)hier_buf(H, "sv_nrm", l, sizeof(double) * nrhs);
  std::vector<double> bn(nrhs), rn(nrhs), target(nrhs), est;
  launch_norms2<double>(ctx, B, n, nrhs, n, nrm);
  HIPCHK(hipMemcpyAsync(bn.data(), nrm, sizeof(double) * nrhs, hipMemcpyDeviceToHost, ctx->stream));
  launch_fill_zero<c128>(ctx, X, (size_t)nrhs * n);
  launch_cast<double, double>(ctx, B, Rr, n, nrhs, n, n);
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (int q = 0; q < nrhs; ++q) {
    if (!std::isfinite(bn[q])) throw DmlmcError(DMLMC_ENUMERIC, "NaN/Inf in the right-hand side");
    bn[q] = std::sqrt(bn[q]);
    rn[q] = bn[q];
  }
  SolveResult out;
  const int m = std::max(2, H->restart);
  const double inner_rel = (prec == DMLMC_MIXED) ? 2e-6 : 0.0;
  while (true) {
    bool all = true;
    double worst = 0.0;
    for (int q = 0; q < nrhs; ++q) {
      const double rel = bn[q] > 0.0 ? rn[q] / bn[q] : 0.0;
      worst = std::max(worst, rel);
      if (rel > rtol) all = false;
    }
    out.relres_max = worst;
    if (all) {
      out.converged = true;
      break;
    }
    if (out.iters >= maxiter) break;
    for (int q = 0; q < nrhs; ++q) target[q] = std::max(0.5 * rtol * bn[q], inner_rel * rn[q]);
    int it;
    if (prec == DMLMC_MIXED)
      it = fgmres_cycle<float>(H, l, Rr, E, nrhs, std::min(m, std::max(1, maxiter - out.iters)), target, est);
    else
      it = fgmres_cycle<double>(H, l, Rr, E, nrhs, std::min(m, std::max(1, maxiter - out.iters)), target, est);
    out.iters += it;
    out.ir_steps += 1;
    launch_add_cast<double>(ctx, E, X, n, nrhs, n, n);
    apply_op<double>(ctx, L, X, Rr, nrhs);
    launch_xmy<double>(ctx, B, Rr, n, nrhs, n, n);
    launch_norms2<double>(ctx, Rr, n, nrhs, n, nrm);
    HIPCHK(hipMemcpyAsync(rn.data(), nrm, sizeof(double) * nrhs, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int q = 0; q < nrhs; ++q) {
      if (!std::isfinite(rn[q])) throw DmlmcError(DMLMC_ENUMERIC, "NaN/Inf in the FP64 residual");
      rn[q] = std::sqrt(rn[q]);
    }
  }
  return out;
}

template void vcycle<float>(dmlmc_hier*, int, const c64*, c64*, int);
template void vcycle<double>(dmlmc_hier*, int, const c128*, c128*, int);
template void smooth<float>(dmlmc_hier*, int, c64*, const c64*, int, int);
template void smooth<double>(dmlmc_hier*, int, c128*, const c128*, int, int);
template void arnoldi_step<double>(dmlmc_ctx*, c128*, c128*, int, int64_t, int, const KrylovArrays&);
template void launch_combine<double, double>(dmlmc_ctx*, const c128*, int, const KrylovArrays&, c128*, int64_t, int);
template void launch_scale_store<double>(dmlmc_ctx*, const c128*, const double*, c128*, int64_t, int);
