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

#include "defl.h"
#include "dense.h"
#include "solver.h"

void readback(dmlmc_ctx* ctx, std::initializer_list<ReadbackPart> parts) {
  size_t total = 0;
  for (const ReadbackPart& p : parts) total += (p.bytes + 15) / 16 * 16;
  if (total > ctx->pinned_bytes) {
    if (ctx->pinned) HIPCHK(hipHostFree(ctx->pinned));
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
    const size_t want = std::max<size_t>(total, 64 * 1024);
    HIPCHK(hipHostMalloc(&ctx->pinned, want, hipHostMallocDefault));
    ctx->pinned_bytes = want;
  }
  if (!ctx->readback_event) HIPCHK(hipEventCreateWithFlags(&ctx->readback_event, hipEventDisableTiming));
  char* stage = static_cast<char*>(ctx->pinned);
  size_t off = 0;
  for (const ReadbackPart& p : parts) {
    HIPCHK(hipMemcpyAsync(stage + off, p.dev, p.bytes, hipMemcpyDeviceToHost, ctx->stream));
    off += (p.bytes + 15) / 16 * 16;
  }
  HIPCHK(hipEventRecord(ctx->readback_event, ctx->stream));
  HIPCHK(hipEventSynchronize(ctx->readback_event));
  off = 0;
  for (const ReadbackPart& p : parts) {
    std::memcpy(p.host, stage + off, p.bytes);
    off += (p.bytes + 15) / 16 * 16;
  }
}

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

__global__ void scale_y_kernel(c128* __restrict__ y, int m, const double* __restrict__ scale, int iters, int nrhs) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  for (int i = 0; i < iters; ++i) y[r * m + i] = scale[(int64_t)i * nrhs + r] * y[r * m + i];
}

// v_out (RV) = w * invb[r]
template <typename RV>
__global__ void scale_store_kernel(const c128* __restrict__ w, const double* __restrict__ invb, Cx<RV>* __restrict__ v,
                                   int64_t n, int64_t ldw, int64_t ldv) {
  const int r = blockIdx.y;
  const double s = invb[r];
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const c128 a = w[r * ldw + p];
    v[r * ldv + p] = cmk((RV)(a.x * s), (RV)(a.y * s));
  }
}

// v[r] *= s[r] in place (FP64)
// dst row i = src row idx[i] (rows of n entries, stride n)
__global__ void gather_rows_kernel(const c128* __restrict__ src, c128* __restrict__ dst, const int* __restrict__ idx,
                                   int64_t n) {
  const int r = blockIdx.y;
  const c128* s = src + (int64_t)idx[r] * n;
  c128* d = dst + (int64_t)r * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) d[i] = s[i];
}

__global__ void scale_inplace_kernel(c128* v, const double* __restrict__ s, int64_t n) {
  const int r = blockIdx.y;
  const double f = s[r];
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const c128 a = v[r * n + p];
    v[r * n + p] = cmk(a.x * f, a.y * f);
  }
}

// x (RX) = sum_i y[r][i] Z_i (RZ)
template <typename RZ, typename RX>
__global__ void combine_kernel(const Cx<RZ>* __restrict__ Z, int k, const c128* __restrict__ y, int ym,
                               Cx<RX>* __restrict__ x, int64_t n, int64_t vstride, int accumulate, int64_t ldz,
                               int64_t ldx) {
  const int r = blockIdx.y;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    double ax = 0.0, ay = 0.0;
    for (int i = 0; i < k; ++i) {
      const c128 yi = y[r * ym + i];
      const Cx<RZ> z = Z[i * vstride + r * ldz + p];
      ax += yi.x * (double)z.x - yi.y * (double)z.y;
      ay += yi.x * (double)z.y + yi.y * (double)z.x;
    }
    if (accumulate) {
      const Cx<RX> x0 = x[r * ldx + p];
      x[r * ldx + p] = cmk((RX)((double)x0.x + ax), (RX)((double)x0.y + ay));
    } else {
      x[r * ldx + p] = cmk((RX)ax, (RX)ay);
    }
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

dmlmc_hier::~dmlmc_hier() {
  for (auto& kv : graphs)
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
}

// Runs body on the context stream through a recorded HIP graph: the first call with a
// key runs it directly (so that every workspace buffer it needs exists), the second
// records and launches it, later ones replay the recording.  A recording is dropped when
// any device buffer was allocated or freed since it was made (its pointers may be stale);
// a recording during which that happens is discarded and the body run directly.  Timing
// runs (events around launches) never record.
template <typename F>
static void run_graphed(dmlmc_hier* H, const std::vector<int64_t>& key, F&& body) {
  dmlmc_ctx* ctx = H->ctx;
  if (!H->use_graphs || ctx->timing) {
    body();
    return;
  }
  const uint64_t now = g_dev_epoch.load();
  auto it = H->graphs.find(key);
  if (it != H->graphs.end()) {
    if (it->second.epoch == now) {
      HIPCHK(hipGraphLaunch(it->second.exec, ctx->stream));
      ++H->graph_launches;
      return;
    }
    (void)hipGraphExecDestroy(it->second.exec);
    H->graphs.erase(it);
    H->graph_seen.erase(key);
  }
  if (!H->graph_seen.count(key)) {
    H->graph_seen.insert(key);
    body();
    return;
  }
  HIPCHK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeRelaxed));
  hipGraph_t g = nullptr;
  try {
    body();
  } catch (...) {
    (void)hipStreamEndCapture(ctx->stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  HIPCHK(hipStreamEndCapture(ctx->stream, &g));
  if (g_dev_epoch.load() != now) {
    (void)hipGraphDestroy(g);
    H->graph_seen.erase(key);
    body();
    return;
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) throw DmlmcError(DMLMC_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  H->graphs[key] = {exec, now};
  HIPCHK(hipGraphLaunch(exec, ctx->stream));
  ++H->graph_launches;
}

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

void krylov_scale_y(dmlmc_ctx* ctx, const KrylovArrays& k, const double* scale, int iters, int nrhs) {
  hipLaunchKernelGGL(scale_y_kernel, dim3(ceil_div(nrhs, 64)), dim3(64), 0, ctx->stream, k.y, k.m, scale, iters, nrhs);
  LAUNCH_CHECK();
}

void krylov_solution(dmlmc_ctx* ctx, const KrylovArrays& k, int iters, int nrhs) {
  hipLaunchKernelGGL(backsub_kernel, dim3(ceil_div(nrhs, 64)), dim3(64), 0, ctx->stream, iters, k.m, k.H, k.g, k.y,
                     nrhs);
  LAUNCH_CHECK();
}

template <typename RZ, typename RX>
void launch_combine(dmlmc_ctx* ctx, const Cx<RZ>* Z, int iters, const KrylovArrays& k, Cx<RX>* x, int64_t n,
                    int nrhs, bool accumulate, int64_t ldz, int64_t ldx) {
  if (ldz <= 0) ldz = n;
  if (ldx <= 0) ldx = n;
  REQUIRE(ldz >= n && ldx >= n, "vector strides below the vector length");
  KTimer kt(ctx, "combine",
            (double)nrhs * n * (iters * sizeof(Cx<RZ>) + (accumulate ? 2 : 1) * sizeof(Cx<RX>)));
  hipLaunchKernelGGL((combine_kernel<RZ, RX>), dim3(gridn(n), nrhs), dim3(256), 0, ctx->stream, Z, iters, k.y, k.m, x,
                     n, (int64_t)nrhs * ldz, accumulate ? 1 : 0, ldz, ldx);
  LAUNCH_CHECK();
}

template <typename RV>
void launch_scale_store(dmlmc_ctx* ctx, const c128* w, const double* invb, Cx<RV>* v, int64_t n, int nrhs,
                        int64_t ldw, int64_t ldv) {
  if (ldw <= 0) ldw = n;
  if (ldv <= 0) ldv = n;
  REQUIRE(ldw >= n && ldv >= n, "vector strides below the vector length");
  hipLaunchKernelGGL((scale_store_kernel<RV>), dim3(gridn(n), nrhs), dim3(256), 0, ctx->stream, w, invb, v, n, ldw,
                     ldv);
  LAUNCH_CHECK();
}

// ---------------------------------------------------------------- coarsest solve
// Fixed-count GMRES from x = 0 on D_L (precision R for the operator and basis, FP64 dots
// and Givens); no host synchronisation.
// With a deflation of this level attached, the deflation space is inverted exactly and
// GMRES runs on the projected remainder only.
template <typename R>
void coarsest_gmres(dmlmc_hier* H, int l, const Cx<R>* b_in, Cx<R>* x, int nrhs) {
  dmlmc_ctx* ctx = H->ctx;
  const Level& L = H->lv[l - 1];
  const int64_t n = L.n();
  const bool f32 = std::is_same<R, float>::value;
  if (f32 && H->coarse_direct_mode != 0 && H->coarse_dinv_n == n) {
    apply_coarse_direct(H, (const c64*)b_in, (c64*)x, nrhs);
    return;
  }
  const dmlmc_defl* D = H->coarse_defl;
  const bool use_defl = D != nullptr && D->level == l;
  const int m = std::max(1, use_defl ? H->coarsest_iters_defl : H->coarsest_iters);
  const Cx<R>* b = b_in;
  c128* e0 = nullptr;
  if (use_defl) {
    c128* b64 = (c128*)hier_buf(H, "cd_b", l, sizeof(c128) * (size_t)nrhs * n);
    c128* r64 = (c128*)hier_buf(H, "cd_r", l, sizeof(c128) * (size_t)nrhs * n);
    e0 = (c128*)hier_buf(H, "cd_e0", l, sizeof(c128) * (size_t)nrhs * n);
    Cx<R>* rR = (Cx<R>*)hier_buf(H, f32 ? "cd_r32" : "cd_r64", l, sizeof(Cx<R>) * (size_t)nrhs * n);
    launch_cast<double, R>(ctx, b_in, b64, n, nrhs, n, n);
    defl_coarse_split(H, D, b64, nrhs, r64, e0, f32 ? DMLMC_MIXED : DMLMC_FP64);
    launch_cast<R, double>(ctx, r64, rR, n, nrhs, n, n);
    b = rR;
  }
  Cx<R>* V = (Cx<R>*)hier_buf(H, f32 ? "cg_V32" : "cg_V64", l, sizeof(Cx<R>) * (size_t)(m + 1) * nrhs * n);
  Cx<R>* wr = (Cx<R>*)hier_buf(H, f32 ? "cg_wr32" : "cg_wr64", l, sizeof(Cx<R>) * (size_t)nrhs * n);
  KrylovArrays k = krylov_arrays(H, "cg_", l, m, nrhs);
  const int64_t vstride = (int64_t)nrhs * n;
  launch_norms2<R>(ctx, b, n, nrhs, n, k.nrm2);
  krylov_init(ctx, k, nrhs);
  if (f32) {
    // single-pass Gram-Schmidt on an unnormalised complex-FP32 basis (FP64 arithmetic)
    double* scale = (double*)hier_buf(H, "cg_sc", l, sizeof(double) * (size_t)(m + 1) * nrhs);
    c64* U = (c64*)V;
    HIPCHK(hipMemcpyAsync(U, b, sizeof(c64) * (size_t)vstride, hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(scale, k.invb, sizeof(double) * nrhs, hipMemcpyDeviceToDevice, ctx->stream));
    for (int j = 0; j < m; ++j) {
      // D (s_j u_j) = s_j (D u_j): the scale enters the Gram-Schmidt step
      apply_op<float>(ctx, L, U + j * vstride, (c64*)wr, nrhs);
      arnoldi_step_cgs1<float>(ctx, U, scale, (const c64*)wr, j, n, nrhs, k, scale + (int64_t)j * nrhs);
    }
    krylov_solution(ctx, k, m, nrhs);
    krylov_scale_y(ctx, k, scale, m, nrhs);
  } else {
    c128* w = (c128*)hier_buf(H, "cg_w", l, sizeof(c128) * (size_t)nrhs * n);
    launch_cast<double, R>(ctx, b, w, n, nrhs, n, n);
    launch_scale_store<R>(ctx, w, k.invb, V, n, nrhs);
    for (int j = 0; j < m; ++j) {
      apply_op<R>(ctx, L, V + j * vstride, wr, nrhs);
      launch_cast<double, R>(ctx, wr, w, n, nrhs, n, n);
      arnoldi_step<R>(ctx, V, w, j, n, nrhs, k);
    }
    krylov_solution(ctx, k, m, nrhs);
  }
  launch_combine<R, R>(ctx, V, m, k, x, n, nrhs, false);
  if (use_defl) launch_add_cast_to<R>(ctx, e0, x, n, nrhs);
}

// ---------------------------------------------------------------- V-cycle
int64_t work_ld(const dmlmc_hier* H, int l) {
  const Level& L = H->lv[l - 1];
  const int64_t n = L.n();
  return (l < (int)H->lv.size() && n >= 4096) ? n + 256 : n;
}

template <typename R>
void smooth(dmlmc_hier* H, int l, Cx<R>* x, const Cx<R>* b, int nrhs, int sweeps, int64_t ld) {
  const Level& L = H->lv[l - 1];
  KTimerGroup group(H->ctx, L.fine ? "sap" : "coarse_gs");  // the colour sweeps run back to back
  for (int s = 0; s < sweeps; ++s) {
    for (int color = 0; color < 2; ++color) {
      if (L.fine)
        launch_sap<R>(H->ctx, L, x, b, nrhs, color, H->sap_mr_iters, ld);
      else
        launch_coarse_gs<R>(H->ctx, L, x, b, nrhs, color, H->smoother_half, ld);
    }
  }
}

template <typename R>
void vcycle(dmlmc_hier* H, int l, const Cx<R>* b, Cx<R>* x, int nrhs, int64_t ld) {
  const int Lmax = (int)H->lv.size();
  const Level& L = H->lv[l - 1];
  const int64_t n = L.n();
  if (ld <= 0) ld = n;
  if (l == Lmax) {
    REQUIRE(ld == n, "coarsest-level vectors are stored unpadded");
    coarsest_gmres<R>(H, l, b, x, nrhs);
    return;
  }
  dmlmc_ctx* ctx = H->ctx;
  const bool f32 = std::is_same<R, float>::value;
  const int64_t ldc = work_ld(H, l + 1);
  Cx<R>* bc = (Cx<R>*)hier_buf(H, f32 ? "vc_b32" : "vc_b64", l + 1, sizeof(Cx<R>) * (size_t)nrhs * ldc);
  Cx<R>* xc = (Cx<R>*)hier_buf(H, f32 ? "vc_x32" : "vc_x64", l + 1, sizeof(Cx<R>) * (size_t)nrhs * ldc);
  if (H->nu_pre > 0) {
    Cx<R>* r = (Cx<R>*)hier_buf(H, f32 ? "vc_r32" : "vc_r64", l, sizeof(Cx<R>) * (size_t)nrhs * ld);
    launch_fill_zero_rows<Cx<R>>(ctx, x, n, nrhs, ld);
    smooth<R>(H, l, x, b, nrhs, H->nu_pre, ld);
    apply_op<R>(ctx, L, x, r, nrhs, false, ld);
    launch_xmy<R>(ctx, b, r, n, nrhs, ld, ld);
    launch_restrict<R>(ctx, L, r, bc, nrhs, ld, ldc);
  } else {
    launch_restrict<R>(ctx, L, b, bc, nrhs, ld, ldc);
  }
  vcycle<R>(H, l + 1, bc, xc, nrhs, ldc);
  launch_prolong<R>(ctx, L, xc, x, nrhs, H->nu_pre > 0, ldc, ld);
  smooth<R>(H, l, x, b, nrhs, L.fine ? H->nu_post : H->nu_post_coarse, ld);
}

// ---------------------------------------------------------------- FGMRES cycle
// Solves A e = r approximately (one cycle of at most m iterations, stopping when every
// residual estimate is <= target[r]) and adds e to x; r, x in FP64, rnorm2 = ||r||^2 per
// RHS (device, as the refinement loop has just computed it).  RP: precision of the
// operator inside the cycle and of the preconditioner.  With u0_ready (complex FP32 only)
// the caller has already stored r in complex FP32 as the first basis vector (unnormalised,
// at the work stride) and r is not read.  Returns the number of iterations.
template <typename RP>
int fgmres_cycle(dmlmc_hier* H, int l, const c128* r, const double* rnorm2, c128* x, int nrhs, int m,
                 const std::vector<double>& target, std::vector<double>& res_host, bool u0_ready = false) {
  dmlmc_ctx* ctx = H->ctx;
  const Level& L = H->lv[l - 1];
  const int64_t n = L.n();
  const bool f32 = std::is_same<RP, float>::value;
  // the complex-FP32 cycle keeps its basis and preconditioned vectors at the padded work
  // stride; r and x (FP64, the caller's) stay unpadded
  const int64_t ldw = f32 ? work_ld(H, l) : n;
  const int64_t vstride = (int64_t)nrhs * ldw;
  Cx<RP>* Z = (Cx<RP>*)hier_buf(H, f32 ? "fg_Z32" : "fg_Z64", l, sizeof(Cx<RP>) * (size_t)m * vstride);
  KrylovArrays k = krylov_arrays(H, "fg_", l, m, nrhs);
  HIPCHK(hipMemcpyAsync(k.nrm2, rnorm2, sizeof(double) * nrhs, hipMemcpyDeviceToDevice, ctx->stream));
  krylov_init(ctx, k, nrhs);
  int it = 0;
  res_host.assign(nrhs, 0.0);
  // complex-FP32 inner cycle: single-pass Gram-Schmidt (FP64 arithmetic) on an
  // unnormalised complex-FP32 basis; FP64 cycle: two passes on an FP64 basis
  c64* U = nullptr;
  double* scale = nullptr;
  c128* V = nullptr;
  c128* w = nullptr;
  Cx<RP>* wr = nullptr;
  if (f32) {
    U = (c64*)hier_buf(H, "fg_U32", l, sizeof(c64) * (size_t)(m + 1) * vstride);
    scale = (double*)hier_buf(H, "fg_sc", l, sizeof(double) * (size_t)(m + 1) * nrhs);
    wr = (Cx<RP>*)hier_buf(H, "fg_wr32", l, sizeof(Cx<RP>) * (size_t)vstride);
    if (u0_ready) {
      // U_0 = r as the caller stored it, its scale 1 / ||r||
      HIPCHK(hipMemcpyAsync(scale, k.invb, sizeof(double) * nrhs, hipMemcpyDeviceToDevice, ctx->stream));
    } else {
      // U_0 = r / ||r|| (scale 1)
      launch_scale_store<float>(ctx, r, k.invb, U, n, nrhs, n, ldw);
      launch_fill_value(ctx, scale, nrhs, 1.0);
    }
  } else {
    V = (c128*)hier_buf(H, "fg_V", l, sizeof(c128) * (size_t)(m + 1) * vstride);
    w = (c128*)hier_buf(H, "fg_w", l, sizeof(c128) * (size_t)vstride);
    launch_scale_store<double>(ctx, r, k.invb, V, n, nrhs);
  }
  for (int j = 0; j < m; ++j) {
    Cx<RP>* zj = Z + j * vstride;
    if (f32) {
      const std::vector<int64_t> key = {l, nrhs, j, m, (int64_t)(uintptr_t)H->coarse_defl, H->coarsest_iters,
                                        H->coarsest_iters_defl, H->nu_pre, H->nu_post, H->nu_post_coarse,
                                        H->sap_mr_iters, H->smoother_half, H->coarse_direct_mode};
      // the preconditioner is homogeneous (M(s u) = s M(u), SAP's minimal-residual steps
      // and the scaled FP16 coarsest solve included), so it runs on the unnormalised U_j:
      // z'_j = M U_j, the Arnoldi step scales A z'_j by s_j in FP64, and the solution
      // update takes y_j s_j
      // on the fine level the operator pass also forms the Gram-Schmidt dots (one read of
      // the new vector less)
      const bool fused = L.fine && n > gs_fused_max_n() && j + 1 <= 8;
      run_graphed(H, key, [&]() {
        vcycle<RP>(H, l, (const Cx<RP>*)(U + j * vstride), zj, nrhs, ldw);
        if (fused) {
          double* part = gs_partials(ctx, n, nrhs, wilson_dots_blocks(L));
          const int G = launch_wilson_dots(ctx, L, (const c64*)zj, (c64*)wr, nrhs, ldw, U, j + 1, vstride,
                                           scale + (int64_t)j * nrhs, part);
          arnoldi_step_cgs1<float>(ctx, U, scale, (const c64*)wr, j, n, nrhs, k, scale + (int64_t)j * nrhs, ldw, G);
        } else {
          apply_op<RP>(ctx, L, zj, wr, nrhs, false, ldw);
          arnoldi_step_cgs1<float>(ctx, U, scale, (const c64*)wr, j, n, nrhs, k, scale + (int64_t)j * nrhs, ldw);
        }
      });
    } else {
      vcycle<RP>(H, l, (const Cx<RP>*)(V + j * vstride), zj, nrhs);
      apply_op<RP>(ctx, L, zj, (Cx<RP>*)w, nrhs);
      arnoldi_step<double>(ctx, V, w, j, n, nrhs, k);
    }
    it = j + 1;
    readback(ctx, {{k.res, res_host.data(), sizeof(double) * nrhs}});
    bool done = true;
    for (int q = 0; q < nrhs; ++q) {
      if (!std::isfinite(res_host[q])) throw DmlmcError(DMLMC_ENUMERIC, "NaN/Inf in the Krylov residual estimate");
      if (res_host[q] > target[q]) done = false;
    }
    if (done) break;
  }
  krylov_solution(ctx, k, it, nrhs);
  if (f32) krylov_scale_y(ctx, k, scale, it, nrhs);
  launch_combine<RP, double>(ctx, Z, it, k, x, n, nrhs, true, ldw, n);
  return it;
}

// ---------------------------------------------------------------- solve with FP64 refinement
SolveResult solve_level(dmlmc_hier* H, int l, const c128* B, c128* X, int nrhs, dmlmc_precision prec, double rtol,
                        int maxiter) {
  dmlmc_ctx* ctx = H->ctx;
  const Level& L = H->lv[l - 1];
  const int64_t n = L.n();
  const bool mixed = prec == DMLMC_MIXED;
  const int m = std::max(2, H->restart);
  // mixed: the residual goes straight into the first basis vector of the complex-FP32
  // cycle (the whole basis is sized here, so the cycle's request never reallocates it);
  // FP64: an FP64 residual vector
  const int64_t ldw = work_ld(H, l);
  c64* U0 = mixed ? (c64*)hier_buf(H, "fg_U32", l, sizeof(c64) * (size_t)(m + 1) * nrhs * ldw) : nullptr;
  c128* Rr = mixed ? nullptr : (c128*)hier_buf(H, "sv_R", l, sizeof(c128) * (size_t)nrhs * n);
  double* nrm = (double*)hier_buf(H, "sv_nrm", l, sizeof(double) * nrhs);
  std::vector<double> bn(nrhs), rn(nrhs), target(nrhs), est;
  launch_norms2<double>(ctx, B, n, nrhs, n, nrm);
  readback(ctx, {{nrm, bn.data(), sizeof(double) * nrhs}});
  // A right-hand side whose entries are far from unit size (root mean square beyond
  // 2^+-8) is solved as 2^-e b with 2^e its root mean square, and the solution scaled
  // back: a power of two is exact in every precision, and the complex-FP32 bulk (whose
  // squares would underflow below ~1e-19 or overflow above ~1e19) then sees unit-sized
  // vectors.  Z2 noise (entries +-1) is never rescaled.
  std::vector<double> rescale(nrhs, 1.0);
  bool any_rescale = false;
  for (int q = 0; q < nrhs; ++q) {
    if (!std::isfinite(bn[q])) throw DmlmcError(DMLMC_ENUMERIC, "NaN/Inf in the right-hand side");
    if (bn[q] > 0.0) {
      const int e = (int)std::lround(0.5 * std::log2(bn[q] / (double)n));
      if (std::abs(e) > 8) {
        rescale[q] = std::ldexp(1.0, -e);
        any_rescale = true;
      }
    }
  }
  if (any_rescale) {
    double* sdev = (double*)hier_buf(H, "sv_rsc", l, sizeof(double) * nrhs);
    c128* Bs = (c128*)hier_buf(H, "sv_Bs", l, sizeof(c128) * (size_t)nrhs * n);
    HIPCHK(hipMemcpyAsync(sdev, rescale.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, ctx->stream));
    launch_scale_store<double>(ctx, B, sdev, Bs, n, nrhs, n, n);
    B = Bs;
    // the norms of the scaled RHS (the first cycle reads them from the device)
    launch_norms2<double>(ctx, B, n, nrhs, n, nrm);
    HIPCHK(hipMemcpyAsync(bn.data(), nrm, sizeof(double) * nrhs, hipMemcpyDeviceToHost, ctx->stream));
  }
  launch_fill_zero<c128>(ctx, X, (size_t)nrhs * n);
  if (mixed)
    launch_cast<float, double>(ctx, B, U0, n, nrhs, n, ldw);  // r = b at x = 0
  else
    launch_cast<double, double>(ctx, B, Rr, n, nrhs, n, n);
  if (any_rescale) HIPCHK(hipStreamSynchronize(ctx->stream));  // the scaled norms' copy into bn
  for (int q = 0; q < nrhs; ++q) {
    bn[q] = std::sqrt(bn[q]);
    rn[q] = bn[q];
  }
  SolveResult out;
  const double inner_rel = (prec == DMLMC_MIXED) ? H->inner_rtol : 0.0;
  // Converged right-hand sides leave the refinement: rows 0..na-1 of X and B (and of the
  // cycle's vectors) hold the active ones, row i being the caller's RHS orig[i]; every
  // RHS's arithmetic is independent of the others in the block, so this only saves the
  // further cycles a converged RHS would otherwise run along with the rest.
  int na = nrhs;
  std::vector<int> orig(nrhs);
  for (int q = 0; q < nrhs; ++q) orig[q] = q;
  bool permuted = false;
  c128* Bw = nullptr;  // working copy of B once rows move
  while (true) {
    std::vector<int> act, conv;
    double worst = 0.0;
    for (int q = 0; q < nrhs; ++q) {  // rows from na on keep the residuals they left with
      const double rel = bn[q] > 0.0 ? rn[q] / bn[q] : 0.0;
      worst = std::max(worst, rel);
      if (q < na) (rel > rtol ? act : conv).push_back(q);
    }
    out.relres_max = worst;
    if (act.empty()) {
      out.converged = true;
      break;
    }
    if (out.iters >= maxiter) break;
    if (!conv.empty()) {
      // move the active rows to the front (stable), the converged ones after them
      std::vector<int> idx(act);
      idx.insert(idx.end(), conv.begin(), conv.end());
      if (!Bw) {
        Bw = (c128*)hier_buf(H, "sv_Bw", l, sizeof(c128) * (size_t)nrhs * n);
        HIPCHK(hipMemcpyAsync(Bw, B, sizeof(c128) * (size_t)nrhs * n, hipMemcpyDeviceToDevice, ctx->stream));
        B = Bw;
      }
      int* idev = (int*)hier_buf(H, "sv_idx", l, sizeof(int) * nrhs);
      c128* tmp = (c128*)hier_buf(H, "sv_tmp", l, sizeof(c128) * (size_t)na * n);
      HIPCHK(hipMemcpyAsync(idev, idx.data(), sizeof(int) * na, hipMemcpyHostToDevice, ctx->stream));
      for (c128* M : {X, Bw}) {
        hipLaunchKernelGGL(gather_rows_kernel, dim3(gridn(n), na), dim3(256), 0, ctx->stream, M, tmp, idev, n);
        LAUNCH_CHECK();
        HIPCHK(hipMemcpyAsync(M, tmp, sizeof(c128) * (size_t)na * n, hipMemcpyDeviceToDevice, ctx->stream));
      }
      auto permute = [&](auto& v) {
        auto w = v;
        for (int i = 0; i < na; ++i) w[i] = v[idx[i]];
        v = w;
      };
      permute(bn);
      permute(rn);
      permute(rescale);
      permute(orig);
      na = (int)act.size();
      permuted = true;
      // the mixed cycle starts from the residual in its first basis vector: rebuild it for
      // the moved rows
      if (mixed) {
        apply_residual_to32(ctx, L, X, B, U0, na, n, ldw);
        launch_norms2<float>(ctx, U0, n, na, ldw, nrm);
      } else {
        apply_residual<double>(ctx, L, X, B, Rr, na);
        launch_norms2<double>(ctx, Rr, n, na, n, nrm);
      }
    }
    for (int q = 0; q < na; ++q) target[q] = std::max(0.5 * rtol * bn[q], inner_rel * rn[q]);
    int it;
    // each cycle adds its correction to X; then r = b - D x (one operator pass, FP64
    // arithmetic; stored in complex FP32 as the next cycle's first basis vector in the
    // mixed form) and ||r||^2 (FP64 sums)
    if (mixed)
      it = fgmres_cycle<float>(H, l, nullptr, nrm, X, na, std::min(m, std::max(1, maxiter - out.iters)), target,
                               est, true);
    else
      it = fgmres_cycle<double>(H, l, Rr, nrm, X, na, std::min(m, std::max(1, maxiter - out.iters)), target, est);
    out.iters += it;
    out.ir_steps += 1;
    if (mixed) {
      apply_residual_to32(ctx, L, X, B, U0, na, n, ldw);
      launch_norms2<float>(ctx, U0, n, na, ldw, nrm);
    } else {
      apply_residual<double>(ctx, L, X, B, Rr, na);
      launch_norms2<double>(ctx, Rr, n, na, n, nrm);
    }
    readback(ctx, {{nrm, rn.data(), sizeof(double) * na}});
    for (int q = 0; q < na; ++q) {
      if (!std::isfinite(rn[q])) throw DmlmcError(DMLMC_ENUMERIC, "NaN/Inf in the FP64 residual");
      rn[q] = std::sqrt(rn[q]);
    }
  }
  if (permuted) {
    // rows back to the caller's order: X row orig[i] = current row i
    std::vector<int> inv(nrhs);
    for (int i = 0; i < nrhs; ++i) inv[orig[i]] = i;
    int* idev = (int*)hier_buf(H, "sv_idx", l, sizeof(int) * nrhs);
    c128* tmp = (c128*)hier_buf(H, "sv_tmp", l, sizeof(c128) * (size_t)nrhs * n);
    HIPCHK(hipMemcpyAsync(idev, inv.data(), sizeof(int) * nrhs, hipMemcpyHostToDevice, ctx->stream));
    hipLaunchKernelGGL(gather_rows_kernel, dim3(gridn(n), nrhs), dim3(256), 0, ctx->stream, X, tmp, idev, n);
    LAUNCH_CHECK();
    HIPCHK(hipMemcpyAsync(X, tmp, sizeof(c128) * (size_t)nrhs * n, hipMemcpyDeviceToDevice, ctx->stream));
    std::vector<double> rs(nrhs);
    for (int i = 0; i < nrhs; ++i) rs[orig[i]] = rescale[i];
    rescale = rs;
  }
  if (any_rescale) {
    for (int q = 0; q < nrhs; ++q) rescale[q] = 1.0 / rescale[q];
    double* sdev = (double*)hier_buf(H, "sv_rsc", l, sizeof(double) * nrhs);
    HIPCHK(hipMemcpyAsync(sdev, rescale.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, ctx->stream));
    hipLaunchKernelGGL(scale_inplace_kernel, dim3(gridn(n), nrhs), dim3(256), 0, ctx->stream, X, sdev, n);
    LAUNCH_CHECK();
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
  return out;
}

template void vcycle<float>(dmlmc_hier*, int, const c64*, c64*, int, int64_t);
template void vcycle<double>(dmlmc_hier*, int, const c128*, c128*, int, int64_t);
template void smooth<float>(dmlmc_hier*, int, c64*, const c64*, int, int, int64_t);
template void smooth<double>(dmlmc_hier*, int, c128*, const c128*, int, int, int64_t);
template void launch_combine<double, double>(dmlmc_ctx*, const c128*, int, const KrylovArrays&, c128*, int64_t, int,
                                             bool, int64_t, int64_t);
template void launch_scale_store<double>(dmlmc_ctx*, const c128*, const double*, c128*, int64_t, int, int64_t,
                                         int64_t);
template void launch_scale_store<float>(dmlmc_ctx*, const c128*, const double*, c64*, int64_t, int, int64_t, int64_t);
