// Hierarchy construction on the device (setup, once per gauge field):
//   * gauge links U_mu = exp(i theta_mu) with the antiperiodic sign folded into the
//     t-links of the last time slice;
//   * test vectors: Z4 start vectors, n_inv steps of V <- orth(D^-1 V) with FGMRES solves
//     to 1e-12 preconditioned by a provisional hierarchy (built from smoothed start
//     vectors, rebuilt from the current vectors after every step);
//   * P: QR with positive real diagonal of every (aggregate, chirality) block of V;
//   * D_{l+1} = P^H D_l P by probing: for each colour class of coarse sites (same-colour
//     sites at distance >= 3 in both directions), the probes P e_k are summed over the
//     class, D_l is applied (multi-RHS stencil) and the result restricted; each coarse
//     site then reads its coupling to the one class member in its neighbourhood;
//   * inverses of the coarse self blocks (Gauss-Jordan with partial pivoting, FP64) for
//     the block Gauss-Seidel smoother.
#include <cmath>

#include "setup.h"
#include "solver.h"

namespace {

__global__ void links_kernel(const double* __restrict__ theta, c128* __restrict__ U64, c64* __restrict__ U32, int Lx,
                             int Lt, int antiperiodic) {
  const int64_t V = (int64_t)Lx * Lt;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * V) return;
  const int mu = (int)(i / V);
  const int64_t s = i % V;
  const int t = (int)(s / Lx);
  double sgn = (mu == 1 && antiperiodic && t == Lt - 1) ? -1.0 : 1.0;
  double sn, cs;
  sincos(theta[i], &sn, &cs);
  U64[i] = cmk(sgn * cs, sgn * sn);
  U32[i] = cmk((float)(sgn * cs), (float)(sgn * sn));
}

// One wavefront per (coarse site, chirality): gather the block of V (rows x N), modified
// Gram-Schmidt in column order (positive real diagonal), store P[cs][c][row][k].
__global__ __launch_bounds__(64) void local_qr_kernel(const c128* __restrict__ V, int64_t n, int Lx, int Lt, int d,
                                                      int ax, int at, int N, c128* __restrict__ P,
                                                      int* __restrict__ fail) {
  extern __shared__ unsigned char smem_raw[];
  c128* B = reinterpret_cast<c128*>(smem_raw);  // [rows][N]
  const int h = d / 2;
  const int rows = ax * at * h;
  const int Lxc = Lx / ax;
  const int64_t blk = blockIdx.x;  // cs * 2 + c
  const int c = (int)(blk % 2);
  const int64_t cs = blk / 2;
  const int X = (int)(cs % Lxc), T = (int)(cs / Lxc);
  for (int row = threadIdx.x; row < rows; row += 64) {
    const int ls = row / h, j = row % h;
    const int lx = ls % ax, lt = ls / ax;
    const int64_t site = (int64_t)(X * ax + lx) + (int64_t)Lx * (T * at + lt);
    const int64_t idx = site * d + c * h + j;
    for (int k = 0; k < N; ++k) B[row * N + k] = V[(int64_t)k * n + idx];
  }
  __syncthreads();
  for (int k = 0; k < N; ++k) {
    for (int jj = 0; jj < k; ++jj) {
      double re = 0.0, im = 0.0;
      for (int row = threadIdx.x; row < rows; row += 64) {
        const c128 q = B[row * N + jj], v = B[row * N + k];
        re += q.x * v.x + q.y * v.y;
        im += q.x * v.y - q.y * v.x;
      }
      for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_xor(re, off, 64);
        im += __shfl_xor(im, off, 64);
      }
      __syncthreads();
      for (int row = threadIdx.x; row < rows; row += 64) {
        const c128 q = B[row * N + jj];
        c128& v = B[row * N + k];
        v.x -= re * q.x - im * q.y;
        v.y -= re * q.y + im * q.x;
      }
      __syncthreads();
    }
    double s = 0.0;
    for (int row = threadIdx.x; row < rows; row += 64) s += cabs2(B[row * N + k]);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    const double nrm = sqrt(s);
    if (nrm == 0.0 || !isfinite(nrm)) {
      if (threadIdx.x == 0) atomicAdd(fail, 1);
    }
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    __syncthreads();
    for (int row = threadIdx.x; row < rows; row += 64) B[row * N + k] = inv * B[row * N + k];
    __syncthreads();
  }
  c128* Pb = P + blk * (int64_t)rows * N;
  for (int e = threadIdx.x; e < rows * N; e += 64) Pb[e] = B[e];
}

// Probe vectors of one colour class: probe_q (q = c * N + k) on the fine level is
// P_Y e_q summed over coarse sites Y of colour (cx, ct) (colour = (X mod mx, T mod mt)).
__global__ void probe_kernel(const c128* __restrict__ P, int Lx, int Lt, int d, int ax, int at, int N, int mx, int mt,
                             int cx, int ct, c128* __restrict__ probes) {
  const int64_t n = (int64_t)Lx * Lt * d;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= n) return;
  const int dof = (int)(tid % d);
  const int64_t site = tid / d;
  const int x = (int)(site % Lx), t = (int)(site / Lx);
  const int X = x / ax, T = t / at;
  const int Lxc = Lx / ax;
  const int h = d / 2;
  const int c = dof / h, j = dof % h;
  const bool mine = (X % mx == cx) && (T % mt == ct);
  const int row = ((x % ax) + ax * (t % at)) * h + j;
  const int rows = ax * at * h;
  const int64_t cs = (int64_t)X + (int64_t)Lxc * T;
  const c128* Pr = P + ((cs * 2 + c) * (int64_t)rows + row) * N;
  for (int q = 0; q < 2 * N; ++q) {
    const int qc = q / N, qk = q % N;
    probes[(int64_t)q * n + tid] = (mine && qc == c) ? Pr[qk] : cmk(0.0, 0.0);
  }
}

// A[X][dir][q * dc + i] = C_q[X][i] for every direction whose neighbour X + dir has the
// colour (cx, ct) and is not a repeat of an earlier direction's site.
__global__ void scatter_kernel(const c128* __restrict__ C, int Lxc, int Ltc, int dc, int mx, int mt, int cx, int ct,
                               c128* __restrict__ A) {
  const int64_t Vc = (int64_t)Lxc * Ltc;
  const int64_t nc = Vc * dc;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (X, i)
  if (tid >= nc) return;
  const int i = (int)(tid % dc);
  const int64_t s = tid / dc;
  const int x = (int)(s % Lxc), t = (int)(s / Lxc);
  const int dx[5] = {0, 1, -1, 0, 0}, dt[5] = {0, 0, 0, 1, -1};
  int64_t nbs[5];
  for (int dir = 0; dir < 5; ++dir) {
    const int xn = (x + dx[dir] + Lxc) % Lxc, tn = (t + dt[dir] + Ltc) % Ltc;
    nbs[dir] = (int64_t)xn + (int64_t)Lxc * tn;
    bool repeat = false;
    for (int e = 0; e < dir; ++e) repeat |= (nbs[e] == nbs[dir]);
    if (repeat) continue;
    if (xn % mx != cx || tn % mt != ct) continue;
    c128* Ab = A + (s * 5 + dir) * (int64_t)dc * dc;
    for (int q = 0; q < dc; ++q) Ab[q * dc + i] = C[(int64_t)q * nc + s * dc + i];
  }
}

// Inverse of every self block (column-major d x d) by Gauss-Jordan with partial pivoting;
// one workgroup of 64 threads per site, augmented matrix in LDS.
__global__ __launch_bounds__(64) void inv_blocks_kernel(const c128* __restrict__ A, int d, c128* __restrict__ Ainv,
                                                        int* __restrict__ fail) {
  extern __shared__ unsigned char smem_raw[];
  c128* M = reinterpret_cast<c128*>(smem_raw);  // [d][2d] row-major
  __shared__ int piv;
  const int64_t s = blockIdx.x;
  const c128* Ab = A + s * 5 * (int64_t)d * d;  // self block = dir 0
  const int w = 2 * d;
  for (int e = threadIdx.x; e < d * w; e += 64) {
    const int i = e / w, j = e % w;
    M[e] = (j < d) ? Ab[j * d + i] : (j - d == i ? cmk(1.0, 0.0) : cmk(0.0, 0.0));
  }
  __syncthreads();
  for (int col = 0; col < d; ++col) {
    if (threadIdx.x == 0) {
      int best = col;
      double bv = cabs2(M[col * w + col]);
      for (int i = col + 1; i < d; ++i) {
        const double v = cabs2(M[i * w + col]);
        if (v > bv) { bv = v; best = i; }
      }
      piv = best;
      if (bv == 0.0) atomicAdd(fail, 1);
    }
    __syncthreads();
    const int p = piv;
    if (p != col) {
      for (int j = threadIdx.x; j < w; j += 64) {
        const c128 tmp = M[col * w + j];
        M[col * w + j] = M[p * w + j];
        M[p * w + j] = tmp;
      }
    }
    __syncthreads();
    const c128 pv = M[col * w + col];
    const double pd = cabs2(pv);
    const c128 ip = pd > 0.0 ? cmk(pv.x / pd, -pv.y / pd) : cmk(0.0, 0.0);
    __syncthreads();
    for (int j = threadIdx.x; j < w; j += 64) M[col * w + j] = M[col * w + j] * ip;
    __syncthreads();
    for (int e = threadIdx.x; e < d * w; e += 64) {
      const int i = e / w, j = e % w;
      if (i == col) continue;
      const c128 f = M[i * w + col];
      if (j == col) continue;
      M[e] = M[e] - f * M[col * w + j];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < d; i += 64)
      if (i != col) M[i * w + col] = cmk(0.0, 0.0);
    __syncthreads();
  }
  c128* Ib = Ainv + s * (int64_t)d * d;
  for (int e = threadIdx.x; e < d * d; e += 64) {
    const int j = e / d, i = e % d;  // column-major output
    Ib[e] = M[i * w + d + j];
  }
}

__global__ void scale_inv_norm_kernel(c128* __restrict__ v, const double* __restrict__ nrm2, int64_t n) {
  const double nn = sqrt(fmax(nrm2[0], 0.0));
  const double s = nn > 0.0 ? 1.0 / nn : 0.0;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
    v[p] = s * v[p];
}

int colour_mod(int extent) {
  if (extent <= 2) return extent;
  for (int c = 3; c <= extent; ++c)
    if (extent % c == 0) return c;
  return extent;
}

// FP32 copies of coarse blocks (d x d each): row-major at d = 16, the layout of the
// matrix-core stencil kernels, column-major (as the FP64 source) otherwise.
__global__ void cast_blocks_kernel(const c128* __restrict__ src, c64* __restrict__ dst, int64_t total, int d,
                                   int rowmajor) {
  const int64_t dd = (int64_t)d * d;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t blk = i / dd;
    const int e = (int)(i % dd);
    const int se = rowmajor ? (e % d) * d + e / d : e;
    dst[i] = ccast<float>(src[blk * dd + se]);
  }
}

// complex-FP16 copies of 16 x 16 row-major FP32 blocks: dst block (b, q) = src block
// (b, q + off) for q < nd, with ns source blocks per site; *overflow is set when an
// entry is not finite or beyond the FP16 range
__global__ void half_blocks_kernel(const c64* __restrict__ src, uint32_t* __restrict__ dst, int64_t nsites, int ns,
                                   int nd, int off, int* __restrict__ overflow) {
  const int64_t total = nsites * nd * 256;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t blk = i / 256;
    const int e = (int)(i % 256);
    const int64_t site = blk / nd;
    const int q = (int)(blk % nd);
    const c64 v = src[(site * ns + q + off) * 256 + e];
    if (!(fabsf(v.x) <= 65000.f && fabsf(v.y) <= 65000.f)) *overflow = 1;
    const _Float16 re = (_Float16)v.x, im = (_Float16)v.y;
    dst[i] = (uint32_t)__builtin_bit_cast(uint16_t, re) | ((uint32_t)__builtin_bit_cast(uint16_t, im) << 16);
  }
}

void half_blocks(dmlmc_ctx* ctx, const c64* src, uint32_t* dst, int64_t nsites, int ns, int nd, int off,
                 int* overflow) {
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(nsites * nd * 256, 256), 8192);
  hipLaunchKernelGGL(half_blocks_kernel, dim3(grid), dim3(256), 0, ctx->stream, src, dst, nsites, ns, nd, off,
                     overflow);
  LAUNCH_CHECK();
}

void cast_blocks(dmlmc_ctx* ctx, const c128* src, c64* dst, int64_t nblocks, int d) {
  const int64_t total = nblocks * d * d;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(total, 256), 8192);
  hipLaunchKernelGGL(cast_blocks_kernel, dim3(grid), dim3(256), 0, ctx->stream, src, dst, total, d, d == 16 ? 1 : 0);
  LAUNCH_CHECK();
}

}  // namespace

void upload_links(dmlmc_ctx* ctx, Level& L, const double* theta_host, int antiperiodic) {
  const int64_t V = L.sites();
  DevBuf th(sizeof(double) * 2 * V);
  HIPCHK(hipMemcpyAsync(th.p, theta_host, sizeof(double) * 2 * V, hipMemcpyHostToDevice, ctx->stream));
  L.U64.alloc(sizeof(c128) * 2 * V);
  L.U32.alloc(sizeof(c64) * 2 * V);
  hipLaunchKernelGGL(links_kernel, dim3(ceil_div(2 * V, 256)), dim3(256), 0, ctx->stream, th.as<double>(),
                     L.U64.as<c128>(), L.U32.as<c64>(), L.Lx, L.Lt, antiperiodic);
  LAUNCH_CHECK();
  HIPCHK(hipStreamSynchronize(ctx->stream));
}

void build_interpolator(dmlmc_ctx* ctx, Level& L, const c128* V, int N) {
  const int rows = L.ax * L.at * (L.dofs / 2);
  const int64_t Vc = (int64_t)(L.Lx / L.ax) * (L.Lt / L.at);
  L.N = N;
  L.P64.alloc(sizeof(c128) * (size_t)Vc * 2 * rows * N);
  DevBuf fail(sizeof(int));
  HIPCHK(hipMemsetAsync(fail.p, 0, sizeof(int), ctx->stream));
  hipLaunchKernelGGL(local_qr_kernel, dim3((unsigned)(Vc * 2)), dim3(64), sizeof(c128) * rows * N, ctx->stream, V,
                     L.n(), L.Lx, L.Lt, L.dofs, L.ax, L.at, N, L.P64.as<c128>(), fail.as<int>());
  LAUNCH_CHECK();
  int nfail = 0;
  HIPCHK(hipMemcpyAsync(&nfail, fail.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (nfail) throw DmlmcError(DMLMC_ENUMERIC, "rank-deficient test vectors on " + std::to_string(nfail) + " blocks");
  L.P32.alloc(sizeof(c64) * (size_t)Vc * 2 * rows * N);
  launch_cast<float, double>(ctx, L.P64.as<c128>(), L.P32.as<c64>(), (int64_t)Vc * 2 * rows * N, 1, 0, 0);
}

Level galerkin_level(dmlmc_ctx* ctx, const Level& F) {
  Level C;
  C.l = F.l + 1;
  C.fine = false;
  C.Lx = F.Lx / F.ax;
  C.Lt = F.Lt / F.at;
  C.dofs = 2 * F.N;
  const int dc = C.dofs;
  const int64_t Vc = C.sites(), nc = C.n(), nf = F.n();
  C.A64.alloc(sizeof(c128) * (size_t)Vc * 5 * dc * dc);
  launch_fill_zero<c128>(ctx, C.A64.as<c128>(), (size_t)Vc * 5 * dc * dc);
  const int mx = colour_mod(C.Lx), mt = colour_mod(C.Lt);
  DevBuf probes(sizeof(c128) * (size_t)dc * nf), Dp(sizeof(c128) * (size_t)dc * nf), Cr(sizeof(c128) * (size_t)dc * nc);
  for (int cx = 0; cx < mx; ++cx) {
    for (int ct = 0; ct < mt; ++ct) {
      hipLaunchKernelGGL(probe_kernel, dim3(ceil_div(nf, 256)), dim3(256), 0, ctx->stream, F.P64.as<c128>(), F.Lx,
                         F.Lt, F.dofs, F.ax, F.at, F.N, mx, mt, cx, ct, probes.as<c128>());
      LAUNCH_CHECK();
      apply_op<double>(ctx, F, probes.as<c128>(), Dp.as<c128>(), dc);
      launch_restrict<double>(ctx, F, Dp.as<c128>(), Cr.as<c128>(), dc);
      hipLaunchKernelGGL(scatter_kernel, dim3(ceil_div(nc, 256)), dim3(256), 0, ctx->stream, Cr.as<c128>(), C.Lx,
                         C.Lt, dc, mx, mt, cx, ct, C.A64.as<c128>());
      LAUNCH_CHECK();
    }
  }
  C.A32.alloc(sizeof(c64) * (size_t)Vc * 5 * dc * dc);
  cast_blocks(ctx, C.A64.as<c128>(), C.A32.as<c64>(), (int64_t)Vc * 5, dc);
  // inverse self blocks for the block Gauss-Seidel smoother
  C.Ainv64.alloc(sizeof(c128) * (size_t)Vc * dc * dc);
  DevBuf fail(sizeof(int));
  HIPCHK(hipMemsetAsync(fail.p, 0, sizeof(int), ctx->stream));
  hipLaunchKernelGGL(inv_blocks_kernel, dim3((unsigned)Vc), dim3(64), sizeof(c128) * dc * 2 * dc, ctx->stream,
                     C.A64.as<c128>(), dc, C.Ainv64.as<c128>(), fail.as<int>());
  LAUNCH_CHECK();
  C.Ainv32.alloc(sizeof(c64) * (size_t)Vc * dc * dc);
  cast_blocks(ctx, C.Ainv64.as<c128>(), C.Ainv32.as<c64>(), (int64_t)Vc, dc);
  if (dc == 16) {
    // the half-precision smoother operands exist only when every entry fits FP16
    DevBuf over(sizeof(int));
    HIPCHK(hipMemsetAsync(over.p, 0, sizeof(int), ctx->stream));
    C.Ahop16.alloc(sizeof(uint32_t) * (size_t)Vc * 4 * 256);
    half_blocks(ctx, C.A32.as<c64>(), C.Ahop16.as<uint32_t>(), Vc, 5, 4, 1, over.as<int>());
    C.Ainv16.alloc(sizeof(uint32_t) * (size_t)Vc * 256);
    half_blocks(ctx, C.Ainv32.as<c64>(), C.Ainv16.as<uint32_t>(), Vc, 1, 1, 0, over.as<int>());
    int novf = 0;
    HIPCHK(hipMemcpyAsync(&novf, over.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (novf) {
      C.Ahop16.release();
      C.Ainv16.release();
    }
  }
  int nfail = 0;
  HIPCHK(hipMemcpyAsync(&nfail, fail.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (nfail) throw DmlmcError(DMLMC_ENUMERIC, "singular coarse self block");
  return C;
}

// Orthonormalise the N columns of V ([N][n], FP64) by classical Gram-Schmidt with one
// reorthogonalisation, in column order (the QR factor with positive real diagonal).
void orthonormalise(dmlmc_hier* H, c128* V, int N, int64_t n) {
  dmlmc_ctx* ctx = H->ctx;
  c128* h = (c128*)hier_buf(H, "or_h", 0, sizeof(c128) * (N + 1) * 2);
  double* nrm = (double*)hier_buf(H, "or_n", 0, sizeof(double) * 2);
  for (int k = 0; k < N; ++k) {
    c128* vk = V + (int64_t)k * n;
    if (k > 0) {
      for (int pass = 0; pass < 2; ++pass) {
        launch_multidot<double>(ctx, V, k, vk, n, 1, n, n, h, N + 1);
        launch_multiaxpy<double>(ctx, V, k, vk, n, 1, n, n, h, N + 1);
      }
    }
    launch_norms2<double>(ctx, vk, n, 1, n, nrm);
    hipLaunchKernelGGL(scale_inv_norm_kernel, dim3((unsigned)std::min<int64_t>(1024, ceil_div(n, 256))), dim3(256), 0,
                       ctx->stream, vk, nrm, n);
    LAUNCH_CHECK();
  }
}

Level clone_operator(dmlmc_ctx* ctx, const Level& S) {
  Level L;
  L.l = S.l;
  L.Lx = S.Lx;
  L.Lt = S.Lt;
  L.dofs = S.dofs;
  L.fine = S.fine;
  L.m0 = S.m0;
  auto cp = [&](DevBuf& d, const DevBuf& s) {
    if (!s.p) return;
    d.alloc(s.bytes);
    HIPCHK(hipMemcpyAsync(d.p, s.p, s.bytes, hipMemcpyDeviceToDevice, ctx->stream));
  };
  cp(L.U64, S.U64);
  cp(L.U32, S.U32);
  cp(L.A64, S.A64);
  cp(L.A32, S.A32);
  cp(L.Ainv64, S.Ainv64);
  cp(L.Ainv32, S.Ainv32);
  cp(L.Ahop16, S.Ahop16);
  cp(L.Ainv16, S.Ainv16);
  return L;
}

// Provisional hierarchy below the operator `top`: every coarsening step uses the real
// step's aggregates and sizes, with test vectors = `smooth_sweeps` smoother sweeps
// applied to the Z4 start vectors (or, for the first step, the given vectors V).
std::unique_ptr<dmlmc_hier> provisional(dmlmc_hier* H, int l, const c128* V_first, int smooth_sweeps) {
  dmlmc_ctx* ctx = H->ctx;
  std::unique_ptr<dmlmc_hier> P(new dmlmc_hier());
  P->ctx = ctx;
  P->sap_mr_iters = H->sap_mr_iters;
  P->nu_pre = H->nu_pre;
  P->nu_post = H->nu_post;
  P->nu_post_coarse = H->nu_post_coarse;
  P->inner_rtol = H->inner_rtol;
  P->smoother_half = H->smoother_half;
  P->coarsest_iters = H->coarsest_iters;
  P->restart = H->restart;
  P->lv.push_back(clone_operator(ctx, H->lv[l - 1]));
  const int L = (int)H->plan.size() + 1;
  for (int s = l; s < L; ++s) {
    Level& F = P->lv.back();
    F.ax = H->plan[s - 1].ax;
    F.at = H->plan[s - 1].at;
    const int N = H->plan[s - 1].ntv;
    const int64_t n = F.n();
    DevBuf tv(sizeof(c128) * (size_t)N * n);
    if (s == l && V_first) {
      HIPCHK(hipMemcpyAsync(tv.p, V_first, tv.bytes, hipMemcpyDeviceToDevice, ctx->stream));
    } else {
      DevBuf z4(sizeof(c128) * (size_t)N * n);
      launch_z4(ctx, z4.as<c128>(), n, H->seed, s, 0, N);
      launch_fill_zero<c128>(ctx, tv.as<c128>(), (size_t)N * n);
      smooth<double>(P.get(), (int)P->lv.size(), tv.as<c128>(), z4.as<c128>(), N, smooth_sweeps);
    }
    build_interpolator(ctx, F, tv.as<c128>(), N);
    P->lv.push_back(galerkin_level(ctx, F));
  }
  return P;
}

void build_levels(dmlmc_hier* H, const std::vector<const c128*>& import_tv) {
  dmlmc_ctx* ctx = H->ctx;
  const int L = (int)H->plan.size() + 1;
  for (int l = 1; l < L; ++l) {
    Level& F = H->lv[l - 1];
    F.ax = H->plan[l - 1].ax;
    F.at = H->plan[l - 1].at;
    const int N = H->plan[l - 1].ntv;
    const int64_t n = F.n();
    DevBuf V(sizeof(c128) * (size_t)N * n);
    if (!import_tv.empty() && import_tv[l - 1]) {
      HIPCHK(hipMemcpyAsync(V.p, import_tv[l - 1], V.bytes, hipMemcpyHostToDevice, ctx->stream));
    } else {
      launch_z4(ctx, V.as<c128>(), n, H->seed, l, 0, N);
      DevBuf X(sizeof(c128) * (size_t)N * n);
      std::unique_ptr<dmlmc_hier> prov;
      for (int step = 0; step < H->n_inv; ++step) {
        // provisional hierarchy: from smoothed start vectors first, then from the
        // current vectors (the solves are exact, so this changes only the work); the
        // solves run complex-FP32 cycles inside FP64 refinement to the FP64 tolerance
        prov = provisional(H, l, step == 0 ? nullptr : V.as<c128>(), 4);
        SolveResult r = solve_level(prov.get(), 1, V.as<c128>(), X.as<c128>(), N, DMLMC_MIXED, 1e-12, 5000);
        if (!r.converged) throw DmlmcError(DMLMC_ENOCONV, "setup solve did not reach 1e-12 at level " + std::to_string(l));
        HIPCHK(hipMemcpyAsync(V.p, X.p, V.bytes, hipMemcpyDeviceToDevice, ctx->stream));
        orthonormalise(H, V.as<c128>(), N, n);
        H->setup_iters += r.iters;
      }
    }
    F.tv_host.resize((size_t)N * n);
    HIPCHK(hipMemcpyAsync(F.tv_host.data(), V.p, V.bytes, hipMemcpyDeviceToHost, ctx->stream));
    build_interpolator(ctx, F, V.as<c128>(), N);
    H->lv.push_back(galerkin_level(ctx, F));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
}
