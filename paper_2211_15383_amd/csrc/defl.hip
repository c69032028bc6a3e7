// Exact deflation of the coarsest operator (eqs. 4-7):
//   * projections C = W^H X and Y = X - W C with W = Gamma5 X_k (n x k) and X (n x b):
//     FP64 forms, and complex-FP32 forms on the matrix cores (v_mfma_f32_16x16x4_f32, four
//     real products per complex product) with FP64 accumulation across K-chunks;
//   * the eigensolver for the k eigenpairs of Q = Gamma5 D_L with the smallest |lambda|:
//     Chebyshev-filtered subspace iteration on Q^2 (filter damps [a, ||Q||^2], a = the
//     largest Ritz value of Q^2 kept in the subspace, degree chosen from the gap to the
//     k-th Ritz value), CholQR2 orthonormalisation, Rayleigh-Ritz with Q^2 on the subspace
//     and then with Q on its k leading vectors; all FP64 on the device except the small
//     dense eigenproblems.
#include <algorithm>
#include <cstdio>
#include <cmath>

#include "defl.h"
#include "tsgemm.h"
#include "eigh_host.h"
#include "jacobi.h"
#include "setup.h"
#include "solver.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int KC = 256;  // K-chunk of the split-K product W^H X

// Partial C over one K-chunk for one 16 x 16 tile (rows i of W^H, columns r of X).
// Operand layout of v_mfma_f32_16x16x4_f32: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; it receives D[4 (l / 16) + v][l % 16], v = 0..3.
__global__ __launch_bounds__(64) void defl_c_mfma_kernel(const c64* __restrict__ W, int k, const c128* __restrict__ X,
                                                         int b, int64_t n, int64_t ldx, c128* __restrict__ part) {
  const int lane = threadIdx.x;
  const int chunk = blockIdx.x;
  const int i0 = blockIdx.y * 16, r0 = blockIdx.z * 16;
  const int row = lane % 16, kk = lane / 16;
  const int iA = i0 + row;   // W row for the A operand
  const int rB = r0 + row;   // X column for the B operand
  floatx4 cre = {0.f, 0.f, 0.f, 0.f}, cim = {0.f, 0.f, 0.f, 0.f};
  const int64_t p0 = (int64_t)chunk * KC;
  const int64_t pend = (p0 + KC < n) ? p0 + KC : n;
  for (int64_t p = p0; p < pend; p += 4) {
    const int64_t pk = p + kk;
    c64 a = cmk(0.f, 0.f), x = cmk(0.f, 0.f);
    if (pk < pend) {
      if (iA < k) a = W[(int64_t)iA * n + pk];
      if (rB < b) {
        const c128 xv = X[(int64_t)rB * ldx + pk];
        x = cmk((float)xv.x, (float)xv.y);
      }
    }
    // conj(W) X: re = Wr Xr + Wi Xi, im = Wr Xi - Wi Xr
    cre = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, x.x, cre, 0, 0, 0);
    cre = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, x.y, cre, 0, 0, 0);
    cim = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, x.y, cim, 0, 0, 0);
    cim = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.y, x.x, cim, 0, 0, 0);
  }
  const int r = r0 + row;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = i0 + 4 * kk + v;
    if (i < k && r < b) part[((int64_t)chunk * b + r) * k + i] = cmk((double)cre[v], (double)cim[v]);
  }
}

// C[r][i] = sum over chunks (FP64)
__global__ void defl_c_reduce_kernel(const c128* __restrict__ part, int nchunks, int k, int b, c128* __restrict__ C) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)k * b) return;
  double re = 0.0, im = 0.0;
  for (int c = 0; c < nchunks; ++c) {
    const c128 v = part[(int64_t)c * k * b + t];
    re += v.x;
    im += v.y;
  }
  C[t] = cmk(re, im);
}

// Y = X - W C on one 16 (p) x 16 (r) tile: A[p][i] = W[i][p], B[i][r] = C[r][i].
__global__ __launch_bounds__(64) void defl_p_mfma_kernel(const c64* __restrict__ W, int k, const c128* __restrict__ C,
                                                         const c128* __restrict__ X, c128* __restrict__ Y, int b,
                                                         int64_t n, int64_t ldx, int64_t ldy, double xscale) {
  const int lane = threadIdx.x;
  const int64_t p0 = (int64_t)blockIdx.x * 16;
  const int r0 = blockIdx.y * 16;
  const int row = lane % 16, kk = lane / 16;
  floatx4 dre = {0.f, 0.f, 0.f, 0.f}, dim = {0.f, 0.f, 0.f, 0.f};
  for (int i0 = 0; i0 < k; i0 += 4) {
    const int i = i0 + kk;
    c64 a = cmk(0.f, 0.f), c = cmk(0.f, 0.f);
    if (i < k) {
      if (p0 + row < n) a = W[(int64_t)i * n + p0 + row];
      if (r0 + row < b) {
        const c128 cv = C[(int64_t)(r0 + row) * k + i];
        c = cmk((float)cv.x, (float)cv.y);
      }
    }
    // W C: re = Wr Cr - Wi Ci, im = Wr Ci + Wi Cr
    dre = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, c.x, dre, 0, 0, 0);
    dre = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.y, c.y, dre, 0, 0, 0);
    dim = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, c.y, dim, 0, 0, 0);
    dim = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, c.x, dim, 0, 0, 0);
  }
  const int r = r0 + row;
  if (r >= b) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t p = p0 + 4 * kk + v;
    if (p < n) {
      const c128 xv = xscale != 0.0 ? X[(int64_t)r * ldx + p] : cmk(0.0, 0.0);
      Y[(int64_t)r * ldy + p] = cmk(xscale * xv.x - (double)dre[v], xscale * xv.y - (double)dim[v]);
    }
  }
}

// Cs[r][i] = sgn * C[r][i] / lambda_i
__global__ void scale_coeffs_kernel(const c128* __restrict__ C, const double* __restrict__ lam, int k, int b,
                                    double sgn, c128* __restrict__ Cs) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)k * b) return;
  const int i = (int)(t % k);
  Cs[t] = (sgn / lam[i]) * C[t];
}

// row-sum bound of |Q| = |D| (Gamma5 only flips signs): max_row sum_j |A[s][dir][i][j]|
__global__ void rowsum_kernel(const c128* __restrict__ A, int64_t sites, int d, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= sites * d) return;
  const int64_t s = t / d;
  const int i = (int)(t % d);
  double sum = 0.0;
  for (int dir = 0; dir < 5; ++dir)
    for (int j = 0; j < d; ++j) sum += sqrt(cabs2(A[(s * 5 + dir) * (int64_t)d * d + j * d + i]));
  out[t] = sum;
}

__global__ void gamma5_kernel(const c128* __restrict__ x, c128* __restrict__ y, int64_t n, int d, int nv) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nv) return;
  const int dof = (int)((t % n) % d);
  const c128 v = x[t];
  y[t] = (dof < d / 2) ? v : cmk(-v.x, -v.y);
}

// y = (2 / e) (Q^2 x - c x) - z  (or without -z when first), elementwise part
__global__ void cheb_kernel(const c128* __restrict__ q2x, const c128* __restrict__ x, const c128* __restrict__ z,
                            c128* __restrict__ y, int64_t total, double alpha, double c, int first) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  c128 v = alpha * (q2x[t] - c * x[t]);
  if (!first) v = v - z[t];
  y[t] = v;
}

// r_i = z_i - theta_i y_i, written over z
__global__ void ritz_res_kernel(c128* __restrict__ z, const c128* __restrict__ y, const double* __restrict__ theta,
                                int64_t n, int nv) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nv) return;
  const int i = (int)(t / n);
  z[t] = z[t] - theta[i] * y[t];
}

}  // namespace

// ------------------------------------------------------------------ projections
void defl_coeffs_fp64(dmlmc_ctx* ctx, const dmlmc_defl* D, const c128* X, int b, int64_t ldx, c128* C) {
  launch_multidot<double>(ctx, D->W64.as<c128>(), D->k, X, D->n, b, ldx, D->n, C, D->k, 0);
}

void defl_project_fp64(dmlmc_ctx* ctx, const dmlmc_defl* D, c128* X, int b, int64_t ldx, const c128* C) {
  launch_multiaxpy<double>(ctx, D->W64.as<c128>(), D->k, X, D->n, b, ldx, D->n, C, D->k, 0, 1.0);
}

void defl_coeffs_mfma(dmlmc_ctx* ctx, const dmlmc_defl* D, const c128* X, int b, int64_t ldx, c128* C,
                      DevBuf& scratch) {
  const int nchunks = (int)ceil_div(D->n, KC);
  scratch.ensure(sizeof(c128) * (size_t)nchunks * D->k * b);
  KTimer kt(ctx, "defl_gemm", 8.0 * D->n * D->k * b);
  dim3 grid(nchunks, (unsigned)ceil_div(D->k, 16), (unsigned)ceil_div(b, 16));
  hipLaunchKernelGGL(defl_c_mfma_kernel, grid, dim3(64), 0, ctx->stream, D->W32.as<c64>(), D->k, X, b, D->n, ldx,
                     scratch.as<c128>());
  LAUNCH_CHECK();
  hipLaunchKernelGGL(defl_c_reduce_kernel, dim3((unsigned)ceil_div((int64_t)D->k * b, 256)), dim3(256), 0,
                     ctx->stream, scratch.as<c128>(), nchunks, D->k, b, C);
  LAUNCH_CHECK();
}

size_t defl_project_scratch_entries(const dmlmc_defl* D, int b) {
  return (size_t)(ceil_div(D->n, KC) + 1) * D->k * b;
}

void defl_project_mfma_into(hipStream_t stream, const dmlmc_defl* D, const c128* X, c128* Y, int b, c128* part) {
  const int nchunks = (int)ceil_div(D->n, KC);
  c128* C = part + (size_t)nchunks * D->k * b;
  dim3 gc(nchunks, (unsigned)ceil_div(D->k, 16), (unsigned)ceil_div(b, 16));
  hipLaunchKernelGGL(defl_c_mfma_kernel, gc, dim3(64), 0, stream, D->W32.as<c64>(), D->k, X, b, D->n, D->n, part);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(defl_c_reduce_kernel, dim3((unsigned)ceil_div((int64_t)D->k * b, 256)), dim3(256), 0, stream,
                     part, nchunks, D->k, b, C);
  LAUNCH_CHECK();
  dim3 gp((unsigned)ceil_div(D->n, 16), (unsigned)ceil_div(b, 16));
  hipLaunchKernelGGL(defl_p_mfma_kernel, gp, dim3(64), 0, stream, D->W32.as<c64>(), D->k, C, X, Y, b, D->n, D->n,
                     D->n, 1.0);
  LAUNCH_CHECK();
}

void defl_project_mfma(dmlmc_ctx* ctx, const dmlmc_defl* D, const c128* X, c128* Y, int b, int64_t ldx, int64_t ldy,
                       const c128* C) {
  KTimer kt(ctx, "defl_gemm", 8.0 * D->n * D->k * b);
  dim3 grid((unsigned)ceil_div(D->n, 16), (unsigned)ceil_div(b, 16));
  hipLaunchKernelGGL(defl_p_mfma_kernel, grid, dim3(64), 0, ctx->stream, D->W32.as<c64>(), D->k, C, X, Y, b, D->n,
                     ldx, ldy, 1.0);
  LAUNCH_CHECK();
}

// Exact solve on the deflation space: with Q x_i = lambda_i x_i, D^-1 W W^H = X Lambda^-1 W^H,
// so for b:  C = W^H b,  e0 = X Lambda^-1 C  and  b - D e0 = (I - W W^H) b = r.
void defl_coarse_split(dmlmc_hier* H, const dmlmc_defl* D, const c128* b, int nrhs, c128* r, c128* e0,
                       dmlmc_precision prec) {
  dmlmc_ctx* ctx = H->ctx;
  const int64_t n = D->n;
  const int k = D->k;
  c128* C = (c128*)hier_buf(H, "dc_C", D->level, sizeof(c128) * (size_t)k * nrhs);
  c128* Cs = (c128*)hier_buf(H, "dc_Cs", D->level, sizeof(c128) * (size_t)k * nrhs);
  const unsigned g = (unsigned)ceil_div((int64_t)k * nrhs, 256);
  if (prec == DMLMC_MIXED) {
    defl_coeffs_mfma(ctx, D, b, nrhs, n, C, hier_devbuf(H, "dc_part", D->level));
    defl_project_mfma(ctx, D, b, r, nrhs, n, n, C);
    hipLaunchKernelGGL(scale_coeffs_kernel, dim3(g), dim3(256), 0, ctx->stream, C, D->lam_dev.as<double>(), k, nrhs,
                       -1.0, Cs);
    LAUNCH_CHECK();
    KTimer kt(ctx, "defl_gemm", 8.0 * n * k * nrhs);
    dim3 grid((unsigned)ceil_div(n, 16), (unsigned)ceil_div(nrhs, 16));
    hipLaunchKernelGGL(defl_p_mfma_kernel, grid, dim3(64), 0, ctx->stream, D->X32.as<c64>(), k, Cs, b, e0, nrhs, n, n,
                       n, 0.0);
    LAUNCH_CHECK();
  } else {
    defl_coeffs_fp64(ctx, D, b, nrhs, n, C);
    HIPCHK(hipMemcpyAsync(r, b, sizeof(c128) * (size_t)n * nrhs, hipMemcpyDeviceToDevice, ctx->stream));
    defl_project_fp64(ctx, D, r, nrhs, n, C);
    hipLaunchKernelGGL(scale_coeffs_kernel, dim3(g), dim3(256), 0, ctx->stream, C, D->lam_dev.as<double>(), k, nrhs,
                       -1.0, Cs);
    LAUNCH_CHECK();
    launch_fill_zero<c128>(ctx, e0, (size_t)n * nrhs);
    launch_multiaxpy<double>(ctx, D->X64.as<c128>(), k, e0, n, nrhs, n, n, Cs, k, 0, 1.0);
  }
}

// X <- (I - W W^H) X  (in place, precision per prec)
void defl_apply(dmlmc_hier* H, const dmlmc_defl* D, c128* X, int b, int64_t ldx, dmlmc_precision prec) {
  dmlmc_ctx* ctx = H->ctx;
  c128* C = (c128*)hier_buf(H, "df_C", D->level, sizeof(c128) * (size_t)D->k * b);
  if (prec == DMLMC_MIXED) {
    defl_coeffs_mfma(ctx, D, X, b, ldx, C, hier_devbuf(H, "df_part", D->level));
    defl_project_mfma(ctx, D, X, X, b, ldx, ldx, C);
  } else {
    defl_coeffs_fp64(ctx, D, X, b, ldx, C);
    defl_project_fp64(ctx, D, X, b, ldx, C);
  }
}

// ------------------------------------------------------------------ eigensolver
namespace {

void applyQ(dmlmc_ctx* ctx, const Level& L, const c128* x, c128* y, int nv) {
  apply_op<double>(ctx, L, x, y, nv, /*gamma5_left=*/true);
}

// M[i][r] = <Y_i, Z_r> (nsY x nv) -> host, row-major
std::vector<std::complex<double>> gram(dmlmc_hier* H, const c128* Y, int nsY, const c128* Z, int nv, int64_t n) {
  dmlmc_ctx* ctx = H->ctx;
  c128* G = (c128*)hier_buf(H, "eg_G", 0, sizeof(c128) * (size_t)nsY * nv);
  ts_gram(ctx, Y, nsY, Z, nv, n, G, hier_devbuf(H, "eg_part", 0));
  std::vector<c128> h((size_t)nsY * nv);
  HIPCHK(hipMemcpyAsync(h.data(), G, sizeof(c128) * h.size(), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  std::vector<std::complex<double>> M((size_t)nsY * nv);
  for (int r = 0; r < nv; ++r)
    for (int i = 0; i < nsY; ++i) M[(size_t)i * nv + r] = std::complex<double>(h[(size_t)r * nsY + i].x, h[(size_t)r * nsY + i].y);
  return M;
}

// out_r = sum_i S[i][r] Y_i (S host nsY x nv row-major); out must not alias Y
void rotate(dmlmc_hier* H, const c128* Y, int nsY, const std::vector<std::complex<double>>& S, int nv, c128* out,
            int64_t n) {
  dmlmc_ctx* ctx = H->ctx;
  std::vector<c128> h((size_t)nv * nsY);
  for (int r = 0; r < nv; ++r)
    for (int i = 0; i < nsY; ++i) h[(size_t)r * nsY + i] = cmk(S[(size_t)i * nv + r].real(), S[(size_t)i * nv + r].imag());
  c128* hd = (c128*)hier_buf(H, "eg_S", 0, sizeof(c128) * h.size());
  HIPCHK(hipMemcpyAsync(hd, h.data(), sizeof(c128) * h.size(), hipMemcpyHostToDevice, ctx->stream));
  ts_rotate(ctx, Y, nsY, hd, nv, n, out);
  HIPCHK(hipStreamSynchronize(ctx->stream));
}

// From this order on, the Rayleigh-Ritz and orthonormalisation matrices are factored on
// the device (parallel Jacobi, jacobi.hip) instead of on the host, whose O(m^3) dense
// solvers take minutes at the orders of a fine-level deflation with k in the thousands.
constexpr int DEVICE_RR_MIN = 512;

// Eigenpairs of the Hermitian Gram-type matrix G (device, column-major m x m): w ascending
// (host), S the eigenvectors (device, column-major, the rotate layout).
void eigh_device(dmlmc_hier* H, const c128* G, int m, c128* S, std::vector<double>& w) {
  const JacobiResult jr = jacobi_eigh(H->ctx, G, m, S, w, hier_devbuf(H, "eg_jac", 0), 1e-12, 40);
  if (!jr.converged) throw DmlmcError(DMLMC_ENUMERIC, "device Jacobi eigensolver did not converge");
  if (H->ctx->verbose)
    std::fprintf(stderr, "[dmlmc] device Rayleigh-Ritz of order %d: %d Jacobi sweeps\n", m, jr.sweeps);
}

// Rayleigh-Ritz step on the device: S (device) and w (host) from M = <A_i, B_r> (na = nb = m)
void rr_device(dmlmc_hier* H, const c128* A, const c128* B, int m, int64_t n, c128* S, std::vector<double>& w) {
  c128* G = (c128*)hier_buf(H, "eg_Gd", 0, sizeof(c128) * (size_t)m * m);
  ts_gram(H->ctx, A, m, B, m, n, G, hier_devbuf(H, "eg_part", 0));
  eigh_device(H, G, m, S, w);
}

// T[i][c] = conj(U(i, c)) sc[c] (U device, column-major m x m): the rows of U diag(sc) as
// vectors, so that their Gram matrix is U diag(sc^2) U^H
__global__ void scaled_rows_kernel(const c128* __restrict__ U, int m, const double* __restrict__ sc,
                                   c128* __restrict__ T) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)m * m) return;
  const int c = (int)(t % m), i = (int)(t / m);
  const c128 u = U[(int64_t)c * m + i];
  T[t] = cmk(u.x * sc[c], -u.y * sc[c]);
}

// Orthonormalise the ns columns of Y, twice: by Cholesky QR (host) below DEVICE_RR_MIN,
// else on the device by the symmetric (Loewdin) form Y <- Y G^-1/2, G = Y^H Y = U diag(g)
// U^H: the orthonormal basis closest to Y, so that a basis of nearly orthogonal Ritz
// vectors stays nearly diagonal for the Rayleigh-Ritz step that follows.  Returns false
// if the Gram matrix is not positive definite.
bool cholqr2(dmlmc_hier* H, c128*& Y, c128*& T, int ns, int64_t n) {
  if (ns >= DEVICE_RR_MIN) {
    dmlmc_ctx* ctx = H->ctx;
    c128* S = (c128*)hier_buf(H, "eg_Sd", 0, sizeof(c128) * (size_t)ns * ns);
    c128* Ur = (c128*)hier_buf(H, "eg_Ur", 0, sizeof(c128) * (size_t)ns * ns);
    c128* Gi = (c128*)hier_buf(H, "eg_Gi", 0, sizeof(c128) * (size_t)ns * ns);
    double* sc = (double*)hier_buf(H, "eg_sc", 0, sizeof(double) * ns);
    std::vector<double> g;
    for (int pass = 0; pass < 2; ++pass) {
      rr_device(H, Y, Y, ns, n, S, g);
      if (!(g[0] > 1e-14 * g[ns - 1])) return false;
      std::vector<double> f(ns);
      for (int c = 0; c < ns; ++c) f[c] = std::pow(g[c], -0.25);
      HIPCHK(hipMemcpyAsync(sc, f.data(), sizeof(double) * ns, hipMemcpyHostToDevice, ctx->stream));
      hipLaunchKernelGGL(scaled_rows_kernel, dim3((unsigned)ceil_div((int64_t)ns * ns, 256)), dim3(256), 0,
                         ctx->stream, S, ns, sc, Ur);
      LAUNCH_CHECK();
      ts_gram(ctx, Ur, ns, Ur, ns, ns, Gi, hier_devbuf(H, "eg_part", 0));  // G^-1/2, column-major
      ts_rotate(ctx, Y, ns, Gi, ns, n, T);
      HIPCHK(hipStreamSynchronize(ctx->stream));
      std::swap(Y, T);
    }
    return true;
  }
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<std::complex<double>> G = gram(H, Y, ns, Y, ns, n);  // G[i][r] = <Y_i, Y_r>
    // G = R^H R with R upper; cholesky_lower gives G = L L^H, so R = L^H and Y R^-1 = Y L^-H
    if (!cholesky_lower(ns, G)) return false;
    lower_inverse(ns, G);  // G = L^-1
    // S = L^-H: S[i][r] = conj(Linv[r][i])
    std::vector<std::complex<double>> S((size_t)ns * ns);
    for (int i = 0; i < ns; ++i)
      for (int r = 0; r < ns; ++r) S[(size_t)i * ns + r] = std::conj(G[(size_t)r * ns + i]);
    rotate(H, Y, ns, S, ns, T, n);
    std::swap(Y, T);
  }
  return true;
}

}  // namespace

// Returns the number of subspace iterations; fills X (k x n, device), lambda (host).
EigResult eig_coarsest(dmlmc_hier* H, int level, int k, double tol, c128* Xout) {
  dmlmc_ctx* ctx = H->ctx;
  const Level& L = H->lv[level - 1];
  const int64_t n = L.n();
  const int ns = (int)std::min<int64_t>(n / 2, k + std::max(8, k / 2));
  REQUIRE(ns >= k, "deflation subspace larger than half the level dimension");
  EigResult res;
  // ||Q||_inf bound
  double qnorm = 0.0;
  if (L.fine) {
    // row sums of |D|: |m0 + 2| on the diagonal, and each of the four hops -(1 -+ s_mu) U / 2
    // has entries of modulus 1/2, two per row
    qnorm = std::fabs(L.m0 + 2.0) + 4.0;
  } else {
    double* rs = (double*)hier_buf(H, "eg_rs", 0, sizeof(double) * n);
    hipLaunchKernelGGL(rowsum_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, ctx->stream,
                       L.A64.as<c128>(), L.sites(), L.dofs, rs);
    LAUNCH_CHECK();
    std::vector<double> h(n);
    HIPCHK(hipMemcpyAsync(h.data(), rs, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    qnorm = *std::max_element(h.begin(), h.end());
  }
  const double bq = qnorm * qnorm * 1.01;
  c128* Y = (c128*)hier_buf(H, "eg_Y", 0, sizeof(c128) * (size_t)ns * n);
  c128* T = (c128*)hier_buf(H, "eg_T", 0, sizeof(c128) * (size_t)ns * n);
  c128* Z = (c128*)hier_buf(H, "eg_Z", 0, sizeof(c128) * (size_t)ns * n);
  c128* Q1 = (c128*)hier_buf(H, "eg_Q1", 0, sizeof(c128) * (size_t)ns * n);
  c128* Y0 = (c128*)hier_buf(H, "eg_Y0", 0, sizeof(c128) * (size_t)ns * n);
  launch_z4(ctx, Y, n, 0x5eed5eedull, level + 64, 0, ns);
  if (!cholqr2(H, Y, T, ns, n)) throw DmlmcError(DMLMC_ENUMERIC, "eigensolver: start block is rank-deficient");
  double a = bq / 64.0;
  std::vector<std::complex<double>> S;
  const int maxit = 100;
  int it = 0;
  std::vector<double> mu, th1;
  std::vector<std::complex<double>> S1;
  for (; it < maxit; ++it) {
    // Rayleigh-Ritz with Q^2 on the whole subspace: Y ordered by the Ritz values mu of Q^2
    applyQ(ctx, L, Y, Z, ns);
    if (ns >= DEVICE_RR_MIN) {
      c128* Sd = (c128*)hier_buf(H, "eg_Sd", 0, sizeof(c128) * (size_t)ns * ns);
      rr_device(H, Z, Z, ns, n, Sd, mu);
      ts_rotate(ctx, Y, ns, Sd, ns, n, T);
    } else {
      std::vector<std::complex<double>> H2 = gram(H, Z, ns, Z, ns, n);
      if (eigh_tridiag(ns, H2, mu, S) < 0) throw DmlmcError(DMLMC_ENUMERIC, "Rayleigh-Ritz eigensolve failed");
      rotate(H, Y, ns, S, ns, T, n);
    }
    std::swap(Y, T);
    // Rayleigh-Ritz with Q on the k leading vectors (their span converges to the invariant
    // subspace of the k smallest |lambda|, which Q maps into itself; an RR with Q on the
    // whole subspace would give spurious Ritz values near 0 from pairs +lambda, -lambda'
    // with similar |lambda| at the subspace boundary)
    applyQ(ctx, L, Y, Z, k);
    if (k >= DEVICE_RR_MIN) {
      c128* Sd = (c128*)hier_buf(H, "eg_Sd", 0, sizeof(c128) * (size_t)ns * ns);
      rr_device(H, Y, Z, k, n, Sd, th1);
      ts_rotate(ctx, Y, k, Sd, k, n, Q1);  // Ritz vectors of Q -> Q1[0..k)
      ts_rotate(ctx, Z, k, Sd, k, n, Y0);  // Q times them -> Y0[0..k)
    } else {
      std::vector<std::complex<double>> H1 = gram(H, Y, k, Z, k, n);
      if (eigh_tridiag(k, H1, th1, S1) < 0) throw DmlmcError(DMLMC_ENUMERIC, "Rayleigh-Ritz eigensolve failed");
      rotate(H, Y, k, S1, k, Q1, n);   // Ritz vectors of Q -> Q1[0..k)
      rotate(H, Z, k, S1, k, Y0, n);   // Q times them -> Y0[0..k)
    }
    double* th = (double*)hier_buf(H, "eg_th", 0, sizeof(double) * k);
    HIPCHK(hipMemcpyAsync(th, th1.data(), sizeof(double) * k, hipMemcpyHostToDevice, ctx->stream));
    hipLaunchKernelGGL(ritz_res_kernel, dim3((unsigned)ceil_div(n * k, 256)), dim3(256), 0, ctx->stream, Y0, Q1, th, n,
                       k);
    LAUNCH_CHECK();
    double* nr = (double*)hier_buf(H, "eg_nr", 0, sizeof(double) * k);
    launch_norms2<double>(ctx, Y0, n, k, n, nr);
    std::vector<double> rn(k);
    HIPCHK(hipMemcpyAsync(rn.data(), nr, sizeof(double) * k, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    double worst = 0.0;
    for (int i = 0; i < k; ++i) worst = std::max(worst, std::sqrt(rn[i]));
    res.max_residual = worst / qnorm;
    if (ctx->verbose)
      std::fprintf(stderr, "[dmlmc] eigensolver level %d, k %d, subspace %d: iteration %d, max residual %.3e (tol %.1e)\n",
                   level, k, ns, it, res.max_residual, tol);
    if (worst <= tol * qnorm) break;
    if (it + 1 == maxit) break;
    // filter interval: damp [a, bq] with a = the largest Ritz value of Q^2 in the subspace
    a = std::min(std::max(mu[ns - 1], 1e-12 * bq), 0.5 * bq);
    const double e = 0.5 * (bq - a), c = 0.5 * (bq + a);
    // degree: the filter should amplify the largest wanted Ritz value of Q^2 (lk) over the
    // damped interval by about e^4 per outer step: T_deg(x_k) = cosh(deg acosh(x_k))
    const double lk = std::max(mu[k - 1], 0.0);
    const double xk = 1.0 + 2.0 * std::max(a - lk, 1e-3 * a) / (bq - a);
    const int deg = (int)std::min(400.0, std::max(8.0, std::ceil(4.0 / std::acosh(xk))));
    res.degree_sum += deg;
    // Chebyshev recurrence on Q^2: T0 = Y, T1 = (Q^2 - c)/e Y, Tj = 2 (Q^2 - c)/e T_{j-1} - T_{j-2}
    c128* prev = Y0;
    c128* cur = Y;
    c128* nxt = T;
    const int64_t tot = n * ns;
    for (int j = 1; j <= deg; ++j) {
      applyQ(ctx, L, cur, Q1, ns);
      applyQ(ctx, L, Q1, Z, ns);
      hipLaunchKernelGGL(cheb_kernel, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, ctx->stream, Z, cur, prev,
                         nxt, tot, (j == 1 ? 1.0 : 2.0) / e, c, j == 1 ? 1 : 0);
      LAUNCH_CHECK();
      c128* t = prev;
      prev = cur;
      cur = nxt;
      nxt = t;
    }
    // cur holds the filtered block; keep the three buffers distinct for the next round
    Y = cur;
    T = nxt;
    Y0 = prev;
    if (!cholqr2(H, Y, T, ns, n)) {
      orthonormalise(H, Y, ns, n);
    }
  }
  res.iters = it;
  res.converged = res.max_residual <= tol;
  // the wanted pairs (Ritz vectors in Q1) in order of |lambda|, then lambda
  std::vector<int> order(k);
  for (int i = 0; i < k; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int i, int j) {
    const double ai = std::fabs(th1[i]), aj = std::fabs(th1[j]);
    return ai < aj || (ai == aj && th1[i] < th1[j]);
  });
  res.lambda.resize(k);
  for (int i = 0; i < k; ++i) {
    res.lambda[i] = th1[order[i]];
    HIPCHK(hipMemcpyAsync(Xout + (int64_t)i * n, Q1 + (int64_t)order[i] * n, sizeof(c128) * n,
                          hipMemcpyDeviceToDevice, ctx->stream));
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return res;
}

void defl_finish(dmlmc_hier* H, dmlmc_defl* D) {
  dmlmc_ctx* ctx = H->ctx;
  const Level& L = H->lv[D->level - 1];
  const int64_t n = D->n;
  D->W64.alloc(sizeof(c128) * (size_t)D->k * n);
  hipLaunchKernelGGL(gamma5_kernel, dim3((unsigned)ceil_div(n * D->k, 256)), dim3(256), 0, ctx->stream,
                     D->X64.as<c128>(), D->W64.as<c128>(), n, L.dofs, D->k);
  LAUNCH_CHECK();
  D->W32.alloc(sizeof(c64) * (size_t)D->k * n);
  launch_cast<float, double>(ctx, D->W64.as<c128>(), D->W32.as<c64>(), n * D->k, 1, 0, 0);
  D->X32.alloc(sizeof(c64) * (size_t)D->k * n);
  launch_cast<float, double>(ctx, D->X64.as<c128>(), D->X32.as<c64>(), n * D->k, 1, 0, 0);
  D->lam_dev.alloc(sizeof(double) * D->k);
  HIPCHK(hipMemcpyAsync(D->lam_dev.p, D->lambda.data(), sizeof(double) * D->k, hipMemcpyHostToDevice, ctx->stream));
  // tr(D^-1 Pi) = sum_i x_i^H Gamma5 x_i / lambda_i = sum_i <x_i, w_i> / lambda_i
  c128* dd = (c128*)hier_buf(H, "df_dd", D->level, sizeof(c128) * D->k);
  launch_dots<double, double>(ctx, D->X64.as<c128>(), D->W64.as<c128>(), n, D->k, n, n, dd);
  std::vector<c128> h(D->k);
  HIPCHK(hipMemcpyAsync(h.data(), dd, sizeof(c128) * D->k, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  double tr = 0.0;
  for (int i = 0; i < D->k; ++i) tr += D->kind == 1 ? h[i].x * D->lambda[i] : h[i].x / D->lambda[i];
  D->tr_defl = tr;
}

// ------------------------------------------------------------------ difference levels
void apply_J(dmlmc_hier* H, int a, int b, const c128* V, c128* W, int nv, dmlmc_precision prec, double rtol) {
  dmlmc_ctx* ctx = H->ctx;
  const Level& La = H->lv[a - 1];
  const Level& Lb = H->lv[b - 1];
  const int64_t na = La.n(), nbn = Lb.n();
  constexpr int CH = 32;  // vectors per multi-RHS solve
  for (int c0 = 0; c0 < nv; c0 += CH) {
    const int m = std::min(CH, nv - c0);
    const c128* v = V + (int64_t)c0 * na;
    c128* w = W + (int64_t)c0 * na;
    c128* t1 = (c128*)hier_buf(H, "jq_t1", a, sizeof(c128) * (size_t)m * na);
    // Q_a^-1 v = D_a^-1 Gamma5 v
    hipLaunchKernelGGL(gamma5_kernel, dim3((unsigned)ceil_div(na * m, 256)), dim3(256), 0, ctx->stream, v, t1, na,
                       La.dofs, m);
    LAUNCH_CHECK();
    SolveResult r1 = solve_level(H, a, t1, w, m, prec, rtol, 5000);
    if (!r1.converged) throw DmlmcError(DMLMC_ENOCONV, "a solve inside the difference operator did not converge");
    // P_ab Q_b^-1 P_ab^H v
    const c128* cur = v;
    for (int l = a; l < b; ++l) {
      c128* nxt = (c128*)hier_buf(H, "jq_r", l + 1, sizeof(c128) * (size_t)m * H->lv[l].n());
      launch_restrict<double>(ctx, H->lv[l - 1], cur, nxt, m);
      cur = nxt;
    }
    c128* t2 = (c128*)hier_buf(H, "jq_t2", b, sizeof(c128) * (size_t)m * nbn);
    c128* z2 = (c128*)hier_buf(H, "jq_z2", b, sizeof(c128) * (size_t)m * nbn);
    hipLaunchKernelGGL(gamma5_kernel, dim3((unsigned)ceil_div(nbn * m, 256)), dim3(256), 0, ctx->stream, cur, t2, nbn,
                       Lb.dofs, m);
    LAUNCH_CHECK();
    SolveResult r2 = solve_level(H, b, t2, z2, m, prec, rtol, 5000);
    if (!r2.converged) throw DmlmcError(DMLMC_ENOCONV, "a solve inside the difference operator did not converge");
    cur = z2;
    for (int l = b - 1; l >= a; --l) {
      c128* nxt = l == a ? t1 : (c128*)hier_buf(H, "jq_p", l, sizeof(c128) * (size_t)m * H->lv[l - 1].n());
      launch_prolong<double>(ctx, H->lv[l - 1], cur, nxt, m, false);
      cur = nxt;
    }
    // w = Q_a^-1 v - P Q_b^-1 P^H v: t1 = w - t1, then w = t1
    launch_xmy<double>(ctx, w, t1, na, m, na, na);
    HIPCHK(hipMemcpyAsync(w, t1, sizeof(c128) * (size_t)m * na, hipMemcpyDeviceToDevice, ctx->stream));
  }
}

double difference_trace_term(dmlmc_hier* H, const dmlmc_defl* D, dmlmc_precision prec, double rtol) {
  dmlmc_ctx* ctx = H->ctx;
  const int64_t n = D->n;
  c128* JX = (c128*)hier_buf(H, "ed_JX", 0, sizeof(c128) * (size_t)D->k * n);
  apply_J(H, D->level, D->level_b, D->X64.as<c128>(), JX, D->k, prec, rtol);
  c128* dd = (c128*)hier_buf(H, "ed_dd", 0, sizeof(c128) * D->k);
  launch_dots<double, double>(ctx, D->W64.as<c128>(), JX, n, D->k, n, n, dd);  // <Gamma5 x_i, J x_i>
  std::vector<c128> h(D->k);
  HIPCHK(hipMemcpyAsync(h.data(), dd, sizeof(c128) * D->k, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  double tr = 0.0;
  for (int i = 0; i < D->k; ++i) tr += h[i].x;
  return tr;
}

namespace {

// indices of the first `count` values ordered by |theta| descending, then theta descending
std::vector<int> largest_first(const std::vector<double>& th, int count) {
  std::vector<int> o(th.size());
  for (size_t i = 0; i < th.size(); ++i) o[i] = (int)i;
  std::sort(o.begin(), o.end(), [&](int i, int j) {
    const double ai = std::fabs(th[i]), aj = std::fabs(th[j]);
    return ai > aj || (ai == aj && th[i] > th[j]);
  });
  o.resize(count);
  return o;
}

}  // namespace

EigResult eig_difference(dmlmc_hier* H, int a, int b, int k, double tol, double solve_rtol, dmlmc_precision prec,
                         c128* Xout) {
  dmlmc_ctx* ctx = H->ctx;
  const int64_t n = H->lv[a - 1].n();
  // the top of the spectrum of J is flat (many |lambda| close to the largest), so the
  // retained subspace carries 32 (or k) vectors beyond the wanted ones
  const int ns = (int)std::min<int64_t>(n / 2 - k, k + std::max(32, k));
  REQUIRE(ns >= k, "deflation subspace too large for the level");
  // block Davidson: the basis grows by the residual block of the k wanted Ritz pairs
  // (orthogonalised against it) until it holds ns + 8 k vectors, then restarts from the
  // ns leading Ritz vectors
  const int cap = (int)std::min<int64_t>(n / 2, ns + 8 * k);
  EigResult res;
  c128* Y = (c128*)hier_buf(H, "ed_Y", 0, sizeof(c128) * (size_t)cap * n);
  c128* Z = (c128*)hier_buf(H, "ed_Z", 0, sizeof(c128) * (size_t)cap * n);
  c128* T = (c128*)hier_buf(H, "ed_T", 0, sizeof(c128) * (size_t)cap * n);
  c128* U = (c128*)hier_buf(H, "ed_U", 0, sizeof(c128) * (size_t)cap * n);
  c128* Rb = (c128*)hier_buf(H, "ed_R", 0, sizeof(c128) * (size_t)k * n);
  c128* Rt = (c128*)hier_buf(H, "ed_Rt", 0, sizeof(c128) * (size_t)k * n);
  c128* C = (c128*)hier_buf(H, "ed_C", 0, sizeof(c128) * (size_t)cap * k);
  launch_z4(ctx, Y, n, 0x5eed5eedull, a + 96, 0, ns);
  if (!cholqr2(H, Y, T, ns, n)) throw DmlmcError(DMLMC_ENUMERIC, "eigensolver: start block is rank-deficient");
  apply_J(H, a, b, Y, Z, ns, prec, solve_rtol);
  int cur = ns;
  const int maxit = 400;
  std::vector<double> th, thk(k);
  std::vector<std::complex<double>> S;
  double* thd = (double*)hier_buf(H, "ed_th", 0, sizeof(double) * k);
  double* nrd = (double*)hier_buf(H, "ed_nr", 0, sizeof(double) * k);
  auto columns = [&](const std::vector<int>& ord, int cnt) {
    std::vector<std::complex<double>> Sc((size_t)cur * cnt);
    for (int c = 0; c < cnt; ++c)
      for (int i = 0; i < cur; ++i) Sc[(size_t)i * cnt + c] = S[(size_t)i * cur + ord[c]];
    return Sc;
  };
  int it = 0;
  for (;; ++it) {
    // Rayleigh-Ritz on span(Y): J is Hermitian, so the projected matrix is symmetrised
    std::vector<std::complex<double>> G = gram(H, Y, cur, Z, cur, n);
    for (int i = 0; i < cur; ++i)
      for (int r = i; r < cur; ++r) {
        const std::complex<double> v = 0.5 * (G[(size_t)i * cur + r] + std::conj(G[(size_t)r * cur + i]));
        G[(size_t)i * cur + r] = v;
        G[(size_t)r * cur + i] = std::conj(v);
      }
    if (eigh_tridiag(cur, G, th, S) < 0) throw DmlmcError(DMLMC_ENUMERIC, "Rayleigh-Ritz eigensolve failed");
    const std::vector<int> ord = largest_first(th, std::min(cur, ns));
    for (int c = 0; c < k; ++c) thk[c] = th[ord[c]];
    // the k wanted Ritz vectors (T) and J applied to them (U); residuals U - theta T -> Rb
    const std::vector<std::complex<double>> Sk = columns(ord, k);
    rotate(H, Y, cur, Sk, k, T, n);
    rotate(H, Z, cur, Sk, k, U, n);
    HIPCHK(hipMemcpyAsync(Rb, U, sizeof(c128) * (size_t)k * n, hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(thd, thk.data(), sizeof(double) * k, hipMemcpyHostToDevice, ctx->stream));
    hipLaunchKernelGGL(ritz_res_kernel, dim3((unsigned)ceil_div(n * k, 256)), dim3(256), 0, ctx->stream, Rb, T, thd, n,
                       k);
    LAUNCH_CHECK();
    launch_norms2<double>(ctx, Rb, n, k, n, nrd);
    std::vector<double> rn(k);
    HIPCHK(hipMemcpyAsync(rn.data(), nrd, sizeof(double) * k, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const double scale = std::fabs(thk[0]);
    double worst = 0.0;
    for (int i = 0; i < k; ++i) worst = std::max(worst, std::sqrt(rn[i]));
    res.max_residual = scale > 0.0 ? worst / scale : worst;
    if (res.max_residual <= tol || it + 1 >= maxit) break;
    if (cur + k > cap) {
      // restart from the ns leading Ritz vectors
      const std::vector<std::complex<double>> Sn = columns(ord, ns);
      rotate(H, Y, cur, Sn, ns, T, n);
      rotate(H, Z, cur, Sn, ns, U, n);
      std::swap(Y, T);
      std::swap(Z, U);
      cur = ns;
    }
    // expansion by the residual block, orthogonalised against the basis twice and within itself
    for (int pass = 0; pass < 2; ++pass) {
      ts_gram(ctx, Y, cur, Rb, k, n, C, hier_devbuf(H, "eg_part", 0));  // C[r][i] = <Y_i, R_r>
      ts_rotate(ctx, Y, cur, C, k, n, Rt);                                 // Rt_r = sum_i C[r][i] Y_i
      launch_xmy<double>(ctx, Rb, Rt, n, k, n, n);                         // Rt = R - Rt
      std::swap(Rb, Rt);
    }
    c128* R = Rb;
    c128* tmp = Rt;
    if (!cholqr2(H, R, tmp, k, n)) orthonormalise(H, R, k, n);
    HIPCHK(hipMemcpyAsync(Y + (int64_t)cur * n, R, sizeof(c128) * (size_t)k * n, hipMemcpyDeviceToDevice, ctx->stream));
    apply_J(H, a, b, Y + (int64_t)cur * n, Z + (int64_t)cur * n, k, prec, solve_rtol);
    cur += k;
  }
  res.iters = it + 1;
  res.converged = res.max_residual <= tol;
  res.lambda.assign(thk.begin(), thk.end());
  HIPCHK(hipMemcpyAsync(Xout, T, sizeof(c128) * (size_t)k * n, hipMemcpyDeviceToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return res;
}
