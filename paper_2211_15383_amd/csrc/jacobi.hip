// Dense Hermitian eigensolver on the device (FP64): parallel cyclic two-sided Jacobi, for
// the Rayleigh-Ritz matrices of the large eigensolves (orders of several thousand), where
// the host tridiagonal solver takes minutes.
//
// The matrix M (order n, even) and the eigenvector matrix V are column-major on the device.
// A sweep is n - 1 rounds of the round-robin (circle) pairing of the indices 0..n-1: in
// round r, pair 0 is (n - 1, r) and pair k >= 1 is ((r + k) mod (n - 1), (r - k) mod (n - 1)),
// so every index is in exactly one pair per round and every (p, q) is met once per sweep.
// All n / 2 rotations of a round are independent and applied at once:
//   * for pair (p, q) with M_pq = |c| e^{i phi}, a = M_pp, b = M_qq, the unitary
//     G = diag(1, e^{-i phi}) R, R = [[cs, sn], [-sn, cs]] the real rotation that
//     annihilates [[a, |c|], [|c|, b]] (t = tan theta from tau = (b - a) / (2 |c|), the
//     smaller root), is skipped when |c| <= 1e-15 sqrt(|a b|) or |c| <= 1e-17 max_i |M_ii|
//     (the largest diagonal entry of the input);
//   * M <- G^H M G on every 2 x 2 block (rows of pair k, columns of pair l), and V <- V G.
// Sweeps repeat until the largest relative off-diagonal entry met in a sweep is below
// tol; the eigenvalues are the diagonal of M.  Each rotation is unitary, so the result
// is accurate to a few ulps of ||M|| times the number of sweeps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "common.h"
#include "jacobi.h"

namespace {

struct Rot {
  double cs, sn;  // real rotation
  double er, ei;  // e^{-i phi}
};

__device__ __forceinline__ void pair_of(int r, int k, int n, int& p, int& q) {
  const int m = n - 1;
  if (k == 0) {
    p = m;
    q = r;
  } else {
    p = (r + k) % m;
    q = (r - k + m) % m;
  }
}

__device__ __forceinline__ unsigned long long dbl_bits(double v) { return (unsigned long long)__double_as_longlong(v); }

// one thread per pair: the rotation of round r; offmax (bits of a non-negative double)
// takes the largest |M_pq| / sqrt(|M_pp M_qq|) met
__global__ __launch_bounds__(256) void jacobi_angles_kernel(const c128* __restrict__ M, int n, int r, double dmax,
                                                            Rot* __restrict__ rot, unsigned long long* offmax) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  double rel = 0.0;
  if (k < n / 2) {
    int p, q;
    pair_of(r, k, n, p, q);
    const double a = M[(int64_t)p * n + p].x, b = M[(int64_t)q * n + q].x;
    const c128 c = M[(int64_t)q * n + p];  // M(p, q), column-major
    const double ac = sqrt(c.x * c.x + c.y * c.y);
    const double scale = sqrt(fabs(a) * fabs(b));
    Rot g{1.0, 0.0, 1.0, 0.0};
    if (ac > 1e-300 && ac > 1e-15 * scale && ac > 1e-17 * dmax) {
      rel = ac / fmax(scale, 1e-15 * dmax);
      const double tau = (b - a) / (2.0 * ac);
      const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
      g.cs = 1.0 / sqrt(1.0 + t * t);
      g.sn = t * g.cs;
      g.er = c.x / ac;
      g.ei = -c.y / ac;
    }
    rot[k] = g;
  }
  // wavefront maximum, then one atomic per wavefront
  for (int off = 32; off > 0; off >>= 1) rel = fmax(rel, __shfl_xor(rel, off, 64));
  if ((threadIdx.x & 63) == 0 && rel > 0.0) atomicMax(offmax, dbl_bits(rel));
}

__device__ __forceinline__ c128 cmul(c128 a, double er, double ei) { return cmk(a.x * er - a.y * ei, a.x * ei + a.y * er); }

// G columns: g_p = (cs, -sn e), g_q = (sn, cs e) with e = e^{-i phi} in the q row:
//   (X G)(:, p) = cs X(:, p) - sn e X(:, q),  (X G)(:, q) = sn X(:, p) + cs e X(:, q)
// G^H rows: (G^H X)(p, :) = cs X(p, :) - sn conj(e) X(q, :),
//           (G^H X)(q, :) = sn X(p, :) + cs conj(e) X(q, :)
// One thread per (k, l): the 2 x 2 block of M at rows of pair k and columns of pair l.
__global__ __launch_bounds__(256) void jacobi_apply_kernel(c128* __restrict__ M, int n, int r,
                                                           const Rot* __restrict__ rot) {
  const int h = n / 2;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)h * h) return;
  const int k = (int)(t % h), l = (int)(t / h);
  int pk, qk, pl, ql;
  pair_of(r, k, n, pk, qk);
  pair_of(r, l, n, pl, ql);
  const Rot gk = rot[k], gl = rot[l];
  c128* cp = M + (int64_t)pl * n;
  c128* cq = M + (int64_t)ql * n;
  const c128 x_pp = cp[pk], x_qp = cp[qk], x_pq = cq[pk], x_qq = cq[qk];
  // columns: Y = X G_l
  const c128 eq_p = cmul(x_pq, gl.er, gl.ei), eq_q = cmul(x_qq, gl.er, gl.ei);
  const c128 y_pp = cmk(gl.cs * x_pp.x - gl.sn * eq_p.x, gl.cs * x_pp.y - gl.sn * eq_p.y);
  const c128 y_qp = cmk(gl.cs * x_qp.x - gl.sn * eq_q.x, gl.cs * x_qp.y - gl.sn * eq_q.y);
  const c128 y_pq = cmk(gl.sn * x_pp.x + gl.cs * eq_p.x, gl.sn * x_pp.y + gl.cs * eq_p.y);
  const c128 y_qq = cmk(gl.sn * x_qp.x + gl.cs * eq_q.x, gl.sn * x_qp.y + gl.cs * eq_q.y);
  // rows: Z = G_k^H Y
  const c128 fq_p = cmul(y_qp, gk.er, -gk.ei), fq_q = cmul(y_qq, gk.er, -gk.ei);
  c128 z_pp = cmk(gk.cs * y_pp.x - gk.sn * fq_p.x, gk.cs * y_pp.y - gk.sn * fq_p.y);
  c128 z_pq = cmk(gk.cs * y_pq.x - gk.sn * fq_q.x, gk.cs * y_pq.y - gk.sn * fq_q.y);
  c128 z_qp = cmk(gk.sn * y_pp.x + gk.cs * fq_p.x, gk.sn * y_pp.y + gk.cs * fq_p.y);
  c128 z_qq = cmk(gk.sn * y_pq.x + gk.cs * fq_q.x, gk.sn * y_pq.y + gk.cs * fq_q.y);
  if (k == l) {
    // the annihilated pair: exact zero off the diagonal, real diagonal
    z_pq = cmk(0.0, 0.0);
    z_qp = cmk(0.0, 0.0);
    z_pp.y = 0.0;
    z_qq.y = 0.0;
  }
  cp[pk] = z_pp;
  cp[qk] = z_qp;
  cq[pk] = z_pq;
  cq[qk] = z_qq;
}

// V <- V G: one thread per (row i, pair l)
__global__ __launch_bounds__(256) void jacobi_vectors_kernel(c128* __restrict__ V, int n, int r,
                                                             const Rot* __restrict__ rot) {
  const int h = n / 2;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * h) return;
  const int i = (int)(t % n), l = (int)(t / n);
  int pl, ql;
  pair_of(r, l, n, pl, ql);
  const Rot g = rot[l];
  c128* cp = V + (int64_t)pl * n;
  c128* cq = V + (int64_t)ql * n;
  const c128 vp = cp[i], vq = cmul(cq[i], g.er, g.ei);
  cp[i] = cmk(g.cs * vp.x - g.sn * vq.x, g.cs * vp.y - g.sn * vq.y);
  cq[i] = cmk(g.sn * vp.x + g.cs * vq.x, g.sn * vp.y + g.cs * vq.y);
}

// The Hermitian part of A (order n, column-major) into the top-left of M (order ne >= n);
// the rest zero, except
// a diagonal value `pad` on the padding indices (kept decoupled: their couplings are 0)
__global__ void jacobi_load_kernel(const c128* __restrict__ A, int n, c128* __restrict__ M, int ne, double pad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)ne * ne) return;
  const int i = (int)(t % ne), j = (int)(t / ne);
  if (i < n && j < n) {
    // Hermitian part (A(i, j) + conj(A(j, i))) / 2: the Gram-type inputs are Hermitian up
    // to rounding
    const c128 u = A[(int64_t)j * n + i], v = A[(int64_t)i * n + j];
    M[t] = cmk(0.5 * (u.x + v.x), 0.5 * (u.y - v.y));
  } else {
    M[t] = cmk(i == j ? pad : 0.0, 0.0);
  }
}

__global__ void jacobi_identity_kernel(c128* __restrict__ V, int ne) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)ne * ne) return;
  V[t] = cmk((t % ne) == (t / ne) ? 1.0 : 0.0, 0.0);
}

__global__ void jacobi_diag_kernel(const c128* __restrict__ M, int ne, double* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ne) d[i] = M[(int64_t)i * ne + i].x;
}

// out column c = V column perm[c], rows < n
__global__ void jacobi_gather_kernel(const c128* __restrict__ V, int ne, const int* __restrict__ perm, int n,
                                     c128* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * n) return;
  const int i = (int)(t % n), c = (int)(t / n);
  out[t] = V[(int64_t)perm[c] * ne + i];
}

__global__ void fill_u64_kernel(unsigned long long* p, unsigned long long v) { *p = v; }

}  // namespace

JacobiResult jacobi_eigh(dmlmc_ctx* ctx, const c128* A, int n, c128* S, std::vector<double>& w, DevBuf& work,
                         double tol, int max_sweeps) {
  REQUIRE(n >= 1, "eigenproblem of order < 1");
  const int ne = n + (n & 1);  // even order: one decoupled padding index if n is odd
  const size_t mat = sizeof(c128) * (size_t)ne * ne;
  const size_t rot_bytes = sizeof(Rot) * (size_t)(ne / 2);
  const size_t need = 2 * mat + rot_bytes + sizeof(double) * ne + sizeof(int) * ne + 64;
  work.ensure(need);
  char* base = static_cast<char*>(work.p);
  c128* M = reinterpret_cast<c128*>(base);
  c128* V = reinterpret_cast<c128*>(base + mat);
  Rot* rot = reinterpret_cast<Rot*>(base + 2 * mat);
  double* d = reinterpret_cast<double*>(base + 2 * mat + rot_bytes);
  int* perm = reinterpret_cast<int*>(base + 2 * mat + rot_bytes + sizeof(double) * ne);
  unsigned long long* offmax =
      reinterpret_cast<unsigned long long*>(base + 2 * mat + rot_bytes + sizeof(double) * ne + sizeof(int) * ne);
  offmax = reinterpret_cast<unsigned long long*>(((uintptr_t)offmax + 7) & ~(uintptr_t)7);
  const int64_t nn = (int64_t)ne * ne;
  // padding value above every eigenvalue of A (Gershgorin bound of the diagonal entries,
  // taken from the diagonal after the load: |lambda| <= ||A||_F <= n max|A_ij|)
  double pad = 0.0;
  if (ne != n) {
    std::vector<c128> h((size_t)n * n);
    HIPCHK(hipMemcpyAsync(h.data(), A, sizeof(c128) * h.size(), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    double fro = 0.0;
    for (const c128& v : h) fro += v.x * v.x + v.y * v.y;
    pad = 2.0 * std::sqrt(fro) + 1.0;
  }
  hipLaunchKernelGGL(jacobi_load_kernel, dim3((unsigned)ceil_div(nn, 256)), dim3(256), 0, ctx->stream, A, n, M, ne, pad);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(jacobi_identity_kernel, dim3((unsigned)ceil_div(nn, 256)), dim3(256), 0, ctx->stream, V, ne);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(jacobi_diag_kernel, dim3((unsigned)ceil_div(ne, 256)), dim3(256), 0, ctx->stream, M, ne, d);
  LAUNCH_CHECK();
  std::vector<double> d0(ne);
  HIPCHK(hipMemcpyAsync(d0.data(), d, sizeof(double) * ne, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  double dmax = 0.0;
  for (double v : d0) dmax = std::max(dmax, std::fabs(v));
  if (!std::isfinite(dmax)) throw DmlmcError(DMLMC_ENUMERIC, "NaN/Inf in the Jacobi eigensolver input");
  const int h = ne / 2;
  const unsigned ga = (unsigned)ceil_div(h, 256);
  const unsigned gm = (unsigned)ceil_div((int64_t)h * h, 256);
  const unsigned gv = (unsigned)ceil_div((int64_t)ne * h, 256);
  JacobiResult res;
  for (int sweep = 0; sweep < max_sweeps && ne > 1; ++sweep) {
    hipLaunchKernelGGL(fill_u64_kernel, dim3(1), dim3(1), 0, ctx->stream, offmax, 0ull);
    LAUNCH_CHECK();
    for (int r = 0; r < ne - 1; ++r) {
      hipLaunchKernelGGL(jacobi_angles_kernel, dim3(ga), dim3(256), 0, ctx->stream, M, ne, r, dmax, rot, offmax);
      hipLaunchKernelGGL(jacobi_apply_kernel, dim3(gm), dim3(256), 0, ctx->stream, M, ne, r, rot);
      hipLaunchKernelGGL(jacobi_vectors_kernel, dim3(gv), dim3(256), 0, ctx->stream, V, ne, r, rot);
    }
    LAUNCH_CHECK();
    unsigned long long bits = 0;
    HIPCHK(hipMemcpyAsync(&bits, offmax, sizeof(bits), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    double rel;
    std::memcpy(&rel, &bits, sizeof(rel));
    res.sweeps = sweep + 1;
    res.offmax = rel;
    if (!std::isfinite(rel)) throw DmlmcError(DMLMC_ENUMERIC, "NaN/Inf in the Jacobi eigensolver");
    if (rel <= tol) break;
  }
  res.converged = res.offmax <= tol;
  hipLaunchKernelGGL(jacobi_diag_kernel, dim3((unsigned)ceil_div(ne, 256)), dim3(256), 0, ctx->stream, M, ne, d);
  LAUNCH_CHECK();
  std::vector<double> dh(ne);
  HIPCHK(hipMemcpyAsync(dh.data(), d, sizeof(double) * ne, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  std::vector<int> order(ne);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return dh[a] < dh[b]; });
  // the padding index carries the largest diagonal value: it sorts last and is dropped
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = dh[order[i]];
  HIPCHK(hipMemcpyAsync(perm, order.data(), sizeof(int) * ne, hipMemcpyHostToDevice, ctx->stream));
  hipLaunchKernelGGL(jacobi_gather_kernel, dim3((unsigned)ceil_div((int64_t)n * n, 256)), dim3(256), 0, ctx->stream, V,
                     ne, perm, n, S);
  LAUNCH_CHECK();
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return res;
}
