// Fused Gram-Schmidt passes of the Arnoldi step (classical Gram-Schmidt with one
// reorthogonalisation, FP64 arithmetic), one launch per pass:
//   A: h1 = V^H w                         (read V, w)
//   B: w' = w - V h1, ||w'||^2             (read V, w; write w')
//   C: h2 = V^H w', then the Hessenberg column, Givens rotation and residual estimate
//      (read V, w')
//   D: v_{j+1} = (w' - V h2) / beta, beta^2 = ||w'||^2 - |h2|^2   (read V, w'; write v)
// Each reduction is finished by the last workgroup of its RHS (partials summed in a fixed
// order, so results are deterministic); the completion counters reset themselves.
#include <cmath>

#include "solver.h"

namespace {

constexpr int NBMAX = 32;        // basis vectors per pass
constexpr int NVMAX = 2 * NBMAX; // reduced doubles per pass

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Reduces acc[0..nv) over the 256-thread block, writes the block partials, and lets the
// last block of RHS r sum all partials into out[0..nv).  Returns true in the last block
// (after out is written and visible to the whole block).
__device__ bool reduce_last_block(double* acc, int nv, double* __restrict__ part, int* __restrict__ counter, int r,
                                  double* __restrict__ out, double* lds /* [4 * NVMAX] */) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int G = gridDim.x;
#pragma unroll
  for (int q = 0; q < NVMAX; ++q) {
    if (q < nv) {
      const double v = wave_sum(acc[q]);
      if (l == 0) lds[w * NVMAX + q] = v;
    }
  }
  __syncthreads();
  double* pr = part + ((int64_t)r * G + blockIdx.x) * nv;
  for (int q = threadIdx.x; q < nv; q += blockDim.x) pr[q] = lds[q] + lds[NVMAX + q] + lds[2 * NVMAX + q] + lds[3 * NVMAX + q];
  __threadfence();
  __shared__ int last;
  __syncthreads();
  if (threadIdx.x == 0) last = (atomicAdd(counter + r, 1) == G - 1);
  __syncthreads();
  if (!last) return false;
  __threadfence();
  const double* base = part + (int64_t)r * G * nv;
  for (int q = threadIdx.x; q < nv; q += blockDim.x) {
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += base[(int64_t)g * nv + q];
    out[q] = s;
  }
  if (threadIdx.x == 0) counter[r] = 0;
  __threadfence_block();
  __syncthreads();
  return true;
}

template <typename RV>
__global__ __launch_bounds__(256) void gs_dots_kernel(const Cx<RV>* __restrict__ V, int nb, const c128* __restrict__ w,
                                                      int64_t n, int64_t vstride, double* __restrict__ part,
                                                      int* __restrict__ counter, c128* __restrict__ h, int hld) {
  __shared__ double lds[4 * NVMAX];
  const int r = blockIdx.y;
  double acc[NVMAX];
#pragma unroll
  for (int q = 0; q < NVMAX; ++q) acc[q] = 0.0;
  const c128* wr = w + (int64_t)r * n;
  const Cx<RV>* Vr = V + (int64_t)r * n;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const c128 b = wr[p];
#pragma unroll
    for (int i = 0; i < NBMAX; ++i) {
      if (i < nb) {
        const Cx<RV> a = Vr[i * vstride + p];
        acc[2 * i] += (double)a.x * b.x + (double)a.y * b.y;
        acc[2 * i + 1] += (double)a.x * b.y - (double)a.y * b.x;
      }
    }
  }
  reduce_last_block(acc, 2 * nb, part, counter, r, (double*)(h + (int64_t)r * hld), lds);
}

template <typename RV>
__global__ __launch_bounds__(256) void gs_update_norm_kernel(const Cx<RV>* __restrict__ V, int nb,
                                                             c128* __restrict__ w, int64_t n, int64_t vstride,
                                                             const c128* __restrict__ h, int hld,
                                                             double* __restrict__ part, int* __restrict__ counter,
                                                             double* __restrict__ nrm2) {
  __shared__ double lds[4 * NVMAX];
  __shared__ c128 hs[NBMAX];
  const int r = blockIdx.y;
  if (threadIdx.x < nb) hs[threadIdx.x] = h[(int64_t)r * hld + threadIdx.x];
  __syncthreads();
  double acc[NVMAX];
#pragma unroll
  for (int q = 0; q < NVMAX; ++q) acc[q] = 0.0;
  c128* wr = w + (int64_t)r * n;
  const Cx<RV>* Vr = V + (int64_t)r * n;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    c128 v = wr[p];
#pragma unroll
    for (int i = 0; i < NBMAX; ++i) {
      if (i < nb) {
        const Cx<RV> a = Vr[i * vstride + p];
        const c128 hi = hs[i];
        v.x -= hi.x * (double)a.x - hi.y * (double)a.y;
        v.y -= hi.x * (double)a.y + hi.y * (double)a.x;
      }
    }
    wr[p] = v;
    acc[0] += v.x * v.x + v.y * v.y;
  }
  reduce_last_block(acc, 1, part, counter, r, nrm2 + r, lds);
}

// Pass C with the Hessenberg bookkeeping done by the last block of each RHS.
template <typename RV>
__global__ __launch_bounds__(256) void gs_dots_finish_kernel(const Cx<RV>* __restrict__ V, int nb,
                                                             const c128* __restrict__ w, int64_t n, int64_t vstride,
                                                             double* __restrict__ part, int* __restrict__ counter,
                                                             int j, int m, const c128* __restrict__ h1,
                                                             c128* __restrict__ h2, int hld,
                                                             const double* __restrict__ nrm2, c128* __restrict__ H,
                                                             double* __restrict__ cs, c128* __restrict__ sn,
                                                             c128* __restrict__ g, double* __restrict__ res,
                                                             double* __restrict__ invb) {
  __shared__ double lds[4 * NVMAX];
  const int r = blockIdx.y;
  double acc[NVMAX];
#pragma unroll
  for (int q = 0; q < NVMAX; ++q) acc[q] = 0.0;
  const c128* wr = w + (int64_t)r * n;
  const Cx<RV>* Vr = V + (int64_t)r * n;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const c128 b = wr[p];
#pragma unroll
    for (int i = 0; i < NBMAX; ++i) {
      if (i < nb) {
        const Cx<RV> a = Vr[i * vstride + p];
        acc[2 * i] += (double)a.x * b.x + (double)a.y * b.y;
        acc[2 * i + 1] += (double)a.x * b.y - (double)a.y * b.x;
      }
    }
  }
  if (!reduce_last_block(acc, 2 * nb, part, counter, r, (double*)(h2 + (int64_t)r * hld), lds)) return;
  if (threadIdx.x != 0) return;
  // Hessenberg column j = h1 + h2; beta = ||w' - V h2|| = sqrt(||w'||^2 - |h2|^2)
  c128* col = H + (int64_t)r * (m + 1) * m + (int64_t)j * (m + 1);
  double h2n = 0.0;
  for (int i = 0; i <= j; ++i) {
    const c128 b2 = h2[(int64_t)r * hld + i];
    h2n += b2.x * b2.x + b2.y * b2.y;
    col[i] = h1[(int64_t)r * hld + i] + b2;
  }
  const double beta = sqrt(fmax(nrm2[r] - h2n, 0.0));
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

template <typename RV>
__global__ __launch_bounds__(256) void gs_update_store_kernel(Cx<RV>* __restrict__ V, int nb,
                                                              const c128* __restrict__ w, int64_t n, int64_t vstride,
                                                              const c128* __restrict__ h, int hld,
                                                              const double* __restrict__ invb) {
  __shared__ c128 hs[NBMAX];
  const int r = blockIdx.y;
  if (threadIdx.x < nb) hs[threadIdx.x] = h[(int64_t)r * hld + threadIdx.x];
  __syncthreads();
  const double sc = invb[r];
  const c128* wr = w + (int64_t)r * n;
  const Cx<RV>* Vr = V + (int64_t)r * n;
  Cx<RV>* out = V + (int64_t)nb * vstride + (int64_t)r * n;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    c128 v = wr[p];
#pragma unroll
    for (int i = 0; i < NBMAX; ++i) {
      if (i < nb) {
        const Cx<RV> a = Vr[i * vstride + p];
        const c128 hi = hs[i];
        v.x -= hi.x * (double)a.x - hi.y * (double)a.y;
        v.y -= hi.x * (double)a.y + hi.y * (double)a.x;
      }
    }
    out[p] = cmk((RV)(v.x * sc), (RV)(v.y * sc));
  }
}

// ---------------------------------------------------------------- single-pass form (mixed path)
// Basis vectors are stored unnormalised in complex FP32 (u_i) with per-vector scales
// s_i = 1 / ||u_i|| (scale[i][r]); all dots and updates accumulate in FP64.
//   A: h_i = s_i <u_i, w>                          (read U, w)
//   B: u_{j+1} = w - sum_i h_i s_i u_i, ||u_{j+1}||^2, then the Hessenberg column,
//      Givens rotation, residual estimate and s_{j+1} in the last block (read U, w; write u)
template <typename RW>
__global__ __launch_bounds__(256) void gs1_dots_kernel(const c64* __restrict__ U, int nb,
                                                       const Cx<RW>* __restrict__ w, int64_t n, int64_t vstride,
                                                       const double* __restrict__ scale, int nrhs,
                                                       double* __restrict__ part, int* __restrict__ counter,
                                                       c128* __restrict__ h, int hld) {
  __shared__ double lds[4 * NVMAX];
  const int r = blockIdx.y;
  double acc[NVMAX];
#pragma unroll
  for (int q = 0; q < NVMAX; ++q) acc[q] = 0.0;
  const Cx<RW>* wr = w + (int64_t)r * n;
  const c64* Ur = U + (int64_t)r * n;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const Cx<RW> bw = wr[p];
    const double bx = (double)bw.x, by = (double)bw.y;
#pragma unroll
    for (int i = 0; i < NBMAX; ++i) {
      if (i < nb) {
        const c64 a = Ur[i * vstride + p];
        acc[2 * i] += (double)a.x * bx + (double)a.y * by;
        acc[2 * i + 1] += (double)a.x * by - (double)a.y * bx;
      }
    }
  }
  __shared__ double hs[2 * NBMAX];
  if (!reduce_last_block(acc, 2 * nb, part, counter, r, hs, lds)) return;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    const double sc = scale[(int64_t)i * nrhs + r];
    h[(int64_t)r * hld + i] = cmk(hs[2 * i] * sc, hs[2 * i + 1] * sc);
  }
}

template <typename RW>
__global__ __launch_bounds__(256) void gs1_update_finish_kernel(c64* __restrict__ U, int nb,
                                                                const Cx<RW>* __restrict__ w, int64_t n,
                                                                int64_t vstride, double* __restrict__ scale, int nrhs,
                                                                double* __restrict__ part, int* __restrict__ counter,
                                                                int j, int m, c128* __restrict__ hcol, int hld,
                                                                c128* __restrict__ H, double* __restrict__ cs,
                                                                c128* __restrict__ sn, c128* __restrict__ g,
                                                                double* __restrict__ res) {
  __shared__ double lds[4 * NVMAX];
  __shared__ c128 hs[NBMAX];
  const int r = blockIdx.y;
  if (threadIdx.x < nb) {
    const c128 hv = hcol[(int64_t)r * hld + threadIdx.x];
    const double sc = scale[(int64_t)threadIdx.x * nrhs + r];
    hs[threadIdx.x] = cmk(hv.x * sc, hv.y * sc);
  }
  __syncthreads();
  double acc[1] = {0.0};
  const Cx<RW>* wr = w + (int64_t)r * n;
  const c64* Ur = U + (int64_t)r * n;
  c64* out = U + (int64_t)nb * vstride + (int64_t)r * n;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const Cx<RW> bw = wr[p];
    double vx = (double)bw.x, vy = (double)bw.y;
#pragma unroll
    for (int i = 0; i < NBMAX; ++i) {
      if (i < nb) {
        const c64 a = Ur[i * vstride + p];
        const c128 hi = hs[i];
        vx -= hi.x * (double)a.x - hi.y * (double)a.y;
        vy -= hi.x * (double)a.y + hi.y * (double)a.x;
      }
    }
    const c64 st = cmk((float)vx, (float)vy);
    out[p] = st;
    acc[0] += (double)st.x * st.x + (double)st.y * st.y;
  }
  __shared__ double nn_s;
  if (!reduce_last_block(acc, 1, part, counter, r, &nn_s, lds)) return;
  const double nn = nn_s;
  if (threadIdx.x != 0) return;
  const double beta = sqrt(fmax(nn, 0.0));
  scale[(int64_t)nb * nrhs + r] = beta > 0.0 ? 1.0 / beta : 0.0;
  c128* col = H + (int64_t)r * (m + 1) * m + (int64_t)j * (m + 1);
  for (int i = 0; i <= j; ++i) col[i] = hcol[(int64_t)r * hld + i];
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
  gr[j + 1] = cmk(-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x));
  gr[j] = c * gj;
  res[r] = sqrt(cabs2(gr[j + 1]));
}

int gs_blocks(int64_t n, int nrhs) {
  const int64_t want = ceil_div(n, 4096);
  const int64_t cap = std::max<int64_t>(1, 2048 / std::max(1, nrhs));
  return (int)std::max<int64_t>(1, std::min(want, cap));
}

}  // namespace

int gs_max_basis() { return NBMAX; }

// One Arnoldi step: orthogonalise w (FP64, [nrhs][n]) against V_0..V_j (RV) by CGS2,
// update the Hessenberg column and rotations, store V_{j+1} = w / ||w||.  w is
// overwritten by the once-orthogonalised vector.
template <typename RV>
void arnoldi_step(dmlmc_ctx* ctx, Cx<RV>* V, c128* w, int j, int64_t n, int nrhs, const KrylovArrays& k) {
  const int nb = j + 1;
  if (nb > NBMAX) throw DmlmcError(DMLMC_EINVAL, "Krylov basis larger than the fused Gram-Schmidt limit");
  const int64_t vstride = (int64_t)nrhs * n;
  const int G = gs_blocks(n, nrhs);
  ctx->scratch_dots.ensure(sizeof(double) * (size_t)nrhs * G * NVMAX);
  double* part = ctx->scratch_dots.as<double>();
  dim3 grid(G, nrhs);
  {
    KTimer kt(ctx, "gs_dots", (double)nrhs * n * (nb * sizeof(Cx<RV>) + sizeof(c128)));
    hipLaunchKernelGGL((gs_dots_kernel<RV>), grid, dim3(256), 0, ctx->stream, V, nb, w, n, vstride, part, k.counter,
                       k.h1, k.hld);
    LAUNCH_CHECK();
  }
  {
    KTimer kt(ctx, "gs_update", (double)nrhs * n * (nb * sizeof(Cx<RV>) + 2 * sizeof(c128)));
    hipLaunchKernelGGL((gs_update_norm_kernel<RV>), grid, dim3(256), 0, ctx->stream, V, nb, w, n, vstride, k.h1,
                       k.hld, part, k.counter, k.nrm2);
    LAUNCH_CHECK();
  }
  {
    KTimer kt(ctx, "gs_dots", (double)nrhs * n * (nb * sizeof(Cx<RV>) + sizeof(c128)));
    hipLaunchKernelGGL((gs_dots_finish_kernel<RV>), grid, dim3(256), 0, ctx->stream, V, nb, w, n, vstride, part,
                       k.counter, j, k.m, k.h1, k.h2, k.hld, k.nrm2, k.H, k.cs, k.sn, k.g, k.res, k.invb);
    LAUNCH_CHECK();
  }
  {
    KTimer kt(ctx, "gs_update", (double)nrhs * n * (nb * sizeof(Cx<RV>) + sizeof(c128) + sizeof(Cx<RV>)));
    hipLaunchKernelGGL((gs_update_store_kernel<RV>), grid, dim3(256), 0, ctx->stream, V, nb, w, n, vstride, k.h2,
                       k.hld, k.invb);
    LAUNCH_CHECK();
  }
}

template <typename RW>
void arnoldi_step_cgs1(dmlmc_ctx* ctx, c64* U, double* scale, const Cx<RW>* w, int j, int64_t n, int nrhs,
                       const KrylovArrays& k) {
  const int nb = j + 1;
  if (nb > NBMAX) throw DmlmcError(DMLMC_EINVAL, "Krylov basis larger than the fused Gram-Schmidt limit");
  const int64_t vstride = (int64_t)nrhs * n;
  const int G = gs_blocks(n, nrhs);
  ctx->scratch_dots.ensure(sizeof(double) * (size_t)nrhs * G * NVMAX);
  double* part = ctx->scratch_dots.as<double>();
  dim3 grid(G, nrhs);
  {
    KTimer kt(ctx, "gs_dots", (double)nrhs * n * (nb * sizeof(c64) + sizeof(Cx<RW>)));
    hipLaunchKernelGGL((gs1_dots_kernel<RW>), grid, dim3(256), 0, ctx->stream, U, nb, w, n, vstride, scale, nrhs,
                       part, k.counter, k.h1, k.hld);
    LAUNCH_CHECK();
  }
  {
    KTimer kt(ctx, "gs_update", (double)nrhs * n * ((nb + 1) * sizeof(c64) + sizeof(Cx<RW>)));
    hipLaunchKernelGGL((gs1_update_finish_kernel<RW>), grid, dim3(256), 0, ctx->stream, U, nb, w, n, vstride, scale,
                       nrhs, part, k.counter, j, k.m, k.h1, k.hld, k.H, k.cs, k.sn, k.g, k.res);
    LAUNCH_CHECK();
  }
}

template void arnoldi_step<double>(dmlmc_ctx*, c128*, c128*, int, int64_t, int, const KrylovArrays&);
template void arnoldi_step_cgs1<float>(dmlmc_ctx*, c64*, double*, const c64*, int, int64_t, int, const KrylovArrays&);
template void arnoldi_step_cgs1<double>(dmlmc_ctx*, c64*, double*, const c128*, int, int64_t, int,
                                        const KrylovArrays&);
template void arnoldi_step<float>(dmlmc_ctx*, c64*, c128*, int, int64_t, int, const KrylovArrays&);
