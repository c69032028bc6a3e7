// Vector kernels: fills, precision casts, per-RHS dot products and norms with FP64
// accumulation (deterministic two-pass reductions), axpy forms, the SplitMix64 counter
// noise, and the block Gram-Schmidt pieces of the Krylov solvers.
#include "common.h"

namespace {

constexpr int RED_BLOCKS = 256;  // partial sums per RHS in the first reduction pass

__global__ void fill_value_kernel(double* __restrict__ p, size_t count, double v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

template <typename T>
__global__ void fill_zero_kernel(T* __restrict__ p, size_t count) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = T{};
}

// p[r * ld + i] = 0 for i < n, row r = blockIdx.y (the entries between n and ld untouched)
template <typename T>
__global__ void fill_zero_rows_kernel(T* __restrict__ p, int64_t n, int64_t ld) {
  T* row = p + (int64_t)blockIdx.y * ld;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    row[i] = T{};
}

template <typename To, typename From>
__global__ void cast_kernel(const Cx<From>* __restrict__ x, Cx<To>* __restrict__ y, int64_t n, int64_t ldx,
                            int64_t ldy) {
  const int r = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[r * ldy + i] = ccast<To>(x[r * ldx + i]);
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  // 256-thread block reduction
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  return t;
}

template <typename RX, typename RY>
__global__ __launch_bounds__(256) void dots_partial(const Cx<RX>* __restrict__ x, const Cx<RY>* __restrict__ y,
                                                    int64_t n, int64_t ldx, int64_t ldy, double* __restrict__ part) {
  __shared__ double sh[8];
  const int r = blockIdx.y;
  double re = 0.0, im = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const Cx<RX> a = x[r * ldx + i];
    const Cx<RY> b = y[r * ldy + i];
    re += (double)a.x * (double)b.x + (double)a.y * (double)b.y;
    im += (double)a.x * (double)b.y - (double)a.y * (double)b.x;
  }
  double sre = block_sum(re, sh);
  double sim = block_sum(im, sh);
  if (threadIdx.x == 0) {
    part[((int64_t)r * gridDim.x + blockIdx.x) * 2 + 0] = sre;
    part[((int64_t)r * gridDim.x + blockIdx.x) * 2 + 1] = sim;
  }
}

template <typename R>
__global__ __launch_bounds__(256) void norms_partial(const Cx<R>* __restrict__ x, int64_t n, int64_t ld,
                                                     double* __restrict__ part) {
  __shared__ double sh[8];
  const int r = blockIdx.y;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += cabs2(x[r * ld + i]);
  double t = block_sum(s, sh);
  if (threadIdx.x == 0) part[(int64_t)r * gridDim.x + blockIdx.x] = t;
}

// out[r * stride + c] = sum_g part[(r * G + g) * width + c] for c < width
__global__ void reduce_partials(const double* __restrict__ part, int G, int width, double* __restrict__ out,
                                int stride) {
  __shared__ double sh[8];
  const int r = blockIdx.x;
  for (int c = 0; c < width; ++c) {
    double s = 0.0;
    for (int g = threadIdx.x; g < G; g += blockDim.x) s += part[((int64_t)r * G + g) * width + c];
    double t = block_sum(s, sh);
    if (threadIdx.x == 0) out[(int64_t)r * stride + c] = t;
    __syncthreads();
  }
}

template <typename R>
__global__ void axpy_dev_kernel(const c128* __restrict__ a, const Cx<R>* __restrict__ x, Cx<R>* __restrict__ y,
                                int64_t n, int64_t ld) {
  const int r = blockIdx.y;
  const Cx<R> ar = ccast<R>(a[r]);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    cfma(y[r * ld + i], ar, x[r * ld + i]);
}

template <typename R>
__global__ void xmy_kernel(const Cx<R>* __restrict__ b, Cx<R>* __restrict__ y, int64_t n, int64_t ldb, int64_t ldy) {
  const int r = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[r * ldy + i] = b[r * ldb + i] - y[r * ldy + i];
}

template <typename RE>
__global__ void add_cast_kernel(const Cx<RE>* __restrict__ e, c128* __restrict__ x, int64_t n, int64_t lde,
                                int64_t ldx) {
  const int r = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[r * ldx + i] = x[r * ldx + i] + ccast<double>(e[r * lde + i]);
}

template <typename RX>
__global__ void add_to_kernel(const c128* __restrict__ e, Cx<RX>* __restrict__ x, int64_t n) {
  const int r = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const Cx<RX> v = x[r * n + i];
    const c128 a = e[r * n + i];
    x[r * n + i] = cmk((RX)((double)v.x + a.x), (RX)((double)v.y + a.y));
  }
}

// SplitMix64 step (Steele, Lea & Flood 2014): add the golden gamma, then mix.
__device__ __forceinline__ uint64_t sm64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <typename R>
__global__ void z2_kernel(Cx<R>* __restrict__ out, int64_t n, uint64_t h1, int64_t sample0, int64_t ld) {
  const int r = blockIdx.y;
  const uint64_t base = sm64(h1 + (uint64_t)(sample0 + r));
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t w = sm64(base + (uint64_t)(j >> 6));
    const R v = ((w >> (j & 63)) & 1ull) ? (R)-1 : (R)1;
    out[r * ld + j] = cmk(v, (R)0);
  }
}

__global__ void z4_kernel(c128* __restrict__ out, int64_t n, uint64_t h1, int vec0) {
  const int r = blockIdx.y;
  const uint64_t base = sm64(h1 + (uint64_t)(vec0 + r));
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t w = sm64(base + (uint64_t)(j >> 5));
    const int c = (int)((w >> (2 * (j & 31))) & 3ull);
    const double re = (c == 0) ? 1.0 : (c == 2 ? -1.0 : 0.0);
    const double im = (c == 1) ? 1.0 : (c == 3 ? -1.0 : 0.0);
    out[(int64_t)r * n + j] = cmk(re, im);
  }
}

// Block Gram-Schmidt pieces.  Basis vector i of RHS r at V + i * vstride + r * ld.
// Partial dots over chunks: part[((r * G + g) * nb + i) * 2 + {0,1}].
template <typename RV>
__global__ __launch_bounds__(256) void multidot_partial(const Cx<RV>* __restrict__ V, int nb,
                                                        const c128* __restrict__ w, int64_t n, int64_t ld,
                                                        int64_t ldv, int64_t vstride, double* __restrict__ part) {
  __shared__ double sh[8];
  const int r = blockIdx.y;
  const int G = gridDim.x;
  for (int i = 0; i < nb; ++i) {
    const Cx<RV>* v = V + i * vstride + r * ldv;
    double re = 0.0, im = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)G * blockDim.x) {
      const Cx<RV> a = v[p];
      const c128 b = w[r * ld + p];
      re += (double)a.x * b.x + (double)a.y * b.y;
      im += (double)a.x * b.y - (double)a.y * b.x;
    }
    double sre = block_sum(re, sh);
    double sim = block_sum(im, sh);
    if (threadIdx.x == 0) {
      part[(((int64_t)r * G + blockIdx.x) * nb + i) * 2 + 0] = sre;
      part[(((int64_t)r * G + blockIdx.x) * nb + i) * 2 + 1] = sim;
    }
    __syncthreads();
  }
}

template <typename RV>
__global__ __launch_bounds__(256) void multiaxpy_kernel(const Cx<RV>* __restrict__ V, int nb, c128* __restrict__ w,
                                                        int64_t n, int64_t ld, int64_t ldv, int64_t vstride,
                                                        const c128* __restrict__ h, int hld, double sgn) {
  const int r = blockIdx.y;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    c128 acc = w[r * ld + p];
    for (int i = 0; i < nb; ++i) {
      const c128 hi = h[(int64_t)r * hld + i];
      const Cx<RV> v = V[i * vstride + r * ldv + p];
      acc.x -= sgn * (hi.x * (double)v.x - hi.y * (double)v.y);
      acc.y -= sgn * (hi.x * (double)v.y + hi.y * (double)v.x);
    }
    w[r * ld + p] = acc;
  }
}

inline unsigned grid_for(int64_t n) { return (unsigned)std::min<int64_t>(std::max<int64_t>(1, ceil_div(n, 256)), 1024); }

}  // namespace

template <typename T>
void launch_fill_zero(dmlmc_ctx* ctx, T* p, size_t count) {
  if (count == 0) return;
  hipLaunchKernelGGL((fill_zero_kernel<T>), dim3(grid_for((int64_t)count)), dim3(256), 0, ctx->stream, p, count);
  LAUNCH_CHECK();
}

template <typename T>
void launch_fill_zero_rows(dmlmc_ctx* ctx, T* p, int64_t n, int nrhs, int64_t ld) {
  if (n == 0 || nrhs == 0) return;
  hipLaunchKernelGGL((fill_zero_rows_kernel<T>), dim3(grid_for(n), nrhs), dim3(256), 0, ctx->stream, p, n, ld);
  LAUNCH_CHECK();
}

template <typename To, typename From>
void launch_cast(dmlmc_ctx* ctx, const Cx<From>* x, Cx<To>* y, int64_t n, int nrhs, int64_t ldx, int64_t ldy) {
  hipLaunchKernelGGL((cast_kernel<To, From>), dim3(grid_for(n), nrhs), dim3(256), 0, ctx->stream, x, y, n, ldx, ldy);
  LAUNCH_CHECK();
}

static double* partial_buf(dmlmc_ctx* ctx, size_t doubles) {
  ctx->scratch_dots.ensure(doubles * sizeof(double));
  return ctx->scratch_dots.as<double>();
}

template <typename RX, typename RY>
void launch_dots(dmlmc_ctx* ctx, const Cx<RX>* x, const Cx<RY>* y, int64_t n, int nrhs, int64_t ldx, int64_t ldy,
                 c128* out) {
  const int G = (int)std::min<int64_t>(RED_BLOCKS, std::max<int64_t>(1, ceil_div(n, 1024)));
  double* part = partial_buf(ctx, (size_t)nrhs * G * 2);
  hipLaunchKernelGGL((dots_partial<RX, RY>), dim3(G, nrhs), dim3(256), 0, ctx->stream, x, y, n, ldx, ldy, part);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(reduce_partials, dim3(nrhs), dim3(256), 0, ctx->stream, part, G, 2, (double*)out, 2);
  LAUNCH_CHECK();
}

template <typename R>
void launch_norms2(dmlmc_ctx* ctx, const Cx<R>* x, int64_t n, int nrhs, int64_t ld, double* out) {
  const int G = (int)std::min<int64_t>(RED_BLOCKS, std::max<int64_t>(1, ceil_div(n, 1024)));
  double* part = partial_buf(ctx, (size_t)nrhs * G);
  hipLaunchKernelGGL((norms_partial<R>), dim3(G, nrhs), dim3(256), 0, ctx->stream, x, n, ld, part);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(reduce_partials, dim3(nrhs), dim3(256), 0, ctx->stream, part, G, 1, out, 1);
  LAUNCH_CHECK();
}

template <typename R>
void launch_axpy_dev(dmlmc_ctx* ctx, const c128* a, const Cx<R>* x, Cx<R>* y, int64_t n, int nrhs, int64_t ld) {
  hipLaunchKernelGGL((axpy_dev_kernel<R>), dim3(grid_for(n), nrhs), dim3(256), 0, ctx->stream, a, x, y, n, ld);
  LAUNCH_CHECK();
}

template <typename R>
void launch_xmy(dmlmc_ctx* ctx, const Cx<R>* b, Cx<R>* y, int64_t n, int nrhs, int64_t ldb, int64_t ldy) {
  hipLaunchKernelGGL((xmy_kernel<R>), dim3(grid_for(n), nrhs), dim3(256), 0, ctx->stream, b, y, n, ldb, ldy);
  LAUNCH_CHECK();
}

template <typename RE>
void launch_add_cast(dmlmc_ctx* ctx, const Cx<RE>* e, c128* x, int64_t n, int nrhs, int64_t lde, int64_t ldx) {
  hipLaunchKernelGGL((add_cast_kernel<RE>), dim3(grid_for(n), nrhs), dim3(256), 0, ctx->stream, e, x, n, lde, ldx);
  LAUNCH_CHECK();
}

template <typename RX>
void launch_add_cast_to(dmlmc_ctx* ctx, const c128* e, Cx<RX>* x, int64_t n, int nrhs) {
  hipLaunchKernelGGL((add_to_kernel<RX>), dim3(grid_for(n), nrhs), dim3(256), 0, ctx->stream, e, x, n);
  LAUNCH_CHECK();
}
template void launch_add_cast_to<float>(dmlmc_ctx*, const c128*, c64*, int64_t, int);
template void launch_add_cast_to<double>(dmlmc_ctx*, const c128*, c128*, int64_t, int);

static uint64_t sm64_host(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <typename R>
void launch_z2(dmlmc_ctx* ctx, Cx<R>* out, int64_t n, uint64_t seed, int level, int64_t sample0, int nrhs,
               int64_t ld) {
  const uint64_t h1 = sm64_host(sm64_host(seed) + (uint64_t)level);
  hipLaunchKernelGGL((z2_kernel<R>), dim3(grid_for(n), nrhs), dim3(256), 0, ctx->stream, out, n, h1, sample0, ld);
  LAUNCH_CHECK();
}

void launch_z4(dmlmc_ctx* ctx, c128* out, int64_t n, uint64_t seed, int level, int vec0, int nvec) {
  const uint64_t h1 = sm64_host(sm64_host(seed) + (uint64_t)level + 32ull);
  hipLaunchKernelGGL(z4_kernel, dim3(grid_for(n), nvec), dim3(256), 0, ctx->stream, out, n, h1, vec0);
  LAUNCH_CHECK();
}

template <typename RV>
void launch_multidot(dmlmc_ctx* ctx, const Cx<RV>* V, int nb, const c128* w, int64_t n, int nrhs, int64_t ld,
                     int64_t vstride, c128* h, int hld, int64_t ldv) {
  if (ldv < 0) ldv = ld;
  const int G = (int)std::min<int64_t>(RED_BLOCKS, std::max<int64_t>(1, ceil_div(n, 2048)));
  double* part = partial_buf(ctx, (size_t)nrhs * G * nb * 2);
  KTimer kt(ctx, "gs_dots", (double)nrhs * n * (nb * sizeof(Cx<RV>) + sizeof(c128)));
  hipLaunchKernelGGL((multidot_partial<RV>), dim3(G, nrhs), dim3(256), 0, ctx->stream, V, nb, w, n, ld, ldv, vstride,
                     part);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(reduce_partials, dim3(nrhs), dim3(256), 0, ctx->stream, part, G, nb * 2, (double*)h, hld * 2);
  LAUNCH_CHECK();
}

template <typename RV>
void launch_multiaxpy(dmlmc_ctx* ctx, const Cx<RV>* V, int nb, c128* w, int64_t n, int nrhs, int64_t ld,
                      int64_t vstride, const c128* h, int hld, int64_t ldv, double sgn) {
  if (ldv < 0) ldv = ld;
  KTimer kt(ctx, "gs_update", (double)nrhs * n * (nb * sizeof(Cx<RV>) + 2 * sizeof(c128)));
  hipLaunchKernelGGL((multiaxpy_kernel<RV>), dim3(grid_for(n), nrhs), dim3(256), 0, ctx->stream, V, nb, w, n, ld,
                     ldv, vstride, h, hld, sgn);
  LAUNCH_CHECK();
}

void launch_fill_value(dmlmc_ctx* ctx, double* p, size_t count, double v) {
  hipLaunchKernelGGL(fill_value_kernel, dim3(grid_for((int64_t)count)), dim3(256), 0, ctx->stream, p, count, v);
  LAUNCH_CHECK();
}

template void launch_fill_zero<c64>(dmlmc_ctx*, c64*, size_t);
template void launch_fill_zero<c128>(dmlmc_ctx*, c128*, size_t);
template void launch_fill_zero<double>(dmlmc_ctx*, double*, size_t);
template void launch_fill_zero_rows<c64>(dmlmc_ctx*, c64*, int64_t, int, int64_t);
template void launch_fill_zero_rows<c128>(dmlmc_ctx*, c128*, int64_t, int, int64_t);
template void launch_cast<float, double>(dmlmc_ctx*, const c128*, c64*, int64_t, int, int64_t, int64_t);
template void launch_cast<double, float>(dmlmc_ctx*, const c64*, c128*, int64_t, int, int64_t, int64_t);
template void launch_cast<double, double>(dmlmc_ctx*, const c128*, c128*, int64_t, int, int64_t, int64_t);
template void launch_cast<float, float>(dmlmc_ctx*, const c64*, c64*, int64_t, int, int64_t, int64_t);
template void launch_dots<double, double>(dmlmc_ctx*, const c128*, const c128*, int64_t, int, int64_t, int64_t, c128*);
template void launch_dots<float, float>(dmlmc_ctx*, const c64*, const c64*, int64_t, int, int64_t, int64_t, c128*);
template void launch_dots<float, double>(dmlmc_ctx*, const c64*, const c128*, int64_t, int, int64_t, int64_t, c128*);
template void launch_norms2<double>(dmlmc_ctx*, const c128*, int64_t, int, int64_t, double*);
template void launch_norms2<float>(dmlmc_ctx*, const c64*, int64_t, int, int64_t, double*);
template void launch_axpy_dev<double>(dmlmc_ctx*, const c128*, const c128*, c128*, int64_t, int, int64_t);
template void launch_axpy_dev<float>(dmlmc_ctx*, const c128*, const c64*, c64*, int64_t, int, int64_t);
template void launch_xmy<double>(dmlmc_ctx*, const c128*, c128*, int64_t, int, int64_t, int64_t);
template void launch_xmy<float>(dmlmc_ctx*, const c64*, c64*, int64_t, int, int64_t, int64_t);
template void launch_add_cast<float>(dmlmc_ctx*, const c64*, c128*, int64_t, int, int64_t, int64_t);
template void launch_add_cast<double>(dmlmc_ctx*, const c128*, c128*, int64_t, int, int64_t, int64_t);
template void launch_z2<double>(dmlmc_ctx*, c128*, int64_t, uint64_t, int, int64_t, int, int64_t);
template void launch_z2<float>(dmlmc_ctx*, c64*, int64_t, uint64_t, int, int64_t, int, int64_t);
template void launch_multidot<double>(dmlmc_ctx*, const c128*, int, const c128*, int64_t, int, int64_t, int64_t, c128*, int,
                                      int64_t);
template void launch_multidot<float>(dmlmc_ctx*, const c64*, int, const c128*, int64_t, int, int64_t, int64_t, c128*, int,
                                     int64_t);
template void launch_multiaxpy<double>(dmlmc_ctx*, const c128*, int, c128*, int64_t, int, int64_t, int64_t, const c128*,
                                       int, int64_t, double);
template void launch_multiaxpy<float>(dmlmc_ctx*, const c64*, int, c128*, int64_t, int, int64_t, int64_t, const c128*,
                                      int, int64_t, double);
