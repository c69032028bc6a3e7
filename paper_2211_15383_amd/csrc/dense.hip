// Direct solve of the coarsest level (d = 16) with its explicit inverse.
//
// Setup: the columns of D_L^-1 come from multi-RHS solves of D_L X = I (blocks of unit
// vectors, FP64 refinement to 1e-10); the inverse is kept in complex FP32, row-major
// [n][n], and on request also in complex FP16 (one power-of-two scale for the whole
// matrix, so that no component exceeds 1).
//
// FP32 apply: Y = D_L^-1 B for a block of RHS on the matrix cores, the same operand layout
// as the coarse stencil (lane (row, kq) takes the quads Dinv[i0 + row][j0 + 4kq ..] and
// B[r0 + row][j0 + 4kq ..], and receives Y[r0 + row][i0 + 4kq + v]); the contraction is
// split over KS waves whose partial tiles are summed by a second kernel in a fixed order.
// At n = 16384 and 32 RHS one apply is 69 GFLOP over a 2.1 GB operand: matrix-core bound
// (~0.44 ms at the FP32 peak), exact to FP32 rounding.
//
// FP16 apply: the same product with v_mfma_f32_16x16x32_f16 (FP32 accumulation).  A
// complex FP16 entry is one 32-bit word (real part in the low half); a lane's eight
// consecutive words of a Dinv row are two K = 32 operands as stored, and the matching
// RHS words become (re, -im) pairs for the real part and (im, re) pairs for the imaginary
// part of the product, two instructions per complex product instead of four.  Each RHS is
// first scaled by a power of two into [-1, 1] and rounded to FP16 (relative rounding
// 2^-11); the reduction undoes both scales.  The operand is half the bytes and the
// instruction count half of the FP32 form, so the apply is HBM-bound (1.07 GB at
// n = 16384).  It is a preconditioner: every solve still stops at its FP64 tolerance.
#include "dense.h"

#include <cmath>

#include "solver.h"

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

struct __align__(16) C64Pair {
  c64 a, b;
};

struct Quad {
  c64 v[4];
};

__device__ __forceinline__ Quad load_quad(const c64* __restrict__ p) {
  const C64Pair* q = reinterpret_cast<const C64Pair*>(p);
  const C64Pair u = q[0], w = q[1];
  Quad r;
  r.v[0] = u.a;
  r.v[1] = u.b;
  r.v[2] = w.a;
  r.v[3] = w.b;
  return r;
}

__device__ __forceinline__ void cmfma(f32x4& dre, f32x4& dim, c64 a, c64 x) {
  dre = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, x.x, dre, 0, 0, 0);
  dre = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.y, x.y, dre, 0, 0, 0);
  dim = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, x.y, dim, 0, 0, 0);
  dim = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, x.x, dim, 0, 0, 0);
}

// grid: (n / (16 TI) / 4 workgroups) x KS; wave (group, ks) accumulates the TI row tiles
// Dinv[i0 + 16 t .. + 16) times B over columns [ks n / KS, (ks + 1) n / KS) for RHS tile
// pairs; every B quad it loads serves TI row tiles.
template <int TI>
__global__ __launch_bounds__(256) void dense_apply_kernel(const c64* __restrict__ Dinv, const c64* __restrict__ B,
                                                          c64* __restrict__ part, int64_t n, int nrhs, int KS) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t grp = (int64_t)blockIdx.x * 4 + w;
  if (grp * 16 * TI >= n) return;  // wave-uniform
  const int ks = blockIdx.y;
  const int64_t i0 = grp * 16 * TI;
  const int64_t kc = n / KS;
  const int64_t j0 = ks * kc;
  const int row = lane & 15, kq = lane >> 4;
  for (int r0 = 0; r0 < nrhs; r0 += 32) {
    const int ra = r0 + row, rb = r0 + 16 + row;
    const bool va = ra < nrhs, vb = rb < nrhs;
    const c64* Ba = B + (int64_t)min(ra, nrhs - 1) * n + 4 * kq;
    const c64* Bb = B + (int64_t)min(rb, nrhs - 1) * n + 4 * kq;
    f32x4 are[TI], aim[TI], bre[TI], bim[TI];
#pragma unroll
    for (int t = 0; t < TI; ++t) are[t] = aim[t] = bre[t] = bim[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int steps = (int)(kc / 16);
    for (int q = 0; q < steps; ++q) {
      const int64_t j = j0 + 16 * (int64_t)q;
      const Quad xa = load_quad(Ba + j);
      const Quad xb = load_quad(Bb + j);
      Quad a[TI];
#pragma unroll
      for (int t = 0; t < TI; ++t) a[t] = load_quad(Dinv + (i0 + 16 * t + row) * n + 4 * kq + j);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const c64 x0 = va ? xa.v[u] : cmk(0.f, 0.f);
        const c64 x1 = vb ? xb.v[u] : cmk(0.f, 0.f);
#pragma unroll
        for (int t = 0; t < TI; ++t) {
          cmfma(are[t], aim[t], a[t].v[u], x0);
          cmfma(bre[t], bim[t], a[t].v[u], x1);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < TI; ++t) {
      c64* pa = part + ((int64_t)ks * nrhs + min(ra, nrhs - 1)) * n + i0 + 16 * t + 4 * kq;
      c64* pb = part + ((int64_t)ks * nrhs + min(rb, nrhs - 1)) * n + i0 + 16 * t + 4 * kq;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (va) pa[v] = cmk(are[t][v], aim[t][v]);
        if (vb) pb[v] = cmk(bre[t][v], bim[t][v]);
      }
    }
  }
}

__global__ void dense_reduce_kernel(const c64* __restrict__ part, int KS, int64_t m, c64* __restrict__ Y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  float sx = 0.f, sy = 0.f;
  for (int k = 0; k < KS; ++k) {
    const c64 v = part[(int64_t)k * m + e];
    sx += v.x;
    sy += v.y;
  }
  Y[e] = cmk(sx, sy);
}

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ half8 as_half8(u32x4 v) { return __builtin_bit_cast(half8, v); }

__device__ __forceinline__ uint32_t pack_half2(float re, float im) {
  const _Float16 a = (_Float16)re, b = (_Float16)im;
  return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
}

// The complex-FP16 inverse is stored in the order the product reads it: for each 16-row
// tile T and 32-column step Q, a 2 KB block holding, for u = 0, 1 and lane = (row, g) =
// row + 16 g, the four words Dinv[16 T + row][32 Q + 8 g + 4 u .. + 3] (block (T, Q) at
// word (T n / 32 + Q) 512).  Each 16-byte load of a wavefront then reads one contiguous
// 1 KB (eight whole 128-byte lines) instead of half of each of 16 lines.
__device__ __forceinline__ int64_t packed16_index(int64_t i, int64_t j, int64_t n) {
  const int64_t T = i / 16, Q = j / 32;
  const int row = (int)(i % 16), c = (int)(j % 32);
  const int g = c / 8, u = (c % 8) / 4, e = c % 4;
  return (T * (n / 32) + Q) * 512 + u * 256 + (row + 16 * g) * 4 + e;
}

// grid: (n / (16 TI) / 4 workgroups) x KS; wave (group, ks) accumulates the TI row tiles
// Dinv[i0 + 16 t .. + 16) times B over columns [ks n / KS, (ks + 1) n / KS), 32 columns
// per step: lane (row, g) holds words j0 + 32 q + 8 g .. + 7 of its Dinv rows (from the
// packed order above) and of its RHS rows, as two K = 32 operands (words 0..3 and 4..7).
template <int TI>
__global__ __launch_bounds__(256) void dense16_apply_kernel(const uint32_t* __restrict__ Dinv,
                                                            const uint32_t* __restrict__ B, c64* __restrict__ part,
                                                            int64_t n, int nrhs, int KS) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t grp = (int64_t)blockIdx.x * 4 + w;
  if (grp * 16 * TI >= n) return;  // wave-uniform
  const int ks = blockIdx.y;
  const int64_t i0 = grp * 16 * TI;
  const int64_t kc = n / KS;
  const int64_t j0 = ks * kc;
  const int row = lane & 15, g = lane >> 4;
  const u32x4 zero = {0u, 0u, 0u, 0u};
  for (int r0 = 0; r0 < nrhs; r0 += 32) {
    const int ra = r0 + row, rb = r0 + 16 + row;
    const bool va = ra < nrhs, vb = rb < nrhs;
    const u32x4* Ba = reinterpret_cast<const u32x4*>(B + (int64_t)min(ra, nrhs - 1) * n + j0 + 8 * g);
    const u32x4* Bb = reinterpret_cast<const u32x4*>(B + (int64_t)min(rb, nrhs - 1) * n + j0 + 8 * g);
    const u32x4* Ar[TI];
#pragma unroll
    for (int t = 0; t < TI; ++t)
      Ar[t] = reinterpret_cast<const u32x4*>(Dinv + ((i0 / 16 + t) * (n / 32) + j0 / 32) * 512) + lane;
    f32x4 are[TI], aim[TI], bre[TI], bim[TI];
#pragma unroll
    for (int t = 0; t < TI; ++t) are[t] = aim[t] = bre[t] = bim[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int steps = (int)(kc / 32);
    for (int q = 0; q < steps; ++q) {
      u32x4 xa[2], xb[2], a[TI][2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        xa[u] = Ba[8 * q + u];
        xb[u] = Bb[8 * q + u];
#pragma unroll
        for (int t = 0; t < TI; ++t) a[t][u] = Ar[t][128 * q + 64 * u];
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        // rows beyond nrhs read a valid row and contribute zeros
        const u32x4 pa = va ? xa[u] : zero, pb = vb ? xb[u] : zero;
        const half8 a_re = as_half8(pa ^ 0x80000000u), a_im = as_half8((pa >> 16) | (pa << 16));
        const half8 b_re = as_half8(pb ^ 0x80000000u), b_im = as_half8((pb >> 16) | (pb << 16));
#pragma unroll
        for (int t = 0; t < TI; ++t) {
          const half8 m = as_half8(a[t][u]);
          are[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(m, a_re, are[t], 0, 0, 0);
          aim[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(m, a_im, aim[t], 0, 0, 0);
          bre[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(m, b_re, bre[t], 0, 0, 0);
          bim[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(m, b_im, bim[t], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < TI; ++t) {
      c64* pa = part + ((int64_t)ks * nrhs + min(ra, nrhs - 1)) * n + i0 + 16 * t + 4 * g;
      c64* pb = part + ((int64_t)ks * nrhs + min(rb, nrhs - 1)) * n + i0 + 16 * t + 4 * g;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (va) pa[v] = cmk(are[t][v], aim[t][v]);
        if (vb) pb[v] = cmk(bre[t][v], bim[t][v]);
      }
    }
  }
}

// 8-bit form of the inverse: a byte holds sign, exponent (4 bits, bias 7) and mantissa (3
// bits), the OCP E4M3 layout that gfx950's FP8 -> FP16 conversion reads (checked against
// every byte pattern on the device).  One conversion widens the two bytes of a complex
// entry to its complex-FP16 word exactly (values below 256, subnormals included).
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void widen8(uint32_t w, uint32_t& lo, uint32_t& hi) {
  lo = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(w, 1.0f, false));
  hi = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(w, 1.0f, true));
}

// As dense16_apply_kernel with the inverse in the 8-bit form: lane (row, g) reads the 16
// bytes of complex entries j0 + 32 q + 8 g .. + 7 of its rows and widens them to the same
// FP16 fragments; the row factors are applied in the reduction.
template <int TI>
__global__ __launch_bounds__(256) void dense8_apply_kernel(const uint32_t* __restrict__ Dinv8,
                                                           const uint32_t* __restrict__ B, c64* __restrict__ part,
                                                           int64_t n, int nrhs, int KS) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t grp = (int64_t)blockIdx.x * 4 + w;
  if (grp * 16 * TI >= n) return;  // wave-uniform
  const int ks = blockIdx.y;
  const int64_t i0 = grp * 16 * TI;
  const int64_t kc = n / KS;
  const int64_t j0 = ks * kc;
  const int row = lane & 15, g = lane >> 4;
  const u32x4 zero = {0u, 0u, 0u, 0u};
  for (int r0 = 0; r0 < nrhs; r0 += 32) {
    const int ra = r0 + row, rb = r0 + 16 + row;
    const bool va = ra < nrhs, vb = rb < nrhs;
    const u32x4* Ba = reinterpret_cast<const u32x4*>(B + (int64_t)min(ra, nrhs - 1) * n + j0 + 8 * g);
    const u32x4* Bb = reinterpret_cast<const u32x4*>(B + (int64_t)min(rb, nrhs - 1) * n + j0 + 8 * g);
    // one 32-bit word holds two complex entries: row i starts at word i n / 2
    const u32x4* Ar[TI];
#pragma unroll
    for (int t = 0; t < TI; ++t)
      Ar[t] = reinterpret_cast<const u32x4*>(Dinv8 + ((i0 + 16 * t + row) * n + j0 + 8 * g) / 2);
    f32x4 are[TI], aim[TI], bre[TI], bim[TI];
#pragma unroll
    for (int t = 0; t < TI; ++t) are[t] = aim[t] = bre[t] = bim[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int steps = (int)(kc / 32);
    for (int q = 0; q < steps; ++q) {
      u32x4 xa[2], xb[2], a8[TI];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        xa[u] = Ba[8 * q + u];
        xb[u] = Bb[8 * q + u];
      }
#pragma unroll
      for (int t = 0; t < TI; ++t) a8[t] = Ar[t][4 * q];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        // rows beyond nrhs read a valid row and contribute zeros
        const u32x4 pa = va ? xa[u] : zero, pb = vb ? xb[u] : zero;
        const half8 a_re = as_half8(pa ^ 0x80000000u), a_im = as_half8((pa >> 16) | (pa << 16));
        const half8 b_re = as_half8(pb ^ 0x80000000u), b_im = as_half8((pb >> 16) | (pb << 16));
#pragma unroll
        for (int t = 0; t < TI; ++t) {
          uint32_t w0, w1, w2, w3;
          widen8(u == 0 ? a8[t].x : a8[t].z, w0, w1);
          widen8(u == 0 ? a8[t].y : a8[t].w, w2, w3);
          const u32x4 wv = {w0, w1, w2, w3};
          const half8 m = as_half8(wv);
          are[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(m, a_re, are[t], 0, 0, 0);
          aim[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(m, a_im, aim[t], 0, 0, 0);
          bre[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(m, b_re, bre[t], 0, 0, 0);
          bim[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(m, b_im, bim[t], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < TI; ++t) {
      c64* pa = part + ((int64_t)ks * nrhs + min(ra, nrhs - 1)) * n + i0 + 16 * t + 4 * g;
      c64* pb = part + ((int64_t)ks * nrhs + min(rb, nrhs - 1)) * n + i0 + 16 * t + 4 * g;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (va) pa[v] = cmk(are[t][v], aim[t][v]);
        if (vb) pb[v] = cmk(bre[t][v], bim[t][v]);
      }
    }
  }
}

__device__ __forceinline__ float block_max_1024(float m, float* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  float r = 0.f;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r = fmaxf(r, red[i]);
  return r;
}

// one workgroup per RHS r: s = 2^-e with max |component| < 2^e, B16[r] = FP16(s B[r]),
// rs[r] = unscale / s (s = 1 for a zero or non-finite RHS, whose NaN/Inf then propagate)
__global__ __launch_bounds__(1024) void dense16_rhs_kernel(const c64* __restrict__ B, int64_t n, float unscale,
                                                           uint32_t* __restrict__ B16, float* __restrict__ rs) {
  __shared__ float red[16];
  const int64_t r = blockIdx.x;
  const c64* b = B + r * n;
  float m = 0.f;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) m = fmaxf(m, fmaxf(fabsf(b[i].x), fabsf(b[i].y)));
  m = block_max_1024(m, red);
  int e = 0;
  if (m > 0.f && isfinite(m)) frexpf(m, &e);  // m = f 2^e, 0.5 <= f < 1
  e = min(max(e, -100), 100);                 // scales stay normal FP32 numbers
  const float s = ldexpf(1.f, -e);
  if (threadIdx.x == 0) rs[r] = unscale * ldexpf(1.f, e);
  uint32_t* o = B16 + r * n;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) o[i] = pack_half2(s * b[i].x, s * b[i].y);
}

// Y[r][i] = rs[r] (rows ? rows[i] : 1) sum_k part[k][r][i]
__global__ void dense16_reduce_kernel(const c64* __restrict__ part, int KS, int64_t n, int64_t m,
                                      const float* __restrict__ rs, const float* __restrict__ rows,
                                      c64* __restrict__ Y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  float sx = 0.f, sy = 0.f;
  for (int k = 0; k < KS; ++k) {
    const c64 v = part[(int64_t)k * m + e];
    sx += v.x;
    sy += v.y;
  }
  const float f = rows ? rs[e / n] * rows[e % n] : rs[e / n];
  Y[e] = cmk(f * sx, f * sy);
}

// per-block maximum |component| of the FP32 inverse
__global__ __launch_bounds__(1024) void absmax_partial_kernel(const c64* __restrict__ A, int64_t m,
                                                              float* __restrict__ part) {
  __shared__ float red[16];
  float v = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    v = fmaxf(v, fmaxf(fabsf(A[i].x), fabsf(A[i].y)));
  v = block_max_1024(v, red);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// A16 = FP16(s A) in the packed order of dense16_apply_kernel (n x n, n % 32 == 0)
__global__ void to_half_kernel(const c64* __restrict__ A, int64_t n, float s, uint32_t* __restrict__ A16) {
  const int64_t m = n * n;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = k / n, j = k % n;
    A16[packed16_index(i, j, n)] = pack_half2(s * A[k].x, s * A[k].y);
  }
}

// Nearest 8-bit float (sign, 4 exponent bits with bias 7, 3 mantissa bits, ties to even)
// for |q| < 256: normal numbers 2^(F-7) (1 + m/8) for exponent field F = 1..14, subnormal
// numbers m/8 2^-6 for F = 0.
__device__ __forceinline__ uint32_t encode8(float q) {
  const uint32_t sign = q < 0.f ? 0x80u : 0u;
  const float a = fabsf(q);
  if (!(a >= 0x1p-10f)) return sign;  // below half the smallest subnormal 2^-9 (or NaN)
  int e;
  frexpf(a, &e);  // a = f 2^e, 0.5 <= f < 1
  int E = e - 1;  // a = (2f) 2^E
  if (E < -6) {
    const int mant = (int)rintf(a * 512.f);  // units of 2^-9
    return sign | (uint32_t)mant;            // mant = 8 is the smallest normal number
  }
  int mant = (int)rintf((ldexpf(a, -E) - 1.f) * 8.f);
  if (mant == 8) {
    mant = 0;
    ++E;
  }
  const int F = min(E + 7, 15);
  return sign | ((uint32_t)F << 3) | (uint32_t)(F == 15 ? min(mant, 6) : mant);
}

// one workgroup per row i: e_i with max |component| < 2^e_i, A8 row = 8-bit form of
// A_i 2^(8 - e_i) (every component below 256), rows[i] = 2^(e_i - 8)
__global__ __launch_bounds__(1024) void to_fp8_rows_kernel(const c64* __restrict__ A, int64_t n,
                                                           uint16_t* __restrict__ A8, float* __restrict__ rows) {
  __shared__ float red[16];
  const int64_t i = blockIdx.x;
  const c64* a = A + i * n;
  float m = 0.f;
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) m = fmaxf(m, fmaxf(fabsf(a[j].x), fabsf(a[j].y)));
  m = block_max_1024(m, red);
  int e = 0;
  if (m > 0.f && isfinite(m)) frexpf(m, &e);
  e = min(max(e, -100), 100);
  const float s = ldexpf(1.f, 8 - e);
  if (threadIdx.x == 0) rows[i] = ldexpf(1.f, e - 8);
  uint16_t* o = A8 + i * n;
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x)
    o[j] = (uint16_t)(encode8(s * a[j].x) | (encode8(s * a[j].y) << 8));
}

// E[r][i] = 1 if i == c0 + r else 0 (unit vectors of columns c0 .. c0 + nb - 1)
__global__ void unit_block_kernel(c128* __restrict__ E, int64_t n, int64_t c0, int nb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nb) return;
  const int64_t r = t / n, i = t % n;
  E[t] = cmk(i == c0 + r ? 1.0 : 0.0, 0.0);
}

// Dinv[i][c0 + r] = X[r][i] (FP32), tiles of 32 x 32 through LDS
__global__ void store_columns_kernel(const c128* __restrict__ X, int64_t n, int64_t c0, int nb,
                                     c64* __restrict__ Dinv) {
  __shared__ c64 tl[32][33];
  const int64_t i0 = (int64_t)blockIdx.x * 32;
  const int r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k;
    const int64_t i = i0 + tx;
    tl[k][tx] = (r < nb && i < n) ? ccast<float>(X[(int64_t)r * n + i]) : cmk(0.f, 0.f);
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int64_t i = i0 + k;
    const int r = r0 + tx;
    if (i < n && r < nb) Dinv[i * n + c0 + r] = tl[tx][k];
  }
}

constexpr int KSPLIT = 16;
constexpr int TILES = 2;     // row tiles of 16 per wavefront
constexpr int KSPLIT16 = 4;  // FP16 form: contraction split and row tiles per wavefront
constexpr int TILES16 = 4;
constexpr int KSPLIT8 = 8;  // 8-bit form (4 .. 16 measure alike)
constexpr int TILES8 = 4;

}  // namespace

void build_coarse_direct(dmlmc_hier* H, const dmlmc_defl* defl, double rtol) {
  dmlmc_ctx* ctx = H->ctx;
  const int L = (int)H->lv.size();
  const Level& C = H->lv[L - 1];
  const int64_t n = C.n();
  REQUIRE(!C.fine && C.dofs == 16, "the direct coarsest solve needs a coarse level with 16 dofs per site");
  REQUIRE(n <= 65536, "the coarsest level is too large for an explicit inverse (n > 65536)");
  REQUIRE(n % (16 * KSPLIT) == 0 && n % (16 * TILES) == 0 && n % (32 * KSPLIT16) == 0 && n % (16 * TILES16) == 0 &&
              n % (32 * KSPLIT8) == 0 && n % (16 * TILES8) == 0,
          "the coarsest dimension must be a multiple of 256");
  struct Restore {
    dmlmc_hier* H;
    const dmlmc_defl* prev;
    int prevd;
    ~Restore() {
      H->coarse_defl = prev;
      H->coarse_direct_mode = prevd;
    }
  } restore{H, H->coarse_defl, H->coarse_direct_mode};
  if (defl) H->coarse_defl = defl;
  H->coarse_direct_mode = 0;  // the columns are computed with the iterative coarsest solve
  H->coarse_dinv.alloc(sizeof(c64) * (size_t)n * n);
  constexpr int NB = 1024;
  c128* E = (c128*)hier_buf(H, "cd_E", L, sizeof(c128) * (size_t)NB * n);
  c128* X = (c128*)hier_buf(H, "cd_X", L, sizeof(c128) * (size_t)NB * n);
  for (int64_t c0 = 0; c0 < n; c0 += NB) {
    const int nb = (int)std::min<int64_t>(NB, n - c0);
    hipLaunchKernelGGL(unit_block_kernel, dim3((unsigned)ceil_div(n * nb, 256)), dim3(256), 0, ctx->stream, E, n, c0,
                       nb);
    LAUNCH_CHECK();
    SolveResult r = solve_level(H, L, E, X, nb, DMLMC_MIXED, rtol, 5000);
    if (!r.converged) throw DmlmcError(DMLMC_ENOCONV, "a column solve of the coarsest inverse did not converge");
    hipLaunchKernelGGL(store_columns_kernel, dim3((unsigned)ceil_div(n, 32), (unsigned)ceil_div(nb, 32)), dim3(256), 0,
                       ctx->stream, X, n, c0, nb, H->coarse_dinv.as<c64>());
    LAUNCH_CHECK();
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  H->coarse_dinv16.release();
  H->coarse_dinv8.release();
  H->coarse_dinv8_rows.release();
  H->coarse_dinv_n = n;
  H->coarse_dinv_rtol = rtol;
}

void build_coarse_direct16(dmlmc_hier* H) {
  dmlmc_ctx* ctx = H->ctx;
  const int64_t n = H->coarse_dinv_n;
  REQUIRE(n > 0, "the FP32 coarsest inverse must be built first");
  const int64_t m = n * n;
  constexpr int NBLK = 1024;
  DevBuf part;
  part.alloc(sizeof(float) * NBLK);
  hipLaunchKernelGGL(absmax_partial_kernel, dim3(NBLK), dim3(1024), 0, ctx->stream, H->coarse_dinv.as<c64>(), m,
                     part.as<float>());
  LAUNCH_CHECK();
  std::vector<float> h(NBLK);
  HIPCHK(hipMemcpyAsync(h.data(), part.p, sizeof(float) * NBLK, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  float amax = 0.f;
  for (float v : h) {
    if (!std::isfinite(v)) throw DmlmcError(DMLMC_ENUMERIC, "NaN/Inf in the coarsest inverse");
    amax = std::max(amax, v);
  }
  int e = 0;
  if (amax > 0.f) std::frexp(amax, &e);  // amax < 2^e
  e = std::min(std::max(e, -100), 100);
  H->coarse_dinv16.alloc(sizeof(uint32_t) * (size_t)m);
  hipLaunchKernelGGL(to_half_kernel, dim3(8192), dim3(256), 0, ctx->stream, H->coarse_dinv.as<c64>(), n,
                     std::ldexp(1.f, -e), H->coarse_dinv16.as<uint32_t>());
  LAUNCH_CHECK();
  HIPCHK(hipStreamSynchronize(ctx->stream));
  H->coarse_dinv16_unscale = std::ldexp(1.f, e);
}

void build_coarse_direct8(dmlmc_hier* H) {
  dmlmc_ctx* ctx = H->ctx;
  const int64_t n = H->coarse_dinv_n;
  REQUIRE(n > 0, "the FP32 coarsest inverse must be built first");
  H->coarse_dinv8.alloc(sizeof(uint16_t) * (size_t)n * n);
  H->coarse_dinv8_rows.alloc(sizeof(float) * (size_t)n);
  hipLaunchKernelGGL(to_fp8_rows_kernel, dim3((unsigned)n), dim3(1024), 0, ctx->stream, H->coarse_dinv.as<c64>(), n,
                     H->coarse_dinv8.as<uint16_t>(), H->coarse_dinv8_rows.as<float>());
  LAUNCH_CHECK();
  HIPCHK(hipStreamSynchronize(ctx->stream));
}

void apply_coarse_direct(dmlmc_hier* H, const c64* B, c64* Y, int nrhs) {
  dmlmc_ctx* ctx = H->ctx;
  const int64_t n = H->coarse_dinv_n;
  REQUIRE(((uintptr_t)B | (uintptr_t)Y) % 16 == 0, "direct coarsest solve needs 16-byte aligned vectors");
  const int64_t m = (int64_t)nrhs * n;
  if (H->coarse_direct_mode == 2 || H->coarse_direct_mode == 3) {
    const bool b8 = H->coarse_direct_mode == 3;
    REQUIRE(b8 ? H->coarse_dinv8.p != nullptr : H->coarse_dinv16.p != nullptr,
            "the reduced-precision coarsest inverse is not built");
    const int L = (int)H->lv.size();
    uint32_t* B16 = (uint32_t*)hier_buf(H, "cd_B16", L, sizeof(uint32_t) * (size_t)m);
    float* rs = (float*)hier_buf(H, "cd_rs", L, sizeof(float) * (size_t)nrhs);
    const int KS = b8 ? KSPLIT8 : KSPLIT16;
    c64* part = (c64*)hier_buf(H, "cd_part16", L, sizeof(c64) * (size_t)KS * m);
    KTimer kt(ctx, b8 ? "coarse_direct8" : "coarse_direct16", (b8 ? 2.0 : 4.0) * n * n + 16.0 * m);
    hipLaunchKernelGGL(dense16_rhs_kernel, dim3((unsigned)nrhs), dim3(1024), 0, ctx->stream, B, n,
                       b8 ? 1.f : H->coarse_dinv16_unscale, B16, rs);
    LAUNCH_CHECK();
    if (b8)
      hipLaunchKernelGGL(dense8_apply_kernel<TILES8>, dim3((unsigned)ceil_div(n / (16 * TILES8), 4), KSPLIT8),
                         dim3(256), 0, ctx->stream, H->coarse_dinv8.as<uint32_t>(), B16, part, n, nrhs, KSPLIT8);
    else
      hipLaunchKernelGGL(dense16_apply_kernel<TILES16>, dim3((unsigned)ceil_div(n / (16 * TILES16), 4), KSPLIT16),
                         dim3(256), 0, ctx->stream, H->coarse_dinv16.as<uint32_t>(), B16, part, n, nrhs, KSPLIT16);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(dense16_reduce_kernel, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, ctx->stream, part, KS,
                       n, m, rs, b8 ? H->coarse_dinv8_rows.as<float>() : (const float*)nullptr, Y);
    LAUNCH_CHECK();
    return;
  }
  c64* part = (c64*)hier_buf(H, "cd_part", (int)H->lv.size(), sizeof(c64) * (size_t)KSPLIT * m);
  KTimer kt(ctx, "coarse_direct", 8.0 * n * n * nrhs);
  hipLaunchKernelGGL(dense_apply_kernel<TILES>, dim3((unsigned)ceil_div(n / (16 * TILES), 4), KSPLIT), dim3(256), 0,
                     ctx->stream, H->coarse_dinv.as<c64>(), B, part, n, nrhs, KSPLIT);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(dense_reduce_kernel, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, ctx->stream, part, KSPLIT, m,
                     Y);
  LAUNCH_CHECK();
}
