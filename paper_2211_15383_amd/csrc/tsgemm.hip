// Tall-skinny FP64 products of the eigensolvers' Rayleigh-Ritz steps, with n (the level
// dimension) up to millions and a few dozen to a few hundred vectors:
//   gram:   G[r][i] = <A_i, B_r> = sum_p conj(A_i[p]) B_r[p]
//   rotate: out_r  = sum_i S[r][i] Y_i
// Vectors are [count][n] complex128.  The Gram product stages 32-row tiles of both
// operands in LDS, the rotation stages the coefficients; they keep a 32 x 32 block of results (gram) or 32 outputs of a row (rotate) per
// workgroup, so every vector is read once per 32 vectors of the other operand instead
// of once per vector.  Gram partial sums are reduced in a fixed order (no atomics).
#include "tsgemm.h"

namespace {

constexpr int GTR = 32;  // rows per LDS tile of the Gram product
constexpr int TR = 64;   // rows per workgroup of the rotation
constexpr int PB = 32;   // result block edge (gram) / outputs per workgroup (rotate)

// grid: (row chunks, ceil(na / PB) * ceil(nb / PB)); a 32 x 32 block of results over 256
// threads: thread t holds i = i0 + t % 32 and r = r0 + t / 32 + 8 q for q < 4.
__global__ __launch_bounds__(256) void gram_partial_kernel(const c128* __restrict__ A, int na,
                                                           const c128* __restrict__ B, int nb, int64_t n,
                                                           c128* __restrict__ part) {
  __shared__ c128 As[GTR][PB + 1];
  __shared__ c128 Bs[GTR][PB + 1];
  const int nib = (na + PB - 1) / PB;
  const int i0 = (blockIdx.y % nib) * PB, r0 = (blockIdx.y / nib) * PB;
  const int t = threadIdx.x;
  const int ii = t % PB, rr = t / PB;  // rr in 0..7
  c128 acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = cmk(0.0, 0.0);
  const int64_t ntiles = (n + GTR - 1) / GTR;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t p0 = tile * GTR;
    // stage: 256 threads load GTR x PB entries of each operand (row-fast across threads)
    for (int e = t; e < GTR * PB; e += 256) {
      const int row = e % GTR, col = e / GTR;
      const int64_t p = p0 + row;
      const int ia = i0 + col, ib = r0 + col;
      As[row][col] = (p < n && ia < na) ? A[(int64_t)ia * n + p] : cmk(0.0, 0.0);
      Bs[row][col] = (p < n && ib < nb) ? B[(int64_t)ib * n + p] : cmk(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int row = 0; row < GTR; ++row) {
      const c128 a = As[row][ii];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const c128 bv = Bs[row][rr + 8 * q];
        acc[q].x += a.x * bv.x + a.y * bv.y;
        acc[q].y += a.x * bv.y - a.y * bv.x;
      }
    }
    __syncthreads();
  }
  // part[chunk][r][i] over the full na x nb result, zero-padded blocks skipped
  c128* out = part + (int64_t)blockIdx.x * na * nb;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = i0 + ii, r = r0 + rr + 8 * q;
    if (i < na && r < nb) out[(int64_t)r * na + i] = acc[q];
  }
}

__global__ void gram_reduce_kernel(const c128* __restrict__ part, int chunks, int64_t m, c128* __restrict__ G) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  c128 s = cmk(0.0, 0.0);
  for (int c = 0; c < chunks; ++c) s = s + part[(int64_t)c * m + e];
  G[e] = s;
}

// grid: (ceil(n / TR), ceil(nr / PB)); thread t: row t % TR of the tile, outputs
// r0 + (t / TR) * 8 + q for q < 8.  S is staged in LDS per 64 input vectors.
__global__ __launch_bounds__(256) void rotate_kernel(const c128* __restrict__ Y, int ny, const c128* __restrict__ S,
                                                     int nr, int64_t n, c128* __restrict__ out) {
  __shared__ c128 Ss[64][PB + 1];
  const int t = threadIdx.x;
  const int row = t % TR, grp = t / TR;  // grp in 0..3
  const int64_t p = (int64_t)blockIdx.x * TR + row;
  const int r0 = blockIdx.y * PB;
  c128 acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = cmk(0.0, 0.0);
  for (int i0 = 0; i0 < ny; i0 += 64) {
    for (int e = t; e < 64 * PB; e += 256) {
      const int ii = e % 64, rr = e / 64;
      const int i = i0 + ii, r = r0 + rr;
      Ss[ii][rr] = (i < ny && r < nr) ? S[(int64_t)r * ny + i] : cmk(0.0, 0.0);
    }
    __syncthreads();
    const int iend = min(64, ny - i0);
    for (int ii = 0; ii < iend; ++ii) {
      const c128 y = p < n ? Y[(int64_t)(i0 + ii) * n + p] : cmk(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const c128 s = Ss[ii][grp * 8 + q];
        acc[q].x += s.x * y.x - s.y * y.y;
        acc[q].y += s.x * y.y + s.y * y.x;
      }
    }
    __syncthreads();
  }
  if (p >= n) return;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int r = r0 + grp * 8 + q;
    if (r < nr) out[(int64_t)r * n + p] = acc[q];
  }
}

}  // namespace

void ts_gram(dmlmc_ctx* ctx, const c128* A, int na, const c128* B, int nb, int64_t n, c128* G, DevBuf& scratch) {
  const int blocks = ((na + PB - 1) / PB) * ((nb + PB - 1) / PB);
  const int64_t ntiles = (n + GTR - 1) / GTR;
  const int chunks = (int)std::max<int64_t>(1, std::min<int64_t>(ntiles, std::max(1, 1024 / blocks)));
  const int64_t m = (int64_t)na * nb;
  scratch.ensure(sizeof(c128) * (size_t)chunks * m);
  hipLaunchKernelGGL(gram_partial_kernel, dim3((unsigned)chunks, (unsigned)blocks), dim3(256), 0, ctx->stream, A, na, B,
                     nb, n, scratch.as<c128>());
  LAUNCH_CHECK();
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, ctx->stream,
                     scratch.as<c128>(), chunks, m, G);
  LAUNCH_CHECK();
}

void ts_rotate(dmlmc_ctx* ctx, const c128* Y, int ny, const c128* S, int nr, int64_t n, c128* out) {
  dim3 grid((unsigned)ceil_div(n, TR), (unsigned)ceil_div(nr, PB));
  hipLaunchKernelGGL(rotate_kernel, grid, dim3(256), 0, ctx->stream, Y, ny, S, nr, n, out);
  LAUNCH_CHECK();
}
