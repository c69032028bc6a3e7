// Direct solve of the coarsest level (d = 16) with its explicit inverse.
//
// Setup: the columns of D_L^-1 come from multi-RHS solves of D_L X = I (blocks of unit
// vectors, FP64 refinement to 1e-10); the inverse is kept in complex FP32, row-major
// [n][n].  Apply: Y = D_L^-1 B for a block of RHS on the matrix cores, the same operand
// layout as the coarse stencil (lane (row, kq) takes the quads Dinv[i0 + row][j0 + 4kq ..]
// and B[r0 + row][j0 + 4kq ..], and receives Y[r0 + row][i0 + 4kq + v]); the contraction
// is split over KS waves whose partial tiles are summed by a second kernel in a fixed
// order.  At n = 16384 and 32 RHS one apply is 69 GFLOP over a 2.1 GB operand: matrix-core
// bound (~0.44 ms at the FP32 peak), comparable to the iterative coarsest solve it
// replaces, and exact to FP32 rounding.
#include "dense.h"
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
constexpr int TILES = 2;  // row tiles of 16 per wavefront

}  // namespace

void build_coarse_direct(dmlmc_hier* H, const dmlmc_defl* defl) {
  dmlmc_ctx* ctx = H->ctx;
  const int L = (int)H->lv.size();
  const Level& C = H->lv[L - 1];
  const int64_t n = C.n();
  REQUIRE(!C.fine && C.dofs == 16, "the direct coarsest solve needs a coarse level with 16 dofs per site");
  REQUIRE(n <= 65536, "the coarsest level is too large for an explicit inverse (n > 65536)");
  REQUIRE(n % (16 * KSPLIT) == 0 && n % (16 * TILES) == 0, "the coarsest dimension must be a multiple of 256");
  struct Restore {
    dmlmc_hier* H;
    const dmlmc_defl* prev;
    bool prevd;
    ~Restore() {
      H->coarse_defl = prev;
      H->coarse_direct_on = prevd;
    }
  } restore{H, H->coarse_defl, H->coarse_direct_on};
  if (defl) H->coarse_defl = defl;
  H->coarse_direct_on = false;  // the columns are computed with the iterative coarsest solve
  H->coarse_dinv.alloc(sizeof(c64) * (size_t)n * n);
  constexpr int NB = 512;
  c128* E = (c128*)hier_buf(H, "cd_E", L, sizeof(c128) * (size_t)NB * n);
  c128* X = (c128*)hier_buf(H, "cd_X", L, sizeof(c128) * (size_t)NB * n);
  for (int64_t c0 = 0; c0 < n; c0 += NB) {
    const int nb = (int)std::min<int64_t>(NB, n - c0);
    hipLaunchKernelGGL(unit_block_kernel, dim3((unsigned)ceil_div(n * nb, 256)), dim3(256), 0, ctx->stream, E, n, c0,
                       nb);
    LAUNCH_CHECK();
    SolveResult r = solve_level(H, L, E, X, nb, DMLMC_MIXED, 1e-10, 5000);
    if (!r.converged) throw DmlmcError(DMLMC_ENOCONV, "a column solve of the coarsest inverse did not converge");
    hipLaunchKernelGGL(store_columns_kernel, dim3((unsigned)ceil_div(n, 32), (unsigned)ceil_div(nb, 32)), dim3(256), 0,
                       ctx->stream, X, n, c0, nb, H->coarse_dinv.as<c64>());
    LAUNCH_CHECK();
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  H->coarse_dinv_n = n;
}

void apply_coarse_direct(dmlmc_hier* H, const c64* B, c64* Y, int nrhs) {
  dmlmc_ctx* ctx = H->ctx;
  const int64_t n = H->coarse_dinv_n;
  REQUIRE(((uintptr_t)B | (uintptr_t)Y) % 16 == 0, "direct coarsest solve needs 16-byte aligned vectors");
  const int64_t m = (int64_t)nrhs * n;
  c64* part = (c64*)hier_buf(H, "cd_part", (int)H->lv.size(), sizeof(c64) * (size_t)KSPLIT * m);
  KTimer kt(ctx, "coarse_direct", 8.0 * n * n * nrhs);
  hipLaunchKernelGGL(dense_apply_kernel<TILES>, dim3((unsigned)ceil_div(n / (16 * TILES), 4), KSPLIT), dim3(256), 0,
                     ctx->stream, H->coarse_dinv.as<c64>(), B, part, n, nrhs, KSPLIT);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(dense_reduce_kernel, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, ctx->stream, part, KSPLIT, m,
                     Y);
  LAUNCH_CHECK();
}
