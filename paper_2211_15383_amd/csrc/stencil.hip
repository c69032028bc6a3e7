// Level operators of the multigrid hierarchy on gfx950:
//   * fine Wilson-Schwinger stencil (spin-projected hops, links folded with the
//     antiperiodic sign), multi-RHS;
//   * coarse nearest-neighbour block stencil (dense d x d blocks, column-major);
//   * SAP smoother on 4x4 (or 2x2) site blocks with local minimal-residual iterations,
//     red/black over blocks, residual b - D x fused in;
//   * red/black point-block Gauss-Seidel on coarse levels (exact inverse self blocks);
//   * restriction P^H and prolongation P on (aggregate, chirality) blocks.
// Vectors are RHS-major: entry i of RHS r is at r * ld + i; complex interleaved.
#include "common.h"

namespace {

template <typename R>
struct __align__(4 * sizeof(R)) Spinor {
  Cx<R> s0, s1;
};

template <typename R>
__device__ __forceinline__ Cx<R> mul_i(Cx<R> a) { return cmk(-a.y, a.x); }
template <typename R>
__device__ __forceinline__ Cx<R> mul_mi(Cx<R> a) { return cmk(a.y, -a.x); }

struct Nbr {
  int64_t xp, xm, tp, tm;
};
__device__ __forceinline__ Nbr neighbours(int64_t s, int Lx, int Lt) {
  int x = (int)(s % Lx), t = (int)(s / Lx);
  Nbr n;
  n.xp = (x + 1 == Lx) ? s - (Lx - 1) : s + 1;
  n.xm = (x == 0) ? s + (Lx - 1) : s - 1;
  n.tp = (t + 1 == Lt) ? s - (int64_t)(Lt - 1) * Lx : s + Lx;
  n.tm = (t == 0) ? s + (int64_t)(Lt - 1) * Lx : s - Lx;
  return n;
}

// Sum of the four hop terms (without the -1/2): returns (acc0, acc1).
// fwd x: (1 - s1) psi = (h, -h), h = p0 - p1; bwd x: (1 + s1) psi = (g, g), g = p0 + p1
// fwd t: (1 - s2) psi = (h, -i h), h = p0 + i p1; bwd t: (1 + s2) psi = (g, i g), g = p0 - i p1
template <typename R>
__device__ __forceinline__ void hops(Cx<R> ux, Cx<R> uxm, Cx<R> ut, Cx<R> utm, Spinor<R> fx, Spinor<R> bx,
                                     Spinor<R> ft, Spinor<R> bt, Cx<R>& a0, Cx<R>& a1) {
  Cx<R> h = ux * (fx.s0 - fx.s1);
  a0 = h;
  a1 = cmk(-h.x, -h.y);
  Cx<R> g = conj(uxm) * (bx.s0 + bx.s1);
  a0 = a0 + g;
  a1 = a1 + g;
  h = ut * (ft.s0 + mul_i(ft.s1));
  a0 = a0 + h;
  a1 = a1 + mul_mi(h);
  g = conj(utm) * (bt.s0 + mul_mi(bt.s1));
  a0 = a0 + g;
  a1 = a1 + mul_i(g);
}

template <typename R, bool G5>
__global__ __launch_bounds__(256) void wilson_kernel(const Cx<R>* __restrict__ U, const Cx<R>* __restrict__ in,
                                                     Cx<R>* __restrict__ out, int Lx, int Lt, R diag, int nrhs,
                                                     int rb, int64_t ldx, int64_t ldy) {
  const int64_t V = (int64_t)Lx * Lt;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= V) return;
  const Nbr nb = neighbours(s, Lx, Lt);
  const Cx<R> ux = U[s], ut = U[V + s], uxm = U[nb.xm], utm = U[V + nb.tm];
  const int r0 = blockIdx.y * rb;
  const int r1 = min(r0 + rb, nrhs);
  const R half = (R)0.5;
  for (int r = r0; r < r1; ++r) {
    const Spinor<R>* p = reinterpret_cast<const Spinor<R>*>(in + r * ldx);
    Spinor<R> c = p[s];
    Cx<R> a0, a1;
    hops(ux, uxm, ut, utm, p[nb.xp], p[nb.xm], p[nb.tp], p[nb.tm], a0, a1);
    Spinor<R> o;
    o.s0 = diag * c.s0 - half * a0;
    o.s1 = diag * c.s1 - half * a1;
    if (G5) o.s1 = cmk(-o.s1.x, -o.s1.y);
    reinterpret_cast<Spinor<R>*>(out + r * ldy)[s] = o;
  }
}

// Coarse block stencil: y_s = sum_dir A[s][dir] x_{s+dir}; blocks column-major
// (A[s][dir][j * d + i] = row i, column j).  Thread per (site, row), RB right-hand sides
// per thread so that every block entry is loaded once per RB vectors.
template <typename R, int RB, bool G5>
__global__ __launch_bounds__(256) void coarse_kernel(const Cx<R>* __restrict__ A, const Cx<R>* __restrict__ in,
                                                     Cx<R>* __restrict__ out, int Lx, int Lt, int d, int spb,
                                                     int nrhs, int64_t ldx, int64_t ldy) {
  const int64_t V = (int64_t)Lx * Lt;
  const int i = threadIdx.x % d;
  const int64_t s = (int64_t)blockIdx.x * spb + threadIdx.x / d;
  if (threadIdx.x >= spb * d || s >= V) return;
  const Nbr nb = neighbours(s, Lx, Lt);
  const int64_t sites[5] = {s, nb.xp, nb.xm, nb.tp, nb.tm};
  const int r0 = blockIdx.y * RB;
  const int nr = min(RB, nrhs - r0);
  Cx<R> acc[RB];
#pragma unroll
  for (int q = 0; q < RB; ++q) acc[q] = cmk((R)0, (R)0);
  const Cx<R>* Ab = A + s * 5 * d * d;
  for (int dir = 0; dir < 5; ++dir) {
    const Cx<R>* Ad = Ab + dir * d * d + i;
    const int64_t base = sites[dir] * d;
    for (int j = 0; j < d; ++j) {
      const Cx<R> a = Ad[j * d];
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        if (q < nr) cfma(acc[q], a, in[(r0 + q) * ldx + base + j]);
      }
    }
  }
  const bool neg = G5 && (i >= d / 2);
#pragma unroll
  for (int q = 0; q < RB; ++q) {
    if (q < nr) out[(r0 + q) * ldy + s * d + i] = neg ? cmk(-acc[q].x, -acc[q].y) : acc[q];
  }
}

// SAP on BSX x BST site blocks (lanes of one block are contiguous within a wavefront).
// For every block of colour `color`: r_B = b_B - (D x)_B, then `mr` minimal-residual
// iterations on the block-restricted operator D_BB (zero outside the block) from e = 0,
// then x_B += e.
template <typename R, int BSX, int BST>
__global__ __launch_bounds__(256) void sap_kernel(const Cx<R>* __restrict__ U, Cx<R>* __restrict__ x,
                                                  const Cx<R>* __restrict__ b, int Lx, int Lt, R diag, int nrhs,
                                                  int rb, int color, int mr) {
  constexpr int BL = BSX * BST;  // lanes per block
  const int64_t V = (int64_t)Lx * Lt;
  const int nbx = Lx / BSX, nbt = Lt / BST;
  const int lane = threadIdx.x % BL;
  const int blk = blockIdx.x * (blockDim.x / BL) + threadIdx.x / BL;
  const int BXi = blk % nbx, BTi = blk / nbx;
  const bool active = (blk < nbx * nbt) && (((BXi + BTi) & 1) == color);
  const int lx = lane % BSX, lt = lane / BSX;
  const int xs = BXi * BSX + lx, ts = BTi * BST + lt;
  const int64_t s = active ? (int64_t)xs + (int64_t)Lx * ts : 0;
  const Nbr nb = neighbours(s, Lx, Lt);
  Cx<R> ux = cmk((R)0, (R)0), ut = ux, uxm = ux, utm = ux;
  if (active) {
    ux = U[s];
    ut = U[V + s];
    uxm = U[nb.xm];
    utm = U[V + nb.tm];
  }
  // in-block neighbour lanes (masks for the block-restricted operator)
  const bool hxp = lx + 1 < BSX, hxm = lx > 0, htp = lt + 1 < BST, htm = lt > 0;
  const int gbase = (threadIdx.x / BL) * BL;  // first lane of my block within the workgroup
  const int wl = (threadIdx.x & 63);           // lane within wavefront
  const int wbase = wl - lane;                 // first lane of my block within the wavefront
  (void)gbase;
  const R half = (R)0.5;
  const int r0 = blockIdx.y * rb;
  const int r1 = min(r0 + rb, nrhs);
  for (int r = r0; r < r1; ++r) {
    Spinor<R>* xp = reinterpret_cast<Spinor<R>*>(x + r * (int64_t)(2 * V));
    const Spinor<R>* bp = reinterpret_cast<const Spinor<R>*>(b + r * (int64_t)(2 * V));
    Spinor<R> rho;
    rho.s0 = rho.s1 = cmk((R)0, (R)0);
    Spinor<R> xc = rho;
    if (active) {
      xc = xp[s];
      Cx<R> a0, a1;
      hops(ux, uxm, ut, utm, xp[nb.xp], xp[nb.xm], xp[nb.tp], xp[nb.tm], a0, a1);
      Spinor<R> bb = bp[s];
      rho.s0 = bb.s0 - (diag * xc.s0 - half * a0);
      rho.s1 = bb.s1 - (diag * xc.s1 - half * a1);
    }
    Spinor<R> e;
    e.s0 = e.s1 = cmk((R)0, (R)0);
    for (int it = 0; it < mr; ++it) {
      // q = D_BB rho, neighbours from lanes of the same block
      Spinor<R> fx, bx, ft, bt;
      const R v[4] = {rho.s0.x, rho.s0.y, rho.s1.x, rho.s1.y};
      R fxv[4], bxv[4], ftv[4], btv[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        fxv[c] = __shfl(v[c], wbase + (hxp ? lane + 1 : lane), 64);
        bxv[c] = __shfl(v[c], wbase + (hxm ? lane - 1 : lane), 64);
        ftv[c] = __shfl(v[c], wbase + (htp ? lane + BSX : lane), 64);
        btv[c] = __shfl(v[c], wbase + (htm ? lane - BSX : lane), 64);
      }
      const R zx = (R)0;
      fx.s0 = hxp ? cmk(fxv[0], fxv[1]) : cmk(zx, zx);
      fx.s1 = hxp ? cmk(fxv[2], fxv[3]) : cmk(zx, zx);
      bx.s0 = hxm ? cmk(bxv[0], bxv[1]) : cmk(zx, zx);
      bx.s1 = hxm ? cmk(bxv[2], bxv[3]) : cmk(zx, zx);
      ft.s0 = htp ? cmk(ftv[0], ftv[1]) : cmk(zx, zx);
      ft.s1 = htp ? cmk(ftv[2], ftv[3]) : cmk(zx, zx);
      bt.s0 = htm ? cmk(btv[0], btv[1]) : cmk(zx, zx);
      bt.s1 = htm ? cmk(btv[2], btv[3]) : cmk(zx, zx);
      Cx<R> a0, a1;
      hops(ux, uxm, ut, utm, fx, bx, ft, bt, a0, a1);
      Spinor<R> q;
      q.s0 = diag * rho.s0 - half * a0;
      q.s1 = diag * rho.s1 - half * a1;
      // alpha = <q, rho> / <q, q> over the block
      R qr_x = q.s0.x * rho.s0.x + q.s0.y * rho.s0.y + q.s1.x * rho.s1.x + q.s1.y * rho.s1.y;
      R qr_y = q.s0.x * rho.s0.y - q.s0.y * rho.s0.x + q.s1.x * rho.s1.y - q.s1.y * rho.s1.x;
      R qq = q.s0.x * q.s0.x + q.s0.y * q.s0.y + q.s1.x * q.s1.x + q.s1.y * q.s1.y;
#pragma unroll
      for (int off = BL / 2; off > 0; off >>= 1) {
        qr_x += __shfl_xor(qr_x, off, 64);
        qr_y += __shfl_xor(qr_y, off, 64);
        qq += __shfl_xor(qq, off, 64);
      }
      const R inv = qq > (R)0 ? (R)1 / qq : (R)0;
      const Cx<R> alpha = cmk(qr_x * inv, qr_y * inv);
      e.s0 = e.s0 + alpha * rho.s0;
      e.s1 = e.s1 + alpha * rho.s1;
      rho.s0 = rho.s0 - alpha * q.s0;
      rho.s1 = rho.s1 - alpha * q.s1;
    }
    if (active) {
      xc.s0 = xc.s0 + e.s0;
      xc.s1 = xc.s1 + e.s1;
      xp[s] = xc;
    }
  }
}

// Red/black point-block Gauss-Seidel on a coarse level: for every site of colour
// `color`, x_s <- x_s + A_ss^-1 (b_s - (D x)_s).  Thread per (site, row); the residual of
// a site is exchanged through LDS.
template <typename R>
__global__ __launch_bounds__(256) void coarse_gs_kernel(const Cx<R>* __restrict__ A, const Cx<R>* __restrict__ Ainv,
                                                        Cx<R>* __restrict__ x, const Cx<R>* __restrict__ b, int Lx,
                                                        int Lt, int d, int spb, int nrhs, int rb, int color,
                                                        int even_lx) {
  extern __shared__ unsigned char smem_raw[];
  Cx<R>* res = reinterpret_cast<Cx<R>*>(smem_raw);
  const int64_t V = (int64_t)Lx * Lt;
  const int i = threadIdx.x % d;
  const int ls = threadIdx.x / d;
  const int64_t k = (int64_t)blockIdx.x * spb + ls;
  int64_t s;
  bool active;
  if (even_lx) {
    // k-th site of colour `color`: t = k / (Lx/2), x = 2 (k % (Lx/2)) + ((t + color) & 1)
    const int64_t half = Lx / 2;
    const int64_t t = k / half;
    s = 2 * (k % half) + ((t + color) & 1) + t * Lx;
    active = (threadIdx.x < spb * d) && (t < Lt);
  } else {
    s = k;
    active = (threadIdx.x < spb * d) && (s < V) && ((((s % Lx) + (s / Lx)) & 1) == color);
  }
  if (!active) s = 0;
  const Nbr nb = neighbours(s, Lx, Lt);
  const int64_t sites[5] = {s, nb.xp, nb.xm, nb.tp, nb.tm};
  const Cx<R>* Ab = A + s * 5 * d * d;
  const int64_t ld = V * d;
  const int r0 = blockIdx.y * rb;
  const int r1 = min(r0 + rb, nrhs);
  for (int r = r0; r < r1; ++r) {
    const Cx<R>* xr = x + r * ld;
    Cx<R> acc = cmk((R)0, (R)0);
    if (active) {
      acc = b[r * ld + s * d + i];
      for (int dir = 0; dir < 5; ++dir) {
        const Cx<R>* Ad = Ab + dir * d * d + i;
        const int64_t base = sites[dir] * d;
        for (int j = 0; j < d; ++j) {
          const Cx<R> a = Ad[j * d];
          const Cx<R> v = xr[base + j];
          acc.x -= a.x * v.x - a.y * v.y;
          acc.y -= a.x * v.y + a.y * v.x;
        }
      }
    }
    __syncthreads();
    res[ls * d + i] = acc;
    __syncthreads();
    if (active) {
      Cx<R> e = cmk((R)0, (R)0);
      const Cx<R>* Ai = Ainv + s * d * d + i;
      for (int j = 0; j < d; ++j) cfma(e, Ai[j * d], res[ls * d + j]);
      Cx<R>* xw = x + r * ld + s * d + i;
      *xw = *xw + e;
    }
  }
}

// Restriction y_c = P^H x_f.  P blocks: P[cs][c][row][k] (row-major, N columns), row =
// local site * h + dof within chirality, local site = lx + ax * lt, h = d_f / 2.
// Thread per (coarse dof, group of RB right-hand sides): each P entry is loaded once per
// RB vectors.
template <typename R, int RB>
__global__ __launch_bounds__(256) void restrict_kernel(const Cx<R>* __restrict__ P, const Cx<R>* __restrict__ xf,
                                                       Cx<R>* __restrict__ yc, int Lxf, int Ltf, int df, int ax,
                                                       int at, int N, int nrhs) {
  const int Lxc = Lxf / ax, Ltc = Ltf / at;
  const int64_t Vc = (int64_t)Lxc * Ltc;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (cs, c, k)
  if (tid >= Vc * 2 * N) return;
  const int k = (int)(tid % N);
  const int c = (int)((tid / N) % 2);
  const int64_t cs = tid / (2 * N);
  const int X = (int)(cs % Lxc), T = (int)(cs / Lxc);
  const int h = df / 2;
  const int rows = ax * at * h;
  const Cx<R>* Pb = P + (cs * 2 + c) * (int64_t)rows * N + k;
  const int64_t ldf = (int64_t)Lxf * Ltf * df, ldc = Vc * 2 * N;
  const int r0 = blockIdx.y * RB;
  const int nr = min(RB, nrhs - r0);
  Cx<R> acc[RB];
#pragma unroll
  for (int q = 0; q < RB; ++q) acc[q] = cmk((R)0, (R)0);
  const Cx<R>* xr = xf + (int64_t)r0 * ldf;
  int row = 0;
  for (int lt = 0; lt < at; ++lt) {
    const int64_t srow = (int64_t)(T * at + lt) * Lxf + (int64_t)X * ax;
    for (int lx = 0; lx < ax; ++lx) {
      const int64_t fbase = (srow + lx) * df + c * h;
      for (int j = 0; j < h; ++j, ++row) {
        const Cx<R> pv = Pb[(int64_t)row * N];
#pragma unroll
        for (int q = 0; q < RB; ++q)
          if (q < nr) cfmac(acc[q], pv, xr[q * ldf + fbase + j]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < RB; ++q)
    if (q < nr) yc[(int64_t)(r0 + q) * ldc + cs * 2 * N + c * N + k] = acc[q];
}

// Prolongation x_f (+)= P e_c; thread per (fine dof, group of RB right-hand sides).
template <typename R, int RB>
__global__ __launch_bounds__(256) void prolong_kernel(const Cx<R>* __restrict__ P, const Cx<R>* __restrict__ ec,
                                                      Cx<R>* __restrict__ xf, int Lxf, int Ltf, int df, int ax, int at,
                                                      int N, int nrhs, int add) {
  const int64_t nf = (int64_t)Lxf * Ltf * df;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= nf) return;
  const int dof = (int)(tid % df);
  const int64_t site = tid / df;
  const int x = (int)(site % Lxf), t = (int)(site / Lxf);
  const int Lxc = Lxf / ax;
  const int64_t Vc = (int64_t)Lxc * (Ltf / at);
  const int64_t cs = (int64_t)(x / ax) + (int64_t)Lxc * (t / at);
  const int h = df / 2;
  const int c = dof / h, j = dof % h;
  const int row = ((x % ax) + ax * (t % at)) * h + j;
  const int rows = ax * at * h;
  const Cx<R>* Pr = P + ((cs * 2 + c) * (int64_t)rows + row) * N;
  const int64_t ldc = Vc * 2 * N;
  const int r0 = blockIdx.y * RB;
  const int nr = min(RB, nrhs - r0);
  const Cx<R>* er = ec + (int64_t)r0 * ldc + cs * 2 * N + c * N;
  Cx<R> acc[RB];
#pragma unroll
  for (int q = 0; q < RB; ++q)
    acc[q] = (add && q < nr) ? xf[(int64_t)(r0 + q) * nf + tid] : cmk((R)0, (R)0);
  for (int kk = 0; kk < N; ++kk) {
    const Cx<R> pv = Pr[kk];
#pragma unroll
    for (int q = 0; q < RB; ++q)
      if (q < nr) cfma(acc[q], pv, er[q * ldc + kk]);
  }
#pragma unroll
  for (int q = 0; q < RB; ++q)
    if (q < nr) xf[(int64_t)(r0 + q) * nf + tid] = acc[q];
}

// ---------------------------------------------------------------- matrix-core forms (d = 16, complex FP32)
// One wavefront computes a 16 (dofs) x 16 (RHS) tile of one site with v_mfma_f32_16x16x4_f32:
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and receives D[4 (l / 16) + v][l % 16].
// A complex product A X takes four real products (re: Ar Xr - Ai Xi, im: Ar Xi + Ai Xr).
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void cmfma(f32x4& dre, f32x4& dim, c64 a, c64 x) {
  dre = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, x.x, dre, 0, 0, 0);
  dre = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.y, x.y, dre, 0, 0, 0);
  dim = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, x.y, dim, 0, 0, 0);
  dim = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, x.x, dim, 0, 0, 0);
}

// The five x tiles (16 RHS x 16 dofs each) a site needs are first staged in LDS with
// 16-byte loads, one 128-byte row per RHS; rows are padded to 17 entries so that the
// B-operand reads (16 lanes, consecutive RHS, one dof) hit distinct banks.
constexpr int XPAD = 17;

struct __align__(16) C64Pair {
  c64 a, b;
};

__device__ __forceinline__ void stage_x_tiles(const c64* __restrict__ x, int64_t ld, const int64_t* sites, int r0,
                                              int nrhs, bool valid, c64 (*Xl)[16][XPAD]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int q = lane + 64 * u;
    const int rr = q >> 3, part = q & 7;
    const bool ok = valid && (r0 + rr < nrhs);
#pragma unroll
    for (int dir = 0; dir < 5; ++dir) {
      C64Pair v;
      if (ok) {
        v = *reinterpret_cast<const C64Pair*>(x + (int64_t)(r0 + rr) * ld + sites[dir] * 16 + 2 * part);
      } else {
        v.a = cmk(0.f, 0.f);
        v.b = v.a;
      }
      Xl[dir][rr][2 * part] = v.a;
      Xl[dir][rr][2 * part + 1] = v.b;
    }
  }
}

// D += sum_dir A[s][dir] X[nb(dir)] for the tile, X from the LDS tiles.
__device__ __forceinline__ void site_product16(const c64* __restrict__ A, int64_t s, c64 (*Xl)[16][XPAD], int row,
                                               int kq, f32x4& dre, f32x4& dim) {
  for (int dir = 0; dir < 5; ++dir) {
    const c64* Ad = A + (s * 5 + dir) * 256;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int j = 4 * t + kq;
      cmfma(dre, dim, Ad[j * 16 + row], Xl[dir][row][j]);
    }
  }
}

template <bool G5>
__global__ __launch_bounds__(256) void coarse16_mfma_kernel(const c64* __restrict__ A, const c64* __restrict__ in,
                                                            c64* __restrict__ out, int Lx, int Lt, int nrhs,
                                                            int64_t ldx, int64_t ldy) {
  __shared__ c64 Xs[4][5][16][XPAD];
  const int64_t V = (int64_t)Lx * Lt;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ntile = (nrhs + 15) / 16;
  const int64_t wave = (int64_t)blockIdx.x * 4 + w;
  const int64_t s0 = wave / ntile;
  const bool valid = s0 < V;  // every wavefront reaches the barrier
  const int64_t s = valid ? s0 : 0;
  const int tile = (int)(wave % ntile);
  const int row = lane & 15, kq = lane >> 4;
  const int rhs = tile * 16 + row;
  const Nbr nb = neighbours(s, Lx, Lt);
  const int64_t sites[5] = {s, nb.xp, nb.xm, nb.tp, nb.tm};
  stage_x_tiles(in, ldx, sites, tile * 16, nrhs, valid, Xs[w]);
  __syncthreads();
  f32x4 dre = {0.f, 0.f, 0.f, 0.f}, dim = {0.f, 0.f, 0.f, 0.f};
  site_product16(A, s, Xs[w], row, kq, dre, dim);
  if (!valid || rhs >= nrhs) return;
  c64* o = out + (int64_t)rhs * ldy + s * 16;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 4 * kq + v;
    const float sg = (G5 && i >= 8) ? -1.f : 1.f;
    o[i] = cmk(sg * dre[v], sg * dim[v]);
  }
}

// Red/black point-block Gauss-Seidel, d = 16: R = b - D x on the colour sites, then
// x += A_ss^-1 R, both products on the matrix cores; R passes through LDS to reach the
// B-operand layout.  Every wavefront reaches the barriers (no early exit).
__global__ __launch_bounds__(256) void coarse16_gs_mfma_kernel(const c64* __restrict__ A, const c64* __restrict__ Ainv,
                                                               c64* __restrict__ x, const c64* __restrict__ b, int Lx,
                                                               int Lt, int nrhs, int color, int even_lx) {
  __shared__ c64 Xs[4][5][16][XPAD];
  __shared__ c64 Rl[4][16][XPAD];  // [wave][rhs][dof]
  const int64_t V = (int64_t)Lx * Lt;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ntile = (nrhs + 15) / 16;
  const int64_t wave = (int64_t)blockIdx.x * 4 + w;
  const int64_t k = wave / ntile;
  const int tile = (int)(wave % ntile);
  int64_t s;
  bool active;
  if (even_lx) {
    const int64_t half = Lx / 2;
    const int64_t t = k / half;
    s = 2 * (k % half) + ((t + color) & 1) + t * Lx;
    active = t < Lt;
  } else {
    s = k;
    active = (s < V) && ((((s % Lx) + (s / Lx)) & 1) == color);
  }
  if (!active) s = 0;
  const int row = lane & 15, kq = lane >> 4;
  const int rhs = tile * 16 + row;
  const bool rv = active && rhs < nrhs;
  const int64_t ld = V * 16;
  const Nbr nb = neighbours(s, Lx, Lt);
  const int64_t sites[5] = {s, nb.xp, nb.xm, nb.tp, nb.tm};
  stage_x_tiles(x, ld, sites, tile * 16, nrhs, active, Xs[w]);
  __syncthreads();
  f32x4 dre = {0.f, 0.f, 0.f, 0.f}, dim = {0.f, 0.f, 0.f, 0.f};
  site_product16(A, s, Xs[w], row, kq, dre, dim);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 4 * kq + v;
    const c64 bb = rv ? b[(int64_t)rhs * ld + s * 16 + i] : cmk(0.f, 0.f);
    Rl[w][row][i] = cmk(bb.x - dre[v], bb.y - dim[v]);
  }
  __syncthreads();
  f32x4 ere = {0.f, 0.f, 0.f, 0.f}, eim = {0.f, 0.f, 0.f, 0.f};
  const c64* Ai = Ainv + s * 256;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int j = 4 * t + kq;
    cmfma(ere, eim, Ai[j * 16 + row], Rl[w][row][j]);
  }
  if (!rv) return;
  c64* xo = x + (int64_t)rhs * ld + s * 16;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 4 * kq + v;
    const c64 o = Xs[w][0][row][i];  // x_s before the update (staged above)
    xo[i] = cmk(o.x + ere[v], o.y + eim[v]);
  }
}

inline int rhs_block_for(int64_t threads, int nrhs) {
  // enough workgroups to fill 256 CUs several times; otherwise split the RHS over y
  const int64_t wgs = ceil_div(threads, 256);
  if (wgs >= 4096) return nrhs;
  int rb = (int)std::max<int64_t>(1, (int64_t)nrhs * wgs / 4096);
  return std::min(rb, nrhs);
}

}  // namespace

template <typename R>
void launch_wilson(dmlmc_ctx* ctx, const Level& L, const Cx<R>* x, Cx<R>* y, int nrhs, int64_t ldx, int64_t ldy,
                   bool gamma5_left) {
  const int64_t V = L.sites();
  const int rb = rhs_block_for(V, nrhs);
  dim3 grid((unsigned)ceil_div(V, 256), (unsigned)ceil_div(nrhs, rb));
  const Cx<R>* U = std::is_same<R, float>::value ? (const Cx<R>*)L.U32.p : (const Cx<R>*)L.U64.p;
  KTimer kt(ctx, "wilson", (double)nrhs * V * 4 * sizeof(Cx<R>) + (double)V * 2 * sizeof(Cx<R>));
  if (gamma5_left)
    hipLaunchKernelGGL((wilson_kernel<R, true>), grid, dim3(256), 0, ctx->stream, U, x, y, L.Lx, L.Lt,
                       (R)(L.m0 + 2.0), nrhs, rb, ldx, ldy);
  else
    hipLaunchKernelGGL((wilson_kernel<R, false>), grid, dim3(256), 0, ctx->stream, U, x, y, L.Lx, L.Lt,
                       (R)(L.m0 + 2.0), nrhs, rb, ldx, ldy);
  LAUNCH_CHECK();
}

template <typename R>
void launch_coarse(dmlmc_ctx* ctx, const Level& L, const Cx<R>* x, Cx<R>* y, int nrhs, int64_t ldx, int64_t ldy,
                   bool gamma5_left) {
  const int d = L.dofs;
  const int spb = std::max(1, 256 / d);
  const int64_t V = L.sites();
  const Cx<R>* A = std::is_same<R, float>::value ? (const Cx<R>*)L.A32.p : (const Cx<R>*)L.A64.p;
  KTimer kt(ctx, "coarse",
            (double)nrhs * L.n() * 2 * sizeof(Cx<R>) + (double)V * 5 * d * d * sizeof(Cx<R>));
  if (std::is_same<R, float>::value && d == 16) {
    const int64_t waves = V * ((nrhs + 15) / 16);
    dim3 grid((unsigned)ceil_div(waves, 4));
    if (gamma5_left)
      hipLaunchKernelGGL((coarse16_mfma_kernel<true>), grid, dim3(256), 0, ctx->stream, (const c64*)A, (const c64*)x,
                         (c64*)y, L.Lx, L.Lt, nrhs, ldx, ldy);
    else
      hipLaunchKernelGGL((coarse16_mfma_kernel<false>), grid, dim3(256), 0, ctx->stream, (const c64*)A, (const c64*)x,
                         (c64*)y, L.Lx, L.Lt, nrhs, ldx, ldy);
    LAUNCH_CHECK();
    return;
  }
  constexpr int RB = 4;
  dim3 grid((unsigned)ceil_div(V, spb), (unsigned)ceil_div(nrhs, RB));
  dim3 block((unsigned)(spb * d));
  if (gamma5_left)
    hipLaunchKernelGGL((coarse_kernel<R, RB, true>), grid, block, 0, ctx->stream, A, x, y, L.Lx, L.Lt, d, spb, nrhs,
                       ldx, ldy);
  else
    hipLaunchKernelGGL((coarse_kernel<R, RB, false>), grid, block, 0, ctx->stream, A, x, y, L.Lx, L.Lt, d, spb,
                       nrhs, ldx, ldy);
  LAUNCH_CHECK();
}

template <typename R>
void apply_op(dmlmc_ctx* ctx, const Level& L, const Cx<R>* x, Cx<R>* y, int nrhs, bool gamma5_left) {
  if (L.fine)
    launch_wilson<R>(ctx, L, x, y, nrhs, L.n(), L.n(), gamma5_left);
  else
    launch_coarse<R>(ctx, L, x, y, nrhs, L.n(), L.n(), gamma5_left);
}

template <typename R>
void launch_sap(dmlmc_ctx* ctx, const Level& L, Cx<R>* x, const Cx<R>* b, int nrhs, int color, int mr_iters) {
  const Cx<R>* U = std::is_same<R, float>::value ? (const Cx<R>*)L.U32.p : (const Cx<R>*)L.U64.p;
  const int64_t V = L.sites();
  const int rb = rhs_block_for(V, nrhs);
  KTimer kt(ctx, "sap", (double)nrhs * V * 2 * sizeof(Cx<R>) * 2.5 + (double)V * sizeof(Cx<R>));
  // 4x4 blocks when the block checkerboard has even extents (no two neighbouring blocks
  // share a colour, also across the periodic boundary), else 2x2 blocks (the fine extents
  // are multiples of 4, so 2x2 block counts are even).
  if (L.Lx % 8 == 0 && L.Lt % 8 == 0) {
    const int nblk = (L.Lx / 4) * (L.Lt / 4);
    dim3 grid((unsigned)ceil_div(nblk, 16), (unsigned)ceil_div(nrhs, rb));
    hipLaunchKernelGGL((sap_kernel<R, 4, 4>), grid, dim3(256), 0, ctx->stream, U, x, b, L.Lx, L.Lt,
                       (R)(L.m0 + 2.0), nrhs, rb, color, mr_iters);
  } else {
    const int nblk = (L.Lx / 2) * (L.Lt / 2);
    dim3 grid((unsigned)ceil_div(nblk, 64), (unsigned)ceil_div(nrhs, rb));
    hipLaunchKernelGGL((sap_kernel<R, 2, 2>), grid, dim3(256), 0, ctx->stream, U, x, b, L.Lx, L.Lt,
                       (R)(L.m0 + 2.0), nrhs, rb, color, mr_iters);
  }
  LAUNCH_CHECK();
}

template <typename R>
void launch_coarse_gs(dmlmc_ctx* ctx, const Level& L, Cx<R>* x, const Cx<R>* b, int nrhs, int color) {
  const int d = L.dofs;
  const int spb = std::max(1, 256 / d);
  const int64_t V = L.sites();
  const Cx<R>* A = std::is_same<R, float>::value ? (const Cx<R>*)L.A32.p : (const Cx<R>*)L.A64.p;
  const Cx<R>* Ai = std::is_same<R, float>::value ? (const Cx<R>*)L.Ainv32.p : (const Cx<R>*)L.Ainv64.p;
  const int even = (L.Lx % 2 == 0) ? 1 : 0;
  const int64_t nsites = even ? V / 2 : V;
  const int rb = rhs_block_for(nsites * d, nrhs);
  KTimer kt(ctx, "coarse_gs",
            (double)nrhs * (V / 2) * d * 4 * sizeof(Cx<R>) + (double)(V / 2) * 6 * d * d * sizeof(Cx<R>));
  if (std::is_same<R, float>::value && d == 16) {
    const int64_t waves = nsites * ((nrhs + 15) / 16);
    hipLaunchKernelGGL(coarse16_gs_mfma_kernel, dim3((unsigned)ceil_div(waves, 4)), dim3(256), 0, ctx->stream,
                       (const c64*)A, (const c64*)Ai, (c64*)x, (const c64*)b, L.Lx, L.Lt, nrhs, color, even);
    LAUNCH_CHECK();
    return;
  }
  dim3 grid((unsigned)ceil_div(nsites, spb), (unsigned)ceil_div(nrhs, rb));
  dim3 block((unsigned)(spb * d));
  size_t shm = (size_t)spb * d * sizeof(Cx<R>);
  hipLaunchKernelGGL((coarse_gs_kernel<R>), grid, block, shm, ctx->stream, A, Ai, x, b, L.Lx, L.Lt, d, spb, nrhs,
                     rb, color, even);
  LAUNCH_CHECK();
}

template <typename R>
void launch_restrict(dmlmc_ctx* ctx, const Level& L, const Cx<R>* xf, Cx<R>* yc, int nrhs) {
  const Cx<R>* P = std::is_same<R, float>::value ? (const Cx<R>*)L.P32.p : (const Cx<R>*)L.P64.p;
  const int64_t Vc = (int64_t)(L.Lx / L.ax) * (L.Lt / L.at);
  const int64_t threads = Vc * 2 * L.N;
  KTimer kt(ctx, "restrict",
            (double)nrhs * (L.n() + threads) * sizeof(Cx<R>) + (double)L.n() * L.N * sizeof(Cx<R>));
  constexpr int RB = 4;
  dim3 grid((unsigned)ceil_div(threads, 256), (unsigned)ceil_div(nrhs, RB));
  hipLaunchKernelGGL((restrict_kernel<R, RB>), grid, dim3(256), 0, ctx->stream, P, xf, yc, L.Lx, L.Lt, L.dofs, L.ax,
                     L.at, L.N, nrhs);
  LAUNCH_CHECK();
}

template <typename R>
void launch_prolong(dmlmc_ctx* ctx, const Level& L, const Cx<R>* ec, Cx<R>* xf, int nrhs, bool add) {
  const Cx<R>* P = std::is_same<R, float>::value ? (const Cx<R>*)L.P32.p : (const Cx<R>*)L.P64.p;
  const int64_t nf = L.n();
  const int64_t nc = (int64_t)(L.Lx / L.ax) * (L.Lt / L.at) * 2 * L.N;
  KTimer kt(ctx, "prolong",
            (double)nrhs * ((add ? 2 : 1) * nf + nc) * sizeof(Cx<R>) + (double)nf * L.N * sizeof(Cx<R>));
  constexpr int RB = 4;
  dim3 grid((unsigned)ceil_div(nf, 256), (unsigned)ceil_div(nrhs, RB));
  hipLaunchKernelGGL((prolong_kernel<R, RB>), grid, dim3(256), 0, ctx->stream, P, ec, xf, L.Lx, L.Lt, L.dofs, L.ax,
                     L.at, L.N, nrhs, add ? 1 : 0);
  LAUNCH_CHECK();
}

#define INST(R)                                                                                                  \
  template void launch_wilson<R>(dmlmc_ctx*, const Level&, const Cx<R>*, Cx<R>*, int, int64_t, int64_t, bool); \
  template void launch_coarse<R>(dmlmc_ctx*, const Level&, const Cx<R>*, Cx<R>*, int, int64_t, int64_t, bool); \
  template void apply_op<R>(dmlmc_ctx*, const Level&, const Cx<R>*, Cx<R>*, int, bool);                        \
  template void launch_sap<R>(dmlmc_ctx*, const Level&, Cx<R>*, const Cx<R>*, int, int, int);                  \
  template void launch_coarse_gs<R>(dmlmc_ctx*, const Level&, Cx<R>*, const Cx<R>*, int, int);                 \
  template void launch_restrict<R>(dmlmc_ctx*, const Level&, const Cx<R>*, Cx<R>*, int);                       \
  template void launch_prolong<R>(dmlmc_ctx*, const Level&, const Cx<R>*, Cx<R>*, int, bool);
INST(float)
INST(double)
