// Level operators of the multigrid hierarchy on gfx950:
//   * fine Wilson-Schwinger stencil (spin-projected hops, links folded with the
//     antiperiodic sign), multi-RHS;
//   * coarse nearest-neighbour block stencil (dense d x d blocks, column-major);
//   * SAP smoother on 8x4, 4x4 or 2x2 site blocks with local minimal-residual iterations,
//     red/black over blocks, residual b - D x fused in;
//   * red/black point-block Gauss-Seidel on coarse levels (exact inverse self blocks);
//   * restriction P^H and prolongation P on (aggregate, chirality) blocks.
// Vectors are RHS-major: entry i of RHS r is at r * ld + i; complex interleaved.
#include "common.h"
#include "tune.h"

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

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).  This
// renumbering hands every XCD a contiguous range of logical workgroups, so neighbouring
// sites (the stencils' re-reads) are fetched through the same L2.  It is a bijection on
// [0, gridDim.x): the largest multiple of 8 is permuted, the tail keeps its numbers.
__device__ __forceinline__ int64_t xcd_block() {
  const int64_t g = blockIdx.x, n = gridDim.x;
  const int64_t full = n & ~(int64_t)7;
  if (g >= full) return g;
  return (g & 7) * (full >> 3) + (g >> 3);
}

// Thread per site, RHS [r0, r1) in sequence; the five spinors of RHS r + 1 are requested
// before RHS r is computed, so a thread always has a full set of loads in flight.
template <typename R, bool G5, typename RO = R>
__global__ __launch_bounds__(256) void wilson_kernel(const Cx<R>* __restrict__ U, const Cx<R>* __restrict__ in,
                                                     Cx<RO>* __restrict__ out, int Lx, int Lt, R diag, int nrhs,
                                                     int rb, int64_t ldx, int64_t ldy,
                                                     const Cx<R>* __restrict__ sub) {
  const int64_t V = (int64_t)Lx * Lt;
  const int64_t s = xcd_block() * blockDim.x + threadIdx.x;
  if (s >= V) return;
  const Nbr nb = neighbours(s, Lx, Lt);
  const Cx<R> ux = U[s], ut = U[V + s], uxm = U[nb.xm], utm = U[V + nb.tm];
  const int r0 = blockIdx.y * rb;
  const int r1 = min(r0 + rb, nrhs);
  const R half = (R)0.5;
  Spinor<R> c, fx, bx, ft, bt;
  {
    const Spinor<R>* p = reinterpret_cast<const Spinor<R>*>(in + r0 * ldx);
    c = p[s];
    fx = p[nb.xp];
    bx = p[nb.xm];
    ft = p[nb.tp];
    bt = p[nb.tm];
  }
  for (int r = r0; r < r1; ++r) {
    const Spinor<R> c0 = c, fx0 = fx, bx0 = bx, ft0 = ft, bt0 = bt;
    if (r + 1 < r1) {
      const Spinor<R>* p = reinterpret_cast<const Spinor<R>*>(in + (r + 1) * ldx);
      c = p[s];
      fx = p[nb.xp];
      bx = p[nb.xm];
      ft = p[nb.tp];
      bt = p[nb.tm];
    }
    __builtin_amdgcn_sched_barrier(0);  // the next RHS's loads go out before this one's arithmetic
    Cx<R> a0, a1;
    hops(ux, uxm, ut, utm, fx0, bx0, ft0, bt0, a0, a1);
    Spinor<R> o;
    o.s0 = diag * c0.s0 - half * a0;
    o.s1 = diag * c0.s1 - half * a1;
    if (G5) o.s1 = cmk(-o.s1.x, -o.s1.y);
    if (sub) {  // residual form: out = sub - D in (sub laid out as in)
      const Spinor<R> bb = reinterpret_cast<const Spinor<R>*>(sub + r * ldx)[s];
      o.s0 = bb.s0 - o.s0;
      o.s1 = bb.s1 - o.s1;
    }
    // the result is not re-read by this launch: non-temporal store (rounded to RO)
    RO* of = reinterpret_cast<RO*>(out + r * ldy + 2 * s);
    __builtin_nontemporal_store((RO)o.s0.x, of);
    __builtin_nontemporal_store((RO)o.s0.y, of + 1);
    __builtin_nontemporal_store((RO)o.s1.x, of + 2);
    __builtin_nontemporal_store((RO)o.s1.y, of + 3);
  }
}

// Coarse block stencil: y_s = sum_dir A[s][dir] x_{s+dir}; blocks column-major
// (A[s][dir][j * d + i] = row i, column j).  Thread per (site, row), RB right-hand sides
// per thread so that every block entry is loaded once per RB vectors.
template <typename R, int RB, bool G5, typename RO = R>
__global__ __launch_bounds__(256) void coarse_kernel(const Cx<R>* __restrict__ A, const Cx<R>* __restrict__ in,
                                                     Cx<RO>* __restrict__ out, int Lx, int Lt, int d, int spb,
                                                     int nrhs, int64_t ldx, int64_t ldy,
                                                     const Cx<R>* __restrict__ sub) {
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
    if (q < nr) {
      const Cx<R> v = neg ? cmk(-acc[q].x, -acc[q].y) : acc[q];
      out[(r0 + q) * ldy + s * d + i] = ccast<RO>(sub ? sub[(r0 + q) * ldx + s * d + i] - v : v);
    }
  }
}

// SAP on BSX x BST site blocks (lanes of one block are contiguous within a wavefront).
// For every block of colour `color`: r_B = b_B - (D x)_B, then `mr` minimal-residual
// iterations on the block-restricted operator D_BB (zero outside the block) from e = 0,
// then x_B += e.
template <typename R, int BSX, int BST>
__global__ __launch_bounds__(256) void sap_kernel(const Cx<R>* __restrict__ U, Cx<R>* __restrict__ x,
                                                  const Cx<R>* __restrict__ b, int Lx, int Lt, R diag, int nrhs,
                                                  int rb, int color, int mr, int64_t ld) {
  constexpr int BL = BSX * BST;  // lanes per block
  const int64_t V = (int64_t)Lx * Lt;
  const int nbx = Lx / BSX, nbt = Lt / BST;  // nbx even: blocks of one colour are every other block of a row
  const int lane = threadIdx.x % BL;
  const int64_t k = xcd_block() * (blockDim.x / BL) + threadIdx.x / BL;  // k-th block of colour `color`
  const int64_t BTi = k / (nbx / 2);
  const int64_t BXi = 2 * (k % (nbx / 2)) + ((BTi + color) & 1);
  const bool active = BTi < nbt;  // uniform over the block's lanes
  const int lx = lane % BSX, lt = lane / BSX;
  const int64_t s = active ? (BXi * BSX + lx) + (int64_t)Lx * (BTi * BST + lt) : 0;
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
  const int wl = (threadIdx.x & 63);  // lane within wavefront
  const int wbase = wl - lane;        // first lane of my block within the wavefront
  const int src_xp = wbase + (hxp ? lane + 1 : lane), src_xm = wbase + (hxm ? lane - 1 : lane);
  const int src_tp = wbase + (htp ? lane + BSX : lane), src_tm = wbase + (htm ? lane - BSX : lane);
  // links of the block-restricted operator: zero on the hops that leave the block
  const Cx<R> zc = cmk((R)0, (R)0);
  const Cx<R> uxb = hxp ? ux : zc, uxmb = hxm ? uxm : zc, utb = htp ? ut : zc, utmb = htm ? utm : zc;
  const R half = (R)0.5;
  const int r0 = blockIdx.y * rb;
  const int r1 = min(r0 + rb, nrhs);
  // x at the site and its four neighbours and b of RHS r + 1 are requested before RHS r
  // is worked on (inactive lanes read site 0 and discard it)
  Spinor<R> xc, fx, bx, ft, bt, bb;
  {
    const Spinor<R>* xp = reinterpret_cast<const Spinor<R>*>(x + r0 * ld);
    xc = xp[s];
    fx = xp[nb.xp];
    bx = xp[nb.xm];
    ft = xp[nb.tp];
    bt = xp[nb.tm];
    bb = reinterpret_cast<const Spinor<R>*>(b + r0 * ld)[s];
  }
  for (int r = r0; r < r1; ++r) {
    const Spinor<R> xc0 = xc, fx0 = fx, bx0 = bx, ft0 = ft, bt0 = bt, bb0 = bb;
    if (r + 1 < r1) {
      const Spinor<R>* xp = reinterpret_cast<const Spinor<R>*>(x + (r + 1) * ld);
      xc = xp[s];
      fx = xp[nb.xp];
      bx = xp[nb.xm];
      ft = xp[nb.tp];
      bt = xp[nb.tm];
      bb = reinterpret_cast<const Spinor<R>*>(b + (r + 1) * ld)[s];
    }
    __builtin_amdgcn_sched_barrier(0);
    Spinor<R> rho;
    {
      Cx<R> a0, a1;
      hops(ux, uxm, ut, utm, fx0, bx0, ft0, bt0, a0, a1);
      rho.s0 = bb0.s0 - (diag * xc0.s0 - half * a0);
      rho.s1 = bb0.s1 - (diag * xc0.s1 - half * a1);
    }
    Spinor<R> e;
    e.s0 = e.s1 = cmk((R)0, (R)0);
    for (int it = 0; it < mr; ++it) {
      // q = D_BB rho, neighbours from lanes of the same block: each lane forms the spin
      // projections the four hops onto its site need and the neighbours take them (two
      // values per hop instead of the whole spinor); the hops that leave the block use the
      // zeroed links
      const Cx<R> pxf = rho.s0 - rho.s1, pxb = rho.s0 + rho.s1;
      const Cx<R> ptf = rho.s0 + mul_i(rho.s1), ptb = rho.s0 + mul_mi(rho.s1);
      const Cx<R> fxp = cmk(__shfl(pxf.x, src_xp, 64), __shfl(pxf.y, src_xp, 64));
      const Cx<R> bxp = cmk(__shfl(pxb.x, src_xm, 64), __shfl(pxb.y, src_xm, 64));
      const Cx<R> ftp = cmk(__shfl(ptf.x, src_tp, 64), __shfl(ptf.y, src_tp, 64));
      const Cx<R> btp = cmk(__shfl(ptb.x, src_tm, 64), __shfl(ptb.y, src_tm, 64));
      Cx<R> a0, a1;
      {
        Cx<R> h = uxb * fxp;
        a0 = h;
        a1 = cmk(-h.x, -h.y);
        Cx<R> g = conj(uxmb) * bxp;
        a0 = a0 + g;
        a1 = a1 + g;
        h = utb * ftp;
        a0 = a0 + h;
        a1 = a1 + mul_mi(h);
        g = conj(utmb) * btp;
        a0 = a0 + g;
        a1 = a1 + mul_i(g);
      }
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
      Spinor<R> xo;
      xo.s0 = xc0.s0 + e.s0;
      xo.s1 = xc0.s1 + e.s1;
      reinterpret_cast<Spinor<R>*>(x + r * ld)[s] = xo;
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
                                                        int even_lx, int64_t ld) {
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
                                                       int at, int N, int nrhs, int64_t ldf, int64_t ldc) {
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
                                                      int N, int nrhs, int add, int64_t ldf, int64_t ldc) {
  const int64_t nf = (int64_t)Lxf * Ltf * df;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= nf) return;
  const int dof = (int)(tid % df);
  const int64_t site = tid / df;
  const int x = (int)(site % Lxf), t = (int)(site / Lxf);
  const int Lxc = Lxf / ax;
  const int64_t cs = (int64_t)(x / ax) + (int64_t)Lxc * (t / at);
  const int h = df / 2;
  const int c = dof / h, j = dof % h;
  const int row = ((x % ax) + ax * (t % at)) * h + j;
  const int rows = ax * at * h;
  const Cx<R>* Pr = P + ((cs * 2 + c) * (int64_t)rows + row) * N;
  const int r0 = blockIdx.y * RB;
  const int nr = min(RB, nrhs - r0);
  const Cx<R>* er = ec + (int64_t)r0 * ldc + cs * 2 * N + c * N;
  Cx<R> acc[RB];
#pragma unroll
  for (int q = 0; q < RB; ++q)
    acc[q] = (add && q < nr) ? xf[(int64_t)(r0 + q) * ldf + tid] : cmk((R)0, (R)0);
  for (int kk = 0; kk < N; ++kk) {
    const Cx<R> pv = Pr[kk];
#pragma unroll
    for (int q = 0; q < RB; ++q)
      if (q < nr) cfma(acc[q], pv, er[q * ldc + kk]);
  }
#pragma unroll
  for (int q = 0; q < RB; ++q)
    if (q < nr) xf[(int64_t)(r0 + q) * ldf + tid] = acc[q];
}

// ---------------------------------------------------------------- matrix-core forms (d = 16, complex FP32)
// One wavefront computes 16 (dofs) x 16 (RHS) tiles of one site with v_mfma_f32_16x16x4_f32:
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and receives D[4 (l / 16) + v][l % 16].
// A complex product A X takes four real products (re: Ar Xr - Ai Xi, im: Ar Xi + Ai Xr).
//
// The contraction over the 16 input dofs is split into four K = 4 steps; step t gives the
// k-th operand slot to dof j = 4k + t.  Lane (row, kq) = (l % 16, l / 16) therefore needs
// A[row][4kq .. 4kq+3] (32 contiguous bytes of a row-major block) and x[rhs row][4kq .. 4kq+3]
// (32 contiguous bytes of a vector), and the D fragment it receives (dofs 4kq .. 4kq+3 of
// RHS row) is already in the B-operand layout of a following product.  Every operand is
// read from global memory with two 16-byte loads per lane; nothing passes through LDS.
// FP32 blocks at d = 16 are stored row-major for this reason (see Level).
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void cmfma(f32x4& dre, f32x4& dim, c64 a, c64 x) {
  dre = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, x.x, dre, 0, 0, 0);
  dre = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.y, x.y, dre, 0, 0, 0);
  dim = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, x.y, dim, 0, 0, 0);
  dim = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, x.x, dim, 0, 0, 0);
}

struct __align__(16) C64Pair {
  c64 a, b;
};

// The fine stencil of a complex-FP32 Arnoldi step fused with the dots of its single-pass
// Gram-Schmidt: y = D z as wilson_kernel computes it (complex FP32, stored rounded to
// complex FP32), and for every RHS r the FP64 dots <u_i, s_r y> (i < nb, s_r = wscale[r],
// the same terms as gs1_dots_kernel) summed over the block's sites, written as block
// partials part[(r G + block) 2 nb + 2 i + (0: re, 1: im)] with G = gridDim.x, so that the
// dots pass need not read y again.  SPT sites per thread (blocks of 256 SPT sites, the
// thread's sites 256 apart); threads beyond the lattice add zeros (no early return: the
// block sums have barriers).
template <int NBT, int SPT>
__global__ __launch_bounds__(256) void wilson_dots_kernel(const c64* __restrict__ U, const c64* __restrict__ in,
                                                          c64* __restrict__ out, int Lx, int Lt, float diag, int nrhs,
                                                          int rb, int64_t ld, const c64* __restrict__ Ub, int nb,
                                                          int64_t vs, const double* __restrict__ wscale,
                                                          double* __restrict__ part) {
  __shared__ double red[4][2 * NBT];
  const int64_t V = (int64_t)Lx * Lt;
  const int64_t blk = xcd_block();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t st[SPT];
  bool act[SPT];
  Nbr nbr[SPT];
  c64 ux[SPT], ut[SPT], uxm[SPT], utm[SPT];
#pragma unroll
  for (int q = 0; q < SPT; ++q) {
    const int64_t sr = (blk * SPT + q) * 256 + threadIdx.x;
    act[q] = sr < V;
    st[q] = act[q] ? sr : 0;
    nbr[q] = neighbours(st[q], Lx, Lt);
    ux[q] = U[st[q]];
    ut[q] = U[V + st[q]];
    uxm[q] = U[nbr[q].xm];
    utm[q] = U[V + nbr[q].tm];
  }
  const int r0 = blockIdx.y * rb;
  const int r1 = min(r0 + rb, nrhs);
  const float half = 0.5f;
  for (int r = r0; r < r1; ++r) {
    const Spinor<float>* p = reinterpret_cast<const Spinor<float>*>(in + r * ld);
    const C64Pair* ur = reinterpret_cast<const C64Pair*>(Ub + r * ld);
    Spinor<float> c[SPT], fx[SPT], bx[SPT], ft[SPT], bt[SPT];
    C64Pair u[SPT][NBT];
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      c[q] = p[st[q]];
      fx[q] = p[nbr[q].xp];
      bx[q] = p[nbr[q].xm];
      ft[q] = p[nbr[q].tp];
      bt[q] = p[nbr[q].tm];
#pragma unroll
      for (int i = 0; i < NBT; ++i)
        if (i < nb) u[q][i] = ur[(int64_t)i * (vs / 2) + st[q]];
    }
    const double ws = wscale[r];
    double acc[2 * NBT];
#pragma unroll
    for (int i = 0; i < 2 * NBT; ++i) acc[i] = 0.0;
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      Cx<float> a0, a1;
      hops(ux[q], uxm[q], ut[q], utm[q], fx[q], bx[q], ft[q], bt[q], a0, a1);
      Spinor<float> o;
      o.s0 = diag * c[q].s0 - half * a0;
      o.s1 = diag * c[q].s1 - half * a1;
      if (act[q]) {
        float* of = reinterpret_cast<float*>(out + r * ld + 2 * st[q]);
        __builtin_nontemporal_store(o.s0.x, of);
        __builtin_nontemporal_store(o.s0.y, of + 1);
        __builtin_nontemporal_store(o.s1.x, of + 2);
        __builtin_nontemporal_store(o.s1.y, of + 3);
        const double b0x = ws * o.s0.x, b0y = ws * o.s0.y, b1x = ws * o.s1.x, b1y = ws * o.s1.y;
#pragma unroll
        for (int i = 0; i < NBT; ++i) {
          if (i < nb) {
            const C64Pair v = u[q][i];
            acc[2 * i] += (double)v.a.x * b0x + (double)v.a.y * b0y + (double)v.b.x * b1x + (double)v.b.y * b1y;
            acc[2 * i + 1] += (double)v.a.x * b0y - (double)v.a.y * b0x + (double)v.b.x * b1y - (double)v.b.y * b1x;
          }
        }
      }
    }
    const int nv = 2 * nb;
#pragma unroll
    for (int i = 0; i < 2 * NBT; ++i) {
      if (i < nv) {
        double v = acc[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[w][i] = v;
      }
    }
    __syncthreads();
    if (threadIdx.x < nv)
      part[((int64_t)r * gridDim.x + blk) * nv + threadIdx.x] =
          red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
    __syncthreads();
  }
}


struct Quad {
  c64 v[4];
};

// Interpolation blocks (and the Gauss-Seidel blocks) are streamed once per launch:
// non-temporal loads keep them from displacing the vectors' neighbour re-reads in the
// caches.  (The coarse stencil reads its blocks with ordinary loads: non-temporal ones
// made its level-2 launch slower, 288 -> 320 us at 1024^2, measured.)  Two 16-byte loads;
// p is 16-byte aligned.
__device__ __forceinline__ Quad load_quad_nt(const c64* __restrict__ p) {
  const f32x4* q = reinterpret_cast<const f32x4*>(p);
  const f32x4 u = __builtin_nontemporal_load(q), w = __builtin_nontemporal_load(q + 1);
  Quad r;
  r.v[0] = cmk(u[0], u[1]);
  r.v[1] = cmk(u[2], u[3]);
  r.v[2] = cmk(w[0], w[1]);
  r.v[3] = cmk(w[2], w[3]);
  return r;
}

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

__device__ __forceinline__ void store_quad(c64* __restrict__ p, f32x4 re, f32x4 im, float sg) {
  C64Pair* q = reinterpret_cast<C64Pair*>(p);
  C64Pair u, w;
  u.a = cmk(sg * re[0], sg * im[0]);
  u.b = cmk(sg * re[1], sg * im[1]);
  w.a = cmk(sg * re[2], sg * im[2]);
  w.b = cmk(sg * re[3], sg * im[3]);
  q[0] = u;
  q[1] = w;
}

// D += A X for one 16 x 16 block (a: lane's A row quarter, x: lane's B quarter).
__device__ __forceinline__ void block_mfma(f32x4& dre, f32x4& dim, const Quad& a, const Quad& x) {
#pragma unroll
  for (int t = 0; t < 4; ++t) cmfma(dre, dim, a.v[t], x.v[t]);
}


__device__ __forceinline__ Quad select_quad(bool keep, const Quad& q) {
  Quad r;
#pragma unroll
  for (int v = 0; v < 4; ++v) r.v[v] = keep ? q.v[v] : cmk(0.f, 0.f);
  return r;
}

// LDS position of 16-byte chunk c (0..7) of staged line L: lines of 8 chunks, unpadded, with
// the chunk index XOR-swizzled by the line, so that the column reads and writes of the
// matrix-core layout (one chunk of each of 8 or 16 consecutive lines) and the row accesses
// of the whole-line loads and stores (the 8 chunks of a line) both fall on distinct banks
__device__ __forceinline__ int sw(int L, int c) { return L * 8 + (c ^ ((L ^ (L >> 3)) & 7)); }

// The 16 RHS rows r0 .. r0+15 (clamped to nrhs - 1) of the 16 complex entries at entry
// offset `off` of v, read with whole-line loads: each of a lane's two 16-byte loads belongs
// to a group of 8 lanes covering one 128-byte line (RHS l / 8 and 8 + l / 8, piece l % 8),
// so each load instruction touches 8 lines instead of 16 half lines.  The two pieces go to
// the wavefront's LDS rows at their swizzled positions (sw); LDS operations of one
// wavefront complete in order.
__device__ __forceinline__ void stage_rows(const c64* __restrict__ v, int64_t ld, int r0, int nrhs, int64_t off,
                                           int lane, float4* __restrict__ rows) {
  const int rr = lane >> 3, pc = lane & 7;
  const int ra = min(r0 + rr, nrhs - 1), rb = min(r0 + 8 + rr, nrhs - 1);
  const float4 A = *reinterpret_cast<const float4*>(v + (int64_t)ra * ld + off + 2 * pc);
  const float4 B = *reinterpret_cast<const float4*>(v + (int64_t)rb * ld + off + 2 * pc);
  rows[sw(rr, pc)] = A;
  rows[sw(8 + rr, pc)] = B;
}

// the 16 rows of a 16 x 16 block (streamed once per launch: non-temporal loads), staged
// as stage_rows does
__device__ __forceinline__ void stage_rows_nt(const c64* __restrict__ A, int lane, float4* __restrict__ rows) {
  const int rr = lane >> 3, pc = lane & 7;
  const f32x4 u = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(A + rr * 16 + 2 * pc));
  const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(A + (8 + rr) * 16 + 2 * pc));
  rows[sw(rr, pc)] = make_float4(u[0], u[1], u[2], u[3]);
  rows[sw(8 + rr, pc)] = make_float4(v[0], v[1], v[2], v[3]);
}

// the quad of lane (row, kq) from staged rows: entries 4 kq .. 4 kq + 3 of RHS row
__device__ __forceinline__ Quad staged_quad(const float4* __restrict__ rows, int lane) {
  const int row = lane & 15, kq = lane >> 4;
  const float4 u = rows[sw(row, 2 * kq)], w = rows[sw(row, 2 * kq + 1)];
  Quad q;
  q.v[0] = cmk(u.x, u.y);
  q.v[1] = cmk(u.z, u.w);
  q.v[2] = cmk(w.x, w.y);
  q.v[3] = cmk(w.z, w.w);
  return q;
}

// y_s = sum_dir A[s][dir] x_{s+dir} (optionally Gamma5 y).  SPLIT = 1: one site per
// wavefront, all RHS in pairs of 16-wide tiles; SPLIT = 2: two wavefronts per site (the
// same workgroup), each taking every other 16-wide tile; SPLIT = 3: one site per
// wavefront, one tile at a time, the blocks and vectors read and the result written by
// whole 128-byte lines staged through LDS (10 KB per wavefront).  Every load of a pass
// is issued before the first product (rows beyond nrhs load a valid row and are zeroed),
// so the wavefront has all its memory requests in flight at once.  Each output tile is the
// same sequence of products in every form.
template <bool G5, int SPLIT>
__global__ __launch_bounds__(256) void coarse16_mfma_kernel(const c64* __restrict__ A, const c64* __restrict__ in,
                                                            c64* __restrict__ out, int Lx, int Lt, int nrhs,
                                                            int64_t ldx, int64_t ldy) {
  const int64_t V = (int64_t)Lx * Lt;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t wv = xcd_block() * 4 + w;
  const int64_t s = wv / (SPLIT == 2 ? 2 : 1);  // SPLIT = 2: two wavefronts per site
  if (s >= V) return;  // wave-uniform: the MFMAs below always run with a full wavefront
  const int row = lane & 15, kq = lane >> 4;
  const Nbr nb = neighbours(s, Lx, Lt);
  const int64_t sites[5] = {s, nb.xp, nb.xm, nb.tp, nb.tm};
  const float sg = (G5 && kq >= 2) ? -1.f : 1.f;
  if constexpr (SPLIT == 3) {
    __shared__ float4 stage[4][5][16 * 8];
    float4(*rows)[16 * 8] = stage[w];
    // a block is 16 rows of 16 complex entries, like 16 RHS rows of a site
    Quad a[5];
#pragma unroll
    for (int dir = 0; dir < 5; ++dir) stage_rows_nt(A + (s * 5 + dir) * 256, lane, rows[dir]);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int dir = 0; dir < 5; ++dir) a[dir] = staged_quad(rows[dir], lane);
    __builtin_amdgcn_wave_barrier();
    for (int r0 = 0; r0 < nrhs; r0 += 16) {
      const int ra = r0 + row;
      const bool va = ra < nrhs;
#pragma unroll
      for (int dir = 0; dir < 5; ++dir) stage_rows(in, ldx, r0, nrhs, sites[dir] * 16, lane, rows[dir]);
      __builtin_amdgcn_wave_barrier();
      Quad xa[5];
#pragma unroll
      for (int dir = 0; dir < 5; ++dir) xa[dir] = staged_quad(rows[dir], lane);
      f32x4 are = {0.f, 0.f, 0.f, 0.f}, aim = are;
#pragma unroll
      for (int dir = 0; dir < 5; ++dir) block_mfma(are, aim, a[dir], select_quad(va, xa[dir]));
      __builtin_amdgcn_wave_barrier();
      float4* o = rows[0];
      o[sw(row, 2 * kq)] = make_float4(sg * are[0], sg * aim[0], sg * are[1], sg * aim[1]);
      o[sw(row, 2 * kq + 1)] = make_float4(sg * are[2], sg * aim[2], sg * are[3], sg * aim[3]);
      __builtin_amdgcn_wave_barrier();
      const int rr = lane >> 3, pc = lane & 7;
      if (r0 + rr < nrhs) *reinterpret_cast<float4*>(out + (int64_t)(r0 + rr) * ldy + s * 16 + 2 * pc) = o[sw(rr, pc)];
      if (r0 + 8 + rr < nrhs)
        *reinterpret_cast<float4*>(out + (int64_t)(r0 + 8 + rr) * ldy + s * 16 + 2 * pc) = o[sw(8 + rr, pc)];
      __builtin_amdgcn_wave_barrier();
    }
    return;
  }
  if constexpr (SPLIT == 2) {
    for (int r0 = 16 * (int)(wv % 2); r0 < nrhs; r0 += 32) {
      const int ra = r0 + row;
      const bool va = ra < nrhs;
      const int64_t oa = (int64_t)min(ra, nrhs - 1) * ldx + 4 * kq;
      Quad a[5], xa[5];
#pragma unroll
      for (int dir = 0; dir < 5; ++dir) {
        a[dir] = load_quad(A + (s * 5 + dir) * 256 + row * 16 + 4 * kq);
        xa[dir] = load_quad(in + oa + sites[dir] * 16);
      }
      __builtin_amdgcn_sched_barrier(0);
      f32x4 are = {0.f, 0.f, 0.f, 0.f}, aim = are;
#pragma unroll
      for (int dir = 0; dir < 5; ++dir) block_mfma(are, aim, a[dir], select_quad(va, xa[dir]));
      if (va) store_quad(out + (int64_t)ra * ldy + s * 16 + 4 * kq, are, aim, sg);
    }
    return;
  }
  for (int r0 = 0; r0 < nrhs; r0 += 32) {
    const int ra = r0 + row, rb = r0 + 16 + row;
    const bool va = ra < nrhs, vb = rb < nrhs;
    const int64_t oa = (int64_t)min(ra, nrhs - 1) * ldx + 4 * kq, ob = (int64_t)min(rb, nrhs - 1) * ldx + 4 * kq;
    Quad a[5], xa[5], xb[5];
#pragma unroll
    for (int dir = 0; dir < 5; ++dir) {
      a[dir] = load_quad(A + (s * 5 + dir) * 256 + row * 16 + 4 * kq);
      xa[dir] = load_quad(in + oa + sites[dir] * 16);
      xb[dir] = load_quad(in + ob + sites[dir] * 16);
    }
    __builtin_amdgcn_sched_barrier(0);  // keep every load above the first product
    f32x4 are = {0.f, 0.f, 0.f, 0.f}, aim = are, bre = are, bim = are;
#pragma unroll
    for (int dir = 0; dir < 5; ++dir) {
      block_mfma(are, aim, a[dir], select_quad(va, xa[dir]));
      block_mfma(bre, bim, a[dir], select_quad(vb, xb[dir]));
    }
    if (va) store_quad(out + (int64_t)ra * ldy + s * 16 + 4 * kq, are, aim, sg);
    if (vb) store_quad(out + (int64_t)rb * ldy + s * 16 + 4 * kq, bre, bim, sg);
  }
}

// FP64 form of the coarse stencil, d = 16, on v_mfma_f64_16x16x4f64 (K = 4, one value per
// lane).  Its result fragment differs from the FP32 instruction's: lane (c, q) receives
// D[q + 4v][c], v < 4.  So lane (row, kq) supplies block row p(row) = 4 (row % 4) + row / 4
// of A (then D row kq + 4v is block row 4kq + v and a lane's four results are contiguous)
// at columns 4kq + t (column-major FP64 blocks: for each t the wavefront's 16 rows read
// one 256-byte column), and x[rhs row][4kq + t], for the four products t; two 16-RHS tiles
// per pass share the block loads.
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void cmfma64(f64x4& dre, f64x4& dim, c128 a, c128 x) {
  dre = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, x.x, dre, 0, 0, 0);
  dre = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, x.y, dre, 0, 0, 0);
  dim = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, x.y, dim, 0, 0, 0);
  dim = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, x.x, dim, 0, 0, 0);
}

template <bool G5, typename RO = double>
__global__ __launch_bounds__(256) void coarse16_f64_mfma_kernel(const c128* __restrict__ A,
                                                                const c128* __restrict__ in, Cx<RO>* __restrict__ out,
                                                                int Lx, int Lt, int nrhs, int64_t ldx, int64_t ldy,
                                                                const c128* __restrict__ sub) {
  const int64_t V = (int64_t)Lx * Lt;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t s = xcd_block() * 4 + w;
  if (s >= V) return;  // wave-uniform
  const int row = lane & 15, kq = lane >> 4;
  const int prow = 4 * (row & 3) + (row >> 2);
  const Nbr nb = neighbours(s, Lx, Lt);
  const int64_t sites[5] = {s, nb.xp, nb.xm, nb.tp, nb.tm};
  const double sg = (G5 && kq >= 2) ? -1.0 : 1.0;
  const c128 zero = cmk(0.0, 0.0);
  for (int r0 = 0; r0 < nrhs; r0 += 32) {
    const int ra = r0 + row, rb = r0 + 16 + row;
    const bool va = ra < nrhs, vb = rb < nrhs;
    const int64_t oa = (int64_t)min(ra, nrhs - 1) * ldx + 4 * kq, ob = (int64_t)min(rb, nrhs - 1) * ldx + 4 * kq;
    f64x4 are = {0.0, 0.0, 0.0, 0.0}, aim = are, bre = are, bim = are;
#pragma unroll
    for (int dir = 0; dir < 5; ++dir) {
      const c128* Ab = A + (s * 5 + dir) * 256 + 64 * kq + prow;
      const c128* xa = in + oa + sites[dir] * 16;
      const c128* xb = in + ob + sites[dir] * 16;
      c128 a[4], u[4], v[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        a[t] = Ab[16 * t];
        u[t] = xa[t];
        v[t] = xb[t];
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        cmfma64(are, aim, a[t], va ? u[t] : zero);
        cmfma64(bre, bim, a[t], vb ? v[t] : zero);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t e = s * 16 + 4 * kq + q;
      const c128 ya = cmk(sg * are[q], sg * aim[q]), yb = cmk(sg * bre[q], sg * bim[q]);
      // residual form: out = sub - D in (sub laid out as in)
      if (va) out[(int64_t)ra * ldy + e] = ccast<RO>(sub ? sub[(int64_t)ra * ldx + e] - ya : ya);
      if (vb) out[(int64_t)rb * ldy + e] = ccast<RO>(sub ? sub[(int64_t)rb * ldx + e] - yb : yb);
    }
  }
}

// Red/black point-block Gauss-Seidel, d = 16, on the sites of one colour:
// x_s = A_ss^-1 (b_s - sum_{dir != self} A[s][dir] x_{s+dir}); the neighbours all have the
// other colour (even extents), so the sweep over one colour is order-independent.  The
// residual fragment stays in registers as the B operand of the inverse-block product.
// H16: the four hop blocks and the inverse self block are read from their complex-FP16
// copies (16 bytes per lane quad instead of 32) and kept packed in registers, and the RHS
// are taken one 16-wide tile at a time.  The hop products run on the FP16 matrix cores
// (the neighbour vectors rounded to complex FP16 after a per-RHS power-of-two scaling, FP32
// accumulation): two instructions per block instead of sixteen FP32 ones, which were half
// of the sweep's time.  The inverse self block is widened to FP32 and applied to the FP32
// residual.  The vectors stay complex FP32.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ half8 as_half8(u32x4 v) { return __builtin_bit_cast(half8, v); }
__device__ __forceinline__ uint32_t pack_half2(float re, float im) {
  const _Float16 a = (_Float16)re, b = (_Float16)im;
  return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
}

__device__ __forceinline__ c64 half2_to_c64(uint32_t w) {
  const _Float16 re = __builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu));
  const _Float16 im = __builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
  return cmk((float)re, (float)im);
}

// One 16-RHS tile of the FP16-block sweep at one site: xa = the four neighbour quads and
// qa = the b quad of RHS row `row` (lane quarter kq); returns the lane's quad of the new x.
// Hop products on the FP16 matrix cores: the neighbour quads of the RHS are scaled by a
// power of two that brings their largest component to [2^14, 2^15) (the same scale for
// the four lanes of the RHS), rounded to complex FP16 and multiplied by the stored
// complex-FP16 blocks with FP32 accumulation, then scaled back.  One
// v_mfma_f32_16x16x32_f16 contracts a whole block row: A = the block words as read (re,
// im interleaved), B = (re, -im) for the real part and (im, re) for the imaginary part
// of the product.  The inverse self block is widened to FP32 and applied to the FP32
// residual.
__device__ __forceinline__ void gs16_tile(const uint4 (&a)[4], const uint4& ai, const Quad (&xa)[4], Quad qa, bool va,
                                          f32x4& ere, f32x4& eim) {
  float mx = 0.f;
#pragma unroll
  for (int dir = 0; dir < 4; ++dir)
#pragma unroll
    for (int q = 0; q < 4; ++q) mx = fmaxf(mx, fmaxf(fabsf(xa[dir].v[q].x), fabsf(xa[dir].v[q].y)));
  mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
  mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
  const int ex = mx > 0.f ? __builtin_amdgcn_frexp_expf(mx) : 0;  // mx = f 2^ex, f in [0.5, 1)
  const float sc = ldexpf(1.f, 15 - ex), unsc = ldexpf(1.f, ex - 15);
  f32x4 are = {0.f, 0.f, 0.f, 0.f}, aim = are;
#pragma unroll
  for (int dir = 0; dir < 4; ++dir) {
    u32x4 w = {0u, 0u, 0u, 0u};
    if (va) {
#pragma unroll
      for (int q = 0; q < 4; ++q) w[q] = pack_half2(sc * xa[dir].v[q].x, sc * xa[dir].v[q].y);
    }
    const half8 b_re = as_half8(w ^ 0x80000000u), b_im = as_half8((w >> 16) | (w << 16));
    const half8 m8 = as_half8(u32x4{a[dir].x, a[dir].y, a[dir].z, a[dir].w});
    are = __builtin_amdgcn_mfma_f32_16x16x32_f16(m8, b_re, are, 0, 0, 0);
    aim = __builtin_amdgcn_mfma_f32_16x16x32_f16(m8, b_im, aim, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) qa.v[v] = cmk(qa.v[v].x - unsc * are[v], qa.v[v].y - unsc * aim[v]);
  ere = f32x4{0.f, 0.f, 0.f, 0.f};
  eim = ere;
  const uint32_t wi[4] = {ai.x, ai.y, ai.z, ai.w};
#pragma unroll
  for (int q = 0; q < 4; ++q) cmfma(ere, eim, half2_to_c64(wi[q]), va ? qa.v[q] : cmk(0.f, 0.f));
}

// SPLIT (FP16 blocks only): 1 = one wavefront per site, its 16-RHS tiles in sequence;
// 2 = two wavefronts per site (same workgroup), each taking every other tile and reading
// the site's blocks; 3 = one wavefront per site, the loads of two tiles in flight together;
// 4 = as 1 with the vectors read by whole-line loads staged through LDS (10 KB per
// wavefront).
template <bool H16, int SPLIT>
__device__ __forceinline__ void coarse16_gs_body(const void* __restrict__ Av, const void* __restrict__ Ainvv,
                                                 c64* __restrict__ x, const c64* __restrict__ b, int Lx, int Lt,
                                                 int nrhs, int color, int64_t ld) {
  static_assert(SPLIT == 1 || (H16 && SPLIT >= 2 && SPLIT <= 4), "split forms only with the FP16 blocks");
  constexpr int WPS = SPLIT == 2 ? 2 : 1;  // wavefronts per site
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t wv = xcd_block() * 4 + w;
  const int64_t k = wv / WPS;
  const int64_t half = Lx / 2;
  const int64_t t = k / half;
  if (t >= Lt) return;  // wave-uniform
  const int64_t s = 2 * (k % half) + ((t + color) & 1) + t * Lx;
  const int row = lane & 15, kq = lane >> 4;
  const Nbr nb = neighbours(s, Lx, Lt);
  const int64_t sites[4] = {nb.xp, nb.xm, nb.tp, nb.tm};
  const int64_t own = s * 16 + 4 * kq;
  if constexpr (H16) {
    const uint32_t* A = static_cast<const uint32_t*>(Av);
    const uint32_t* Ainv = static_cast<const uint32_t*>(Ainvv);
    // the blocks are read once per launch: non-temporal loads
    uint4 a[4];
#pragma unroll
    for (int dir = 0; dir < 4; ++dir) {
      const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(A + (s * 4 + dir) * 256 + row * 16 + 4 * kq));
      a[dir] = make_uint4(v.x, v.y, v.z, v.w);
    }
    const u32x4 vi = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(Ainv + s * 256 + row * 16 + 4 * kq));
    const uint4 ai = make_uint4(vi.x, vi.y, vi.z, vi.w);
    if constexpr (SPLIT == 3) {
      for (int r0 = 0; r0 < nrhs; r0 += 32) {
        const int ra = r0 + row, rb = r0 + 16 + row;
        const bool va = ra < nrhs, vb = rb < nrhs;
        const int64_t oa = (int64_t)min(ra, nrhs - 1) * ld + 4 * kq, ob = (int64_t)min(rb, nrhs - 1) * ld + 4 * kq;
        Quad xa[4], xb[4];
#pragma unroll
        for (int dir = 0; dir < 4; ++dir) {
          xa[dir] = load_quad(x + oa + sites[dir] * 16);
          xb[dir] = load_quad(x + ob + sites[dir] * 16);
        }
        const Quad qa = load_quad(b + oa - 4 * kq + own);
        const Quad qb = load_quad(b + ob - 4 * kq + own);
        __builtin_amdgcn_sched_barrier(0);  // keep every load above the first product
        f32x4 ere, eim;
        gs16_tile(a, ai, xa, qa, va, ere, eim);
        if (va) store_quad(x + (int64_t)ra * ld + own, ere, eim, 1.f);
        gs16_tile(a, ai, xb, qb, vb, ere, eim);
        if (vb) store_quad(x + (int64_t)rb * ld + own, ere, eim, 1.f);
      }
    } else if constexpr (SPLIT == 4) {
      __shared__ float4 stage[4][5][16 * 8];
      float4(*rows)[16 * 8] = stage[w];
      for (int r0 = 0; r0 < nrhs; r0 += 16) {
        const int ra = r0 + row;
        const bool va = ra < nrhs;
#pragma unroll
        for (int dir = 0; dir < 4; ++dir) stage_rows(x, ld, r0, nrhs, sites[dir] * 16, lane, rows[dir]);
        stage_rows(b, ld, r0, nrhs, s * 16, lane, rows[4]);
        __builtin_amdgcn_wave_barrier();
        Quad xa[4];
#pragma unroll
        for (int dir = 0; dir < 4; ++dir) xa[dir] = staged_quad(rows[dir], lane);
        const Quad qa = staged_quad(rows[4], lane);
        f32x4 ere, eim;
        gs16_tile(a, ai, xa, qa, va, ere, eim);
        // the new x goes out the same way: the lane's quad into LDS row `row`, then whole-line
        // 16-byte stores (rows staged by the b vector above are free again)
        __builtin_amdgcn_wave_barrier();
        float4* out = rows[4];
        out[sw(row, 2 * kq)] = make_float4(ere[0], eim[0], ere[1], eim[1]);
        out[sw(row, 2 * kq + 1)] = make_float4(ere[2], eim[2], ere[3], eim[3]);
        __builtin_amdgcn_wave_barrier();
        {
          const int rr = lane >> 3, pc = lane & 7;
          if (r0 + rr < nrhs)
            *reinterpret_cast<float4*>(x + (int64_t)(r0 + rr) * ld + s * 16 + 2 * pc) = out[sw(rr, pc)];
          if (r0 + 8 + rr < nrhs)
            *reinterpret_cast<float4*>(x + (int64_t)(r0 + 8 + rr) * ld + s * 16 + 2 * pc) = out[sw(8 + rr, pc)];
        }
        __builtin_amdgcn_wave_barrier();  // the next tile's staging writes come after these reads
      }
    } else {
      for (int r0 = 16 * (int)(wv % WPS); r0 < nrhs; r0 += 16 * WPS) {
        const int ra = r0 + row;
        const bool va = ra < nrhs;
        const int64_t oa = (int64_t)min(ra, nrhs - 1) * ld + 4 * kq;
        Quad xa[4];
#pragma unroll
        for (int dir = 0; dir < 4; ++dir) xa[dir] = load_quad(x + oa + sites[dir] * 16);
        const Quad qa = load_quad(b + oa - 4 * kq + own);
        __builtin_amdgcn_sched_barrier(0);  // keep every load above the first product
        f32x4 ere, eim;
        gs16_tile(a, ai, xa, qa, va, ere, eim);
        if (va) store_quad(x + (int64_t)ra * ld + own, ere, eim, 1.f);
      }
    }
  } else {
    const c64* A = static_cast<const c64*>(Av);
    const c64* Ainv = static_cast<const c64*>(Ainvv);
    for (int r0 = 0; r0 < nrhs; r0 += 32) {
      const int ra = r0 + row, rb = r0 + 16 + row;
      const bool va = ra < nrhs, vb = rb < nrhs;
      const int64_t oa = (int64_t)min(ra, nrhs - 1) * ld + 4 * kq, ob = (int64_t)min(rb, nrhs - 1) * ld + 4 * kq;
      Quad a[4], xa[4], xb[4];
#pragma unroll
      for (int dir = 0; dir < 4; ++dir) {
        a[dir] = load_quad(A + (s * 5 + dir + 1) * 256 + row * 16 + 4 * kq);
        xa[dir] = load_quad(x + oa + sites[dir] * 16);
        xb[dir] = load_quad(x + ob + sites[dir] * 16);
      }
      const Quad ai = load_quad(Ainv + s * 256 + row * 16 + 4 * kq);
      Quad qa = load_quad(b + oa - 4 * kq + own);
      Quad qb = load_quad(b + ob - 4 * kq + own);
      __builtin_amdgcn_sched_barrier(0);  // keep every load above the first product
      f32x4 are = {0.f, 0.f, 0.f, 0.f}, aim = are, bre = are, bim = are;
#pragma unroll
      for (int dir = 0; dir < 4; ++dir) {
        block_mfma(are, aim, a[dir], select_quad(va, xa[dir]));
        block_mfma(bre, bim, a[dir], select_quad(vb, xb[dir]));
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        qa.v[v] = cmk(qa.v[v].x - are[v], qa.v[v].y - aim[v]);
        qb.v[v] = cmk(qb.v[v].x - bre[v], qb.v[v].y - bim[v]);
      }
      f32x4 ere = {0.f, 0.f, 0.f, 0.f}, eim = ere, fre = ere, fim = ere;
      block_mfma(ere, eim, ai, select_quad(va, qa));
      block_mfma(fre, fim, ai, select_quad(vb, qb));
      if (va) store_quad(x + (int64_t)ra * ld + own, ere, eim, 1.f);
      if (vb) store_quad(x + (int64_t)rb * ld + own, fre, fim, 1.f);
    }
  }
}

template <bool H16, int SPLIT>
__global__ __launch_bounds__(256) void coarse16_gs_mfma_kernel(const void* __restrict__ Av,
                                                               const void* __restrict__ Ainvv, c64* __restrict__ x,
                                                               const c64* __restrict__ b, int Lx, int Lt, int nrhs,
                                                               int color, int64_t ld) {
  coarse16_gs_body<H16, SPLIT>(Av, Ainvv, x, b, Lx, Lt, nrhs, color, ld);
}

// The staged form (SPLIT = 4) fits in 128 registers without spilling: four wavefronts per
// SIMD instead of three (level 2 at 1024^2: about 2 % faster); the other forms would spill.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void coarse16_gs_mfma_staged_kernel(
    const void* __restrict__ Av, const void* __restrict__ Ainvv, c64* __restrict__ x, const c64* __restrict__ b,
    int Lx, int Lt, int nrhs, int color, int64_t ld) {
  coarse16_gs_body<true, 4>(Av, Ainvv, x, b, Lx, Lt, nrhs, color, ld);
}

// ---------------------------------------------------------------- matrix-core transfers (2N = 16, complex FP32)
// Per aggregate, prolongation is X_f (E x b) (+)= P_full (E x 16) E_c (16 x b) and
// restriction Y_c (16 x b) = P_full^H X_f, with E = ax at d_f fine entries ordered
// (lt, lx, dof) and P_full[e][c N + k] = P[cs][c][row(e)][k] when chirality(e) = c, else 0.
// Entries 4q .. 4q+3 of an aggregate are contiguous in memory (ax d_f % 4 == 0), so the
// B operands and D fragments of both products move as 32-byte quads.
struct AggMap {
  int Lxf, df, ax, at, N, h, rows, E, Lxc;
  __device__ __forceinline__ int64_t fine_offset(int64_t cs, int e) const {
    const int X = (int)(cs % Lxc), T = (int)(cs / Lxc);
    const int lt = e / (ax * df), rem = e % (ax * df);
    return ((int64_t)(T * at + lt) * Lxf + (int64_t)X * ax) * df + rem;
  }
  // index of P[cs][c][row(e)][0] for entry e, and its chirality c
  __device__ __forceinline__ int64_t prow(int64_t cs, int e, int& c) const {
    const int lt = e / (ax * df), rem = e % (ax * df);
    const int lx = rem / df, dof = rem % df;
    c = dof / h;
    const int row = (lx + ax * lt) * h + dof % h;
    return ((cs * 2 + c) * (int64_t)rows + row) * N;
  }
};

// One wavefront per (aggregate, group of MT 16-entry tiles), all RHS, two 16-RHS tiles at
// a time; the group's interpolation quads (and, when adding, the old fine values) are all
// requested before the first product.
template <int MT>
__global__ __launch_bounds__(256) void prolong16_mfma_kernel(const c64* __restrict__ P, const c64* __restrict__ ec,
                                                             c64* __restrict__ xf, AggMap g, int64_t Vc, int nrhs,
                                                             int add, int64_t ldf, int64_t ldc) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int groups = g.E / 16 / MT;
  const int64_t wave = xcd_block() * 4 + w;
  const int64_t cs = wave / groups;
  if (cs >= Vc) return;  // wave-uniform
  const int grp = (int)(wave % groups);
  const int row = lane & 15, kq = lane >> 4;
  // coarse dof 4 kq + t has chirality kq / 2 and test vector 4 (kq % 2) + t
  const int cj = kq >> 1, k0 = 4 * (kq & 1);
  Quad a[MT];
  int64_t fo[MT];
#pragma unroll
  for (int u = 0; u < MT; ++u) {
    const int mt = grp * MT + u;
    int ce;
    const int64_t pr = g.prow(cs, 16 * mt + row, ce);
    a[u] = select_quad(ce == cj, load_quad_nt(P + pr + k0));
    fo[u] = g.fine_offset(cs, 16 * mt + 4 * kq);
  }
  for (int r0 = 0; r0 < nrhs; r0 += 32) {
    const int ra = r0 + row, rb = r0 + 16 + row;
    const bool va = ra < nrhs, vb = rb < nrhs;
    const int64_t oa = (int64_t)min(ra, nrhs - 1) * ldf, ob = (int64_t)min(rb, nrhs - 1) * ldf;
    // rows beyond nrhs load a valid row and are zeroed (no divergent loads)
    const Quad ea = select_quad(va, load_quad(ec + (int64_t)min(ra, nrhs - 1) * ldc + cs * 16 + 4 * kq));
    const Quad eb = select_quad(vb, load_quad(ec + (int64_t)min(rb, nrhs - 1) * ldc + cs * 16 + 4 * kq));
    Quad xa[MT], xb[MT];
    if (add) {
#pragma unroll
      for (int u = 0; u < MT; ++u) {
        xa[u] = load_quad(xf + oa + fo[u]);
        xb[u] = load_quad(xf + ob + fo[u]);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < MT; ++u) {
      f32x4 are = {0.f, 0.f, 0.f, 0.f}, aim = are, bre = are, bim = are;
      block_mfma(are, aim, a[u], ea);
      block_mfma(bre, bim, a[u], eb);
      if (add) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          are[v] += xa[u].v[v].x;
          aim[v] += xa[u].v[v].y;
          bre[v] += xb[u].v[v].x;
          bim[v] += xb[u].v[v].y;
        }
      }
      if (va) store_quad(xf + oa + fo[u], are, aim, 1.f);
      if (vb) store_quad(xf + ob + fo[u], bre, bim, 1.f);
    }
  }
}

// Prolongation for d_f = 16, where each 16-entry tile of an aggregate is one fine site
// (its 16 entries of one RHS are one 128-byte line): as prolong16_mfma_kernel, one 16-RHS
// tile at a time, with the coarse vector read, the old fine values read (when adding) and
// the results written by whole lines staged through LDS.  The same products and sums.
template <int MT>
__global__ __launch_bounds__(256) void prolong16_staged_kernel(const c64* __restrict__ P, const c64* __restrict__ ec,
                                                               c64* __restrict__ xf, AggMap g, int64_t Vc, int nrhs,
                                                               int add, int64_t ldf, int64_t ldc) {
  __shared__ float4 stage[4][2][16 * 8];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int groups = g.E / 16 / MT;
  const int64_t wave = xcd_block() * 4 + w;
  const int64_t cs = wave / groups;
  if (cs >= Vc) return;  // wave-uniform; no workgroup barrier below
  const int grp = (int)(wave % groups);
  const int row = lane & 15, kq = lane >> 4;
  const int cj = kq >> 1, k0 = 4 * (kq & 1);
  float4(*rows)[16 * 8] = stage[w];
  Quad a[MT];
  int64_t fs[MT];
#pragma unroll
  for (int u = 0; u < MT; ++u) {
    const int mt = grp * MT + u;
    int ce;
    const int64_t pr = g.prow(cs, 16 * mt + row, ce);
    a[u] = select_quad(ce == cj, load_quad_nt(P + pr + k0));
    fs[u] = g.fine_offset(cs, 16 * mt);  // the tile's site: entries fs .. fs + 15
  }
  const int rr = lane >> 3, pc = lane & 7;
  for (int r0 = 0; r0 < nrhs; r0 += 16) {
    const bool va = r0 + row < nrhs;
    stage_rows(ec, ldc, r0, nrhs, cs * 16, lane, rows[0]);
    __builtin_amdgcn_wave_barrier();
    const Quad ea = select_quad(va, staged_quad(rows[0], lane));
#pragma unroll
    for (int u = 0; u < MT; ++u) {
      f32x4 are = {0.f, 0.f, 0.f, 0.f}, aim = are;
      block_mfma(are, aim, a[u], ea);
      if (add) {
        stage_rows(xf, ldf, r0, nrhs, fs[u], lane, rows[1]);
        __builtin_amdgcn_wave_barrier();
        const Quad xo = staged_quad(rows[1], lane);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          are[v] += xo.v[v].x;
          aim[v] += xo.v[v].y;
        }
      }
      __builtin_amdgcn_wave_barrier();
      rows[1][sw(row, 2 * kq)] = make_float4(are[0], aim[0], are[1], aim[1]);
      rows[1][sw(row, 2 * kq + 1)] = make_float4(are[2], aim[2], are[3], aim[3]);
      __builtin_amdgcn_wave_barrier();
      if (r0 + rr < nrhs) *reinterpret_cast<float4*>(xf + (int64_t)(r0 + rr) * ldf + fs[u] + 2 * pc) = rows[1][sw(rr, pc)];
      if (r0 + 8 + rr < nrhs)
        *reinterpret_cast<float4*>(xf + (int64_t)(r0 + 8 + rr) * ldf + fs[u] + 2 * pc) = rows[1][sw(8 + rr, pc)];
      __builtin_amdgcn_wave_barrier();
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// Prolongation for aggregates whose rows are half a 128-byte line (a_x d_f = 8 entries,
// the fine level of 2 dofs on 4-site-wide aggregates): one wavefront per pair of
// aggregates adjacent in x (X even), whose rows share lines, all TT = a_t / 2 tiles of
// both, one 16-RHS tile at a time.  The two coarse vectors are read, and the 16 x a_t fine
// lines written (and, when adding, read), by whole lines staged through LDS.  Each entry
// is the product of prolong16_mfma_kernel, plus the old value when adding, in the same
// order.
template <int TT>
__global__ __launch_bounds__(256) void prolong16_pair_kernel(const c64* __restrict__ P, const c64* __restrict__ ec,
                                                             c64* __restrict__ xf, AggMap g, int64_t Vc, int nrhs,
                                                             int add, int64_t ldf, int64_t ldc) {
  constexpr int NL = 16 * 2 * TT;  // lines of one RHS tile: 16 RHS x a_t fine rows
  __shared__ float4 stage[4][NL * 8];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t cs0 = 2 * (xcd_block() * 4 + w);
  if (cs0 >= Vc) return;  // wave-uniform; no workgroup barrier below
  const int row = lane & 15, kq = lane >> 4;
  const int cj = kq >> 1, k0 = 4 * (kq & 1);
  float4* lines = stage[w];
  Quad a[2][TT];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int u = 0; u < TT; ++u) {
      int ce;
      const int64_t pr = g.prow(cs0 + p, 16 * u + row, ce);
      a[p][u] = select_quad(ce == cj, load_quad_nt(P + pr + k0));
    }
  const int rr = lane >> 3, pc = lane & 7;
  // fine row lt of the pair starts at aggregate cs0's row lt (16 entries: cs0's 8, then cs0 + 1's)
  int64_t fl[2 * TT];
#pragma unroll
  for (int lt = 0; lt < 2 * TT; ++lt) fl[lt] = g.fine_offset(cs0, 8 * lt) + 2 * pc;
  for (int r0 = 0; r0 < nrhs; r0 += 16) {
    const bool va = r0 + row < nrhs;
    stage_rows(ec, ldc, r0, nrhs, cs0 * 16, lane, lines);
    stage_rows(ec, ldc, r0, nrhs, (cs0 + 1) * 16, lane, lines + 16 * 8);
    __builtin_amdgcn_wave_barrier();
    const Quad e0 = select_quad(va, staged_quad(lines, lane));
    const Quad e1 = select_quad(va, staged_quad(lines + 16 * 8, lane));
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int u = 0; u < TT; ++u) {
        f32x4 re = {0.f, 0.f, 0.f, 0.f}, im = re;
        block_mfma(re, im, a[p][u], p ? e1 : e0);
        // entries 16 u + 4 kq .. + 3: fine row 2 u + kq / 2, entries 4 (kq % 2) .. of its 8
        const int L = (2 * u + (kq >> 1)) * 16 + row, c = 4 * p + 2 * (kq & 1);
        lines[sw(L, c)] = make_float4(re[0], im[0], re[1], im[1]);
        lines[sw(L, c + 1)] = make_float4(re[2], im[2], re[3], im[3]);
      }
    __builtin_amdgcn_wave_barrier();
    float4 old[NL / 8];
    if (add) {
#pragma unroll
      for (int i = 0; i < NL / 8; ++i) {
        const int li = 8 * i + rr, r = min(r0 + (li & 15), nrhs - 1);
        old[i] = *reinterpret_cast<const float4*>(xf + (int64_t)r * ldf + fl[li >> 4]);
      }
    }
#pragma unroll
    for (int i = 0; i < NL / 8; ++i) {
      const int li = 8 * i + rr, r = r0 + (li & 15);
      float4 v = lines[sw(li, pc)];
      if (add) {
        v.x = v.x + old[i].x;
        v.y = v.y + old[i].y;
        v.z = v.z + old[i].z;
        v.w = v.w + old[i].w;
      }
      if (r < nrhs) *reinterpret_cast<float4*>(xf + (int64_t)r * ldf + fl[li >> 4]) = v;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// WPA wavefronts per aggregate (WPA = min(4, E / 16)), 4 / WPA aggregates per workgroup:
// the aggregate's 16-entry tiles are dealt round-robin to its wavefronts, each of which
// requests the loads of up to UT tiles before multiplying; the partial 16 x 32 results
// of the wavefronts meet in LDS.  Every wavefront reaches the barriers.
template <int UT>
__global__ __launch_bounds__(256) void restrict16_mfma_kernel(const c64* __restrict__ P, const c64* __restrict__ xf,
                                                              c64* __restrict__ yc, AggMap g, int64_t Vc, int nrhs,
                                                              int wpa, int64_t ldf, int64_t ldc) {
  __shared__ f32x4 part[4][4][64];  // [wave][are, aim, bre, bim][lane]
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t cs_raw = xcd_block() * (4 / wpa) + w / wpa;
  const bool valid = cs_raw < Vc;
  const int64_t cs = valid ? cs_raw : Vc - 1;
  const int sub = w % wpa;
  const int row = lane & 15, kq = lane >> 4;
  // A operand: lane (row, kq) supplies conj(P_full[e][row]) for e = 16 kt + 4 kq + t
  const int cj = row >> 3, kj = row & 7;
  const int ntile = g.E / 16;
  for (int r0 = 0; r0 < nrhs; r0 += 32) {
    const int ra = r0 + row, rb = r0 + 16 + row;
    const bool va = ra < nrhs, vb = rb < nrhs;
    f32x4 are = {0.f, 0.f, 0.f, 0.f}, aim = are, bre = are, bim = are;
    const int64_t oa = (int64_t)min(ra, nrhs - 1) * ldf, ob = (int64_t)min(rb, nrhs - 1) * ldf;
    for (int kt0 = sub; kt0 < ntile; kt0 += UT * wpa) {
      Quad a[UT], xa[UT], xb[UT];
#pragma unroll
      for (int u = 0; u < UT; ++u) {
        const int kt = kt0 + u * wpa;
        if (kt >= ntile) continue;  // wave-uniform
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          int ce;
          const int64_t pr = g.prow(cs, 16 * kt + 4 * kq + t, ce);
          const float* pf = reinterpret_cast<const float*>(P + pr + kj);
          const c64 pv = cmk(__builtin_nontemporal_load(pf), __builtin_nontemporal_load(pf + 1));
          a[u].v[t] = ce == cj ? cmk(pv.x, -pv.y) : cmk(0.f, 0.f);
        }
        const int64_t fo = g.fine_offset(cs, 16 * kt + 4 * kq);
        xa[u] = load_quad(xf + oa + fo);
        xb[u] = load_quad(xf + ob + fo);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < UT; ++u) {
        if (kt0 + u * wpa < ntile) {  // wave-uniform
          block_mfma(are, aim, a[u], select_quad(va, xa[u]));
          block_mfma(bre, bim, a[u], select_quad(vb, xb[u]));
        }
      }
    }
    part[w][0][lane] = are;
    part[w][1][lane] = aim;
    part[w][2][lane] = bre;
    part[w][3][lane] = bim;
    __syncthreads();
    if (sub == 0 && valid) {
      for (int q = 1; q < wpa; ++q) {
        are += part[w + q][0][lane];
        aim += part[w + q][1][lane];
        bre += part[w + q][2][lane];
        bim += part[w + q][3][lane];
      }
      if (va) store_quad(yc + (int64_t)ra * ldc + cs * 16 + 4 * kq, are, aim, 1.f);
      if (vb) store_quad(yc + (int64_t)rb * ldc + cs * 16 + 4 * kq, bre, bim, 1.f);
    }
    __syncthreads();
  }
}

// Restriction for the pair shape of prolong16_pair_kernel with at most three tiles per
// aggregate (where restrict16_mfma_kernel takes one wavefront per aggregate): one
// wavefront per pair of aggregates adjacent in x, one 16-RHS tile at a time; the 16 x a_t
// fine lines are read, and the two aggregates' coarse results written, by whole lines
// staged through LDS.  Each result is the sum of restrict16_mfma_kernel's products in its
// order (tile 0, 1, ...).
template <int TT>
__global__ __launch_bounds__(256) void restrict16_pair_kernel(const c64* __restrict__ P, const c64* __restrict__ xf,
                                                              c64* __restrict__ yc, AggMap g, int64_t Vc, int nrhs,
                                                              int64_t ldf, int64_t ldc) {
  constexpr int NL = 16 * 2 * TT;
  __shared__ float4 stage[4][NL * 8];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t cs0 = 2 * (xcd_block() * 4 + w);
  if (cs0 >= Vc) return;  // wave-uniform; no workgroup barrier below
  const int row = lane & 15, kq = lane >> 4;
  const int cj = row >> 3, kj = row & 7;
  float4* lines = stage[w];
  Quad a[2][TT];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int u = 0; u < TT; ++u)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        int ce;
        const int64_t pr = g.prow(cs0 + p, 16 * u + 4 * kq + t, ce);
        const float* pf = reinterpret_cast<const float*>(P + pr + kj);
        const c64 pv = cmk(__builtin_nontemporal_load(pf), __builtin_nontemporal_load(pf + 1));
        a[p][u].v[t] = ce == cj ? cmk(pv.x, -pv.y) : cmk(0.f, 0.f);
      }
  const int rr = lane >> 3, pc = lane & 7;
  int64_t fl[2 * TT];
#pragma unroll
  for (int lt = 0; lt < 2 * TT; ++lt) fl[lt] = g.fine_offset(cs0, 8 * lt) + 2 * pc;
  for (int r0 = 0; r0 < nrhs; r0 += 16) {
    const bool va = r0 + row < nrhs;
    float4 in[NL / 8];
#pragma unroll
    for (int i = 0; i < NL / 8; ++i) {
      const int li = 8 * i + rr, r = min(r0 + (li & 15), nrhs - 1);
      in[i] = *reinterpret_cast<const float4*>(xf + (int64_t)r * ldf + fl[li >> 4]);
    }
#pragma unroll
    for (int i = 0; i < NL / 8; ++i) lines[sw(8 * i + rr, pc)] = in[i];
    __builtin_amdgcn_wave_barrier();
    f32x4 re[2], im[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      re[p] = f32x4{0.f, 0.f, 0.f, 0.f};
      im[p] = re[p];
#pragma unroll
      for (int u = 0; u < TT; ++u) {
        const int L = (2 * u + (kq >> 1)) * 16 + row, c = 4 * p + 2 * (kq & 1);
        const float4 x0 = lines[sw(L, c)], x1 = lines[sw(L, c + 1)];
        Quad xq;
        xq.v[0] = cmk(x0.x, x0.y);
        xq.v[1] = cmk(x0.z, x0.w);
        xq.v[2] = cmk(x1.x, x1.y);
        xq.v[3] = cmk(x1.z, x1.w);
        block_mfma(re[p], im[p], a[p][u], select_quad(va, xq));
      }
    }
    __builtin_amdgcn_wave_barrier();
    // coarse rows: RHS row r of the pair is 32 entries (two lines), entries 16 p + 4 kq ..
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      lines[sw(2 * row + p, 2 * kq)] = make_float4(re[p][0], im[p][0], re[p][1], im[p][1]);
      lines[sw(2 * row + p, 2 * kq + 1)] = make_float4(re[p][2], im[p][2], re[p][3], im[p][3]);
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int li = 8 * i + rr, r = r0 + (li >> 1);
      if (r < nrhs)
        *reinterpret_cast<float4*>(yc + (int64_t)r * ldc + (cs0 + (li & 1)) * 16 + 2 * pc) = lines[sw(li, pc)];
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// the fine rows of an aggregate are half a 128-byte line and pairs of aggregates adjacent in
// x share them (tiles per aggregate: a_t / 2)
bool transfer16_pair_ok(const Level& L) {
  return L.ax * L.dofs == 8 && (L.Lx / L.ax) % 2 == 0 && (L.at == 2 || L.at == 4 || L.at == 8);
}

bool transfer16_ok(const Level& L) {
  const int E = L.ax * L.at * L.dofs;
  return L.N == 8 && L.dofs % 2 == 0 && (L.ax * L.dofs) % 4 == 0 && E % 16 == 0;
}

AggMap agg_map(const Level& L) {
  AggMap g;
  g.Lxf = L.Lx;
  g.df = L.dofs;
  g.ax = L.ax;
  g.at = L.at;
  g.N = L.N;
  g.h = L.dofs / 2;
  g.rows = L.ax * L.at * g.h;
  g.E = L.ax * L.at * L.dofs;
  g.Lxc = L.Lx / L.ax;
  return g;
}

inline int rhs_block_for(int64_t threads, int nrhs) {
  // enough workgroups to fill 256 CUs several times; otherwise split the RHS over y
  const int64_t wgs = ceil_div(threads, 256);
  if (wgs >= 4096) return nrhs;
  int rb = (int)std::max<int64_t>(1, (int64_t)nrhs * wgs / 4096);
  return std::min(rb, nrhs);
}

}  // namespace

bool transfer16_available(const Level& L) { return transfer16_ok(L); }
bool transfer16_pair_available(const Level& L) { return transfer16_ok(L) && transfer16_pair_ok(L); }

// whether the staged transfers run (built-in rule from 16384 fine sites on: measured at
// 1024^2, where the level-1 and level-2 transfers gain and the 64^2-site ones do not)
static bool prolong_staged_rule(const Level& L) {
  return L.kv[KV_PROLONG_STAGED] == 2 || (L.kv[KV_PROLONG_STAGED] == 0 && L.sites() >= 16384);
}
bool restrict16_pair_selected(const Level& L) {
  const int v = L.kv[KV_RESTRICT_STAGED];
  return transfer16_pair_available(L) && L.at <= 4 && (v == 2 || (v == 0 && L.sites() >= 16384));
}
bool prolong16_pair_selected(const Level& L) { return transfer16_pair_available(L) && prolong_staged_rule(L); }

template <typename R>
void launch_wilson(dmlmc_ctx* ctx, const Level& L, const Cx<R>* x, Cx<R>* y, int nrhs, int64_t ldx, int64_t ldy,
                   bool gamma5_left, const Cx<R>* sub) {
  const int64_t V = L.sites();
  // at most 8 RHS per thread: more workgroups in flight; links are re-read nrhs / 8 times
  const int rb = L.kv[KV_WILSON_RB] > 0 ? std::min(L.kv[KV_WILSON_RB], nrhs) : std::min(8, rhs_block_for(V, nrhs));
  dim3 grid((unsigned)ceil_div(V, 256), (unsigned)ceil_div(nrhs, rb));
  const Cx<R>* U = std::is_same<R, float>::value ? (const Cx<R>*)L.U32.p : (const Cx<R>*)L.U64.p;
  REQUIRE(!(sub && gamma5_left), "the residual form has no Gamma5");
  KTimer kt(ctx, "wilson", (double)nrhs * V * (sub ? 6 : 4) * sizeof(Cx<R>) + (double)V * 2 * sizeof(Cx<R>));
  if (gamma5_left)
    hipLaunchKernelGGL((wilson_kernel<R, true>), grid, dim3(256), 0, ctx->stream, U, x, y, L.Lx, L.Lt,
                       (R)(L.m0 + 2.0), nrhs, rb, ldx, ldy, (const Cx<R>*)nullptr);
  else
    hipLaunchKernelGGL((wilson_kernel<R, false>), grid, dim3(256), 0, ctx->stream, U, x, y, L.Lx, L.Lt,
                       (R)(L.m0 + 2.0), nrhs, rb, ldx, ldy, sub);
  LAUNCH_CHECK();
}

constexpr int WD_SPT = 2;  // sites per thread of the fused stencil-and-dots kernel

int wilson_dots_blocks(const Level& L) { return (int)ceil_div(L.sites(), 256 * WD_SPT); }

int launch_wilson_dots(dmlmc_ctx* ctx, const Level& L, const c64* z, c64* y, int nrhs, int64_t ld, const c64* Ub,
                       int nb, int64_t vs, const double* wscale, double* part) {
  REQUIRE(L.fine && nb >= 1 && nb <= 8, "the fused stencil-and-dots pass runs on the fine level with at most 8 basis vectors");
  REQUIRE(ld >= L.n() && ld % 2 == 0 && vs % 2 == 0 && ((uintptr_t)Ub % 16) == 0,
          "the fused stencil-and-dots pass needs even strides and a 16-byte aligned basis");
  const int64_t V = L.sites();
  const int G = wilson_dots_blocks(L);
  const int rb = L.kv[KV_WILSON_RB] > 0 ? std::min(L.kv[KV_WILSON_RB], nrhs)
                                        : std::min(8, rhs_block_for(ceil_div(V, WD_SPT), nrhs));
  dim3 grid((unsigned)G, (unsigned)ceil_div(nrhs, rb));
  KTimer kt(ctx, "wilson",
            (double)nrhs * V * 4 * sizeof(c64) + (double)V * 2 * sizeof(c64) + (double)nrhs * L.n() * nb * sizeof(c64));
  if (nb <= 4)
    hipLaunchKernelGGL((wilson_dots_kernel<4, WD_SPT>), grid, dim3(256), 0, ctx->stream, L.U32.as<c64>(), z, y, L.Lx,
                       L.Lt, (float)(L.m0 + 2.0), nrhs, rb, ld, Ub, nb, vs, wscale, part);
  else
    hipLaunchKernelGGL((wilson_dots_kernel<8, WD_SPT>), grid, dim3(256), 0, ctx->stream, L.U32.as<c64>(), z, y, L.Lx,
                       L.Lt, (float)(L.m0 + 2.0), nrhs, rb, ld, Ub, nb, vs, wscale, part);
  LAUNCH_CHECK();
  return G;
}

template <typename R>
void launch_coarse(dmlmc_ctx* ctx, const Level& L, const Cx<R>* x, Cx<R>* y, int nrhs, int64_t ldx, int64_t ldy,
                   bool gamma5_left, const Cx<R>* sub) {
  const int d = L.dofs;
  const int spb = std::max(1, 256 / d);
  const int64_t V = L.sites();
  const Cx<R>* A = std::is_same<R, float>::value ? (const Cx<R>*)L.A32.p : (const Cx<R>*)L.A64.p;
  REQUIRE(!(sub && gamma5_left), "the residual form has no Gamma5");
  KTimer kt(ctx, "coarse",
            (double)nrhs * L.n() * (sub ? 3 : 2) * sizeof(Cx<R>) + (double)V * 5 * d * d * sizeof(Cx<R>));
  if (std::is_same<R, float>::value && d == 16) {
    REQUIRE(sub == nullptr, "the complex-FP32 matrix-core stencil has no residual form");
    REQUIRE(ldx % 2 == 0 && ldy % 2 == 0 && ((uintptr_t)x | (uintptr_t)y) % 16 == 0,
            "matrix-core coarse stencil needs 16-byte aligned RHS rows");
    // built-in rule: whole-line traffic staged through LDS (measured at 1024^2 with the
    // swizzled LDS rows: 65536 sites 290 -> 267 us, 4096 sites 21.9 -> 20.1 us, 1024 sites
    // 8.0 -> 7.0 us against the best of the other forms)
    const int split = L.kv[KV_COARSE_SPLIT] > 0 ? L.kv[KV_COARSE_SPLIT] : 3;
    dim3 grid((unsigned)ceil_div(V * (split == 2 ? 2 : 1), 4));
    if (split == 3) {
      if (gamma5_left)
        hipLaunchKernelGGL((coarse16_mfma_kernel<true, 3>), grid, dim3(256), 0, ctx->stream, (const c64*)A,
                           (const c64*)x, (c64*)y, L.Lx, L.Lt, nrhs, ldx, ldy);
      else
        hipLaunchKernelGGL((coarse16_mfma_kernel<false, 3>), grid, dim3(256), 0, ctx->stream, (const c64*)A,
                           (const c64*)x, (c64*)y, L.Lx, L.Lt, nrhs, ldx, ldy);
    } else if (split == 2) {
      if (gamma5_left)
        hipLaunchKernelGGL((coarse16_mfma_kernel<true, 2>), grid, dim3(256), 0, ctx->stream, (const c64*)A,
                           (const c64*)x, (c64*)y, L.Lx, L.Lt, nrhs, ldx, ldy);
      else
        hipLaunchKernelGGL((coarse16_mfma_kernel<false, 2>), grid, dim3(256), 0, ctx->stream, (const c64*)A,
                           (const c64*)x, (c64*)y, L.Lx, L.Lt, nrhs, ldx, ldy);
    } else if (gamma5_left) {
      hipLaunchKernelGGL((coarse16_mfma_kernel<true, 1>), grid, dim3(256), 0, ctx->stream, (const c64*)A,
                         (const c64*)x, (c64*)y, L.Lx, L.Lt, nrhs, ldx, ldy);
    } else {
      hipLaunchKernelGGL((coarse16_mfma_kernel<false, 1>), grid, dim3(256), 0, ctx->stream, (const c64*)A,
                         (const c64*)x, (c64*)y, L.Lx, L.Lt, nrhs, ldx, ldy);
    }
    LAUNCH_CHECK();
    return;
  }
  if (std::is_same<R, double>::value && d == 16 && nrhs >= 8) {
    // FP64 matrix cores pay from a few RHS on (a 16-wide tile); single vectors keep the
    // scalar kernel
    dim3 grid((unsigned)ceil_div(V, 4));
    if (gamma5_left)
      hipLaunchKernelGGL((coarse16_f64_mfma_kernel<true>), grid, dim3(256), 0, ctx->stream, (const c128*)A,
                         (const c128*)x, (c128*)y, L.Lx, L.Lt, nrhs, ldx, ldy, (const c128*)nullptr);
    else
      hipLaunchKernelGGL((coarse16_f64_mfma_kernel<false>), grid, dim3(256), 0, ctx->stream, (const c128*)A,
                         (const c128*)x, (c128*)y, L.Lx, L.Lt, nrhs, ldx, ldy, (const c128*)sub);
    LAUNCH_CHECK();
    return;
  }
  constexpr int RB = 4;
  dim3 grid((unsigned)ceil_div(V, spb), (unsigned)ceil_div(nrhs, RB));
  dim3 block((unsigned)(spb * d));
  if (gamma5_left)
    hipLaunchKernelGGL((coarse_kernel<R, RB, true>), grid, block, 0, ctx->stream, A, x, y, L.Lx, L.Lt, d, spb, nrhs,
                       ldx, ldy, (const Cx<R>*)nullptr);
  else
    hipLaunchKernelGGL((coarse_kernel<R, RB, false>), grid, block, 0, ctx->stream, A, x, y, L.Lx, L.Lt, d, spb,
                       nrhs, ldx, ldy, sub);
  LAUNCH_CHECK();
}

template <typename R>
void apply_op(dmlmc_ctx* ctx, const Level& L, const Cx<R>* x, Cx<R>* y, int nrhs, bool gamma5_left, int64_t ld) {
  if (ld <= 0) ld = L.n();
  if (L.fine)
    launch_wilson<R>(ctx, L, x, y, nrhs, ld, ld, gamma5_left, nullptr);
  else
    launch_coarse<R>(ctx, L, x, y, nrhs, ld, ld, gamma5_left, nullptr);
}

template <typename R>
void apply_residual(dmlmc_ctx* ctx, const Level& L, const Cx<R>* x, const Cx<R>* b, Cx<R>* r, int nrhs) {
  if (L.fine)
    launch_wilson<R>(ctx, L, x, r, nrhs, L.n(), L.n(), false, b);
  else
    launch_coarse<R>(ctx, L, x, r, nrhs, L.n(), L.n(), false, b);
}

void apply_residual_to32(dmlmc_ctx* ctx, const Level& L, const c128* x, const c128* b, c64* r, int nrhs, int64_t ldx,
                         int64_t ldr) {
  if (ldx <= 0) ldx = L.n();
  if (ldr <= 0) ldr = L.n();
  REQUIRE(ldx >= L.n() && ldr >= L.n() && ldx % 2 == 0 && ldr % 2 == 0,
          "residual vectors need even strides of at least the level size");
  const int64_t V = L.sites();
  // reads x and b (FP64), writes r (complex FP32)
  const double vec_bytes = (double)nrhs * L.n() * (2 * sizeof(c128) + sizeof(c64));
  if (L.fine) {
    const int rb = std::min(8, rhs_block_for(V, nrhs));
    dim3 grid((unsigned)ceil_div(V, 256), (unsigned)ceil_div(nrhs, rb));
    KTimer kt(ctx, "wilson", vec_bytes + (double)V * 2 * sizeof(c128));
    hipLaunchKernelGGL((wilson_kernel<double, false, float>), grid, dim3(256), 0, ctx->stream, L.U64.as<c128>(), x,
                       r, L.Lx, L.Lt, L.m0 + 2.0, nrhs, rb, ldx, ldr, b);
    LAUNCH_CHECK();
    return;
  }
  const int d = L.dofs;
  KTimer kt(ctx, "coarse", vec_bytes + (double)V * 5 * d * d * sizeof(c128));
  if (d == 16 && nrhs >= 8) {
    hipLaunchKernelGGL((coarse16_f64_mfma_kernel<false, float>), dim3((unsigned)ceil_div(V, 4)), dim3(256), 0,
                       ctx->stream, L.A64.as<c128>(), x, r, L.Lx, L.Lt, nrhs, ldx, ldr, b);
    LAUNCH_CHECK();
    return;
  }
  constexpr int RB = 4;
  const int spb = std::max(1, 256 / d);
  dim3 grid((unsigned)ceil_div(V, spb), (unsigned)ceil_div(nrhs, RB));
  hipLaunchKernelGGL((coarse_kernel<double, RB, false, float>), grid, dim3((unsigned)(spb * d)), 0, ctx->stream,
                     L.A64.as<c128>(), x, r, L.Lx, L.Lt, d, spb, nrhs, ldx, ldr, b);
  LAUNCH_CHECK();
}

template <typename R>
void launch_sap(dmlmc_ctx* ctx, const Level& L, Cx<R>* x, const Cx<R>* b, int nrhs, int color, int mr_iters,
                int64_t ld) {
  if (ld <= 0) ld = L.n();
  REQUIRE(ld >= L.n() && ld % 2 == 0, "SAP vectors need an even stride of at least the level size");
  const Cx<R>* U = std::is_same<R, float>::value ? (const Cx<R>*)L.U32.p : (const Cx<R>*)L.U64.p;
  const int64_t V = L.sites();
  // 4 RHS per thread (more workgroups in flight) unless tuned
  const int rb = L.kv[KV_SAP_RB] > 0 ? std::min(L.kv[KV_SAP_RB], nrhs) : std::min(4, rhs_block_for(V, nrhs));
  // algorithmic bytes of one colour: x of every site (the colour's own and its halo) read
  // once, b read and x written on the colour's sites (two vector passes), and the links
  KTimer kt(ctx, "sap", (double)nrhs * V * 2 * sizeof(Cx<R>) * 2 + (double)V * 2 * sizeof(Cx<R>));
  // 8x4 blocks when the block checkerboard has even extents (no two neighbouring blocks
  // share a colour, also across the periodic boundary): a block row of one RHS is then
  // 8 sites x 2 spins = one 128-byte line in complex FP32, so a colour's sweep touches
  // only its own lines besides the halo.  Else 4x4, else 2x2 blocks (the fine extents are
  // multiples of 4, so 2x2 block counts are even).
  REQUIRE(L.Lx % 4 == 0 && L.Lt % 4 == 0, "SAP needs fine extents divisible by 4");
  if (L.Lx % 16 == 0 && L.Lt % 8 == 0) {
    const int nblk = (L.Lx / 8) * (L.Lt / 4) / 2;  // blocks of one colour
    dim3 grid((unsigned)ceil_div(nblk, 8), (unsigned)ceil_div(nrhs, rb));
    hipLaunchKernelGGL((sap_kernel<R, 8, 4>), grid, dim3(256), 0, ctx->stream, U, x, b, L.Lx, L.Lt,
                       (R)(L.m0 + 2.0), nrhs, rb, color, mr_iters, ld);
  } else if (L.Lx % 8 == 0 && L.Lt % 8 == 0) {
    const int nblk = (L.Lx / 4) * (L.Lt / 4) / 2;  // blocks of one colour
    dim3 grid((unsigned)ceil_div(nblk, 16), (unsigned)ceil_div(nrhs, rb));
    hipLaunchKernelGGL((sap_kernel<R, 4, 4>), grid, dim3(256), 0, ctx->stream, U, x, b, L.Lx, L.Lt,
                       (R)(L.m0 + 2.0), nrhs, rb, color, mr_iters, ld);
  } else {
    const int nblk = (L.Lx / 2) * (L.Lt / 2) / 2;
    dim3 grid((unsigned)ceil_div(nblk, 64), (unsigned)ceil_div(nrhs, rb));
    hipLaunchKernelGGL((sap_kernel<R, 2, 2>), grid, dim3(256), 0, ctx->stream, U, x, b, L.Lx, L.Lt,
                       (R)(L.m0 + 2.0), nrhs, rb, color, mr_iters, ld);
  }
  LAUNCH_CHECK();
}

template <typename R>
void launch_coarse_gs(dmlmc_ctx* ctx, const Level& L, Cx<R>* x, const Cx<R>* b, int nrhs, int color, bool half,
                      int64_t ld) {
  if (ld <= 0) ld = L.n();
  REQUIRE(ld >= L.n(), "Gauss-Seidel vectors need a stride of at least the level size");
  const int d = L.dofs;
  const int spb = std::max(1, 256 / d);
  const int64_t V = L.sites();
  const Cx<R>* A = std::is_same<R, float>::value ? (const Cx<R>*)L.A32.p : (const Cx<R>*)L.A64.p;
  const Cx<R>* Ai = std::is_same<R, float>::value ? (const Cx<R>*)L.Ainv32.p : (const Cx<R>*)L.Ainv64.p;
  const int even = (L.Lx % 2 == 0) ? 1 : 0;
  const int64_t nsites = even ? V / 2 : V;
  const int rb = rhs_block_for(nsites * d, nrhs);
  if (std::is_same<R, float>::value && d == 16) {
    // direct form: reads b and the neighbours' x, writes x (three vector passes over the
    // colour's sites) and the four hop blocks and the inverse self block
    REQUIRE(even && L.Lt % 2 == 0, "block Gauss-Seidel needs even extents");
    REQUIRE(((uintptr_t)x | (uintptr_t)b) % 16 == 0 && ld % 2 == 0,
            "matrix-core Gauss-Seidel needs 16-byte aligned vectors");
    const bool h16 = half && L.Ahop16.p && L.Ainv16.p;
    // built-in rule: vectors through whole-line loads and stores staged in LDS (measured at
    // 1024^2: level 2, 32768 sites per colour, 127 -> 118 us; level 3, 2048 sites, 11.4 ->
    // 10.3 us), and two wavefronts per site on the smallest launches (512 sites: 5.8 ->
    // 4.4 us)
    const int gs_form = L.kv[KV_GS_SPLIT] > 0 ? L.kv[KV_GS_SPLIT] : (nsites < 1024 ? 2 : 4);
    KTimer kt(ctx, "coarse_gs",
              (double)nrhs * (V / 2) * d * 3 * sizeof(Cx<R>) + (double)(V / 2) * 5 * d * d * (h16 ? 4 : sizeof(Cx<R>)));
    if (h16 && gs_form == 2)
      hipLaunchKernelGGL((coarse16_gs_mfma_kernel<true, 2>), dim3((unsigned)ceil_div(nsites * 2, 4)), dim3(256), 0,
                         ctx->stream, L.Ahop16.p, L.Ainv16.p, (c64*)x, (const c64*)b, L.Lx, L.Lt, nrhs, color, ld);
    else if (h16 && gs_form == 3)
      hipLaunchKernelGGL((coarse16_gs_mfma_kernel<true, 3>), dim3((unsigned)ceil_div(nsites, 4)), dim3(256), 0,
                         ctx->stream, L.Ahop16.p, L.Ainv16.p, (c64*)x, (const c64*)b, L.Lx, L.Lt, nrhs, color, ld);
    else if (h16 && gs_form == 4)
      hipLaunchKernelGGL(coarse16_gs_mfma_staged_kernel, dim3((unsigned)ceil_div(nsites, 4)), dim3(256), 0,
                         ctx->stream, L.Ahop16.p, L.Ainv16.p, (c64*)x, (const c64*)b, L.Lx, L.Lt, nrhs, color, ld);
    else if (h16)
      hipLaunchKernelGGL((coarse16_gs_mfma_kernel<true, 1>), dim3((unsigned)ceil_div(nsites, 4)), dim3(256), 0,
                         ctx->stream, L.Ahop16.p, L.Ainv16.p, (c64*)x, (const c64*)b, L.Lx, L.Lt, nrhs, color, ld);
    else
      hipLaunchKernelGGL((coarse16_gs_mfma_kernel<false, 1>), dim3((unsigned)ceil_div(nsites, 4)), dim3(256), 0,
                         ctx->stream, (const void*)A, (const void*)Ai, (c64*)x, (const c64*)b, L.Lx, L.Lt, nrhs,
                         color, ld);
    LAUNCH_CHECK();
    return;
  }
  KTimer kt(ctx, "coarse_gs",
            (double)nrhs * (V / 2) * d * 4 * sizeof(Cx<R>) + (double)(V / 2) * 6 * d * d * sizeof(Cx<R>));
  dim3 grid((unsigned)ceil_div(nsites, spb), (unsigned)ceil_div(nrhs, rb));
  dim3 block((unsigned)(spb * d));
  size_t shm = (size_t)spb * d * sizeof(Cx<R>);
  hipLaunchKernelGGL((coarse_gs_kernel<R>), grid, block, shm, ctx->stream, A, Ai, x, b, L.Lx, L.Lt, d, spb, nrhs,
                     rb, color, even, ld);
  LAUNCH_CHECK();
}

template <typename R>
void launch_restrict(dmlmc_ctx* ctx, const Level& L, const Cx<R>* xf, Cx<R>* yc, int nrhs, int64_t ldf,
                     int64_t ldc) {
  const Cx<R>* P = std::is_same<R, float>::value ? (const Cx<R>*)L.P32.p : (const Cx<R>*)L.P64.p;
  const int64_t Vc = (int64_t)(L.Lx / L.ax) * (L.Lt / L.at);
  const int64_t threads = Vc * 2 * L.N;
  if (ldf <= 0) ldf = L.n();
  if (ldc <= 0) ldc = threads;
  REQUIRE(ldf >= L.n() && ldc >= threads && ldf % 2 == 0 && ldc % 2 == 0,
          "restriction vectors need even strides of at least the level sizes");
  KTimer kt(ctx, "restrict",
            (double)nrhs * (L.n() + threads) * sizeof(Cx<R>) + (double)L.n() * L.N * sizeof(Cx<R>));
  if (std::is_same<R, float>::value && transfer16_ok(L)) {
    REQUIRE(((uintptr_t)xf | (uintptr_t)yc) % 16 == 0, "matrix-core restriction needs 16-byte aligned vectors");
    const AggMap g = agg_map(L);
    // rows of half a line: pairs of aggregates staged through LDS
    if (restrict16_pair_selected(L)) {
      const dim3 grid((unsigned)ceil_div(Vc / 2, 4));
      if (L.at == 4)
        hipLaunchKernelGGL(restrict16_pair_kernel<2>, grid, dim3(256), 0, ctx->stream, (const c64*)P, (const c64*)xf,
                           (c64*)yc, g, Vc, nrhs, ldf, ldc);
      else
        hipLaunchKernelGGL(restrict16_pair_kernel<1>, grid, dim3(256), 0, ctx->stream, (const c64*)P, (const c64*)xf,
                           (c64*)yc, g, Vc, nrhs, ldf, ldc);
      LAUNCH_CHECK();
      return;
    }
    const int wpa = g.E / 16 >= 4 ? 4 : 1;  // wavefronts per aggregate
    const dim3 grid((unsigned)ceil_div(Vc, 4 / wpa));
    // built-in rule (measured at 1024^2): one tile per batch of loads when an aggregate's
    // tiles are dealt to four wavefronts (level 2: 96 -> 78 us), else two
    const int ut = L.kv[KV_RESTRICT_UT] > 0 ? L.kv[KV_RESTRICT_UT] : (wpa == 4 ? 1 : 2);
    if (ut == 1)
      hipLaunchKernelGGL(restrict16_mfma_kernel<1>, grid, dim3(256), 0, ctx->stream, (const c64*)P, (const c64*)xf,
                         (c64*)yc, g, Vc, nrhs, wpa, ldf, ldc);
    else if (ut == 2)
      hipLaunchKernelGGL(restrict16_mfma_kernel<2>, grid, dim3(256), 0, ctx->stream, (const c64*)P, (const c64*)xf,
                         (c64*)yc, g, Vc, nrhs, wpa, ldf, ldc);
    else
      hipLaunchKernelGGL(restrict16_mfma_kernel<4>, grid, dim3(256), 0, ctx->stream, (const c64*)P, (const c64*)xf,
                         (c64*)yc, g, Vc, nrhs, wpa, ldf, ldc);
    LAUNCH_CHECK();
    return;
  }
  constexpr int RB = 4;
  dim3 grid((unsigned)ceil_div(threads, 256), (unsigned)ceil_div(nrhs, RB));
  hipLaunchKernelGGL((restrict_kernel<R, RB>), grid, dim3(256), 0, ctx->stream, P, xf, yc, L.Lx, L.Lt, L.dofs, L.ax,
                     L.at, L.N, nrhs, ldf, ldc);
  LAUNCH_CHECK();
}

template <typename R>
void launch_prolong(dmlmc_ctx* ctx, const Level& L, const Cx<R>* ec, Cx<R>* xf, int nrhs, bool add, int64_t ldc,
                    int64_t ldf) {
  const Cx<R>* P = std::is_same<R, float>::value ? (const Cx<R>*)L.P32.p : (const Cx<R>*)L.P64.p;
  const int64_t nf = L.n();
  const int64_t nc = (int64_t)(L.Lx / L.ax) * (L.Lt / L.at) * 2 * L.N;
  if (ldf <= 0) ldf = nf;
  if (ldc <= 0) ldc = nc;
  REQUIRE(ldf >= nf && ldc >= nc && ldf % 2 == 0 && ldc % 2 == 0,
          "prolongation vectors need even strides of at least the level sizes");
  KTimer kt(ctx, "prolong",
            (double)nrhs * ((add ? 2 : 1) * nf + nc) * sizeof(Cx<R>) + (double)nf * L.N * sizeof(Cx<R>));
  if (std::is_same<R, float>::value && transfer16_ok(L)) {
    REQUIRE(((uintptr_t)ec | (uintptr_t)xf) % 16 == 0, "matrix-core prolongation needs 16-byte aligned vectors");
    const AggMap g = agg_map(L);
    const int tiles = g.E / 16;
    const int tuned = L.kv[KV_PROLONG_MT];
    const int mtw = (tuned > 0 && tiles % tuned == 0) ? tuned
                                                      : (tiles % 4 == 0 ? std::min(4, tiles) : (tiles % 2 == 0 ? 2 : 1));
    const int64_t Vc = nc / 16;
    const dim3 grid((unsigned)ceil_div(Vc * (tiles / mtw), 4));
    // 16 dofs per fine site, or rows of half a line (pairs of aggregates): whole-line traffic
    // staged through LDS; built-in rule from 16384 fine sites on (measured at 1024^2: 256^2
    // sites, 95 -> 72 us; 64^2 sites, no gain)
    const bool staged = (L.dofs == 16 || transfer16_pair_ok(L)) && prolong_staged_rule(L);
    if (prolong16_pair_selected(L)) {
      const dim3 pgrid((unsigned)ceil_div(Vc / 2, 4));
      if (L.at == 8)
        hipLaunchKernelGGL(prolong16_pair_kernel<4>, pgrid, dim3(256), 0, ctx->stream, (const c64*)P, (const c64*)ec,
                           (c64*)xf, g, Vc, nrhs, add ? 1 : 0, ldf, ldc);
      else if (L.at == 4)
        hipLaunchKernelGGL(prolong16_pair_kernel<2>, pgrid, dim3(256), 0, ctx->stream, (const c64*)P, (const c64*)ec,
                           (c64*)xf, g, Vc, nrhs, add ? 1 : 0, ldf, ldc);
      else
        hipLaunchKernelGGL(prolong16_pair_kernel<1>, pgrid, dim3(256), 0, ctx->stream, (const c64*)P, (const c64*)ec,
                           (c64*)xf, g, Vc, nrhs, add ? 1 : 0, ldf, ldc);
      LAUNCH_CHECK();
      return;
    }
    if (staged) {
      if (mtw == 4)
        hipLaunchKernelGGL(prolong16_staged_kernel<4>, grid, dim3(256), 0, ctx->stream, (const c64*)P, (const c64*)ec,
                           (c64*)xf, g, Vc, nrhs, add ? 1 : 0, ldf, ldc);
      else if (mtw == 2)
        hipLaunchKernelGGL(prolong16_staged_kernel<2>, grid, dim3(256), 0, ctx->stream, (const c64*)P, (const c64*)ec,
                           (c64*)xf, g, Vc, nrhs, add ? 1 : 0, ldf, ldc);
      else
        hipLaunchKernelGGL(prolong16_staged_kernel<1>, grid, dim3(256), 0, ctx->stream, (const c64*)P, (const c64*)ec,
                           (c64*)xf, g, Vc, nrhs, add ? 1 : 0, ldf, ldc);
      LAUNCH_CHECK();
      return;
    }
    if (mtw == 4)
      hipLaunchKernelGGL(prolong16_mfma_kernel<4>, grid, dim3(256), 0, ctx->stream, (const c64*)P, (const c64*)ec,
                         (c64*)xf, g, Vc, nrhs, add ? 1 : 0, ldf, ldc);
    else if (mtw == 2)
      hipLaunchKernelGGL(prolong16_mfma_kernel<2>, grid, dim3(256), 0, ctx->stream, (const c64*)P, (const c64*)ec,
                         (c64*)xf, g, Vc, nrhs, add ? 1 : 0, ldf, ldc);
    else
      hipLaunchKernelGGL(prolong16_mfma_kernel<1>, grid, dim3(256), 0, ctx->stream, (const c64*)P, (const c64*)ec,
                         (c64*)xf, g, Vc, nrhs, add ? 1 : 0, ldf, ldc);
    LAUNCH_CHECK();
    return;
  }
  constexpr int RB = 4;
  dim3 grid((unsigned)ceil_div(nf, 256), (unsigned)ceil_div(nrhs, RB));
  hipLaunchKernelGGL((prolong_kernel<R, RB>), grid, dim3(256), 0, ctx->stream, P, ec, xf, L.Lx, L.Lt, L.dofs, L.ax,
                     L.at, L.N, nrhs, add ? 1 : 0, ldf, ldc);
  LAUNCH_CHECK();
}

#define INST(R)                                                                                                  \
  template void launch_wilson<R>(dmlmc_ctx*, const Level&, const Cx<R>*, Cx<R>*, int, int64_t, int64_t, bool,     \
                                 const Cx<R>*);                                                                  \
  template void launch_coarse<R>(dmlmc_ctx*, const Level&, const Cx<R>*, Cx<R>*, int, int64_t, int64_t, bool,     \
                                 const Cx<R>*);                                                                  \
  template void apply_op<R>(dmlmc_ctx*, const Level&, const Cx<R>*, Cx<R>*, int, bool, int64_t);               \
  template void apply_residual<R>(dmlmc_ctx*, const Level&, const Cx<R>*, const Cx<R>*, Cx<R>*, int);          \
  template void launch_sap<R>(dmlmc_ctx*, const Level&, Cx<R>*, const Cx<R>*, int, int, int, int64_t);         \
  template void launch_coarse_gs<R>(dmlmc_ctx*, const Level&, Cx<R>*, const Cx<R>*, int, int, bool, int64_t);  \
  template void launch_restrict<R>(dmlmc_ctx*, const Level&, const Cx<R>*, Cx<R>*, int, int64_t, int64_t);     \
  template void launch_prolong<R>(dmlmc_ctx*, const Level&, const Cx<R>*, Cx<R>*, int, bool, int64_t, int64_t);
INST(float)
INST(double)
