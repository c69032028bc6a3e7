// Gram-Schmidt passes of the Arnoldi step, FP64 arithmetic.
//
// Two-pass form (classical Gram-Schmidt with one reorthogonalisation, FP64 basis):
//   A: h1 = V^H w                        (read V, w)
//   B: w' = w - V h1, ||w'||^2            (read V, w; write w')
//   C: h2 = V^H w', Hessenberg column, Givens rotation, residual estimate
//   D: v_{j+1} = (w' - V h2) / beta, beta^2 = ||w'||^2 - |h2|^2
// Single-pass form (complex-FP32 cycles: unnormalised FP32 basis u_i, scales s_i = 1/||u_i||):
//   A: h_i = s_i <u_i, w>                (read U, w)
//   B: u_{j+1} = w - sum_i h_i s_i u_i, ||u_{j+1}||^2, Hessenberg column, Givens, s_{j+1}
//
// Small vectors (n <= 16384, the coarsest levels) take the single-pass step in one
// 1024-thread workgroup per RHS: dots, reduction, update, norm and the Givens step in
// one launch, the basis re-read from L2.
//
// Reductions: each workgroup reduces in LDS; with one workgroup per RHS the workgroup
// finishes the pass itself, otherwise it writes partial sums and a small kernel (one
// workgroup per RHS) adds them in a fixed order.  No atomics or device-scope fences.
#include <cmath>

#include "solver.h"

namespace {

constexpr int NBMAX = 32;         // basis vectors per pass
constexpr int NVMAX = 2 * NBMAX;  // reduced doubles per pass

enum FinishMode { FIN_STORE = 0, FIN_SCALED = 1, FIN_CGS2 = 2, FIN_CGS1 = 3 };

struct Fin {
  int mode = FIN_STORE;
  int j = 0, m = 0, hld = 0, nrhs = 0;
  double* out = nullptr;        // FIN_STORE: nv doubles per RHS at out + r * ostride
  int ostride = 0;
  const c128* h1 = nullptr;     // FIN_CGS2: first-pass coefficients; FIN_CGS1: the coefficients
  c128* h = nullptr;            // FIN_SCALED / FIN_CGS2: where the (scaled) coefficients go
  double* scale = nullptr;      // FIN_SCALED / FIN_CGS1: [i][nrhs]
  const double* nrm2 = nullptr; // FIN_CGS2: ||w'||^2
  c128* H = nullptr;
  double* cs = nullptr;
  c128* sn = nullptr;
  c128* g = nullptr;
  double* res = nullptr;
  double* invb = nullptr;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// acc[0..nv) summed over the 256-thread block into red[0..nv) (LDS); all threads return
// after red is complete.
template <int NV>
__device__ void block_reduce(const double (&acc)[NV], int nv, double* lds /* [4][NVMAX] */, double* red) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    if (q < nv) {
      const double v = wave_sum(acc[q]);
      if (l == 0) lds[w * NVMAX + q] = v;
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nv; q += blockDim.x)
    red[q] = lds[q] + lds[NVMAX + q] + lds[2 * NVMAX + q] + lds[3 * NVMAX + q];
  __syncthreads();
}

// Hessenberg column j (col rows 0..j hold the Gram-Schmidt coefficients) and beta:
// previous rotations, a new rotation, g and the residual estimate.
__device__ void hessenberg_update(const Fin& f, int r, double beta) {
  const int m = f.m, j = f.j;
  c128* col = f.H + (int64_t)r * (m + 1) * m + (int64_t)j * (m + 1);
  for (int i = 0; i < j; ++i) {
    const double c = f.cs[r * m + i];
    const c128 s = f.sn[r * m + i];
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
  f.cs[r * m + j] = c;
  f.sn[r * m + j] = s;
  c128* gr = f.g + (int64_t)r * (m + 1);
  const c128 gj = gr[j];
  gr[j + 1] = cmk(-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x));  // -conj(s) g_j
  gr[j] = c * gj;
  f.res[r] = sqrt(cabs2(gr[j + 1]));
}

// Completes a pass for RHS r from the reduced sums red[0..nv) (whole block calls it).
__device__ void finish_pass(const Fin& f, int r, int nv, const double* red) {
  const int nb = f.j + 1;
  switch (f.mode) {
    case FIN_STORE:
      for (int q = threadIdx.x; q < nv; q += blockDim.x) f.out[(int64_t)r * f.ostride + q] = red[q];
      break;
    case FIN_SCALED:
      for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        const double sc = f.scale[(int64_t)i * f.nrhs + r];
        f.h[(int64_t)r * f.hld + i] = cmk(red[2 * i] * sc, red[2 * i + 1] * sc);
      }
      break;
    case FIN_CGS2:
      if (threadIdx.x == 0) {
        c128* col = f.H + (int64_t)r * (f.m + 1) * f.m + (int64_t)f.j * (f.m + 1);
        double h2n = 0.0;
        for (int i = 0; i < nb; ++i) {
          const c128 b2 = cmk(red[2 * i], red[2 * i + 1]);
          h2n += b2.x * b2.x + b2.y * b2.y;
          f.h[(int64_t)r * f.hld + i] = b2;
          col[i] = f.h1[(int64_t)r * f.hld + i] + b2;
        }
        const double beta = sqrt(fmax(f.nrm2[r] - h2n, 0.0));
        hessenberg_update(f, r, beta);
        f.invb[r] = beta > 0.0 ? 1.0 / beta : 0.0;
      }
      break;
    case FIN_CGS1:
      if (threadIdx.x == 0) {
        const double beta = sqrt(fmax(red[0], 0.0));
        f.scale[(int64_t)nb * f.nrhs + r] = beta > 0.0 ? 1.0 / beta : 0.0;
        c128* col = f.H + (int64_t)r * (f.m + 1) * f.m + (int64_t)f.j * (f.m + 1);
        for (int i = 0; i < nb; ++i) col[i] = f.h1[(int64_t)r * f.hld + i];
        hessenberg_update(f, r, beta);
      }
      break;
  }
}

// Block reduce, then either finish (one workgroup per RHS) or write partials.
template <int NV>
__device__ void reduce_or_partial(const double (&acc)[NV], int nv, double* lds, double* red, double* __restrict__ part,
                                  const Fin& f, int r) {
  block_reduce(acc, nv, lds, red);
  if (gridDim.x == 1) {
    finish_pass(f, r, nv, red);
  } else {
    double* pr = part + ((int64_t)r * gridDim.x + blockIdx.x) * nv;
    for (int q = threadIdx.x; q < nv; q += blockDim.x) pr[q] = red[q];
  }
}

// One wavefront per RHS: lane l adds the partials of blocks l, l + 64, ... into four
// running sums (blocks l + 256 i + 64 u go to sum u, so that four loads are in flight and
// no add waits on the previous one), then the wavefront sums across lanes.
__global__ __launch_bounds__(64) void partial_finish_kernel(const double* __restrict__ part, int G, int nv, Fin f) {
  __shared__ double red[NVMAX];
  const int r = blockIdx.x, l = threadIdx.x;
  const double* base = part + (int64_t)r * G * nv;
  for (int q = 0; q < nv; ++q) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int g = l;
    for (; g + 192 < G; g += 256) {
      s0 += base[(int64_t)g * nv + q];
      s1 += base[(int64_t)(g + 64) * nv + q];
      s2 += base[(int64_t)(g + 128) * nv + q];
      s3 += base[(int64_t)(g + 192) * nv + q];
    }
    for (; g < G; g += 64) s0 += base[(int64_t)g * nv + q];
    double s = (s0 + s1) + (s2 + s3);
    s = wave_sum(s);
    if (l == 0) red[q] = s;
  }
  __syncthreads();
  finish_pass(f, r, nv, red);
}

template <typename R>
struct __align__(4 * sizeof(R)) Pair {
  Cx<R> a, b;
};

// ---------------------------------------------------------------- two-pass form kernels
template <typename RV>
__global__ __launch_bounds__(256) void gs_dots_kernel(const Cx<RV>* __restrict__ V, int nb, const c128* __restrict__ w,
                                                      int64_t n, int64_t vstride, double* __restrict__ part, Fin f) {
  __shared__ double lds[4 * NVMAX];
  __shared__ double red[NVMAX];
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
  reduce_or_partial(acc, 2 * nb, lds, red, part, f, r);
}

template <typename RV>
__global__ __launch_bounds__(256) void gs_update_norm_kernel(const Cx<RV>* __restrict__ V, int nb,
                                                             c128* __restrict__ w, int64_t n, int64_t vstride,
                                                             const c128* __restrict__ h, int hld,
                                                             double* __restrict__ part, Fin f) {
  __shared__ double lds[4 * NVMAX];
  __shared__ double red[NVMAX];
  __shared__ c128 hs[NBMAX];
  const int r = blockIdx.y;
  if (threadIdx.x < nb) hs[threadIdx.x] = h[(int64_t)r * hld + threadIdx.x];
  __syncthreads();
  double acc[1] = {0.0};
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
  reduce_or_partial(acc, 1, lds, red, part, f, r);
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

// ---------------------------------------------------------------- single-pass form kernels
// UNR element pairs per thread and pass: their loads are all issued before the first
// product, and each pair's terms are added in the order of the pairs (the sums do not
// depend on UNR; at 1024^2, four pairs per pass against one: dots 15.1 -> 14.6 ms and
// updates 20.7 -> 20.0 ms per estimate).
template <typename RW, int NBT, int UNR>
__global__ __launch_bounds__(256) void gs1_dots_kernel(const c64* __restrict__ U, int nb,
                                                       const Cx<RW>* __restrict__ w, int64_t n, int64_t vstride,
                                                       const double* __restrict__ wscale, double* __restrict__ part,
                                                       Fin f, int64_t ld) {
  __shared__ double lds[4 * NVMAX];
  __shared__ double red[NVMAX];
  const int r = blockIdx.y;
  const double ws = wscale ? wscale[r] : 1.0;
  double acc[2 * NBT];
#pragma unroll
  for (int q = 0; q < 2 * NBT; ++q) acc[q] = 0.0;
  // element pairs (n is even): 16-byte loads of the FP32 basis
  const Pair<RW>* wr = reinterpret_cast<const Pair<RW>*>(w + (int64_t)r * ld);
  const Pair<float>* Ur = reinterpret_cast<const Pair<float>*>(U + (int64_t)r * ld);
  const int64_t np = n / 2, vs = vstride / 2, S = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += UNR * S) {
    Pair<RW> bw[UNR];
    Pair<float> u[UNR][NBT];
#pragma unroll
    for (int k = 0; k < UNR; ++k) {
      const int64_t q = p + k * S < np ? p + k * S : p;
      bw[k] = wr[q];
#pragma unroll
      for (int i = 0; i < NBT; ++i)
        if (i < nb) u[k][i] = Ur[i * vs + q];
    }
#pragma unroll
    for (int k = 0; k < UNR; ++k) {
      if (p + k * S < np) {
        const double b0x = ws * bw[k].a.x, b0y = ws * bw[k].a.y, b1x = ws * bw[k].b.x, b1y = ws * bw[k].b.y;
#pragma unroll
        for (int i = 0; i < NBT; ++i) {
          if (i < nb) {
            const Pair<float> ui = u[k][i];
            acc[2 * i] += (double)ui.a.x * b0x + (double)ui.a.y * b0y + (double)ui.b.x * b1x + (double)ui.b.y * b1y;
            acc[2 * i + 1] += (double)ui.a.x * b0y - (double)ui.a.y * b0x + (double)ui.b.x * b1y - (double)ui.b.y * b1x;
          }
        }
      }
    }
  }
  reduce_or_partial(acc, 2 * nb, lds, red, part, f, r);
}

template <typename RW, int NBT, int UNR>
__global__ __launch_bounds__(256) void gs1_update_kernel(c64* __restrict__ U, int nb, const Cx<RW>* __restrict__ w,
                                                         int64_t n, int64_t vstride, const c128* __restrict__ h,
                                                         int hld, const double* __restrict__ scale, int nrhs,
                                                         const double* __restrict__ wscale, double* __restrict__ part,
                                                         Fin f, int64_t ld) {
  __shared__ double lds[4 * NVMAX];
  __shared__ double red[NVMAX];
  __shared__ c128 hs[NBMAX];
  const int r = blockIdx.y;
  const double ws = wscale ? wscale[r] : 1.0;
  if (threadIdx.x < nb) {
    const c128 hv = h[(int64_t)r * hld + threadIdx.x];
    const double sc = scale[(int64_t)threadIdx.x * nrhs + r];
    hs[threadIdx.x] = cmk(hv.x * sc, hv.y * sc);
  }
  __syncthreads();
  double acc[1] = {0.0};
  const Pair<RW>* wr = reinterpret_cast<const Pair<RW>*>(w + (int64_t)r * ld);
  const Pair<float>* Ur = reinterpret_cast<const Pair<float>*>(U + (int64_t)r * ld);
  Pair<float>* out = reinterpret_cast<Pair<float>*>(U + (int64_t)nb * vstride + (int64_t)r * ld);
  const int64_t np = n / 2, vs = vstride / 2, S = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += UNR * S) {
    Pair<RW> bw[UNR];
    Pair<float> u[UNR][NBT];
#pragma unroll
    for (int k = 0; k < UNR; ++k) {
      const int64_t q = p + k * S < np ? p + k * S : p;
      bw[k] = wr[q];
#pragma unroll
      for (int i = 0; i < NBT; ++i)
        if (i < nb) u[k][i] = Ur[i * vs + q];
    }
#pragma unroll
    for (int k = 0; k < UNR; ++k) {
      if (p + k * S < np) {
        double v0x = ws * bw[k].a.x, v0y = ws * bw[k].a.y, v1x = ws * bw[k].b.x, v1y = ws * bw[k].b.y;
#pragma unroll
        for (int i = 0; i < NBT; ++i) {
          if (i < nb) {
            const Pair<float> ui = u[k][i];
            const c128 hi = hs[i];
            v0x -= hi.x * (double)ui.a.x - hi.y * (double)ui.a.y;
            v0y -= hi.x * (double)ui.a.y + hi.y * (double)ui.a.x;
            v1x -= hi.x * (double)ui.b.x - hi.y * (double)ui.b.y;
            v1y -= hi.x * (double)ui.b.y + hi.y * (double)ui.b.x;
          }
        }
        Pair<float> st;
        st.a = cmk((float)v0x, (float)v0y);
        st.b = cmk((float)v1x, (float)v1y);
        out[p + k * S] = st;
        acc[0] += (double)st.a.x * st.a.x + (double)st.a.y * st.a.y + (double)st.b.x * st.b.x + (double)st.b.y * st.b.y;
      }
    }
  }
  reduce_or_partial(acc, 1, lds, red, part, f, r);
}

// Sums v[0..15] over the 64 lanes of a wavefront by recursive halving: at each exchange a
// lane keeps half of its values and adds the partner's copy of that half (17 shuffles
// instead of 96).  Lane l ends with the total of value (l >> 2) & 15 in v[0].
__device__ __forceinline__ void wave_sum16(double (&v)[16]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int step = 0; step < 4; ++step) {
    const int half = 8 >> step;
    const int mask = 32 >> step;
    const bool hi = (lane & mask) != 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (i < half) {
        const double a = v[i], b = v[half + i];
        const double send = hi ? a : b;
        const double recv = __shfl_xor(send, mask, 64);
        v[i] = (hi ? b : a) + recv;
      }
    }
  }
  v[0] += __shfl_xor(v[0], 2, 64);
  v[0] += __shfl_xor(v[0], 1, 64);
}

// Whole single-pass step for RHS blockIdx.x in one workgroup of 1024 threads; element
// pair p of the vectors belongs to thread p % 1024 (PPT pairs per thread, n <= 2048 PPT).
constexpr int FUSED_THREADS = 1024;
constexpr int FUSED_PPT = 8;
constexpr int FUSED_CHUNK = 8;  // basis vectors per reduction round (16 doubles: wave_sum16)

template <typename RW>
__global__ __launch_bounds__(FUSED_THREADS) void gs1_fused_kernel(c64* __restrict__ U, int nb,
                                                                  const Cx<RW>* __restrict__ w, int64_t n,
                                                                  int64_t vstride, const double* __restrict__ wscale,
                                                                  Fin f, int64_t ld) {
  constexpr int NW = FUSED_THREADS / 64;
  __shared__ double lds[NW][2 * FUSED_CHUNK];
  __shared__ double red[NVMAX];
  __shared__ c128 cf[NBMAX];  // h_i s_i, the coefficients of the unnormalised u_i
  const int r = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nrhs = f.nrhs;
  const double ws = wscale ? wscale[r] : 1.0;
  const int64_t np = n / 2, vs = vstride / 2;
  const Pair<RW>* wr = reinterpret_cast<const Pair<RW>*>(w + (int64_t)r * ld);
  const Pair<float>* Ur = reinterpret_cast<const Pair<float>*>(U + (int64_t)r * ld);
  // h_i = s_i <u_i, ws w>, FUSED_CHUNK basis vectors per reduction round (w is re-read
  // from L2 per round rather than held in registers)
  for (int c0 = 0; c0 < nb; c0 += FUSED_CHUNK) {
    double acc[2 * FUSED_CHUNK];
#pragma unroll
    for (int q = 0; q < 2 * FUSED_CHUNK; ++q) acc[q] = 0.0;
#pragma unroll 2
    for (int q = 0; q < FUSED_PPT; ++q) {
      const int64_t p = tid + (int64_t)q * FUSED_THREADS;
      if (p < np) {
        const Pair<RW> b = wr[p];
#pragma unroll
        for (int i = 0; i < FUSED_CHUNK; ++i) {
          if (c0 + i < nb) {
            const Pair<float> u = Ur[(c0 + i) * vs + p];
            acc[2 * i] += (double)u.a.x * b.a.x + (double)u.a.y * b.a.y + (double)u.b.x * b.b.x +
                          (double)u.b.y * b.b.y;
            acc[2 * i + 1] += (double)u.a.x * b.a.y - (double)u.a.y * b.a.x + (double)u.b.x * b.b.y -
                              (double)u.b.y * b.b.x;
          }
        }
      }
    }
    wave_sum16(acc);
    if ((lane & 3) == 0) lds[wv][(lane >> 2) & 15] = acc[0];
    __syncthreads();
    if (tid < 2 * FUSED_CHUNK && c0 + tid / 2 < nb) {
      double sum = 0.0;
      for (int k = 0; k < NW; ++k) sum += lds[k][tid];
      red[2 * c0 + tid] = sum;
    }
    __syncthreads();
  }
  if (tid < nb) {
    const double sc = f.scale[(int64_t)tid * nrhs + r];
    const c128 h = cmk(ws * sc * red[2 * tid], ws * sc * red[2 * tid + 1]);
    f.h[(int64_t)r * f.hld + tid] = h;
    cf[tid] = cmk(h.x * sc, h.y * sc);
  }
  __syncthreads();
  // u_{j+1} = ws w - sum_i (h_i s_i) u_i, its norm from the stored FP32 values
  Pair<float>* out = reinterpret_cast<Pair<float>*>(U + (int64_t)nb * vstride + (int64_t)r * ld);
  double nrm = 0.0;
#pragma unroll
  for (int q = 0; q < FUSED_PPT; ++q) {
    const int64_t p = tid + (int64_t)q * FUSED_THREADS;
    if (p < np) {
      const Pair<RW> b = wr[p];
      double v0x = ws * b.a.x, v0y = ws * b.a.y, v1x = ws * b.b.x, v1y = ws * b.b.y;
      for (int i = 0; i < nb; ++i) {
        const Pair<float> u = Ur[i * vs + p];
        const c128 hi = cf[i];
        v0x -= hi.x * (double)u.a.x - hi.y * (double)u.a.y;
        v0y -= hi.x * (double)u.a.y + hi.y * (double)u.a.x;
        v1x -= hi.x * (double)u.b.x - hi.y * (double)u.b.y;
        v1y -= hi.x * (double)u.b.y + hi.y * (double)u.b.x;
      }
      Pair<float> st;
      st.a = cmk((float)v0x, (float)v0y);
      st.b = cmk((float)v1x, (float)v1y);
      out[p] = st;
      nrm += (double)st.a.x * st.a.x + (double)st.a.y * st.a.y + (double)st.b.x * st.b.x + (double)st.b.y * st.b.y;
    }
  }
  nrm = wave_sum(nrm);
  if (lane == 0) lds[wv][0] = nrm;
  __syncthreads();
  if (tid == 0) {
    double sum = 0.0;
    for (int k = 0; k < NW; ++k) sum += lds[k][0];
    const double beta = sqrt(fmax(sum, 0.0));
    f.scale[(int64_t)nb * nrhs + r] = beta > 0.0 ? 1.0 / beta : 0.0;
    c128* col = f.H + (int64_t)r * (f.m + 1) * f.m + (int64_t)f.j * (f.m + 1);
    for (int i = 0; i < nb; ++i) col[i] = f.h[(int64_t)r * f.hld + i];
    hessenberg_update(f, r, beta);
  }
}

// Workgroups per RHS: about 8 element pairs per thread (two passes of four), at most
// 16384 / nrhs in total (bounds the partial sums; at 1024^2 against 16 pairs and 2048 in
// total: dots and updates 34.3 -> 33.1 ms per estimate).  One workgroup per RHS finishes
// the pass in the same launch.
int gs_blocks(int64_t n, int nrhs) {
  nrhs = std::max(1, nrhs);
  int64_t g = ceil_div(n, 2 * 256 * 8);
  g = std::min<int64_t>(g, std::max(1, 16384 / nrhs));
  return (int)std::max<int64_t>(1, g);
}

void launch_partial_finish(dmlmc_ctx* ctx, const double* part, int G, int nv, const Fin& f, int nrhs) {
  if (G <= 1) return;
  hipLaunchKernelGGL(partial_finish_kernel, dim3(nrhs), dim3(64), 0, ctx->stream, part, G, nv, f);
  LAUNCH_CHECK();
}

Fin base_fin(const KrylovArrays& k, int j, int nrhs) {
  Fin f;
  f.j = j;
  f.m = k.m;
  f.hld = k.hld;
  f.nrhs = nrhs;
  f.H = k.H;
  f.cs = k.cs;
  f.sn = k.sn;
  f.g = k.g;
  f.res = k.res;
  f.invb = k.invb;
  return f;
}

}  // namespace

int gs_max_basis() { return NBMAX; }

// One Arnoldi step, two-pass form: orthogonalise w (FP64, [nrhs][n]) against V_0..V_j,
// update the Hessenberg column and rotations, store V_{j+1} = w / ||w||.
template <typename RV>
void arnoldi_step(dmlmc_ctx* ctx, Cx<RV>* V, c128* w, int j, int64_t n, int nrhs, const KrylovArrays& k) {
  const int nb = j + 1;
  if (nb > NBMAX) throw DmlmcError(DMLMC_EINVAL, "Krylov basis larger than the Gram-Schmidt limit");
  const int64_t vstride = (int64_t)nrhs * n;
  const int G = gs_blocks(2 * n, nrhs);  // one element per thread and iteration here
  ctx->scratch_dots.ensure(sizeof(double) * (size_t)nrhs * G * NVMAX);
  double* part = ctx->scratch_dots.as<double>();
  dim3 grid(G, nrhs);
  Fin fa = base_fin(k, j, nrhs);
  fa.mode = FIN_STORE;
  fa.out = (double*)k.h1;
  fa.ostride = 2 * k.hld;
  {
    KTimer kt(ctx, "gs_dots", (double)nrhs * n * (nb * sizeof(Cx<RV>) + sizeof(c128)));
    hipLaunchKernelGGL((gs_dots_kernel<RV>), grid, dim3(256), 0, ctx->stream, V, nb, w, n, vstride, part, fa);
    LAUNCH_CHECK();
    launch_partial_finish(ctx, part, G, 2 * nb, fa, nrhs);
  }
  Fin fb = base_fin(k, j, nrhs);
  fb.mode = FIN_STORE;
  fb.out = k.nrm2;
  fb.ostride = 1;
  {
    KTimer kt(ctx, "gs_update", (double)nrhs * n * (nb * sizeof(Cx<RV>) + 2 * sizeof(c128)));
    hipLaunchKernelGGL((gs_update_norm_kernel<RV>), grid, dim3(256), 0, ctx->stream, V, nb, w, n, vstride, k.h1,
                       k.hld, part, fb);
    LAUNCH_CHECK();
    launch_partial_finish(ctx, part, G, 1, fb, nrhs);
  }
  Fin fc = base_fin(k, j, nrhs);
  fc.mode = FIN_CGS2;
  fc.h1 = k.h1;
  fc.h = k.h2;
  fc.nrm2 = k.nrm2;
  {
    KTimer kt(ctx, "gs_dots", (double)nrhs * n * (nb * sizeof(Cx<RV>) + sizeof(c128)));
    hipLaunchKernelGGL((gs_dots_kernel<RV>), grid, dim3(256), 0, ctx->stream, V, nb, w, n, vstride, part, fc);
    LAUNCH_CHECK();
    launch_partial_finish(ctx, part, G, 2 * nb, fc, nrhs);
  }
  {
    KTimer kt(ctx, "gs_update", (double)nrhs * n * (nb * sizeof(Cx<RV>) + sizeof(c128) + sizeof(Cx<RV>)));
    hipLaunchKernelGGL((gs_update_store_kernel<RV>), grid, dim3(256), 0, ctx->stream, V, nb, w, n, vstride, k.h2,
                       k.hld, k.invb);
    LAUNCH_CHECK();
  }
}

// One Arnoldi step, single-pass form on an unnormalised complex-FP32 basis.
int64_t gs_fused_max_n() { return 2 * (int64_t)FUSED_THREADS * FUSED_PPT; }

double* gs_partials(dmlmc_ctx* ctx, int64_t n, int nrhs, int extra_G) {
  const int G = std::max(gs_blocks(n, nrhs), extra_G);
  ctx->scratch_dots.ensure(sizeof(double) * (size_t)nrhs * G * NVMAX);
  return ctx->scratch_dots.as<double>();
}

template <typename RW>
void arnoldi_step_cgs1(dmlmc_ctx* ctx, c64* U, double* scale, const Cx<RW>* w, int j, int64_t n, int nrhs,
                       const KrylovArrays& k, const double* wscale, int64_t ld, int dots_G) {
  const int nb = j + 1;
  if (nb > NBMAX) throw DmlmcError(DMLMC_EINVAL, "Krylov basis larger than the Gram-Schmidt limit");
  if (ld <= 0) ld = n;
  REQUIRE(ld >= n && ld % 2 == 0, "Gram-Schmidt vectors need an even stride of at least their length");
  const int64_t vstride = (int64_t)nrhs * ld;
  if (n <= 2 * (int64_t)FUSED_THREADS * FUSED_PPT) {
    Fin f = base_fin(k, j, nrhs);
    f.mode = FIN_CGS1;
    f.h = k.h1;
    f.scale = scale;
    KTimer kt(ctx, "gs_fused", (double)nrhs * n * ((2 * nb + 1) * sizeof(c64) + sizeof(Cx<RW>)));
    hipLaunchKernelGGL((gs1_fused_kernel<RW>), dim3(nrhs), dim3(FUSED_THREADS), 0, ctx->stream, U, nb, w, n, vstride,
                       wscale, f, ld);
    LAUNCH_CHECK();
    return;
  }
  const int G = gs_blocks(n, nrhs);
  double* part = gs_partials(ctx, n, nrhs, dots_G);
  dim3 grid(G, nrhs);
  Fin fa = base_fin(k, j, nrhs);
  fa.mode = FIN_SCALED;
  fa.h = k.h1;
  fa.scale = scale;
  if (dots_G > 0) {
    // the dots were formed with w (launch_wilson_dots): only their partial sums remain
    KTimer kt(ctx, "gs_dots", 0.0);
    launch_partial_finish(ctx, part, dots_G, 2 * nb, fa, nrhs);
  } else {
    KTimer kt(ctx, "gs_dots", (double)nrhs * n * (nb * sizeof(c64) + sizeof(Cx<RW>)));
    // the basis count rounded up to 4, 8, 16 or 32 sizes the registers (and occupancy)
    if (nb <= 4)
      hipLaunchKernelGGL((gs1_dots_kernel<RW, 4, 4>), grid, dim3(256), 0, ctx->stream, U, nb, w, n, vstride, wscale, part,
                         fa, ld);
    else if (nb <= 8)
      hipLaunchKernelGGL((gs1_dots_kernel<RW, 8, 2>), grid, dim3(256), 0, ctx->stream, U, nb, w, n, vstride, wscale, part,
                         fa, ld);
    else if (nb <= 16)
      hipLaunchKernelGGL((gs1_dots_kernel<RW, 16, 1>), grid, dim3(256), 0, ctx->stream, U, nb, w, n, vstride, wscale,
                         part, fa, ld);
    else
      hipLaunchKernelGGL((gs1_dots_kernel<RW, NBMAX, 1>), grid, dim3(256), 0, ctx->stream, U, nb, w, n, vstride, wscale,
                         part, fa, ld);
    LAUNCH_CHECK();
    launch_partial_finish(ctx, part, G, 2 * nb, fa, nrhs);
  }
  Fin fb = base_fin(k, j, nrhs);
  fb.mode = FIN_CGS1;
  fb.h1 = k.h1;
  fb.scale = scale;
  {
    KTimer kt(ctx, "gs_update", (double)nrhs * n * ((nb + 1) * sizeof(c64) + sizeof(Cx<RW>)));
#define GS1_UPDATE(NBT, UNR)                                                                                      \
  hipLaunchKernelGGL((gs1_update_kernel<RW, NBT, UNR>), grid, dim3(256), 0, ctx->stream, U, nb, w, n, vstride, k.h1, \
                     k.hld, scale, nrhs, wscale, part, fb, ld)
    if (nb <= 4)
      GS1_UPDATE(4, 4);
    else if (nb <= 8)
      GS1_UPDATE(8, 2);
    else if (nb <= 16)
      GS1_UPDATE(16, 1);
    else
      GS1_UPDATE(NBMAX, 1);
#undef GS1_UPDATE
    LAUNCH_CHECK();
    launch_partial_finish(ctx, part, G, 1, fb, nrhs);
  }
}

template void arnoldi_step<double>(dmlmc_ctx*, c128*, c128*, int, int64_t, int, const KrylovArrays&);
template void arnoldi_step<float>(dmlmc_ctx*, c64*, c128*, int, int64_t, int, const KrylovArrays&);
template void arnoldi_step_cgs1<float>(dmlmc_ctx*, c64*, double*, const c64*, int, int64_t, int, const KrylovArrays&,
                                       const double*, int64_t, int);
template void arnoldi_step_cgs1<double>(dmlmc_ctx*, c64*, double*, const c128*, int, int64_t, int,
                                        const KrylovArrays&, const double*, int64_t, int);
