// Internal declarations of the dmlmc library (host + device).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstring>
#include <initializer_list>
#include <map>
#include <set>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "dmlmc.h"

// ------------------------------------------------------------------ complex arithmetic
template <typename R>
struct __align__(2 * sizeof(R)) Cx {
  R x, y;
};
using c64 = Cx<float>;
using c128 = Cx<double>;

template <typename R>
__host__ __device__ __forceinline__ Cx<R> cmk(R a, R b) {
  Cx<R> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename R>
__host__ __device__ __forceinline__ Cx<R> operator+(Cx<R> a, Cx<R> b) { return cmk(a.x + b.x, a.y + b.y); }
template <typename R>
__host__ __device__ __forceinline__ Cx<R> operator-(Cx<R> a, Cx<R> b) { return cmk(a.x - b.x, a.y - b.y); }
template <typename R>
__host__ __device__ __forceinline__ Cx<R> operator*(Cx<R> a, Cx<R> b) {
  return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename R>
__host__ __device__ __forceinline__ Cx<R> operator*(R s, Cx<R> a) { return cmk(s * a.x, s * a.y); }
template <typename R>
__host__ __device__ __forceinline__ Cx<R> conj(Cx<R> a) { return cmk(a.x, -a.y); }
// conj(a) * b
template <typename R>
__host__ __device__ __forceinline__ Cx<R> cdot(Cx<R> a, Cx<R> b) {
  return cmk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// acc += a * b
template <typename R>
__host__ __device__ __forceinline__ void cfma(Cx<R>& acc, Cx<R> a, Cx<R> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
template <typename R>
__host__ __device__ __forceinline__ void cfmac(Cx<R>& acc, Cx<R> a, Cx<R> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}
template <typename R>
__host__ __device__ __forceinline__ double cabs2(Cx<R> a) {
  return (double)a.x * (double)a.x + (double)a.y * (double)a.y;
}
template <typename To, typename From>
__host__ __device__ __forceinline__ Cx<To> ccast(Cx<From> a) {
  return cmk((To)a.x, (To)a.y);
}

// ------------------------------------------------------------------ errors
struct DmlmcError : std::runtime_error {
  dmlmc_status status;
  DmlmcError(dmlmc_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define HIPCHK(expr)                                                                          \
  do {                                                                                        \
    hipError_t _e = (expr);                                                                   \
    if (_e != hipSuccess)                                                                     \
      throw DmlmcError(_e == hipErrorOutOfMemory ? DMLMC_ENOMEM : DMLMC_EHIP,                 \
                       std::string(#expr) + ": " + hipGetErrorString(_e) + " at " __FILE__ ":" + \
                           std::to_string(__LINE__));                                         \
  } while (0)

#define REQUIRE(cond, msg)                                                  \
  do {                                                                      \
    if (!(cond)) throw DmlmcError(DMLMC_EINVAL, std::string("invalid argument: ") + (msg)); \
  } while (0)

#define LAUNCH_CHECK() HIPCHK(hipGetLastError())

// ------------------------------------------------------------------ device memory
// Bumped by every device allocation and free: a recorded HIP graph made before a bump may
// hold pointers to memory that has moved, and is re-recorded.
inline std::atomic<uint64_t> g_dev_epoch{0};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(size_t b) { alloc(b); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t b) {
    release();
    if (b == 0) return;
    HIPCHK(hipMalloc(&p, b));
    bytes = b;
    ++g_dev_epoch;
  }
  // grows (never shrinks); contents are not preserved
  void ensure(size_t b) { if (b > bytes) alloc(b); }
  void release() { if (p) { (void)hipFree(p); p = nullptr; bytes = 0; ++g_dev_epoch; } }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

// ------------------------------------------------------------------ timing of kernel classes
struct TimerClass {
  int64_t launches = 0;
  double ms = 0.0;
  double bytes = 0.0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  std::vector<double> pending_bytes;
  std::vector<int64_t> pending_launches;
};

struct dmlmc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  bool timing = false;
  int verbose = 0;  // > 0: long phases (eigensolver iterations) print progress lines to stderr
  std::set<std::string> timing_only;  // empty: every class
  std::map<std::string, TimerClass> timers;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> event_pool;
  DevBuf scratch_dots;   // reduction partials
  DevBuf scratch_small;  // small per-RHS device results
  void* noalloc_scratch = nullptr;  // device address of the allocation-free entry point's array
  // open KTimerGroup: launches of this class are counted into it instead of timed alone
  const char* group_cls = nullptr;
  double group_bytes = 0.0;
  int64_t group_launches = 0;
  // pinned host staging of small device results read back during a solve (readback)
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  hipEvent_t readback_event = nullptr;
};

// Copies small device arrays to host memory and waits for them: the copies go to the
// context's pinned buffer (direct transfers, no pageable staging), one event on the
// context stream is waited for, then the values are copied out.  Each part is
// {device source, host destination, bytes}.
struct ReadbackPart {
  const void* dev;
  void* host;
  size_t bytes;
};
void readback(dmlmc_ctx* ctx, std::initializer_list<ReadbackPart> parts);

// RAII bracket around one launch of a timed kernel class.
struct KTimer {
  dmlmc_ctx* ctx;
  const char* cls;
  double bytes;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  KTimer(dmlmc_ctx* c, const char* k, double b);
  ~KTimer();
};
// One event pair around a run of back-to-back launches of one class (the colour sweeps of
// a smoother): each KTimer of that class inside only adds its launch and bytes, so the
// class's launch time is the run's elapsed time over its launches, without an event pair
// between every two launches.
struct KTimerGroup {
  dmlmc_ctx* ctx;
  const char* cls;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  KTimerGroup(dmlmc_ctx* c, const char* k);
  ~KTimerGroup();
};
void timing_collect(dmlmc_ctx* ctx);

// ------------------------------------------------------------------ hierarchy objects
// Launch variants of the tuned kernels.  A variant changes only how a launch divides its
// work over threads and wavefronts, never the arithmetic of any output entry, so every
// variant gives bitwise the same results.  Value 0 takes the built-in rule.
enum KernelVariant {
  KV_WILSON_RB = 0,  // fine stencil: RHS per thread (1, 2, 4, 8)
  KV_COARSE_SPLIT,   // complex-FP32 coarse stencil, d = 16: wavefronts per site (1: both 16-RHS tiles, 2: one each);
                     // 3: whole-line traffic staged through LDS
  KV_SAP_RB,         // SAP colour sweep: RHS per thread (1, 2, 4, 8)
  KV_GS_SPLIT,       // complex-FP16-block Gauss-Seidel, d = 16: 1, 2 wavefronts per site; 3: tile pairs in
                     // flight; 4: whole-line vector loads and stores staged in LDS
  KV_RESTRICT_UT,    // matrix-core restriction: 16-entry tiles whose loads a wavefront issues at once (1, 2, 4)
  KV_PROLONG_MT,     // matrix-core prolongation: 16-entry tiles per wavefront (1, 2, 4; dividing the tile count)
  KV_PROLONG_STAGED,  // prolongation with 16 dofs on the fine side, or fine rows of half a line: 1 = direct
                      // loads and stores, 2 = whole-line vector traffic staged through LDS
  KV_RESTRICT_STAGED,  // restriction with fine rows of half a line: 1 = direct, 2 = staged through LDS
  KV_COUNT
};

struct Level {
  int l = 1;              // 1-based
  int kv[KV_COUNT] = {};  // launch variants (KernelVariant), 0 = built-in rule
  int Lx = 0, Lt = 0, dofs = 2;
  bool fine = true;
  double m0 = 0.0;
  // fine level: links U[mu][site] with the antiperiodic sign folded into U_t(., Lt-1)
  DevBuf U64, U32;
  // coarse levels: blocks A[site][5][d][d] and inverse self blocks [site][d][d]; FP64
  // blocks column-major (entry (i, j) at j * d + i); FP32 blocks the same except at
  // d = 16, where they are row-major (entry (i, j) at i * 16 + j, the matrix-core layout)
  DevBuf A64, A32, Ainv64, Ainv32;
  // d = 16: complex-FP16 copies (real part in the low half of a 32-bit word, row-major) of
  // the four hop blocks [site][4][16][16] and of the inverse self blocks, read by the
  // half-precision operands form of the coarse Gauss-Seidel smoother
  DevBuf Ahop16, Ainv16;
  // interpolation to level l+1 (if not coarsest): blocks P[cs][chir][row][k]
  int ax = 0, at = 0, N = 0;
  DevBuf P64, P32;
  std::vector<c128> tv_host;  // test vectors used for P (ntv x n), kept for export
  int64_t sites() const { return (int64_t)Lx * Lt; }
  int64_t n() const { return sites() * dofs; }
  int rows_per_block() const { return ax * at * (dofs / 2); }
};

struct Workspace;  // per-level scratch for V-cycles and solves (solver.hip)

struct CoarsenStep {
  int ax = 0, at = 0, ntv = 0;
};

// Reduction of the FP64 residual that ends one complex-FP32 FGMRES cycle (measured at
// 1024^2: the total iteration count is the same for targets from 2e-6 to 1e-2, while
// shorter cycles keep the Gram-Schmidt bases short)
constexpr double INNER_RTOL_DEFAULT = 1e-2;

struct dmlmc_hier {
  dmlmc_ctx* ctx = nullptr;
  std::vector<Level> lv;
  std::vector<CoarsenStep> plan;  // coarsening steps 1..L-1
  uint64_t seed = 0;
  int n_inv = 3;
  int64_t setup_iters = 0;
  const dmlmc_defl* attached = nullptr;
  // deflation of the coarsest level used inside V-cycles (exact solve on its span, GMRES
  // on the rest); set for the duration of an estimate, or by dmlmc_set_deflation
  const dmlmc_defl* coarse_defl = nullptr;
  int tuned_block = 0;  // RHS block chosen by the autotuner (0: not tuned)
  // explicit coarsest inverse for the complex-FP32 coarsest solves: complex FP32 [n][n],
  // and its complex-FP16 copy (scaled by 2^-e so that every component is below 1;
  // coarse_dinv16_unscale = 2^e; stored in 2 KB blocks of 16 rows x 32 columns in the
  // order of the matrix-core product's loads), and its 8-bit copy (two bytes per complex entry, each
  // row scaled by its own power of two, coarse_dinv8_rows[i] = 2^(e_i - 8)); mode 0 off, 1 FP32
  // inverse, 2 FP16 inverse, 3 8-bit inverse
  DevBuf coarse_dinv;
  DevBuf coarse_dinv16;
  DevBuf coarse_dinv8;
  DevBuf coarse_dinv8_rows;
  int64_t coarse_dinv_n = 0;
  double coarse_dinv_rtol = 0.0;  // residual tolerance of the column solves it was built with
  float coarse_dinv16_unscale = 1.f;
  int coarse_direct_mode = 0;
  // recorded FGMRES iterations (preconditioner + operator + Gram-Schmidt) of the
  // complex-FP32 cycles, keyed by everything their launches depend on
  bool use_graphs = true;
  struct GraphRec {
    hipGraphExec_t exec = nullptr;
    uint64_t epoch = 0;
  };
  std::map<std::vector<int64_t>, GraphRec> graphs;
  std::set<std::vector<int64_t>> graph_seen;
  int64_t graph_launches = 0;
  int coarsest_iters_defl = 8;
  // solver knobs (not part of the math; iteration counts only)
  int sap_mr_iters = 2;
  int nu_pre = 0, nu_post = 2, nu_post_coarse = 2;  // post-smoothing: fine level, coarse levels
  double inner_rtol = INNER_RTOL_DEFAULT;            // reduction per complex-FP32 FGMRES cycle
  bool smoother_half = true;  // complex-FP32 coarse Gauss-Seidel reads the FP16 block copies
  int coarsest_iters = 24;
  int restart = 16;
  std::vector<std::unique_ptr<Workspace>> ws;  // indexed by level-1
  ~dmlmc_hier();
};

struct dmlmc_defl {
  dmlmc_ctx* ctx = nullptr;
  int level = 0, k = 0;
  // kind 0: eigenpairs of Q_L = Gamma5 D_L (coarsest term; tr_defl = sum x^H Gamma5 x / lambda);
  // kind 1: eigenpairs of J = Q_a^-1 - P_ab Q_b^-1 P_ab^H of the term (a = level, b = level_b)
  // (tr_defl = sum lambda x^H Gamma5 x, the trace of the term on the deflated space)
  int kind = 0, level_b = 0;
  int64_t n = 0;
  DevBuf X64;     // eigenvectors of Q, [k][n]
  DevBuf W64, W32;// Gamma5 X, [k][n]
  DevBuf X32;     // eigenvectors of Q in FP32, [k][n]
  DevBuf lam_dev; // eigenvalues on the device, [k]
  std::vector<double> lambda;
  double tr_defl = 0.0;
  int eig_iters = 0;            // outer subspace iterations (0 when imported)
  int64_t eig_degree_sum = 0;   // Chebyshev degrees summed (Q^2 applications per vector)
  double eig_residual = 0.0;    // max ||Q x - lambda x|| / ||Q||_bound at exit
};

// ------------------------------------------------------------------ kernel launchers
// precision tag: R = float -> c64 path, R = double -> c128 path
// Vectors of nrhs right-hand sides are stored one after another, RHS r at r * ld; ld = 0
// stands for the level size n.  y = D x (or Gamma5 D x); with sub given, the residual
// form y = sub - D x
template <typename R>
void launch_wilson(dmlmc_ctx* ctx, const Level& L, const Cx<R>* x, Cx<R>* y, int nrhs, int64_t ldx,
                   int64_t ldy, bool gamma5_left, const Cx<R>* sub = nullptr);
template <typename R>
void launch_coarse(dmlmc_ctx* ctx, const Level& L, const Cx<R>* x, Cx<R>* y, int nrhs, int64_t ldx,
                   int64_t ldy, bool gamma5_left, const Cx<R>* sub = nullptr);
template <typename R>
void apply_op(dmlmc_ctx* ctx, const Level& L, const Cx<R>* x, Cx<R>* y, int nrhs, bool gamma5_left = false,
              int64_t ld = 0);
// y = D z on the fine level in complex FP32 fused with the dots <u_i, wscale[r] y> of a
// single-pass Gram-Schmidt step (basis u_i, i < nb <= 8, at Ub + i * vs, RHS r at r * ld):
// writes G = wilson_dots_blocks(L) block partials per RHS, 2 nb doubles each, to part
// (layout of the Gram-Schmidt partial sums) and returns G
int wilson_dots_blocks(const Level& L);
int launch_wilson_dots(dmlmc_ctx* ctx, const Level& L, const c64* z, c64* y, int nrhs, int64_t ld, const c64* Ub,
                       int nb, int64_t vs, const double* wscale, double* part);
// r = b - D x in one pass (the refinement residual)
template <typename R>
void apply_residual(dmlmc_ctx* ctx, const Level& L, const Cx<R>* x, const Cx<R>* b, Cx<R>* r, int nrhs);
// r = b - D x computed in FP64 and stored in complex FP32 (x, b at stride ldx, r at ldr;
// 0: the level size): the first Krylov vector of a complex-FP32 refinement cycle
void apply_residual_to32(dmlmc_ctx* ctx, const Level& L, const c128* x, const c128* b, c64* r, int nrhs,
                         int64_t ldx = 0, int64_t ldr = 0);
template <typename R>
void launch_sap(dmlmc_ctx* ctx, const Level& L, Cx<R>* x, const Cx<R>* b, int nrhs, int color,
                int mr_iters, int64_t ld = 0);
template <typename R>
void launch_coarse_gs(dmlmc_ctx* ctx, const Level& L, Cx<R>* x, const Cx<R>* b, int nrhs, int color,
                      bool half = false, int64_t ld = 0);
template <typename R>
void launch_restrict(dmlmc_ctx* ctx, const Level& L, const Cx<R>* xf, Cx<R>* yc, int nrhs, int64_t ldf = 0,
                     int64_t ldc = 0);
template <typename R>
void launch_prolong(dmlmc_ctx* ctx, const Level& L, const Cx<R>* ec, Cx<R>* xf, int nrhs, bool add,
                    int64_t ldc = 0, int64_t ldf = 0);

// BLAS-like (blas.hip)
template <typename T>
void launch_fill_zero(dmlmc_ctx* ctx, T* p, size_t count);
// zeroes entries 0 .. n-1 of nrhs rows at stride ld (the entries between n and ld untouched)
template <typename T>
void launch_fill_zero_rows(dmlmc_ctx* ctx, T* p, int64_t n, int nrhs, int64_t ld);
void launch_fill_value(dmlmc_ctx* ctx, double* p, size_t count, double v);
template <typename To, typename From>
void launch_cast(dmlmc_ctx* ctx, const Cx<From>* x, Cx<To>* y, int64_t n, int nrhs, int64_t ldx, int64_t ldy);
// per-RHS dots out[r] = sum_i conj(x[r][i]) y[r][i] (FP64 accumulation), out on device
template <typename RX, typename RY>
void launch_dots(dmlmc_ctx* ctx, const Cx<RX>* x, const Cx<RY>* y, int64_t n, int nrhs, int64_t ldx,
                 int64_t ldy, c128* out);
// per-RHS squared norms (FP64), out on device
template <typename R>
void launch_norms2(dmlmc_ctx* ctx, const Cx<R>* x, int64_t n, int nrhs, int64_t ld, double* out);
// y[r] = a[r] * x[r] + y[r]   (a on device, per RHS)
template <typename R>
void launch_axpy_dev(dmlmc_ctx* ctx, const c128* a, const Cx<R>* x, Cx<R>* y, int64_t n, int nrhs, int64_t ld);
// y = b - y (residual from y = D x), in place
template <typename R>
void launch_xmy(dmlmc_ctx* ctx, const Cx<R>* b, Cx<R>* y, int64_t n, int nrhs, int64_t ldb, int64_t ldy);
// x64 += (double) e32
template <typename RE>
void launch_add_cast(dmlmc_ctx* ctx, const Cx<RE>* e, c128* x, int64_t n, int nrhs, int64_t lde, int64_t ldx);
// x (RX) += e (FP64), [nrhs][n]
template <typename RX>
void launch_add_cast_to(dmlmc_ctx* ctx, const c128* e, Cx<RX>* x, int64_t n, int nrhs);
// Z2 noise
template <typename R>
void launch_z2(dmlmc_ctx* ctx, Cx<R>* out, int64_t n, uint64_t seed, int level, int64_t sample0, int nrhs,
               int64_t ld);
void launch_z4(dmlmc_ctx* ctx, c128* out, int64_t n, uint64_t seed, int level, int vec0, int nvec);

// Block inner products with a set of nb vectors V_i: vector i of RHS r at
// V + i * vstride + r * ldv (ldv = 0: one set shared by all RHS; ldv < 0: ldv = ld).
//  h[r][i] = <V_i[r], w[r]> for i < nb (FP64 accumulation)
template <typename RV>
void launch_multidot(dmlmc_ctx* ctx, const Cx<RV>* V, int nb, const c128* w, int64_t n, int nrhs,
                     int64_t ld, int64_t vstride, c128* h /* [nrhs][hld] */, int hld, int64_t ldv = -1);
//  w[r] -= sgn * sum_i h[r][i] V_i[r]
template <typename RV>
void launch_multiaxpy(dmlmc_ctx* ctx, const Cx<RV>* V, int nb, c128* w, int64_t n, int nrhs, int64_t ld,
                      int64_t vstride, const c128* h, int hld, int64_t ldv = -1, double sgn = 1.0);

// helpers
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
