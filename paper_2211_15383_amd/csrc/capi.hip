// C ABI of the library: argument validation (before any device work), object lifetimes,
// error translation (no exception crosses the ABI) and kernel-class timing.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "defl.h"
#include "dense.h"
#include "mlmc.h"
#include "noalloc.h"
#include "setup.h"
#include "solver.h"
#include "tune.h"

namespace {

std::string g_create_error;

template <typename F>
dmlmc_status guarded(dmlmc_ctx* ctx, F&& f) {
  try {
    if (ctx) {
      ctx->err.clear();
      HIPCHK(hipSetDevice(ctx->device));
    }
    f();
    return DMLMC_OK;
  } catch (const DmlmcError& e) {
    if (ctx) ctx->err = e.what(); else g_create_error = e.what();
    return e.status;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->err = "host allocation failed"; else g_create_error = "host allocation failed";
    return DMLMC_ENOMEM;
  } catch (const std::exception& e) {
    if (ctx) ctx->err = e.what(); else g_create_error = e.what();
    return DMLMC_EHIP;
  }
}

void check_hier(const dmlmc_ctx* ctx, const dmlmc_hier* h) {
  REQUIRE(h != nullptr, "hierarchy is NULL");
  if (h->ctx != ctx) throw DmlmcError(DMLMC_ESTATE, "hierarchy belongs to another context");
}

void check_level(const dmlmc_hier* h, int level) {
  REQUIRE(level >= 1 && level <= (int)h->lv.size(), "level out of range");
}

}  // namespace

// ---------------------------------------------------------------- timing
namespace {
bool class_timed(const dmlmc_ctx* ctx, const char* k) {
  return ctx && ctx->timing && (ctx->timing_only.empty() || ctx->timing_only.count(k));
}

void take_events(dmlmc_ctx* ctx, hipEvent_t& e0, hipEvent_t& e1) {
  if (!ctx->event_pool.empty()) {
    e0 = ctx->event_pool.back().first;
    e1 = ctx->event_pool.back().second;
    ctx->event_pool.pop_back();
  } else {
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
  }
}
}  // namespace

KTimer::KTimer(dmlmc_ctx* c, const char* k, double b) : ctx(c), cls(k), bytes(b) {
  if (!class_timed(ctx, k)) return;
  if (ctx->group_cls && std::strcmp(ctx->group_cls, k) == 0) {
    ctx->group_bytes += b;
    ctx->group_launches += 1;
    return;
  }
  take_events(ctx, e0, e1);
  HIPCHK(hipEventRecord(e0, ctx->stream));
}

KTimer::~KTimer() {
  if (!e0) return;
  (void)hipEventRecord(e1, ctx->stream);
  TimerClass& t = ctx->timers[cls];
  t.pending.emplace_back(e0, e1);
  t.pending_bytes.push_back(bytes);
  t.pending_launches.push_back(1);
}

KTimerGroup::KTimerGroup(dmlmc_ctx* c, const char* k) : ctx(c), cls(k) {
  if (!class_timed(ctx, k) || ctx->group_cls) return;
  take_events(ctx, e0, e1);
  ctx->group_cls = k;
  ctx->group_bytes = 0.0;
  ctx->group_launches = 0;
  HIPCHK(hipEventRecord(e0, ctx->stream));
}

KTimerGroup::~KTimerGroup() {
  if (!e0) return;
  (void)hipEventRecord(e1, ctx->stream);
  ctx->group_cls = nullptr;
  if (ctx->group_launches == 0) {
    ctx->event_pool.emplace_back(e0, e1);
    return;
  }
  TimerClass& t = ctx->timers[cls];
  t.pending.emplace_back(e0, e1);
  t.pending_bytes.push_back(ctx->group_bytes);
  t.pending_launches.push_back(ctx->group_launches);
}

void timing_collect(dmlmc_ctx* ctx) {
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (auto& kv : ctx->timers) {
    TimerClass& t = kv.second;
    for (size_t i = 0; i < t.pending.size(); ++i) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, t.pending[i].first, t.pending[i].second));
      t.ms += ms;
      t.launches += t.pending_launches[i];
      t.bytes += t.pending_bytes[i];
      ctx->event_pool.push_back(t.pending[i]);
    }
    t.pending.clear();
    t.pending_bytes.clear();
    t.pending_launches.clear();
  }
}

extern "C" {

const char* dmlmc_version(void) { return "dmlmc 0.1 (gfx950)"; }

dmlmc_status dmlmc_create(dmlmc_ctx** out, int device, void* hip_stream) {
  if (!out) {
    g_create_error = "invalid argument: out is NULL";
    return DMLMC_EINVAL;
  }
  *out = nullptr;
  if (device < 0) {
    g_create_error = "invalid argument: device index out of range";
    return DMLMC_EINVAL;
  }
  dmlmc_ctx* ctx = nullptr;
  dmlmc_status st = guarded(nullptr, [&]() {
    int count = 0;
    HIPCHK(hipGetDeviceCount(&count));
    REQUIRE(device >= 0 && device < count, "device index out of range");
    HIPCHK(hipSetDevice(device));
    ctx = new dmlmc_ctx();
    ctx->device = device;
    if (hip_stream) {
      ctx->stream = (hipStream_t)hip_stream;
    } else {
      HIPCHK(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
      ctx->own_stream = true;
    }
    ctx->noalloc_scratch = noalloc_scratch_address();
  });
  if (st != DMLMC_OK) {
    delete ctx;
    return st;
  }
  *out = ctx;
  return DMLMC_OK;
}

void dmlmc_destroy(dmlmc_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& kv : ctx->timers)
    for (auto& e : kv.second.pending) ctx->event_pool.push_back(e);
  for (auto& e : ctx->event_pool) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  ctx->scratch_dots.release();
  ctx->scratch_small.release();
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->readback_event) (void)hipEventDestroy(ctx->readback_event);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}


const char* dmlmc_last_error(const dmlmc_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

dmlmc_status dmlmc_build_hierarchy(dmlmc_ctx* ctx, const dmlmc_lattice* lat, const dmlmc_mg_params* mg,
                                   dmlmc_hier** out) {
  if (!ctx) return DMLMC_EINVAL;
  return guarded(ctx, [&]() {
    REQUIRE(out != nullptr && lat != nullptr && mg != nullptr && lat->theta != nullptr, "NULL pointer");
    *out = nullptr;
    REQUIRE(mg->nlevels >= 1 && mg->nlevels <= 8, "nlevels must be in 1..8");
    REQUIRE(lat->Lx >= 4 && lat->Lt >= 4 && lat->Lx % 4 == 0 && lat->Lt % 4 == 0,
            "fine lattice extents must be multiples of 4 (SAP blocks)");
    REQUIRE(std::isfinite(lat->m0), "m0 is not finite");
    REQUIRE(mg->n_inv >= 1 || mg->import_tv != nullptr || mg->nlevels == 1, "n_inv must be >= 1");
    // geometry of every coarsening step
    int Lx = lat->Lx, Lt = lat->Lt, d = 2;
    for (int s = 0; s + 1 < mg->nlevels; ++s) {
      const int ax = mg->agg[s][0], at = mg->agg[s][1], N = mg->ntv[s];
      REQUIRE(ax >= 1 && at >= 1 && N >= 1, "aggregates and test vectors must be positive");
      REQUIRE(Lx % ax == 0 && Lt % at == 0, "lattice extent not divisible by the aggregate");
      REQUIRE(Lx / ax >= 2 && Lt / at >= 2, "coarse lattice extent must be at least 2");
      REQUIRE(ax * at * (d / 2) >= N, "more test vectors than rows per aggregate and chirality");
      Lx /= ax;
      Lt /= at;
      d = 2 * N;
      REQUIRE(d <= 64, "at most 32 test vectors per chirality");
      if (s + 2 < mg->nlevels) REQUIRE(Lx % 2 == 0 && Lt % 2 == 0, "smoothed coarse levels need even extents");
    }
    std::unique_ptr<dmlmc_hier> H(new dmlmc_hier());
    H->ctx = ctx;
    H->seed = mg->seed;
    H->n_inv = mg->n_inv;
    for (int s = 0; s + 1 < mg->nlevels; ++s) {
      CoarsenStep st;
      st.ax = mg->agg[s][0];
      st.at = mg->agg[s][1];
      st.ntv = mg->ntv[s];
      H->plan.push_back(st);
    }
    Level F;
    F.l = 1;
    F.fine = true;
    F.Lx = lat->Lx;
    F.Lt = lat->Lt;
    F.dofs = 2;
    F.m0 = lat->m0;
    upload_links(ctx, F, lat->theta, lat->antiperiodic_t);
    H->lv.push_back(std::move(F));
    std::vector<const c128*> imp;
    if (mg->import_tv) {
      for (int s = 0; s + 1 < mg->nlevels; ++s) imp.push_back((const c128*)mg->import_tv[s]);
    }
    build_levels(H.get(), imp);
    *out = H.release();
  });
}

void dmlmc_free_hierarchy(dmlmc_hier* h) {
  if (!h) return;
  if (h->ctx) {
    (void)hipSetDevice(h->ctx->device);
    (void)hipStreamSynchronize(h->ctx->stream);
  }
  delete h;
}

dmlmc_status dmlmc_level_info(const dmlmc_hier* h, int level, int* Lx, int* Lt, int* dofs) {
  if (!h || level < 1 || level > (int)h->lv.size()) return DMLMC_EINVAL;
  const Level& L = h->lv[level - 1];
  if (Lx) *Lx = L.Lx;
  if (Lt) *Lt = L.Lt;
  if (dofs) *dofs = L.dofs;
  return DMLMC_OK;
}

dmlmc_status dmlmc_export_level(dmlmc_ctx* ctx, const dmlmc_hier* h, int level, void* P_host, void* Dc_host,
                                void* tv_host) {
  if (!ctx) return DMLMC_EINVAL;
  return guarded(ctx, [&]() {
    check_hier(ctx, h);
    check_level(h, level);
    const Level& L = h->lv[level - 1];
    const int Lmax = (int)h->lv.size();
    REQUIRE(!(P_host || tv_host) || level < Lmax, "P and test vectors exist only below the coarsest level");
    REQUIRE(!Dc_host || level >= 2, "block stencil exists only on coarse levels");
    if (P_host) {
      const Level& C = h->lv[level];
      const int64_t nf = L.n(), nc = C.n();
      const int rows = L.rows_per_block(), N = L.N, h2 = L.dofs / 2;
      std::vector<c128> Pb((size_t)C.sites() * 2 * rows * N);
      HIPCHK(hipMemcpy(Pb.data(), L.P64.p, sizeof(c128) * Pb.size(), hipMemcpyDeviceToHost));
      c128* P = (c128*)P_host;
      std::memset(P, 0, sizeof(c128) * (size_t)nf * nc);
      const int Lxc = C.Lx;
      for (int64_t cs = 0; cs < C.sites(); ++cs) {
        const int X = (int)(cs % Lxc), T = (int)(cs / Lxc);
        for (int c = 0; c < 2; ++c)
          for (int row = 0; row < rows; ++row) {
            const int ls = row / h2, j = row % h2;
            const int64_t site = (int64_t)(X * L.ax + ls % L.ax) + (int64_t)L.Lx * (T * L.at + ls / L.ax);
            const int64_t fi = site * L.dofs + c * h2 + j;
            for (int k = 0; k < N; ++k)
              P[fi * nc + cs * 2 * N + c * N + k] = Pb[((cs * 2 + c) * rows + row) * N + k];
          }
      }
    }
    if (tv_host) std::memcpy(tv_host, L.tv_host.data(), sizeof(c128) * L.tv_host.size());
    if (Dc_host) {
      const int d = L.dofs;
      std::vector<c128> A((size_t)L.sites() * 5 * d * d);
      HIPCHK(hipMemcpy(A.data(), L.A64.p, sizeof(c128) * A.size(), hipMemcpyDeviceToHost));
      c128* o = (c128*)Dc_host;
      for (int64_t b = 0; b < L.sites() * 5; ++b)
        for (int i = 0; i < d; ++i)
          for (int j = 0; j < d; ++j) o[(b * d + i) * d + j] = A[(b * d + j) * d + i];  // column- to row-major
    }
  });
}

dmlmc_status dmlmc_deflate(dmlmc_ctx* ctx, dmlmc_hier* h, int level, int k, double eig_rtol, const void* import_X,
                           const double* import_lambda, dmlmc_defl** out, double* tr_defl_out) {
  if (!ctx) return DMLMC_EINVAL;
  dmlmc_status conv = DMLMC_OK;
  dmlmc_status st = guarded(ctx, [&]() {
    REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    check_hier(ctx, h);
    check_level(h, level);
    const Level& L = h->lv[level - 1];
    REQUIRE(k >= 1 && (int64_t)k * 4 <= L.n(), "k must be in 1..n_level/4");
    REQUIRE((import_X == nullptr) == (import_lambda == nullptr), "import_X and import_lambda go together");
    REQUIRE(import_X != nullptr || eig_rtol > 0.0, "eig_rtol must be positive");
    std::unique_ptr<dmlmc_defl> D(new dmlmc_defl());
    D->ctx = ctx;
    D->level = level;
    D->k = k;
    D->n = L.n();
    D->X64.alloc(sizeof(c128) * (size_t)k * D->n);
    if (import_X) {
      HIPCHK(hipMemcpy(D->X64.p, import_X, sizeof(c128) * (size_t)k * D->n, hipMemcpyHostToDevice));
      D->lambda.assign(import_lambda, import_lambda + k);
      for (double v : D->lambda) REQUIRE(std::isfinite(v) && v != 0.0, "imported eigenvalue is zero or not finite");
    } else {
      EigResult r = eig_coarsest(h, level, k, eig_rtol, D->X64.as<c128>());
      D->lambda = r.lambda;
      D->eig_iters = r.iters;
      D->eig_degree_sum = r.degree_sum;
      D->eig_residual = r.max_residual;
      if (!r.converged) conv = DMLMC_ENOCONV;
    }
    defl_finish(h, D.get());
    if (tr_defl_out) *tr_defl_out = D->tr_defl;
    *out = D.release();
  });
  if (st == DMLMC_OK && conv != DMLMC_OK) {
    ctx->err = "eigensolver stopped at its iteration limit";
    return conv;
  }
  return st;
}

dmlmc_status dmlmc_deflation_info(const dmlmc_defl* d, int* iters, int64_t* degree_sum, double* max_residual) {
  if (!d) return DMLMC_EINVAL;
  if (iters) *iters = d->eig_iters;
  if (degree_sum) *degree_sum = d->eig_degree_sum;
  if (max_residual) *max_residual = d->eig_residual;
  return DMLMC_OK;
}

void dmlmc_free_deflation(dmlmc_defl* d) {
  if (!d) return;
  if (d->ctx) {
    (void)hipSetDevice(d->ctx->device);
    (void)hipStreamSynchronize(d->ctx->stream);
  }
  delete d;
}

dmlmc_status dmlmc_export_deflation(dmlmc_ctx* ctx, const dmlmc_defl* d, void* X_host, double* lambda_host) {
  if (!ctx) return DMLMC_EINVAL;
  return guarded(ctx, [&]() {
    REQUIRE(d != nullptr, "deflation is NULL");
    if (d->ctx != ctx) throw DmlmcError(DMLMC_ESTATE, "deflation belongs to another context");
    if (X_host) HIPCHK(hipMemcpy(X_host, d->X64.p, sizeof(c128) * (size_t)d->k * d->n, hipMemcpyDeviceToHost));
    if (lambda_host) std::memcpy(lambda_host, d->lambda.data(), sizeof(double) * d->k);
  });
}

dmlmc_status dmlmc_solve_multi_rhs(dmlmc_ctx* ctx, const dmlmc_hier* h, int level, const dmlmc_defl* proj,
                                   const void* B, void* X, int nrhs, int64_t ld, dmlmc_precision prec, double rtol,
                                   int maxiter, dmlmc_solve_stats* stats) {
  if (!ctx) return DMLMC_EINVAL;
  SolveResult r;
  dmlmc_status st = guarded(ctx, [&]() {
    check_hier(ctx, h);
    check_level(h, level);
    REQUIRE(B != nullptr && X != nullptr, "NULL vector");
    REQUIRE(B != X, "B and X must not alias");
    REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    dmlmc_hier* H = const_cast<dmlmc_hier*>(h);
    const int64_t n = H->lv[level - 1].n();
    REQUIRE(ld >= n, "ld smaller than the level dimension");
    REQUIRE(prec == DMLMC_FP64 || prec == DMLMC_MIXED, "unknown precision");
    REQUIRE(rtol > 0.0 && maxiter >= 1, "rtol must be > 0 and maxiter >= 1");
    if (proj) {
      if (proj->ctx != ctx) throw DmlmcError(DMLMC_ESTATE, "deflation belongs to another context");
      REQUIRE(proj->level == level, "deflation is for another level");
    }
    c128* Bc = (c128*)hier_buf(H, "api_B", level, sizeof(c128) * (size_t)nrhs * n);
    c128* Xc = (c128*)hier_buf(H, "api_X", level, sizeof(c128) * (size_t)nrhs * n);
    launch_cast<double, double>(ctx, (const c128*)B, Bc, n, nrhs, ld, n);
    if (proj) defl_apply(H, proj, Bc, nrhs, n, prec);
    r = solve_level(H, level, Bc, Xc, nrhs, prec, rtol, maxiter);
    launch_cast<double, double>(ctx, Xc, (c128*)X, n, nrhs, n, ld);
    HIPCHK(hipStreamSynchronize(ctx->stream));
  });
  if (stats) {
    stats->iters = r.iters;
    stats->ir_steps = r.ir_steps;
    stats->converged = r.converged ? 1 : 0;
    stats->relres_max = r.relres_max;
  }
  if (st == DMLMC_OK && !r.converged) {
    ctx->err = "rtol not reached within maxiter";
    return DMLMC_ENOCONV;
  }
  return st;
}

dmlmc_status dmlmc_mlmc_trace(dmlmc_ctx* ctx, const dmlmc_hier* h, const dmlmc_defl* coarsest,
                              const dmlmc_mlmc_params* p, dmlmc_trace_result* out) {
  if (!ctx) return DMLMC_EINVAL;
  return guarded(ctx, [&]() {
    check_hier(ctx, h);
    REQUIRE(p != nullptr && out != nullptr, "NULL pointer");
    const int L = (int)h->lv.size();
    REQUIRE(p->rhs_block >= 0 && p->rhs_block <= 512, "rhs_block must be in 0..512 (0: tuned)");
    REQUIRE(p->eps > 0.0 || p->fixed_counts, "eps must be positive");
    REQUIRE(p->rtol > 0.0, "rtol must be positive");
    REQUIRE(p->prec == DMLMC_FP64 || p->prec == DMLMC_MIXED, "unknown precision");
    for (int l = 0; l < L; ++l) {
      REQUIRE(p->n0[l] >= 1, "n0 must be >= 1 on every level");
      REQUIRE(!p->samples_out[l] || p->max_samples[l] >= 1, "samples_out needs max_samples");
    }
    if (coarsest) {
      if (coarsest->ctx != ctx) throw DmlmcError(DMLMC_ESTATE, "deflation belongs to another context");
      REQUIRE(coarsest->level == L && coarsest->kind == 0, "deflation must be of the coarsest level");
    }
    REQUIRE(!p->skip[0] && !p->skip[L - 1], "the finest and the coarsest level cannot be skipped");
    for (int l = 1; l < L; ++l) {
      const dmlmc_defl* t = p->term_defl[l - 1];
      if (!t) continue;
      if (t->ctx != ctx) throw DmlmcError(DMLMC_ESTATE, "deflation belongs to another context");
      REQUIRE(!p->skip[l - 1], "a term deflation is given for a skipped level");
      int nx = l + 1;
      while (nx < L && p->skip[nx - 1]) ++nx;
      REQUIRE(t->kind == 1 && t->level == l && t->level_b == nx,
              "term deflation does not match the term (a, b) of the telescoping sum");
    }
    REQUIRE(p->term_defl[L - 1] == nullptr, "the coarsest term is deflated through the coarsest argument");
    std::memset(out, 0, sizeof(*out));
    run_mlmc(const_cast<dmlmc_hier*>(h), coarsest, p, out);
  });
}

dmlmc_status dmlmc_hutchinson_trace(dmlmc_ctx* ctx, const dmlmc_hier* h, const dmlmc_defl* fine,
                                    const dmlmc_defl* coarsest, const dmlmc_mlmc_params* p, dmlmc_trace_result* out) {
  if (!ctx) return DMLMC_EINVAL;
  return guarded(ctx, [&]() {
    check_hier(ctx, h);
    REQUIRE(p != nullptr && out != nullptr, "NULL pointer");
    const int L = (int)h->lv.size();
    REQUIRE(p->rhs_block >= 0 && p->rhs_block <= 512, "rhs_block must be in 0..512 (0: tuned)");
    REQUIRE(p->eps > 0.0 || p->fixed_counts, "eps must be positive");
    REQUIRE(p->rtol > 0.0, "rtol must be positive");
    REQUIRE(p->prec == DMLMC_FP64 || p->prec == DMLMC_MIXED, "unknown precision");
    REQUIRE(p->n0[0] >= 1, "n0[0] must be >= 1");
    REQUIRE(!p->samples_out[0] || p->max_samples[0] >= 1, "samples_out needs max_samples");
    for (int l = 0; l < 8; ++l) {
      REQUIRE(!p->skip[l] && !p->term_defl[l], "skip and term_defl do not apply to the single-level estimator");
      REQUIRE(l == 0 || !p->samples_out[l], "only samples_out[0] applies to the single-level estimator");
    }
    if (fine) {
      if (fine->ctx != ctx) throw DmlmcError(DMLMC_ESTATE, "deflation belongs to another context");
      REQUIRE(fine->kind == 0 && fine->level == 1, "fine must be a deflation of level 1 (dmlmc_deflate)");
    }
    if (coarsest) {
      if (coarsest->ctx != ctx) throw DmlmcError(DMLMC_ESTATE, "deflation belongs to another context");
      REQUIRE(coarsest->level == L && coarsest->kind == 0, "deflation must be of the coarsest level");
    }
    std::memset(out, 0, sizeof(*out));
    run_hutchinson(const_cast<dmlmc_hier*>(h), fine, coarsest, p, out);
  });
}

dmlmc_status dmlmc_deflate_difference(dmlmc_ctx* ctx, dmlmc_hier* h, int a, int b, int k, double eig_rtol,
                                      double solve_rtol, dmlmc_precision prec, const void* import_X,
                                      const double* import_lambda, double corr_rtol, dmlmc_defl** out,
                                      double* corr_out) {
  if (!ctx) return DMLMC_EINVAL;
  dmlmc_status conv = DMLMC_OK;
  dmlmc_status st = guarded(ctx, [&]() {
    REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    check_hier(ctx, h);
    const int L = (int)h->lv.size();
    REQUIRE(a >= 1 && a < b && b <= L, "need 1 <= a < b <= L");
    const int64_t na = h->lv[a - 1].n();
    REQUIRE(k >= 1 && (int64_t)k * 4 <= na, "k must be in 1..n_a/4");
    REQUIRE((import_X == nullptr) == (import_lambda == nullptr), "import_X and import_lambda go together");
    REQUIRE(import_X != nullptr || (eig_rtol > 0.0 && solve_rtol > 0.0), "tolerances must be positive");
    REQUIRE(prec == DMLMC_FP64 || prec == DMLMC_MIXED, "unknown precision");
    std::unique_ptr<dmlmc_defl> D(new dmlmc_defl());
    D->ctx = ctx;
    D->level = a;
    D->level_b = b;
    D->kind = 1;
    D->k = k;
    D->n = na;
    D->X64.alloc(sizeof(c128) * (size_t)k * na);
    if (import_X) {
      HIPCHK(hipMemcpy(D->X64.p, import_X, sizeof(c128) * (size_t)k * na, hipMemcpyHostToDevice));
      D->lambda.assign(import_lambda, import_lambda + k);
      for (double v : D->lambda) REQUIRE(std::isfinite(v), "imported eigenvalue is not finite");
    } else {
      EigResult r = eig_difference(h, a, b, k, eig_rtol, solve_rtol, prec, D->X64.as<c128>());
      D->lambda = r.lambda;
      D->eig_iters = r.iters;
      D->eig_residual = r.max_residual;
      if (!r.converged) conv = DMLMC_ENOCONV;
    }
    defl_finish(h, D.get());
    if (corr_rtol > 0.0) D->tr_defl = difference_trace_term(h, D.get(), prec, corr_rtol);
    if (corr_out) *corr_out = D->tr_defl;
    *out = D.release();
  });
  if (st == DMLMC_OK && conv != DMLMC_OK) {
    ctx->err = "eigensolver stopped at its iteration limit";
    return conv;
  }
  return st;
}

dmlmc_status dmlmc_coarsest_direct(dmlmc_ctx* ctx, dmlmc_hier* h, const dmlmc_defl* coarsest, int enable) {
  if (!ctx) return DMLMC_EINVAL;
  return guarded(ctx, [&]() {
    check_hier(ctx, h);
    REQUIRE(enable >= 0 && enable <= 3, "enable must be 0, 1, 2 or 3");
    if (coarsest) {
      if (coarsest->ctx != ctx) throw DmlmcError(DMLMC_ESTATE, "deflation belongs to another context");
      REQUIRE(coarsest->kind == 0 && coarsest->level == (int)h->lv.size(), "deflation must be of the coarsest level");
    }
    if (!enable) {
      h->coarse_direct_mode = 0;
      h->coarse_dinv.release();
      h->coarse_dinv16.release();
      h->coarse_dinv8.release();
      h->coarse_dinv8_rows.release();
      h->coarse_dinv_n = 0;
      return;
    }
    // column tolerance: well below the rounding of the copy that is applied (FP32: 1e-8;
    // the FP16 and 8-bit copies round at ~5e-4 and ~6e-2): the inverse is a preconditioner
    // component, so its accuracy only moves iteration counts
    const double rtol = enable == 1 ? 1e-8 : 1e-6;
    if (h->coarse_dinv_n != 0 && h->coarse_dinv_rtol > rtol) {
      h->coarse_dinv.release();
      h->coarse_dinv16.release();
      h->coarse_dinv8.release();
      h->coarse_dinv8_rows.release();
      h->coarse_dinv_n = 0;
    }
    if (h->coarse_dinv_n == 0) build_coarse_direct(h, coarsest, rtol);
    if (enable == 2 && h->coarse_dinv16.p == nullptr) build_coarse_direct16(h);
    if (enable == 3 && h->coarse_dinv8.p == nullptr) build_coarse_direct8(h);
    h->coarse_direct_mode = enable;
  });
}

dmlmc_status dmlmc_tune_rhs_block(dmlmc_ctx* ctx, dmlmc_hier* h, const dmlmc_defl* coarsest, const int* candidates,
                                  int ncand, dmlmc_precision prec, double rtol, uint64_t noise_seed, int* best,
                                  double* sec_per_sample) {
  if (!ctx) return DMLMC_EINVAL;
  return guarded(ctx, [&]() {
    check_hier(ctx, h);
    REQUIRE(candidates != nullptr && best != nullptr, "NULL pointer");
    REQUIRE(ncand >= 1 && ncand <= 16, "ncand must be in 1..16");
    for (int c = 0; c < ncand; ++c) REQUIRE(candidates[c] >= 1 && candidates[c] <= 512, "candidates must be in 1..512");
    REQUIRE(rtol > 0.0, "rtol must be positive");
    REQUIRE(prec == DMLMC_FP64 || prec == DMLMC_MIXED, "unknown precision");
    const int L = (int)h->lv.size();
    if (coarsest) {
      if (coarsest->ctx != ctx) throw DmlmcError(DMLMC_ESTATE, "deflation belongs to another context");
      REQUIRE(coarsest->level == L, "deflation must be of the coarsest level");
    }
    *best = tune_rhs_block(h, coarsest, candidates, ncand, prec, rtol, noise_seed, sec_per_sample);
  });
}

dmlmc_status dmlmc_tune_kernels(dmlmc_ctx* ctx, dmlmc_hier* h, int nrhs, int reps, const char* cache_path, int* picks,
                                double* best_us, double* default_us) {
  if (!ctx) return DMLMC_EINVAL;
  return guarded(ctx, [&]() {
    check_hier(ctx, h);
    REQUIRE(nrhs >= 1 && nrhs <= 512, "nrhs must be in 1..512");
    REQUIRE(reps >= 1 && reps <= 1000, "reps must be in 1..1000");
    static_assert(DMLMC_KV_COUNT == KV_COUNT, "kernel variant ids of the header and the library differ");
    tune_kernels(h, nrhs, reps, cache_path, picks, best_us, default_us);
  });
}

dmlmc_status dmlmc_set_kernel_variant(dmlmc_hier* h, int level, int kernel, int value) {
  if (!h) return DMLMC_EINVAL;
  return guarded(h->ctx, [&]() { set_kernel_variant(h, level, kernel, value); });
}

dmlmc_status dmlmc_get_kernel_variant(const dmlmc_hier* h, int level, int kernel, int* value) {
  if (!h || !value || level < 1 || level > (int)h->lv.size() || kernel < 0 || kernel >= KV_COUNT) return DMLMC_EINVAL;
  *value = h->lv[level - 1].kv[kernel];
  return DMLMC_OK;
}

dmlmc_status dmlmc_set_deflation(dmlmc_hier* h, const dmlmc_defl* d) {
  if (!h) return DMLMC_EINVAL;
  if (d && d->ctx != h->ctx) return DMLMC_ESTATE;
  h->attached = d;
  h->coarse_defl = (d && d->kind == 0 && d->level == (int)h->lv.size()) ? d : nullptr;
  return DMLMC_OK;
}

dmlmc_status dmlmc_set_solver_params(dmlmc_hier* h, const dmlmc_solver_params* p) {
  if (!h || !p) return DMLMC_EINVAL;
  auto ok = [](int v, int lo, int hi) { return v < 0 || (v >= lo && v <= hi); };
  const int maxb = gs_max_basis() - 1;
  if (!ok(p->sap_mr_iters, 0, 64) || !ok(p->nu_pre, 0, 16) || !ok(p->nu_post, 0, 16) ||
      !ok(p->coarsest_iters, 1, maxb) || !ok(p->coarsest_iters_defl, 1, maxb) || !ok(p->restart, 2, maxb) ||
      !ok(p->use_graphs, 0, 1) || !ok(p->nu_post_coarse, 0, 16) || !ok(p->smoother_half, 0, 1))
    return DMLMC_EINVAL;
  if (p->inner_rtol >= 0.0 && !(p->inner_rtol > 0.0 && p->inner_rtol < 1.0)) return DMLMC_EINVAL;
  auto pick = [](int v, int cur) { return v >= 0 ? v : cur; };
  const int nu_pre = pick(p->nu_pre, h->nu_pre);
  const int nu_post = pick(p->nu_post, h->nu_post);
  const int nu_post_coarse = pick(p->nu_post_coarse, h->nu_post_coarse);
  // every level must smooth at least once per V-cycle
  if (nu_pre == 0 && (nu_post == 0 || nu_post_coarse == 0)) return DMLMC_EINVAL;
  h->nu_pre = nu_pre;
  h->nu_post = nu_post;
  h->nu_post_coarse = nu_post_coarse;
  if (p->sap_mr_iters >= 0) h->sap_mr_iters = p->sap_mr_iters;
  if (p->coarsest_iters >= 0) h->coarsest_iters = p->coarsest_iters;
  if (p->coarsest_iters_defl >= 0) h->coarsest_iters_defl = p->coarsest_iters_defl;
  if (p->restart >= 0) h->restart = p->restart;
  if (p->use_graphs >= 0) h->use_graphs = p->use_graphs != 0;
  if (p->inner_rtol >= 0.0) h->inner_rtol = p->inner_rtol;
  if (p->smoother_half >= 0) h->smoother_half = p->smoother_half != 0;
  return DMLMC_OK;
}

dmlmc_status dmlmc_get_solver_params(const dmlmc_hier* h, dmlmc_solver_params* p) {
  if (!h || !p) return DMLMC_EINVAL;
  p->sap_mr_iters = h->sap_mr_iters;
  p->nu_pre = h->nu_pre;
  p->nu_post = h->nu_post;
  p->coarsest_iters = h->coarsest_iters;
  p->coarsest_iters_defl = h->coarsest_iters_defl;
  p->restart = h->restart;
  p->use_graphs = h->use_graphs ? 1 : 0;
  p->nu_post_coarse = h->nu_post_coarse;
  p->inner_rtol = h->inner_rtol;
  p->smoother_half = h->smoother_half ? 1 : 0;
  return DMLMC_OK;
}

dmlmc_status dmlmc_z2_noise(dmlmc_ctx* ctx, int64_t n, uint64_t seed, int level, int64_t sample0, int nrhs, void* out,
                            dmlmc_precision prec) {
  if (!ctx) return DMLMC_EINVAL;
  return guarded(ctx, [&]() {
    REQUIRE(out != nullptr && n >= 1 && nrhs >= 1 && level >= 0 && sample0 >= 0, "invalid noise request");
    if (prec == DMLMC_MIXED)
      launch_z2<float>(ctx, (c64*)out, n, seed, level, sample0, nrhs, n);
    else
      launch_z2<double>(ctx, (c128*)out, n, seed, level, sample0, nrhs, n);
    HIPCHK(hipStreamSynchronize(ctx->stream));
  });
}

dmlmc_status dmlmc_apply_strided(dmlmc_ctx* ctx, const dmlmc_hier* h, int op, int level, const void* in,
                                 int64_t ld_in, void* out, int64_t ld_out, int nrhs, dmlmc_precision prec,
                                 uint64_t arg) {
  if (!ctx) return DMLMC_EINVAL;
  return guarded(ctx, [&]() {
    check_hier(ctx, h);
    check_level(h, level);
    REQUIRE(in != nullptr && out != nullptr && nrhs >= 1, "NULL vector or nrhs < 1");
    REQUIRE(prec == DMLMC_FP64 || prec == DMLMC_MIXED, "unknown precision");
    dmlmc_hier* H = const_cast<dmlmc_hier*>(h);
    const Level& L = H->lv[level - 1];
    const int Lmax = (int)H->lv.size();
    const bool f32 = prec == DMLMC_MIXED;
    const int64_t n = L.n();
    const int64_t nc = level < Lmax ? H->lv[level].n() : 0;
    // the level each vector lives on
    const int64_t n_in = op == DMLMC_OP_PROLONG ? nc : n;
    const int64_t n_out = op == DMLMC_OP_RESTRICT ? nc : n;
    if (op == DMLMC_OP_RESTRICT || op == DMLMC_OP_PROLONG)
      REQUIRE(level < Lmax, "no transfer below the coarsest level");
    if (ld_in == 0) ld_in = n_in;
    if (ld_out == 0) ld_out = n_out;
    REQUIRE(ld_in >= n_in && ld_out >= n_out && ld_in % 2 == 0 && ld_out % 2 == 0,
            "strides must be even and at least the vector length");
    switch (op) {
      case DMLMC_OP_D:
      case DMLMC_OP_GAMMA5_D: {
        const bool g5 = op == DMLMC_OP_GAMMA5_D;
        if (L.fine) {
          if (f32) launch_wilson<float>(ctx, L, (const c64*)in, (c64*)out, nrhs, ld_in, ld_out, g5);
          else launch_wilson<double>(ctx, L, (const c128*)in, (c128*)out, nrhs, ld_in, ld_out, g5);
        } else {
          if (f32) launch_coarse<float>(ctx, L, (const c64*)in, (c64*)out, nrhs, ld_in, ld_out, g5);
          else launch_coarse<double>(ctx, L, (const c128*)in, (c128*)out, nrhs, ld_in, ld_out, g5);
        }
        break;
      }
      case DMLMC_OP_RESTRICT:
        if (f32) launch_restrict<float>(ctx, L, (const c64*)in, (c64*)out, nrhs, ld_in, ld_out);
        else launch_restrict<double>(ctx, L, (const c128*)in, (c128*)out, nrhs, ld_in, ld_out);
        break;
      case DMLMC_OP_PROLONG:
        if (f32) launch_prolong<float>(ctx, L, (const c64*)in, (c64*)out, nrhs, false, ld_in, ld_out);
        else launch_prolong<double>(ctx, L, (const c128*)in, (c128*)out, nrhs, false, ld_in, ld_out);
        break;
      case DMLMC_OP_SMOOTH:
        REQUIRE(level < Lmax, "the coarsest level has no smoother");
        REQUIRE(arg >= 1 && arg <= 1000, "sweeps must be in 1..1000");
        REQUIRE(ld_in == ld_out, "the smoother takes one stride for b and x");
        if (f32) smooth<float>(H, level, (c64*)out, (const c64*)in, nrhs, (int)arg, ld_in);
        else smooth<double>(H, level, (c128*)out, (const c128*)in, nrhs, (int)arg, ld_in);
        break;
      case DMLMC_OP_VCYCLE:
        REQUIRE(ld_in == ld_out, "the V-cycle takes one stride for its input and output");
        REQUIRE(level < Lmax || ld_in == n, "coarsest-level vectors are unpadded");
        if (f32) vcycle<float>(H, level, (const c64*)in, (c64*)out, nrhs, ld_in);
        else vcycle<double>(H, level, (const c128*)in, (c128*)out, nrhs, ld_in);
        break;
      case DMLMC_OP_DEFL_C:
      case DMLMC_OP_DEFL_P: {
        // DMLMC_OP_DEFL_C writes [nrhs][k] coefficients, not a level vector
        REQUIRE(ld_in == n && (op == DMLMC_OP_DEFL_C || ld_out == n), "the deflation operators take unpadded vectors");
        const dmlmc_defl* D = H->attached;
        REQUIRE(D != nullptr, "no deflation attached (dmlmc_set_deflation)");
        REQUIRE(D->level == level, "attached deflation is for another level");
        // complex128 vectors for both precisions; prec selects FP64 or FP32 matrix-core kernels
        c128* C = (c128*)hier_buf(H, "api_C", level, sizeof(c128) * (size_t)D->k * nrhs);
        if (f32) defl_coeffs_mfma(ctx, D, (const c128*)in, nrhs, n, C, hier_devbuf(H, "api_part", level));
        else defl_coeffs_fp64(ctx, D, (const c128*)in, nrhs, n, C);
        if (op == DMLMC_OP_DEFL_C) {
          HIPCHK(hipMemcpyAsync(out, C, sizeof(c128) * (size_t)D->k * nrhs, hipMemcpyDeviceToDevice, ctx->stream));
        } else if (f32) {
          defl_project_mfma(ctx, D, (const c128*)in, (c128*)out, nrhs, n, n, C);
        } else {
          HIPCHK(hipMemcpyAsync(out, in, sizeof(c128) * (size_t)n * nrhs, hipMemcpyDeviceToDevice, ctx->stream));
          defl_project_fp64(ctx, D, (c128*)out, nrhs, n, C);
        }
        break;
      }
      default:
        REQUIRE(false, "unknown operator");
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
  });
}

dmlmc_status dmlmc_deflate_project_noalloc(dmlmc_ctx* ctx, const dmlmc_defl* d, const void* in, void* out,
                                           int nrhs) {
  if (!ctx) return DMLMC_EINVAL;
  return guarded(ctx, [&]() {
    REQUIRE(d != nullptr, "deflation is NULL");
    if (d->ctx != ctx) throw DmlmcError(DMLMC_ESTATE, "deflation belongs to another context");
    REQUIRE(in != nullptr && out != nullptr && nrhs >= 1, "NULL vector or nrhs < 1");
    const size_t bytes = sizeof(c128) * (size_t)d->n * nrhs;
    const char* a = (const char*)in;
    const char* b = (const char*)out;
    REQUIRE(a + bytes <= b || b + bytes <= a, "in and out overlap");
    deflate_project_noalloc(ctx, d, in, out, nrhs);
  });
}

dmlmc_status dmlmc_apply(dmlmc_ctx* ctx, const dmlmc_hier* h, int op, int level, const void* in, void* out, int nrhs,
                         dmlmc_precision prec, uint64_t arg) {
  return dmlmc_apply_strided(ctx, h, op, level, in, 0, out, 0, nrhs, prec, arg);
}

dmlmc_status dmlmc_work_stride(const dmlmc_hier* h, int level, int64_t* ld) {
  if (!h || !ld || level < 1 || level > (int)h->lv.size()) return DMLMC_EINVAL;
  *ld = work_ld(h, level);
  return DMLMC_OK;
}

dmlmc_status dmlmc_set_verbose(dmlmc_ctx* ctx, int level) {
  if (!ctx || level < 0) return DMLMC_EINVAL;
  ctx->verbose = level;
  return DMLMC_OK;
}

dmlmc_status dmlmc_timing_enable(dmlmc_ctx* ctx, int enable) {
  if (!ctx) return DMLMC_EINVAL;
  return guarded(ctx, [&]() {
    timing_collect(ctx);
    ctx->timing = enable != 0;
  });
}

dmlmc_status dmlmc_timing_select(dmlmc_ctx* ctx, const char* classes) {
  if (!ctx) return DMLMC_EINVAL;
  return guarded(ctx, [&]() {
    timing_collect(ctx);
    ctx->timing_only.clear();
    if (!classes) return;
    std::string all(classes), cur;
    for (char c : all + ",") {
      if (c == ',') {
        if (!cur.empty()) ctx->timing_only.insert(cur);
        cur.clear();
      } else if (c != ' ') {
        cur += c;
      }
    }
  });
}

dmlmc_status dmlmc_timing_reset(dmlmc_ctx* ctx) {
  if (!ctx) return DMLMC_EINVAL;
  return guarded(ctx, [&]() {
    timing_collect(ctx);
    for (auto& kv : ctx->timers) {
      kv.second.launches = 0;
      kv.second.ms = 0.0;
      kv.second.bytes = 0.0;
    }
  });
}

dmlmc_status dmlmc_timing_get(dmlmc_ctx* ctx, const char* cls, int64_t* launches, double* ms, double* bytes) {
  if (!ctx || !cls) return DMLMC_EINVAL;
  return guarded(ctx, [&]() {
    timing_collect(ctx);
    auto it = ctx->timers.find(cls);
    if (launches) *launches = it == ctx->timers.end() ? 0 : it->second.launches;
    if (ms) *ms = it == ctx->timers.end() ? 0.0 : it->second.ms;
    if (bytes) *bytes = it == ctx->timers.end() ? 0.0 : it->second.bytes;
  });
}

}  // extern "C"
