// Multigrid multilevel Monte Carlo estimate of tr(D^-1) (eq. 11) with exact deflation of
// the coarsest term (eq. 5).  Samples are drawn in blocks of RHS; every block of a
// difference level l < L draws its Z2 noise X on the device, solves D_l Z = X and
// D_{l+1} Z' = P_l^H X (multi-RHS, per-RHS Krylov spaces) and forms
// s = x^H z - y^H z' with FP64 dots; the coarsest level solves D_L Z = (I - W W^H) X and
// forms s = x^H z.  Sample values go to the host, where the FP64 accumulation, the error
// estimate and the multilevel sample allocation run.
#include <chrono>
#include <cmath>
#include <complex>

#include "defl.h"
#include "mlmc.h"
#include "solver.h"

namespace {

double level_work(const dmlmc_hier* H, int l) {
  const Level& L = H->lv[l - 1];
  return l == 1 ? 18.0 * L.sites() : 5.0 * L.dofs * L.dofs * L.sites();
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// Samples x^H D_l^-1 (x - W W^H x) of the Z2 block X [b][n_l] (W of `defl`, a deflation
// of level l, or none), appended to out: the coarsest term of eq. 11 (l = L) and the
// plain deflated Hutchinson estimator at the fine level (l = 1).
static int deflated_block(dmlmc_hier* H, const dmlmc_defl* defl, int l, const c128* X, int b,
                          const dmlmc_mlmc_params* p, std::vector<std::complex<double>>& out) {
  dmlmc_ctx* ctx = H->ctx;
  const int64_t n = H->lv[l - 1].n();
  const int maxit = p->maxiter > 0 ? p->maxiter : 2000;
  c128* Z = (c128*)hier_buf(H, "ml_Z", l, sizeof(c128) * (size_t)b * n);
  c128* s1 = (c128*)hier_buf(H, "ml_s1", l, sizeof(c128) * b);
  c128* Xt = (c128*)hier_buf(H, "ml_Xt", l, sizeof(c128) * (size_t)b * n);
  HIPCHK(hipMemcpyAsync(Xt, X, sizeof(c128) * (size_t)b * n, hipMemcpyDeviceToDevice, ctx->stream));
  if (defl) defl_apply(H, defl, Xt, b, n, p->prec);
  SolveResult r = solve_level(H, l, Xt, Z, b, p->prec, p->rtol, maxit);
  if (!r.converged) throw DmlmcError(DMLMC_ENOCONV, "sample solve did not converge at level " + std::to_string(l));
  launch_dots<double, double>(ctx, X, Z, n, b, n, n, s1);
  std::vector<c128> h1(b);
  readback(ctx, {{s1, h1.data(), sizeof(c128) * b}});
  for (int q = 0; q < b; ++q) out.emplace_back(h1[q].x, h1[q].y);
  return r.iters;
}

// Sample values of indices [i0, i0 + b) of the term that starts at level l, appended to
// out.  l < L: the difference term (l, lb) with lb the next level kept (l + 1, or further
// when levels are skipped, eq. 12), deflated by tdefl when given (Sec. 4.2); l = L: the
// coarsest term, deflated by defl.
static int sample_block(dmlmc_hier* H, const dmlmc_defl* defl, int l, int64_t i0, int b,
                        const dmlmc_mlmc_params* p, std::vector<std::complex<double>>& out, int lb = 0,
                        const dmlmc_defl* tdefl = nullptr) {
  dmlmc_ctx* ctx = H->ctx;
  const int L = (int)H->lv.size();
  const Level& F = H->lv[l - 1];
  const int64_t n = F.n();
  c128* X = (c128*)hier_buf(H, "ml_X", l, sizeof(c128) * (size_t)b * n);
  c128* Z = (c128*)hier_buf(H, "ml_Z", l, sizeof(c128) * (size_t)b * n);
  c128* s1 = (c128*)hier_buf(H, "ml_s1", l, sizeof(c128) * b);
  launch_z2<double>(ctx, X, n, p->noise_seed, l, i0, b, n);
  int iters = 0;
  const int maxit = p->maxiter > 0 ? p->maxiter : 2000;
  if (l < L) {
    if (lb == 0) lb = l + 1;
    const int64_t nc = H->lv[lb - 1].n();
    // x~ = x - V V^H x for a deflated term
    const c128* Xr = X;
    if (tdefl) {
      c128* Xt = (c128*)hier_buf(H, "ml_Xt", l, sizeof(c128) * (size_t)b * n);
      HIPCHK(hipMemcpyAsync(Xt, X, sizeof(c128) * (size_t)b * n, hipMemcpyDeviceToDevice, ctx->stream));
      defl_apply(H, tdefl, Xt, b, n, p->prec);
      Xr = Xt;
    }
    // y = P^H x and y~ = P^H x~ through the levels between l and lb
    auto restrict_to = [&](const c128* src, const char* tag) -> c128* {
      const c128* cur = src;
      c128* nxt = nullptr;
      for (int m = l; m < lb; ++m) {
        nxt = (c128*)hier_buf(H, m + 1 == lb ? tag : "ml_Rm", m + 1, sizeof(c128) * (size_t)b * H->lv[m].n());
        launch_restrict<double>(ctx, H->lv[m - 1], cur, nxt, b);
        cur = nxt;
      }
      return nxt;
    };
    c128* Zc = (c128*)hier_buf(H, "ml_Zc", lb, sizeof(c128) * (size_t)b * nc);
    c128* s2 = (c128*)hier_buf(H, "ml_s2", l, sizeof(c128) * b);
    SolveResult r1 = solve_level(H, l, Xr, Z, b, p->prec, p->rtol, maxit);
    c128* Y = restrict_to(X, "ml_Y");
    const c128* Yr = tdefl ? restrict_to(Xr, "ml_Yt") : Y;
    SolveResult r2 = solve_level(H, lb, Yr, Zc, b, p->prec, p->rtol, maxit);
    if (!r1.converged || !r2.converged)
      throw DmlmcError(DMLMC_ENOCONV, "sample solve did not converge at level " + std::to_string(l));
    iters = r1.iters + r2.iters;
    launch_dots<double, double>(ctx, X, Z, n, b, n, n, s1);
    launch_dots<double, double>(ctx, Y, Zc, nc, b, nc, nc, s2);
    std::vector<c128> h1(b), h2(b);
    readback(ctx, {{s1, h1.data(), sizeof(c128) * b}, {s2, h2.data(), sizeof(c128) * b}});
    for (int q = 0; q < b; ++q) out.emplace_back(h1[q].x - h2[q].x, h1[q].y - h2[q].y);
  } else {
    iters = deflated_block(H, defl, l, X, b, p, out);
  }
  return iters;
}

void run_mlmc(dmlmc_hier* H, const dmlmc_defl* defl, const dmlmc_mlmc_params* p, dmlmc_trace_result* res) {
  const int L = (int)H->lv.size();
  // the coarsest deflation also serves the coarsest solve inside every V-cycle
  struct Restore {
    dmlmc_hier* H;
    const dmlmc_defl* prev;
    ~Restore() { H->coarse_defl = prev; }
  } restore{H, H->coarse_defl};
  if (defl) H->coarse_defl = defl;
  const int blk = p->rhs_block > 0 ? p->rhs_block : H->tuned_block;
  if (blk < 1) throw DmlmcError(DMLMC_ESTATE, "rhs_block = 0 but the hierarchy has no tuned block size");
  const double t0 = now_s();
  // the levels kept in the telescoping sum; next[l] = the level a term starting at l joins
  std::vector<int> next(L + 1, 0);
  std::vector<bool> kept(L + 1, false);
  {
    int prev = 0;
    for (int l = 1; l <= L; ++l) {
      if (l > 1 && l < L && p->skip[l - 1]) continue;
      kept[l] = true;
      if (prev) next[prev] = l;
      prev = l;
    }
  }
  std::vector<std::vector<std::complex<double>>> S(L);
  std::vector<int64_t> target(L, 0), cap(L, 0);
  std::vector<double> cost(L, 0.0), level_time(L, 0.0);
  std::vector<int64_t> iters(L, 0);
  auto roundup = [&](int64_t m) { return ((m + blk - 1) / blk) * blk; };
  double tr_defl = defl ? defl->tr_defl : 0.0;
  for (int l = 1; l <= L; ++l) {
    if (!kept[l]) continue;
    cost[l - 1] = level_work(H, l) + (l < L ? level_work(H, next[l]) : 0.0);
    target[l - 1] = roundup(std::max(1, p->n0[l - 1]));
    cap[l - 1] = p->max_samples[l - 1] > 0 ? p->max_samples[l - 1] : ((int64_t)1 << 40);
    if (l < L && p->term_defl[l - 1]) tr_defl += p->term_defl[l - 1]->tr_defl;
  }
  double T = 0.0, Ti = 0.0, err = INFINITY;
  std::vector<double> var(L, 0.0);
  std::vector<std::complex<double>> mean(L);
  while (true) {
    for (int l = 1; l <= L; ++l) {
      if (!kept[l]) continue;
      auto& s = S[l - 1];
      while ((int64_t)s.size() < std::min(target[l - 1], cap[l - 1])) {
        const int64_t i0 = (int64_t)s.size();
        const int b = (int)std::min<int64_t>(blk, std::min(target[l - 1], cap[l - 1]) - i0);
        const double ts = now_s();
        iters[l - 1] += sample_block(H, defl, l, i0, b, p, s, l < L ? next[l] : 0,
                                     l < L ? p->term_defl[l - 1] : nullptr);
        level_time[l - 1] += now_s() - ts;
      }
    }
    // estimate (FP64 on the host)
    T = tr_defl;
    Ti = 0.0;
    double vn = 0.0;
    for (int l = 0; l < L; ++l) {
      if (!kept[l + 1]) continue;
      const auto& s = S[l];
      std::complex<double> m(0.0, 0.0);
      for (auto v : s) m += v;
      m /= (double)s.size();
      mean[l] = m;
      double v2 = 0.0;
      for (auto v : s) v2 += std::norm(v - m);
      var[l] = s.size() > 1 ? v2 / (double)(s.size() - 1) : 0.0;
      T += m.real();
      Ti += m.imag();
      vn += var[l] / (double)s.size();
    }
    err = T != 0.0 ? std::sqrt(vn) / std::fabs(T) : INFINITY;
    if (p->fixed_counts || err <= p->eps) break;
    // multilevel allocation
    double sum = 0.0;
    for (int l = 0; l < L; ++l)
      if (kept[l + 1]) sum += std::sqrt(var[l] * cost[l]);
    bool grew = false;
    for (int l = 0; l < L; ++l) {
      if (!kept[l + 1]) continue;
      const double want = std::ceil(std::sqrt(var[l] / cost[l]) * sum / (p->eps * p->eps * T * T));
      int64_t t = roundup(std::max<int64_t>((int64_t)want, (int64_t)S[l].size()));
      t = std::min(t, cap[l]);
      if (t > (int64_t)S[l].size()) {
        target[l] = t;
        grew = true;
      }
    }
    if (!grew) break;
  }
  res->trace = T;
  res->trace_imag = Ti;
  res->rel_err = err;
  res->tr_defl = tr_defl;
  for (int l = 0; l < L && l < 8; ++l) {
    res->N[l] = (int64_t)S[l].size();
    res->mean_re[l] = mean[l].real();
    res->mean_im[l] = mean[l].imag();
    res->var[l] = var[l];
    res->cost_s[l] = level_time[l];
    res->iters[l] = iters[l];
    if (p->samples_out[l]) {
      const int64_t m = std::min<int64_t>((int64_t)S[l].size(), p->max_samples[l]);
      for (int64_t i = 0; i < m; ++i) {
        p->samples_out[l][2 * i] = S[l][i].real();
        p->samples_out[l][2 * i + 1] = S[l][i].imag();
      }
    }
  }
  res->t_trace_s = now_s() - t0;
}

int tune_rhs_block(dmlmc_hier* H, const dmlmc_defl* defl, const int* cand, int ncand, dmlmc_precision prec,
                   double rtol, uint64_t noise_seed, double* sec_per_sample) {
  const int L = (int)H->lv.size();
  struct Restore {
    dmlmc_hier* H;
    const dmlmc_defl* prev;
    ~Restore() { H->coarse_defl = prev; }
  } restore{H, H->coarse_defl};
  if (defl) H->coarse_defl = defl;
  dmlmc_mlmc_params p{};
  p.noise_seed = noise_seed;
  p.prec = prec;
  p.rtol = rtol;
  p.maxiter = 2000;
  const int64_t base = (int64_t)1 << 62;  // sample indices no estimate uses
  int best = cand[0];
  double best_t = INFINITY;
  std::vector<std::complex<double>> sink;
  for (int c = 0; c < ncand; ++c) {
    const int b = cand[c];
    double t = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      t = 0.0;
      for (int l = 1; l <= L; ++l) {
        sink.clear();
        HIPCHK(hipStreamSynchronize(H->ctx->stream));
        const double t0 = now_s();
        sample_block(H, defl, l, base + (int64_t)pass * 512, b, &p, sink);
        t += (now_s() - t0) / b;
      }
    }
    if (sec_per_sample) sec_per_sample[c] = t;
    if (t < best_t) {
      best_t = t;
      best = b;
    }
  }
  H->tuned_block = best;
  return best;
}

void run_hutchinson(dmlmc_hier* H, const dmlmc_defl* fine, const dmlmc_defl* coarsest, const dmlmc_mlmc_params* p,
                    dmlmc_trace_result* res) {
  const int L = (int)H->lv.size();
  struct Restore {
    dmlmc_hier* H;
    const dmlmc_defl* prev;
    ~Restore() { H->coarse_defl = prev; }
  } restore{H, H->coarse_defl};
  // the V-cycles' coarsest solve: the given coarsest deflation (for a one-level hierarchy
  // the fine deflation is that of the coarsest level)
  if (coarsest)
    H->coarse_defl = coarsest;
  else if (L == 1 && fine)
    H->coarse_defl = fine;
  const int blk = p->rhs_block > 0 ? p->rhs_block : H->tuned_block;
  if (blk < 1) throw DmlmcError(DMLMC_ESTATE, "rhs_block = 0 but the hierarchy has no tuned block size");
  const double t0 = now_s();
  auto roundup = [&](int64_t m) { return ((m + blk - 1) / blk) * blk; };
  const int64_t n = H->lv[0].n();
  const int64_t cap = p->max_samples[0] > 0 ? p->max_samples[0] : ((int64_t)1 << 40);
  int64_t target = roundup(std::max(1, p->n0[0]));
  const double tr_defl = fine ? fine->tr_defl : 0.0;
  std::vector<std::complex<double>> S;
  int64_t iters = 0;
  double T = 0.0, Ti = 0.0, err = INFINITY, var = 0.0, level_time = 0.0;
  std::complex<double> mean(0.0, 0.0);
  while (true) {
    while ((int64_t)S.size() < std::min(target, cap)) {
      const int64_t i0 = (int64_t)S.size();
      const int b = (int)std::min<int64_t>(blk, std::min(target, cap) - i0);
      const double ts = now_s();
      c128* X = (c128*)hier_buf(H, "ml_X", 1, sizeof(c128) * (size_t)b * n);
      launch_z2<double>(H->ctx, X, n, p->noise_seed, 1, i0, b, n);
      iters += deflated_block(H, fine, 1, X, b, p, S);
      level_time += now_s() - ts;
    }
    mean = std::complex<double>(0.0, 0.0);
    for (auto v : S) mean += v;
    mean /= (double)S.size();
    double v2 = 0.0;
    for (auto v : S) v2 += std::norm(v - mean);
    var = S.size() > 1 ? v2 / (double)(S.size() - 1) : 0.0;
    T = tr_defl + mean.real();
    Ti = mean.imag();
    err = T != 0.0 ? std::sqrt(var / (double)S.size()) / std::fabs(T) : INFINITY;
    if (p->fixed_counts || err <= p->eps) break;
    // one level: N = V / (eps T)^2, the multilevel rule with a single term
    const double want = std::ceil(var / (p->eps * p->eps * T * T));
    const int64_t t = std::min(roundup(std::max<int64_t>((int64_t)want, (int64_t)S.size())), cap);
    if (t <= (int64_t)S.size()) break;
    target = t;
  }
  res->trace = T;
  res->trace_imag = Ti;
  res->rel_err = err;
  res->tr_defl = tr_defl;
  res->N[0] = (int64_t)S.size();
  res->mean_re[0] = mean.real();
  res->mean_im[0] = mean.imag();
  res->var[0] = var;
  res->cost_s[0] = level_time;
  res->iters[0] = iters;
  if (p->samples_out[0]) {
    const int64_t m = std::min<int64_t>((int64_t)S.size(), p->max_samples[0]);
    for (int64_t i = 0; i < m; ++i) {
      p->samples_out[0][2 * i] = S[i].real();
      p->samples_out[0][2 * i + 1] = S[i].imag();
    }
  }
  res->t_trace_s = now_s() - t0;
}
