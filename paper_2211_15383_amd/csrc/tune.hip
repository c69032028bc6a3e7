// Launch-variant autotuner of the hot complex-FP32 kernels of a hierarchy.
//
// Every tuned kernel has variants that divide the same work differently over threads and
// wavefronts (RHS per thread, wavefronts per site, tiles whose loads a wavefront issues at
// once); the arithmetic of each output entry is the same in all of them, so a choice never
// changes a result bit.  For each level and each kernel that runs there, the tuner times
// every variant at the level's real shape (nrhs right-hand sides at the solver's work
// stride, complex FP32) with HIP events and keeps the fastest; the built-in rule stays unless
// a variant beats it by more than 2 %.
// Choices are cached per process by (device architecture, kernel, level shape, nrhs, stride)
// and, when a cache file is named, read from and written back to it (one "key value" line
// per choice), so later hierarchies of the same shapes skip the timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "common.h"
#include "solver.h"
#include "tune.h"

namespace {

std::mutex g_cache_mu;
std::map<std::string, int> g_cache;

const char* kv_name(int k) {
  static const char* names[KV_COUNT] = {"wilson_rb", "coarse_split",   "sap_rb",         "gs_split",
                                        "restrict_ut", "prolong_mt", "prolong_staged", "restrict_staged"};
  return names[k];
}

std::string arch_name(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string a(prop.gcnArchName);
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

std::string cache_key(const std::string& arch, int k, const Level& L, int nrhs, int64_t ld) {
  std::ostringstream s;
  s << arch << '|' << kv_name(k) << '|' << L.Lx << 'x' << L.Lt << 'x' << L.dofs << "|N" << L.N << "|a" << L.ax << 'x'
    << L.at << "|b" << nrhs << "|ld" << ld << (L.Ahop16.p ? "|h16" : "");
  return s.str();
}

void load_cache_file(const std::string& path) {
  std::ifstream f(path);
  std::string key;
  int v;
  while (f >> key >> v) g_cache[key] = v;
}

void save_cache_file(const std::string& path) {
  const std::string tmp = path + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) throw DmlmcError(DMLMC_EINVAL, "cannot write the tuning cache file " + path);
    for (const auto& kv : g_cache) f << kv.first << ' ' << kv.second << '\n';
  }
  if (std::rename(tmp.c_str(), path.c_str()) != 0)
    throw DmlmcError(DMLMC_EINVAL, "cannot replace the tuning cache file " + path);
}

// candidate values of kernel k on level L (empty: the kernel does not run there)
std::vector<int> candidates(const dmlmc_hier* H, const Level& L, int k) {
  const bool last = L.l == (int)H->lv.size();
  const bool coarse16 = !L.fine && L.dofs == 16;
  const bool transfer = !last && transfer16_available(L);
  switch (k) {
    case KV_WILSON_RB: return L.fine ? std::vector<int>{1, 2, 4, 8} : std::vector<int>{};
    case KV_SAP_RB: return L.fine ? std::vector<int>{1, 2, 4, 8} : std::vector<int>{};
    case KV_COARSE_SPLIT: return coarse16 ? std::vector<int>{1, 2, 3} : std::vector<int>{};
    case KV_GS_SPLIT: return (coarse16 && L.Ahop16.p && L.Ainv16.p) ? std::vector<int>{1, 2, 3, 4} : std::vector<int>{};
    case KV_RESTRICT_UT: return (transfer && !restrict16_pair_selected(L)) ? std::vector<int>{1, 2, 4} : std::vector<int>{};
    case KV_PROLONG_STAGED:
      return (transfer && (L.dofs == 16 || transfer16_pair_available(L))) ? std::vector<int>{1, 2} : std::vector<int>{};
    case KV_RESTRICT_STAGED:
      return (transfer && transfer16_pair_available(L) && L.at <= 4) ? std::vector<int>{1, 2} : std::vector<int>{};
    case KV_PROLONG_MT: {
      if (!transfer || prolong16_pair_selected(L)) return {};
      const int tiles = L.ax * L.at * L.dofs / 16;
      std::vector<int> v;
      for (int m : {1, 2, 4})
        if (tiles % m == 0) v.push_back(m);
      return v;
    }
    default: return {};
  }
}

}  // namespace

void tune_kernels(dmlmc_hier* H, int nrhs, int reps, const char* cache_path, int* picks, double* best_us,
                  double* default_us) {
  dmlmc_ctx* ctx = H->ctx;
  const int nl = (int)H->lv.size();
  const std::string arch = arch_name(ctx->device);
  std::lock_guard<std::mutex> lock(g_cache_mu);
  if (cache_path && *cache_path) load_cache_file(cache_path);
  const bool timing = ctx->timing;
  ctx->timing = false;  // no class events around the launches timed here
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  bool tuned_any = false;
  try {
    for (int li = 0; li < nl; ++li) {
      Level& L = H->lv[li];
      const int l = li + 1;
      const int64_t ld = work_ld(H, l);
      for (int k = 0; k < KV_COUNT; ++k) {
        const int slot = li * KV_COUNT + k;
        if (picks) picks[slot] = -1;
        if (best_us) best_us[slot] = 0.0;
        if (default_us) default_us[slot] = 0.0;
      }
      std::vector<std::vector<int>> cand(KV_COUNT);
      bool any = false;
      for (int k = 0; k < KV_COUNT; ++k) {
        cand[k] = candidates(H, L, k);
        any = any || !cand[k].empty();
      }
      if (!any) continue;
      // operands: x, y on this level, xc, yc on the next (transfers); x holds Z2 noise
      c64* x = (c64*)hier_buf(H, "tn_x", l, sizeof(c64) * (size_t)nrhs * ld);
      c64* y = (c64*)hier_buf(H, "tn_y", l, sizeof(c64) * (size_t)nrhs * ld);
      c64 *xc = nullptr, *yc = nullptr;
      int64_t ldc = 0;
      if (li + 1 < nl) {
        ldc = work_ld(H, l + 1);
        xc = (c64*)hier_buf(H, "tn_xc", l, sizeof(c64) * (size_t)nrhs * ldc);
        yc = (c64*)hier_buf(H, "tn_yc", l, sizeof(c64) * (size_t)nrhs * ldc);
        launch_z2<float>(ctx, xc, H->lv[li + 1].n(), 0x7475ull, l + 1, 0, nrhs, ldc);
      }
      launch_z2<float>(ctx, x, L.n(), 0x7475ull, l, 0, nrhs, ld);
      launch_z2<float>(ctx, y, L.n(), 0x7476ull, l, 0, nrhs, ld);
      // the staged-transfer choices come before the tile counts of the kernels they replace
      static const int order[KV_COUNT] = {KV_WILSON_RB,      KV_SAP_RB,          KV_COARSE_SPLIT, KV_GS_SPLIT,
                                          KV_PROLONG_STAGED, KV_RESTRICT_STAGED, KV_RESTRICT_UT,  KV_PROLONG_MT};
      for (int k : order) {
        cand[k] = candidates(H, L, k);
        if (cand[k].empty()) continue;
        auto run = [&]() {
          switch (k) {
            case KV_WILSON_RB: launch_wilson<float>(ctx, L, x, y, nrhs, ld, ld, false); break;
            case KV_COARSE_SPLIT: launch_coarse<float>(ctx, L, x, y, nrhs, ld, ld, false); break;
            case KV_SAP_RB: launch_sap<float>(ctx, L, y, x, nrhs, 0, H->sap_mr_iters, ld); break;
            case KV_GS_SPLIT: launch_coarse_gs<float>(ctx, L, y, x, nrhs, 0, true, ld); break;
            case KV_RESTRICT_UT: launch_restrict<float>(ctx, L, x, yc, nrhs, ld, ldc); break;
            case KV_PROLONG_MT: launch_prolong<float>(ctx, L, xc, y, nrhs, false, ldc, ld); break;
            case KV_PROLONG_STAGED: launch_prolong<float>(ctx, L, xc, y, nrhs, false, ldc, ld); break;
            case KV_RESTRICT_STAGED: launch_restrict<float>(ctx, L, x, yc, nrhs, ld, ldc); break;
          }
        };
        auto time_value = [&](int v) {
          L.kv[k] = v;
          run();  // warm-up
          HIPCHK(hipEventRecord(e0, ctx->stream));
          for (int r = 0; r < reps; ++r) run();
          HIPCHK(hipEventRecord(e1, ctx->stream));
          HIPCHK(hipEventSynchronize(e1));
          float ms = 0.f;
          HIPCHK(hipEventElapsedTime(&ms, e0, e1));
          return 1e3 * (double)ms / reps;
        };
        const int slot = li * KV_COUNT + k;
        const std::string key = cache_key(arch, k, L, nrhs, ld);
        auto hit = g_cache.find(key);
        if (hit != g_cache.end() && (hit->second == 0 || std::find(cand[k].begin(), cand[k].end(), hit->second) !=
                                                               cand[k].end())) {
          L.kv[k] = hit->second;
          if (picks) picks[slot] = hit->second;
          continue;
        }
        // a variant replaces the built-in rule only when it is faster by more than 2 %
        // (launch times scatter by about 1 %; a tie keeps the rule)
        const double t0 = time_value(0);
        int best = 0;
        double tb = t0, tv = 0.0;
        int bv = 0;
        for (int v : cand[k]) {
          const double t = time_value(v);
          if (bv == 0 || t < tv) {
            tv = t;
            bv = v;
          }
        }
        if (bv != 0 && tv < 0.98 * t0) {
          best = bv;
          tb = tv;
        }
        L.kv[k] = best;
        g_cache[key] = best;
        tuned_any = true;
        if (picks) picks[slot] = best;
        if (best_us) best_us[slot] = tb;
        if (default_us) default_us[slot] = t0;
      }
      HIPCHK(hipStreamSynchronize(ctx->stream));
      for (const char* b : {"tn_x", "tn_y", "tn_xc", "tn_yc"}) hier_devbuf(H, b, l).release();
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->timing = timing;
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->timing = timing;
  ++g_dev_epoch;  // recorded graphs hold the launches of the previous variants
  if (tuned_any && cache_path && *cache_path) save_cache_file(cache_path);
}

void set_kernel_variant(dmlmc_hier* H, int level, int kernel, int value) {
  REQUIRE(level >= 1 && level <= (int)H->lv.size(), "level out of range");
  REQUIRE(kernel >= 0 && kernel < KV_COUNT, "unknown kernel id");
  static const std::vector<int> allowed[KV_COUNT] = {{0, 1, 2, 4, 8}, {0, 1, 2, 3}, {0, 1, 2, 4, 8}, {0, 1, 2, 3, 4},
                                                     {0, 1, 2, 4},    {0, 1, 2, 4}, {0, 1, 2},    {0, 1, 2}};
  REQUIRE(std::find(allowed[kernel].begin(), allowed[kernel].end(), value) != allowed[kernel].end(),
          "value not allowed for this kernel");
  H->lv[level - 1].kv[kernel] = value;
  ++g_dev_epoch;
}
