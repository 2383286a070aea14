// Launch-shape tuner.  For a plan it times every compiled variant of the per-iteration kernels
// on the plan's own buffers (HIP events on the plan's stream, one warm-up launch, then a few
// timed ones) and keeps the fastest:
//   time FFTs (steps (a) and (c)): transforms per workgroup NB, NB/2, NB/4, or NB with 1024
//   threads and radix-8 passes;
//   matvec: the three-stage register FFT (L >= 256), or LDS Stockham passes with the default
//   workgroup size, the other size (256 <-> 512), or radix 8 (1024 threads for L = 8192);
//   triangular solves (exact spatial solver): one workgroup per block, or a persistent grid.
// Results are cached per shape in the process and, when the environment variable
// RFDE_TUNE_CACHE names a file, in that file (lines "key value"), so a shape is timed once.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>

#include "rfde_internal.hpp"

namespace rfde {
namespace {

std::mutex g_mu;
std::map<std::string, int> g_cache;
bool g_loaded = false;

const char* cache_path() {
  const char* p = std::getenv("RFDE_TUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

void load_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const char* path = cache_path();
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char key[256];
  int val;
  while (std::fscanf(f, "%255s %d", key, &val) == 2) g_cache[key] = val;
  std::fclose(f);
}

void store_locked(const std::string& key, int val) {
  g_cache[key] = val;
  const char* path = cache_path();
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d\n", key.c_str(), val);
  std::fclose(f);
}

bool lookup(const std::string& key, int* val) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_locked();
  auto it = g_cache.find(key);
  if (it == g_cache.end()) return false;
  *val = it->second;
  return true;
}

void remember(const std::string& key, int val) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_locked();
  store_locked(key, val);
}

std::string key_of(const char* kind, const Plan& p, long a, long b) {
  char buf[128];
  std::snprintf(buf, sizeof buf, "%s_%ld_%ld_%d", kind, a, b, p.opts.precond_bits);
  return buf;
}

// Mean ms of `reps` launches of fn after one warm-up launch.
template <typename F>
int time_ms(Plan& p, F fn, int reps, double* ms) {
  RFDE_TRY(fn());
  RFDE_HIP(hipEventRecord(p.ev[2], p.stream));
  for (int r = 0; r < reps; ++r) RFDE_TRY(fn());
  RFDE_HIP(hipEventRecord(p.ev[3], p.stream));
  RFDE_HIP(hipEventSynchronize(p.ev[3]));
  float t = 0.f;
  RFDE_HIP(hipEventElapsedTime(&t, p.ev[2], p.ev[3]));
  *ms = t / reps;
  return RFDE_OK;
}

}  // namespace

int tune_plan(Plan& p, int what, rfde_tune_report* rep) {
  rfde_tune_report r{};
  const size_t N = p.N();
  // inputs for timing: zeros (the kernels' cost does not depend on the values)
  RFDE_HIP(hipMemsetAsync(p.wvec, 0, N * sizeof(double), p.stream));
  RFDE_HIP(hipMemsetAsync(p.xvec, 0, N * sizeof(double), p.stream));
  const int reps = 3;

  // time FFTs: forward + inverse together
  const std::string kt = key_of("time", p, p.Lt, p.S);
  int best = p.tv_time;
  if (!(what & 1)) {
  } else if (lookup(kt, &best)) {
    r.from_cache |= 1;
  } else {
    double bms = 1e300;
    const int nv = p.Lt == p.Nt ? 4 : 3;  // variant 3 exists for power-of-two N_t only
    for (int v = 0; v < nv; ++v) {
      p.tv_time = v;
      double ms = 0;
      RFDE_TRY(time_ms(p, [&]() -> int {
        RFDE_TRY(launch_time_fwd(p, p.wvec, p.zf));
        return launch_time_inv(p, p.zf, p.xvec);
      }, reps, &ms));
      r.ms_time[v] = ms;
      if (ms < bms) { bms = ms; best = v; }
    }
    remember(kt, best);
  }
  p.tv_time = best;
  r.time_variant = best;

  // matvec (1D)
  best = p.tv_matvec;
  if (p.dim == 1 && (what & 2)) {
    const std::string km = key_of("matvec", p, p.L, p.Nt);
    if (lookup(km, &best)) {
      r.from_cache |= 2;
    } else {
      double bms = 1e300;
      for (int v = 0; v < 4; ++v) {
        p.tv_matvec = v;
        double ms = 0;
        RFDE_TRY(time_ms(p, [&]() -> int { return launch_matvec(p, p.wvec, p.xvec); }, reps, &ms));
        r.ms_matvec[v] = ms;
        if (ms < bms) { bms = ms; best = v; }
      }
      remember(km, best);
    }
  }
  p.tv_matvec = best;
  r.matvec_variant = best;

  // triangular solves: out of place into the (m N doubles) Z basis, which holds the nf x M
  // complex outputs whenever m >= 2
  best = p.trsv_cap;
  const size_t csz = p.opts.precond_bits == 32 ? 8 : 16;
  if ((what & 4) && p.factor_bytes && (size_t)p.nf * p.S * csz <= (size_t)p.opts.restart * N * sizeof(double)) {
    const std::string ks = key_of("trsv", p, p.T, p.nb);
    if (lookup(ks, &best)) {
      r.from_cache |= 4;
    } else {
      static const int caps[5] = {0, 256, 512, 1024, 2048};
      double bms = 1e300;
      for (int c = 0; c < 5; ++c) {
        r.trsv_caps[c] = caps[c];
        if (caps[c] != 0 && caps[c] >= p.nb) { r.ms_trsv[c] = -1.0; continue; }
        p.trsv_cap = caps[c];
        double ms = 0;
        RFDE_TRY(time_ms(p, [&]() -> int { return launch_trsv(p, p.zf, p.zbuf); }, 2, &ms));
        r.ms_trsv[c] = ms;
        if (ms < bms) { bms = ms; best = caps[c]; }
      }
      remember(ks, best);
    }
  }
  p.trsv_cap = best;
  r.trsv_grid_cap = best;
  RFDE_HIP(hipStreamSynchronize(p.stream));
  if (rep) *rep = r;
  return RFDE_OK;
}

}  // namespace rfde

extern "C" int rfde_plan_autotune(rfde_plan plan, rfde_tune_report* report) {
  rfde::Plan* p = reinterpret_cast<rfde::Plan*>(plan);
  if (!p) return RFDE_EINVAL;
  return rfde::tune_plan(*p, 7, report);
}

extern "C" int rfde_plan_set_variants(rfde_plan plan, int time_variant, int matvec_variant,
                                      int trsv_grid_cap) {
  rfde::Plan* p = reinterpret_cast<rfde::Plan*>(plan);
  if (!p || time_variant < 0 || time_variant > 3 || matvec_variant < 0 || matvec_variant > 3 ||
      trsv_grid_cap < 0)
    return RFDE_EINVAL;
  p->tv_time = time_variant;
  p->tv_matvec = matvec_variant;
  p->trsv_cap = trsv_grid_cap;
  return RFDE_OK;
}
