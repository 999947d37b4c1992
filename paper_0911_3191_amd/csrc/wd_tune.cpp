// Autotuner for the dslash launch shape: right-hand sides per thread (nr),
// y-sub-slabs of an XCD's sweep (nsub, shortens the reuse distance of the
// t-neighbours), for the 16-bit formats LDS staging of the x/y neighbours
// (lds), and for binary16 with 12-real links one thread per site looping
// over every right-hand side (rloop).  (link_nt, a cache hint for link loads, is still parsed
// but the kernels no longer use it and it is not searched.)
//
// The first eager launch for a (lattice, precision, nrhs) times each
// candidate with HIP events on the caller's stream, using the plain
// out = D in form on the caller's own fields, and keeps the fastest.
// Launches made while the stream is being captured into a graph, or whose
// output aliases their xpay source, use the default shape instead and do not
// tune.  WD_TUNE=0 disables tuning; WD_TUNE_CACHE=<file> keeps the choices
// across processes (one "Lx Ly Lz Lt prec nrhs flags nr block gslow nsub
// link_nt lds rloop" line per entry, flags = 1 for 8-real links + 2 for temporal
// gauge + 4 for UKQCD-basis fields); WD_TUNE_VERBOSE=1 prints every timed candidate to stderr;
// WD_DSLASH_SHAPE="nr,gslow,nsub[,link_nt[,out_nt[,wgs[,lds[,rloop]]]]]" forces a shape
// (the RHS-group-slowest order, streaming output stores and the occupancy
// cap are not searched: none paid on the lattices measured).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <algorithm>

#include "wd_internal.h"

namespace wd {

namespace {

using Key = std::tuple<int, int, int, int, int, int>;  // dims, prec, nrhs, link and basis flags

std::mutex g_mu;
std::map<Key, LaunchCfg> g_cache;
bool g_loaded = false;

Key key_of(const wd_gauge* g, wd_prec prec, int nrhs, int basis) {
  const Geom& geo = g->geom;
  return Key{geo.L[0], geo.L[1], geo.L[2], geo.L[3] * 8 + static_cast<int>(prec), nrhs,
             (g->recon == 8 ? 1 : 0) | (g->tgauge ? 2 : 0) | (basis == kBasisUK ? 4 : 0)};
}

LaunchCfg default_cfg(wd_prec, int nrhs) { return LaunchCfg{nrhs == 1 ? 1 : 2, 256}; }

const char* cache_path() {
  const char* p = std::getenv("WD_TUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

void load_cache_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const char* path = cache_path();
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  int lx, ly, lz, lt, prec, nrhs, flags, nr, block, gslow, nsub, nt, lds, rloop;
  while (std::fscanf(f, "%d %d %d %d %d %d %d %d %d %d %d %d %d %d", &lx, &ly, &lz, &lt, &prec, &nrhs, &flags, &nr,
                     &block, &gslow, &nsub, &nt, &lds, &rloop) == 14) {
    if (nr >= 1 && nr <= 4 && block == 256 && (gslow == 0 || gslow == 1) && nsub >= 1 && nsub <= 8 &&
        (nt == 0 || nt == 1) && (lds == 0 || lds == 1) && (rloop == 0 || rloop == 1)) {
      LaunchCfg c{nr, block, gslow, nsub, nt};
      c.lds = lds;
      c.rloop = rloop;
      g_cache[Key{lx, ly, lz, lt * 8 + prec, nrhs, flags}] = c;
    }
  }
  std::fclose(f);
}

void save_entry_locked(const Key& k, const LaunchCfg& c) {
  const char* path = cache_path();
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%d %d %d %d %d %d %d %d %d %d %d %d %d %d\n", std::get<0>(k), std::get<1>(k), std::get<2>(k),
               std::get<3>(k) / 8, std::get<3>(k) % 8, std::get<4>(k), std::get<5>(k), c.nr, c.block, c.gslow,
               c.nsub, c.link_nt, c.lds, c.rloop);
  std::fclose(f);
}

bool tuning_enabled() {
  const char* e = std::getenv("WD_TUNE");
  return !(e && e[0] == '0');
}

bool verbose() {
  const char* e = std::getenv("WD_TUNE_VERBOSE");
  return e && e[0] == '1';
}

// Milliseconds per launch of configuration c (plain out = D in), or -1.
float time_cfg(const wd_gauge* g, wd_prec prec, const DslashArgs& plain, const LaunchCfg& c,
               hipStream_t s) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1.0f;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1.0f;
  }
  launch_dslash_cfg(g, prec, plain, c, s);  // warm-up
  const int reps = 2;
  (void)hipEventRecord(e0, s);
  for (int i = 0; i < reps; ++i) launch_dslash_cfg(g, prec, plain, c, s);
  (void)hipEventRecord(e1, s);
  float ms = -1.0f;
  if (hipGetLastError() == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
      hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
    ms /= reps;
  else
    ms = -1.0f;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

LaunchCfg run_tuner(const wd_gauge* g, wd_prec prec, const DslashArgs& d, hipStream_t s) {
  DslashArgs plain = d;
  plain.xpay = nullptr;
  plain.dot = DOT_NONE;
  plain.y = nullptr;
  LaunchCfg best = default_cfg(prec, d.out.nrhs);
  float best_ms = -1.0f;
  // Kernels carry 1..4 RHS slots per thread (one RHS also tries a two-slot
  // thread: its empty slot costs arithmetic but no memory traffic, and in FP64
  // the two-slot kernel has measured faster).
  const bool slab = g->geom.L[2] % 8 == 0;
  for (int nr = 1; nr <= 4; ++nr) {
    if (nr > std::max(d.out.nrhs, 2)) break;
    if (g->recon == 8 && nr > 2) break;  // 8-real kernels exist for two slots
    for (int nsub = 1; nsub <= (slab ? 4 : 1); nsub *= 2) {
      if (g->geom.L[1] % nsub) continue;
      for (int v = 0; v < 4; ++v) {
        const int nt = v & 1, lds = v >> 1;
        if (nt) continue;  // the link cache hint is not used by the kernels
        if (lds && !(is_half(prec) && nr <= 3 && g->recon == 12 && slab)) continue;
        const int gslow = 0;
        LaunchCfg c{nr, 256, gslow, nsub, nt};
        c.lds = lds;
        // the better of two timings, so a clock ramp-up does not decide
        float ms = time_cfg(g, prec, plain, c, s);
        const float ms2 = time_cfg(g, prec, plain, c, s);
        if (ms2 > 0.0f && (ms < 0.0f || ms2 < ms)) ms = ms2;
        if (verbose())
          std::fprintf(stderr, "[wd tune] %dx%dx%dx%d prec %d nrhs %d: nr %d nsub %d link_nt %d lds %d -> %.1f us\n",
                       g->geom.L[0], g->geom.L[1], g->geom.L[2], g->geom.L[3], (int)prec, d.out.nrhs,
                       nr, nsub, nt, lds, ms * 1e3f);
        if (ms > 0.0f && (best_ms < 0.0f || ms < best_ms)) {
          best_ms = ms;
          best = c;
        }
      }
    }
  }
  // binary16 with 12-real links: one thread per site over every RHS
  if (prec == WD_HALF_F16 && g->recon == 12 && d.out.nrhs >= 2) {
    for (int nsub = 1; nsub <= (slab ? 8 : 1); nsub *= 2) {
      if (g->geom.L[1] % nsub) continue;
      for (int lds = 0; lds <= (slab ? 1 : 0); ++lds) {
        LaunchCfg c{1, 256, 0, nsub, 0};
        c.rloop = 1;
        c.lds = lds;
        float ms = time_cfg(g, prec, plain, c, s);
        const float ms2 = time_cfg(g, prec, plain, c, s);
        if (ms2 > 0.0f && (ms < 0.0f || ms2 < ms)) ms = ms2;
        if (verbose())
          std::fprintf(stderr, "[wd tune] %dx%dx%dx%d prec %d nrhs %d: rhs loop nsub %d lds %d -> %.1f us\n",
                       g->geom.L[0], g->geom.L[1], g->geom.L[2], g->geom.L[3], (int)prec, d.out.nrhs, nsub, lds,
                       ms * 1e3f);
        if (ms > 0.0f && (best_ms < 0.0f || ms < best_ms)) {
          best_ms = ms;
          best = c;
        }
      }
    }
  }
  return best;
}

}  // namespace

LaunchCfg tuned_dslash_config(const wd_gauge* g, wd_prec prec, const DslashArgs& d, hipStream_t s) {
  const int nrhs = d.out.nrhs;
  // WD_DSLASH_SHAPE="nr,gslow,nsub[,link_nt]" forces one shape (tests sweep them with it)
  if (const char* f = std::getenv("WD_DSLASH_SHAPE")) {
    int nr = 1, gslow = 0, nsub = 1, nt = 0, ont = 0, wgs = 0, lds = 0, rloop = 0;
    const int n = std::sscanf(f, "%d,%d,%d,%d,%d,%d,%d,%d", &nr, &gslow, &nsub, &nt, &ont, &wgs, &lds, &rloop);
    if (n >= 3 && nr >= 1 && nr <= 4 && (gslow == 0 || gslow == 1) && nsub >= 1 && nsub <= 8 &&
        (nt == 0 || nt == 1) && (ont == 0 || ont == 1) && wgs >= 0 && wgs <= 8 && (lds == 0 || lds == 1) &&
        (rloop == 0 || rloop == 1))
      return LaunchCfg{nr, 256, gslow, nsub, nt, ont, wgs, lds, rloop};
  }
  const Key k = key_of(g, prec, nrhs, d.basis);
  {
    std::lock_guard<std::mutex> lock(g_mu);
    load_cache_locked();
    auto it = g_cache.find(k);
    if (it != g_cache.end()) return it->second;
  }
  if (!tuning_enabled() || d.no_tune) return default_cfg(prec, nrhs);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
    return default_cfg(prec, nrhs);
  if (d.xpay && d.xpay->ptr == d.out.ptr) return default_cfg(prec, nrhs);
  if (d.rhs_map) return default_cfg(prec, nrhs);  // a launch over part of the batch does not tune
  const LaunchCfg best = run_tuner(g, prec, d, s);
  std::lock_guard<std::mutex> lock(g_mu);
  g_cache[k] = best;
  save_entry_locked(k, best);
  return best;
}

void tune_dslash(const wd_gauge* g, wd_prec prec, Field out, Field in, int basis, hipStream_t s) {
  DslashArgs d;
  d.out = out;
  d.in = in;
  d.out_parity = 1;
  d.basis = basis;
  (void)tuned_dslash_config(g, prec, d, s);
}

}  // namespace wd
