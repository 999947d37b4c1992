// Autotuner for the dslash launch shape.  Searched, per launch key:
//   nr     right-hand sides per thread (1..4);
//   nsub   y-sub-slabs of an XCD's sweep (shortens the reuse distance of the
//          t-neighbours);
//   lds    16-bit formats: LDS staging of the x/y neighbours;
//   rloop  binary16 with 12-real links: one thread per site looping over
//          every right-hand side;
//   block  workgroup size (128 or 256; 512 for the RHS loop);
//   wgs    cap on workgroups per CU, i.e. on waves per SIMD (LDS reserved
//          so that only that many fit).
// Launches with a fused dot product keep one sub-slab and 256-thread
// workgroups, so each partial record covers a fixed set of sites and the
// reductions give the same bits for every tuned shape; their search covers
// nr, lds, rloop and wgs.  (link_nt, a cache hint for link loads, and out_nt
// are still parsed but not searched: neither paid on the lattices measured.)
//
// A key is (lattice, precision, RHS count of the launch, link format and
// basis, form), the form being adjoint or not, xpay or not, the fused dot,
// and whether the launch covers a mapped subset of the batch (the solvers'
// reliable-update launches over the updating right-hand sides).  The first
// eager launch of a key times each candidate with HIP events on the caller's
// stream, in that launch's own form and on its own fields (outputs are
// rewritten, inputs only read, so the repeats are harmless), and keeps the
// fastest: the best of two timings of five launches each, after a warm-up.
// The search is greedy: nr, nsub, lds and rloop first, then the workgroup
// size for the winner, then the occupancy cap for that; a subset launch
// stops after the first stage with one sub-slab.  Last, the (up to four)
// shapes within 3% of the fastest are timed again over 20 launches each, in
// two interleaved rounds, and the best of those longer timings wins: five
// launches cannot separate shapes that close.  Launches made
// while the stream is being captured into a graph, or whose output aliases
// one of their inputs (xpay source, y, in), use the default shape and do not
// tune.
//
// WD_TUNE=0 disables tuning; WD_TUNE_CACHE=<file> keeps the choices across
// processes (one "Lx Ly Lz Lt prec nrhs flags form nr block gslow nsub
// link_nt lds rloop wgs" line per entry; flags = 1 for 8-real links + 2 for
// temporal gauge + 4 for UKQCD-basis fields; form = 1 adjoint + 2 xpay +
// 4 * dot mode + 32 mapped subset); WD_TUNE_VERBOSE=1 prints every timed
// candidate to stderr (the final re-timings marked "re-timed");
// WD_DSLASH_SHAPE="nr,gslow,nsub[,link_nt[,out_nt[,wgs
// [,lds[,rloop[,block]]]]]]" forces a shape (the RHS-group-slowest order is
// not searched: it never paid).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>
#include <vector>

#include "wd_internal.h"

namespace wd {

namespace {

using Key = std::tuple<int, int, int, int, int, int, int>;  // Lx, Ly, Lz, Lt*8+prec, nrhs, flags, form

std::mutex g_mu;
std::map<Key, LaunchCfg> g_cache;
bool g_loaded = false;

int launch_rhs(const DslashArgs& d) { return d.rhs_map ? d.n_map : d.out.nrhs; }

bool has_dot(const DslashArgs& d) { return d.xpay && d.dot != DOT_NONE; }

int form_of(const DslashArgs& d) {
  return (d.dagger ? 1 : 0) | (d.xpay ? 2 : 0) | ((d.xpay ? d.dot : 0) << 2) | (d.rhs_map ? 32 : 0);
}

Key key_of(const wd_gauge* g, wd_prec prec, const DslashArgs& d) {
  const Geom& geo = g->geom;
  return Key{geo.L[0], geo.L[1], geo.L[2], geo.L[3] * 8 + static_cast<int>(prec), launch_rhs(d),
             (g->recon == 8 ? 1 : 0) | (g->tgauge ? 2 : 0) | (d.basis == kBasisUK ? 4 : 0), form_of(d)};
}

LaunchCfg default_cfg(int nrhs) { return LaunchCfg{nrhs == 1 ? 1 : 2, 256}; }

// A configuration the launchers accept: 128 or 256 threads (512 for the RHS
// loop), slots 1..4 (1 for the RHS loop), caps 0 or 2..8.
bool valid_cfg(const LaunchCfg& c) {
  const bool block_ok = c.block == 128 || c.block == 256 || (c.rloop && c.block == 512);
  return block_ok && c.nr >= 1 && c.nr <= 4 && !(c.rloop && c.nr != 1) && (c.gslow == 0 || c.gslow == 1) &&
         c.nsub >= 1 && c.nsub <= 8 && (c.link_nt == 0 || c.link_nt == 1) && (c.out_nt == 0 || c.out_nt == 1) &&
         (c.wgs == 0 || (c.wgs >= 2 && c.wgs <= 8)) && (c.lds == 0 || c.lds == 1) && (c.rloop == 0 || c.rloop == 1);
}

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
  int v[16];
  while (std::fscanf(f, "%d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5],
                     &v[6], &v[7], &v[8], &v[9], &v[10], &v[11], &v[12], &v[13], &v[14], &v[15]) == 16) {
    LaunchCfg c{v[8], v[9], v[10], v[11], v[12]};
    c.lds = v[13];
    c.rloop = v[14];
    c.wgs = v[15];
    if (valid_cfg(c)) g_cache[Key{v[0], v[1], v[2], v[3] * 8 + v[4], v[5], v[6], v[7]}] = c;
  }
  std::fclose(f);
}

void save_entry_locked(const Key& k, const LaunchCfg& c) {
  const char* path = cache_path();
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d\n", std::get<0>(k), std::get<1>(k),
               std::get<2>(k), std::get<3>(k) / 8, std::get<3>(k) % 8, std::get<4>(k), std::get<5>(k),
               std::get<6>(k), c.nr, c.block, c.gslow, c.nsub, c.link_nt, c.lds, c.rloop, c.wgs);
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

constexpr int kReps = 5;       // launches per timing in the search
constexpr int kLongReps = 20;  // launches per timing of the finalists
constexpr int kFinalists = 4;
constexpr float kFinalistBand = 1.03f;

// Milliseconds per launch of configuration c in the launch's own form, or -1.
float time_cfg(const wd_gauge* g, wd_prec prec, const DslashArgs& d, const LaunchCfg& c, hipStream_t s,
               int reps = kReps) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1.0f;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1.0f;
  }
  launch_dslash_cfg(g, prec, d, c, s);  // warm-up
  (void)hipEventRecord(e0, s);
  for (int i = 0; i < reps; ++i) launch_dslash_cfg(g, prec, d, c, s);
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

struct Search {
  const wd_gauge* g;
  wd_prec prec;
  const DslashArgs& d;
  hipStream_t s;
  LaunchCfg best;
  float best_ms = -1.0f;
  std::vector<std::pair<LaunchCfg, float>> tried;  // every shape that launched, with its time

  void report(const LaunchCfg& c, const char* tag, float ms) const {
    if (verbose())
      std::fprintf(stderr,
                   "[wd tune] %dx%dx%dx%d prec %d nrhs %d form %d: nr %d nsub %d lds %d rloop %d block %d wgs %d"
                   "%s -> %.1f us\n",
                   g->geom.L[0], g->geom.L[1], g->geom.L[2], g->geom.L[3], (int)prec, launch_rhs(d), form_of(d),
                   c.nr, c.nsub, c.lds, c.rloop, c.block, c.wgs, tag, ms * 1e3f);
  }

  // the better of two timings, so that a clock ramp-up does not decide
  void try_cfg(const LaunchCfg& c) {
    float ms = time_cfg(g, prec, d, c, s);
    const float ms2 = time_cfg(g, prec, d, c, s);
    if (ms2 > 0.0f && (ms < 0.0f || ms2 < ms)) ms = ms2;
    report(c, "", ms);
    if (ms <= 0.0f) return;
    tried.emplace_back(c, ms);
    if (best_ms < 0.0f || ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }

  // the shapes within the band of the fastest, timed again over longer runs
  // in interleaved rounds; the best longer timing wins
  void refine() {
    std::vector<std::pair<LaunchCfg, float>> fin;
    for (const auto& t : tried)
      if (t.second <= best_ms * kFinalistBand) fin.push_back(t);
    if (fin.size() < 2) return;
    std::stable_sort(fin.begin(), fin.end(), [](const auto& a, const auto& b) { return a.second < b.second; });
    if (fin.size() > (size_t)kFinalists) fin.resize(kFinalists);
    std::vector<float> t(fin.size(), -1.0f);
    for (int round = 0; round < 2; ++round)
      for (size_t i = 0; i < fin.size(); ++i) {
        const float ms = time_cfg(g, prec, d, fin[i].first, s, kLongReps);
        if (ms > 0.0f && (t[i] < 0.0f || ms < t[i])) t[i] = ms;
      }
    int k = -1;
    for (size_t i = 0; i < fin.size(); ++i) {
      report(fin[i].first, " re-timed", t[i]);
      if (t[i] > 0.0f && (k < 0 || t[i] < t[k])) k = (int)i;
    }
    if (k >= 0) {
      best = fin[k].first;
      best_ms = t[k];
    }
  }
};

LaunchCfg run_tuner(const wd_gauge* g, wd_prec prec, const DslashArgs& d, hipStream_t s) {
  const int n = launch_rhs(d);
  const bool dot = has_dot(d);
  // a subset launch (one key per subset size, tuned when that size first
  // occurs inside a solve) searches the slots only, to keep that first time short
  const bool mapped = d.rhs_map != nullptr;
  const bool slab = g->geom.L[2] % 8 == 0;
  const int max_nsub = (dot || mapped) ? 1 : (slab ? 4 : 1);
  Search S{g, prec, d, s, default_cfg(n)};
  // 1. slots, sub-slabs, LDS staging.  One RHS also tries a two-slot thread:
  // its empty slot costs arithmetic but no memory traffic, and in FP64 the
  // two-slot kernel has measured faster.
  for (int nr = 1; nr <= 4; ++nr) {
    if (nr > std::max(n, 2)) break;
    if (g->recon == 8 && nr > 2) break;  // 8-real kernels exist for one and two slots
    for (int nsub = 1; nsub <= max_nsub; nsub *= 2) {
      if (g->geom.L[1] % nsub) continue;
      for (int lds = 0; lds <= 1; ++lds) {
        if (lds && !(is_half(prec) && nr <= 3 && g->recon == 12 && slab)) continue;
        LaunchCfg c{nr, 256, 0, nsub, 0};
        c.lds = lds;
        S.try_cfg(c);
      }
    }
  }
  //    binary16 with 12-real links: one thread per site over every RHS
  if (prec == WD_HALF_F16 && g->recon == 12 && n >= 2) {
    for (int nsub = 1; nsub <= ((dot || mapped) ? 1 : (slab ? 8 : 1)); nsub *= 2) {
      if (g->geom.L[1] % nsub) continue;
      for (int lds = 0; lds <= (slab ? 1 : 0); ++lds) {
        LaunchCfg c{1, 256, 0, nsub, 0};
        c.rloop = 1;
        c.lds = lds;
        S.try_cfg(c);
      }
    }
  }
  if (mapped) return S.best;
  // 2. workgroup size of the winner (fused dots keep 256)
  if (!dot) {
    const LaunchCfg w = S.best;
    for (int block : {128, 512}) {
      if (block == 512 && !w.rloop) continue;
      LaunchCfg c = w;
      c.block = block;
      S.try_cfg(c);
    }
  }
  // 3. occupancy cap of the winner: at most wgs workgroups per CU
  {
    const LaunchCfg w = S.best;
    const int per_wg = w.block / 64;  // waves per workgroup
    for (int wgs : {2, 3, 4, 6}) {
      if (wgs * per_wg > 32) continue;  // no tighter than the 8 waves per SIMD a CU holds
      LaunchCfg c = w;
      c.wgs = wgs;
      S.try_cfg(c);
    }
  }
  // 4. the finalists, timed again over longer runs
  S.refine();
  return S.best;
}

}  // namespace

LaunchCfg tuned_dslash_config(const wd_gauge* g, wd_prec prec, const DslashArgs& d, hipStream_t s) {
  const int nrhs = launch_rhs(d);
  // WD_DSLASH_SHAPE forces one shape (tests sweep them with it)
  if (const char* f = std::getenv("WD_DSLASH_SHAPE")) {
    int nr = 1, gslow = 0, nsub = 1, nt = 0, ont = 0, wgs = 0, lds = 0, rloop = 0, block = 256;
    const int n = std::sscanf(f, "%d,%d,%d,%d,%d,%d,%d,%d,%d", &nr, &gslow, &nsub, &nt, &ont, &wgs, &lds, &rloop,
                              &block);
    const LaunchCfg c{nr, block, gslow, nsub, nt, ont, wgs, lds, rloop};
    if (n >= 3 && valid_cfg(c)) return c;
  }
  const Key k = key_of(g, prec, d);
  {
    std::lock_guard<std::mutex> lock(g_mu);
    load_cache_locked();
    auto it = g_cache.find(k);
    if (it != g_cache.end()) return it->second;
  }
  if (!tuning_enabled() || d.no_tune) return default_cfg(nrhs);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return default_cfg(nrhs);
  // repeated launches must leave the result unchanged: no output may alias an input
  if ((d.xpay && d.xpay->ptr == d.out.ptr) || (d.y && d.y->ptr == d.out.ptr) || d.in.ptr == d.out.ptr)
    return default_cfg(nrhs);
  const LaunchCfg best = run_tuner(g, prec, d, s);
  std::lock_guard<std::mutex> lock(g_mu);
  g_cache[k] = best;
  save_entry_locked(k, best);
  return best;
}

void tune_dslash(const wd_gauge* g, wd_prec prec, const DslashArgs& d, hipStream_t s) {
  (void)tuned_dslash_config(g, prec, d, s);
}

}  // namespace wd
