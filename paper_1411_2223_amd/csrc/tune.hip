// tune.hip -- autotuner for the Dslash launch (QUDA's automatic choice of
// running parameters is the idea, section "CPS & QUDA"; this one is written
// for gfx950): times each candidate RHS tile (columns per thread) on the
// caller's own buffers and keeps the fastest per (device, lattice, link tier,
// vector tiers, epilogue, columns).  Results live in memory and, when the
// environment variable ASQ_TUNE_CACHE names a file, in that file as one JSON
// object mapping each key to its launch variant code.
// ASQ_TUNE=0 turns timing off and uses the built-in defaults.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "asq_internal.h"

namespace asq {
namespace {

std::mutex g_mu;
std::map<std::string, int> g_cache;
bool g_loaded = false;

std::string key_of(const asq_gauge* g, int link, int in, int out, int epi, int ncol) {
  char buf[160];
  hipDeviceProp_t prop;
  const char* arch = "gfx";
  if (hipGetDeviceProperties(&prop, g->device) == hipSuccess) arch = prop.gcnArchName;
  snprintf(buf, sizeof(buf), "%s/%dx%dx%dx%d/L%d/I%d/O%d/E%d/N%d", arch, g->geom.X, g->geom.Y, g->geom.Z,
           g->geom.T, link, in, out, epi, ncol);
  for (char* c = buf; *c; ++c)
    if (*c == ' ' || *c == ':') *c = '_';
  return buf;
}

void load_cache_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const char* path = getenv("ASQ_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  // the file this library writes: one "key": code pair per line
  char line[256], k[200];
  int v;
  while (fgets(line, sizeof(line), f))
    if (sscanf(line, " \"%199[^\"]\" : %d", k, &v) == 2) g_cache[k] = v;
  fclose(f);
}

void save_cache_locked() {
  const char* path = getenv("ASQ_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "w");
  if (!f) return;
  fprintf(f, "{\n");
  size_t n = 0;
  for (auto& kv : g_cache)
    fprintf(f, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++n < g_cache.size() ? "," : "");
  fprintf(f, "}\n");
  fclose(f);
}

int default_rtile(int link, int ncol) {
  if (ncol <= 1) return 1;
  if (link == LINK_F64_R18) return 2;
  return ncol >= 4 ? 4 : 2;
}

bool tuning_on() {
  const char* e = getenv("ASQ_TUNE");
  return !(e && e[0] == '0');
}

}  // namespace

// ASQ_VARIANT=<code> (decimal) replaces the tuned launch variant wherever the
// library builds that variant for the tier (tests use it to run every variant
// through the solver epilogues).
int forced_variant(int link, int in) {
  const char* e = getenv("ASQ_VARIANT");
  if (!e || !*e) return -1;
  const int v = atoi(e);
  return variant_built(link, in, v) ? v : -1;
}

int tuned_rtile(const asq_gauge* g, int link, int in, int out, int epi, int ncol) {
  const int fv = forced_variant(link, in);
  // a forced tile wider than the batch, or whose LDS window does not fit this
  // lattice, is ignored, except the matrix-core form, which masks its idle
  // columns; that form takes alpha from the column state, so it is not forced
  // where the update launch forms alpha itself
  if (fv >= 0 && !(fv & kMfmaBit) && (fv & 0xff) <= (ncol > 1 ? ncol : 1) && variant_fits(g->geom, in, fv)) return fv;
  if (fv >= 0 && (fv & kMfmaBit) && ncol > kFoldAlphaMaxTile) return fv;
  std::lock_guard<std::mutex> lk(g_mu);
  load_cache_locked();
  auto it = g_cache.find(key_of(g, link, in, out, epi, ncol));
  // a cache file may come from another build: only variants the tuner itself
  // could have chosen are taken from it
  if (it != g_cache.end() && variant_built(link, in, it->second) && !(it->second & kMfmaBit) &&
      (it->second & 0xff) <= (ncol > 1 ? ncol : 1) && variant_fits(g->geom, in, it->second))
    return it->second;
  return default_rtile(link, ncol);
}

// True when tune_dslash would time candidates for this configuration (timing
// on, no recorded winner), so the caller can put trial data in place first.
bool tune_pending(const asq_gauge* g, int link, int in, int ncol, int epi_timed) {
  if (!tuning_on()) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  load_cache_locked();
  return g_cache.count(key_of(g, link, in, in, epi_timed, ncol)) == 0;
}

// Time the PLAIN Dslash (the loop shared by every epilogue) for each tile on
// in_buf -> out_buf and record the winner for every epilogue; with
// epi = EPI_CANON, time and record the public operator on the canonical
// layouts instead.  Buffers are the caller's: in_buf is only read, out_buf is
// scratch.  persist = false keeps the winners out of the ASQ_TUNE_CACHE file
// (timings taken while other work may share the device).
int tune_dslash(const asq_gauge* g, int link, int in, int ncol, const void* in_buf, void* out_buf,
                hipStream_t s, int epi_timed, bool persist) {
  const std::string kp = key_of(g, link, in, in, epi_timed, ncol);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache_locked();
    if (g_cache.count(kp)) return ASQ_OK;
  }
  int best = default_rtile(link, ncol);
  int best_update = best;  // the UPDATE epilogue's pick: no tile wider than 8 columns
  if (tuning_on()) {
    DslashArgs a;
    memset(&a, 0, sizeof(a));
    a.g = g->geom;
    a.out_parity = 1;
    a.ncol = ncol;
    a.links = g->links[link];
    a.in = in_buf;
    a.out = out_buf;
    a.mask = MASK_ALL;
    a.nblk = g->nblk;
    a.coeff_fat = g->desc.fat_scale;
    a.coeff_long = g->desc.long_scale;
    hipEvent_t e0, e1;
    ASQ_HIP_TRY(hipEventCreate(&e0));
    ASQ_HIP_TRY(hipEventCreate(&e1));
    float best_ms = 1e30f, best_update_ms = 1e30f;
    // columns per thread x hop-loop form x block order (orders differ only when
    // there are several tiles) x XCD slabs or one global sweep (of single blocks
    // or of runs of blocks per XCD)
    std::vector<int> cands;
    for (int gs = 0; gs < 2; ++gs)
      for (int order = 0; order < 4; ++order)
        for (int pipe = 0; pipe < 2; ++pipe)
          for (int cols : {1, 2, 4, 6, 8, 12})
            if (order == 0 || (ncol + cols - 1) / cols >= 2) cands.push_back(make_rtile(cols, pipe, order, gs != 0));
    // runs of 16, 64 or 256 blocks per XCD inside the sweep: pipelined loop, the
    // first two block orders
    for (int chunk = 1; chunk <= 3; ++chunk)
      for (int order = 0; order < 2; ++order)
        for (int cols : {1, 2, 4, 6, 8, 12})
          if (order == 0 || (ncol + cols - 1) / cols >= 2) cands.push_back(make_rtile(cols, true, order, true, chunk));
    // one-column tiles with streamed links, where the tier has that form
    {
      const size_t n = cands.size();
      for (size_t q = 0; q < n; ++q)
        if ((cands[q] & 0xff) == 1 && variant_built(link, in, cands[q] | kStreamBit)) cands.push_back(cands[q] | kStreamBit);
    }
    // and every pipelined candidate with the LDS window (the canonical layouts
    // refuse it, and so do windows too large for LDS; a candidate that fails to
    // launch is skipped)
    {
      const size_t n = cands.size();
      for (size_t q = 0; q < n; ++q)
        if (variant_built(link, in, cands[q] | kLdsBit)) cands.push_back(cands[q] | kLdsBit);
    }
    // The solver runs D_oe forwards and D_eo backwards, so each sweep starts on
    // the links and vectors the previous one left in the memory-side cache; the
    // candidates are timed in that pattern (pairs of launches), best of two.
    auto pair = [&](int r) {
      bool ok = true;
      for (int k = 0; k < 2 && ok; ++k) {
        a.out_parity = k ? 0 : 1;
        a.reverse = k;
        ok = launch_dslash(link, in, in, epi_timed, r, a, s) == ASQ_OK;
      }
      return ok;
    };
    for (int r : cands) {
      const int cols = r & 0xff;
      if (cols > 1 && cols > ncol) continue;  // a wider tile than the batch only wastes lanes
      if (!pair(r)) continue;  // warm-up
      // a candidate whose timing fails is skipped
      float ms = 1e30f;
      bool ok = true;
      for (int rep = 0; rep < 2 && ok; ++rep) {
        ok = hipEventRecord(e0, s) == hipSuccess && pair(r) && pair(r) && hipEventRecord(e1, s) == hipSuccess &&
             hipEventSynchronize(e1) == hipSuccess;
        float t = 0;
        ok = ok && hipEventElapsedTime(&t, e0, e1) == hipSuccess;
        if (ok && t < ms) ms = t;
      }
      if (!ok) continue;
      if (log_enabled()) fprintf(stderr, "[asq] tune %s R=%d %.3f ms\n", kp.c_str(), r, ms / 4);
      if (ms < best_ms) {
        best_ms = ms;
        best = r;
      }
      // the UPDATE epilogue also keeps r, x and the direction of every column of
      // the tile live: the 12-column tile loses occupancy there that the plain
      // loop timed here does not show
      if (cols <= 8 && ms < best_update_ms) {
        best_update_ms = ms;
        best_update = r;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (epi_timed == EPI_CANON) {
    g_cache[kp] = best;
  } else {
    for (int epi = EPI_PLAIN; epi <= EPI_RESID; ++epi)
      for (int out = VEC_F64; out <= VEC_F16; ++out)
        g_cache[key_of(g, link, in, out, epi, ncol)] = epi == EPI_UPDATE ? best_update : best;
  }
  if (persist) save_cache_locked();
  return ASQ_OK;
}

}  // namespace asq
