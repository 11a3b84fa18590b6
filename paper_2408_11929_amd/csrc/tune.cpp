// Autotuner of the sweep's segment plan.
//
// A sweep launch can run on one, two or sixteen workgroups per chain (plans
// 0, 2, 1), or on one workgroup per tile of two right-hand sides (choice 3).  Which is fastest depends on the strips (band half-width, rows),
// the number of chains in the launch and the device, so the engine measures
// every plan that fits a launch the first time it meets a launch of that
// shape, keeps the fastest, and reuses it for every later launch of the same
// shape.  Shapes are keyed by precision, blocked term count, segments per
// workgroup, band half-width, mesh size, strip count and the chain count
// rounded up to a power of two.  The choices can be saved to and loaded from
// a JSON file (and are, when HH_TUNE_CACHE names one), so that a deployment
// replays them instead of measuring again.
//
// Tuning is off unless asked for (hh_autotune or HH_AUTOTUNE=1): the plans
// add the same terms in different orders, so a measured choice, which can
// vary with timing noise from one process to the next, would make the last
// bits of a result vary with it.  With tuning off, a loaded or saved choice
// is still used, and otherwise the fixed rule of sweep_plan_for.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "tune.h"

namespace hh {

namespace {

std::mutex g_mu;
std::map<TuneKey, TuneEntry> g_table;
int g_enabled = -1;  // -1: not yet read from the environment
bool g_loaded = false;

const char* cache_path() {
  const char* p = std::getenv("HH_TUNE_CACHE");
  return p && *p ? p : nullptr;
}

// The file format is the one tune_save writes: one JSON object per entry.
bool load_locked(const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
  std::fclose(f);
  size_t pos = 0;
  int loaded = 0;
  while ((pos = text.find("{\"precision\"", pos)) != std::string::npos) {
    TuneKey k{};
    TuneEntry e{};
    const int n = std::sscanf(text.c_str() + pos,
                              "{\"precision\": %d, \"KP\": %d, \"P\": %d, \"kmax\": %d, \"n\": %d, "
                              "\"N\": %d, \"chains\": %d, \"plan\": %d, \"ms\": [%lf, %lf, %lf, %lf]",
                              &k.prec, &k.KP, &k.P, &k.kmax, &k.n, &k.N, &k.chains, &e.plan,
                              &e.ms[0], &e.ms[1], &e.ms[2], &e.ms[3]);
    if (n == 12 && e.plan >= 0 && e.plan < HH_NCHOICE) {
      g_table[k] = e;
      ++loaded;
    }
    pos += 1;
  }
  return loaded > 0 || text.find("\"entries\"") != std::string::npos;
}

bool save_locked(const char* path) {
  FILE* f = std::fopen(path, "w");
  if (!f) return false;
  std::fprintf(f, "{\"entries\": [\n");
  size_t i = 0;
  for (const auto& kv : g_table) {
    const TuneKey& k = kv.first;
    const TuneEntry& e = kv.second;
    std::fprintf(f,
                 "  {\"precision\": %d, \"KP\": %d, \"P\": %d, \"kmax\": %d, \"n\": %d, \"N\": %d, "
                 "\"chains\": %d, \"plan\": %d, \"ms\": [%.6f, %.6f, %.6f, %.6f]}%s\n",
                 k.prec, k.KP, k.P, k.kmax, k.n, k.N, k.chains, e.plan, e.ms[0], e.ms[1], e.ms[2],
                 e.ms[3], ++i < g_table.size() ? "," : "");
  }
  std::fprintf(f, "]}\n");
  return std::fclose(f) == 0;
}

void ensure_loaded_locked() {
  if (g_loaded) return;
  g_loaded = true;
  if (const char* p = cache_path()) load_locked(p);
}

}  // namespace

int tune_bucket(int chains) {
  int b = 1;
  while (b < chains) b *= 2;
  return b;
}

bool tune_enabled() {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_enabled < 0) {
    const char* e = std::getenv("HH_AUTOTUNE");
    g_enabled = e && std::atoi(e) > 0 ? 1 : 0;
  }
  return g_enabled == 1;
}

void tune_set_enabled(bool on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_enabled = on ? 1 : 0;
}

bool tune_lookup(const TuneKey& k, int& plan) {
  std::lock_guard<std::mutex> lk(g_mu);
  ensure_loaded_locked();
  auto it = g_table.find(k);
  if (it == g_table.end()) return false;
  plan = it->second.plan;
  return true;
}

void tune_store(const TuneKey& k, const TuneEntry& e) {
  std::lock_guard<std::mutex> lk(g_mu);
  ensure_loaded_locked();
  g_table[k] = e;
  if (const char* p = cache_path()) save_locked(p);
}

bool tune_save(const char* path) {
  std::lock_guard<std::mutex> lk(g_mu);
  return save_locked(path);
}

bool tune_load(const char* path) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_loaded = true;
  return load_locked(path);
}

void tune_clear() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
  g_loaded = true;
}

size_t tune_entries() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_table.size();
}

}  // namespace hh
