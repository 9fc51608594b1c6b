// In-process autotuner: the first call of a tunable launch with a new shape
// times every variant on the caller's own data (HIP events on the caller's
// stream, one untimed launch then the median of three) and keeps the fastest;
// later calls with that shape reuse the choice.  Choices can be persisted as
// JSON lines in the file named by the environment variable AWG_TUNE_CACHE
// (read once at the first lookup, appended after each new measurement).
// Every variant of a tunable kernel computes bit-identical results, so the
// choice affects time only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "awg_common.h"
#include "awg_tune.h"

namespace awg {
namespace {

struct Choice {
  int variant = 0;
  std::vector<double> us;   // measured time per variant (microseconds)
};

std::mutex g_mu;
std::map<std::string, Choice> g_cache;
bool g_loaded = false;
bool g_enabled = true;

void load_file() {
  if (g_loaded) return;
  g_loaded = true;
  const char* path = std::getenv("AWG_TUNE_CACHE");
  if (!path || !*path) return;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    // {"key":"...","variant":V}
    const size_t k0 = line.find("\"key\":\"");
    const size_t v0 = line.find("\"variant\":");
    if (k0 == std::string::npos || v0 == std::string::npos) continue;
    const size_t ks = k0 + 7, ke = line.find('"', ks);
    if (ke == std::string::npos) continue;
    Choice c;
    c.variant = std::atoi(line.c_str() + v0 + 10);
    g_cache[line.substr(ks, ke - ks)] = c;
  }
}

void append_file(const std::string& key, const Choice& c) {
  const char* path = std::getenv("AWG_TUNE_CACHE");
  if (!path || !*path) return;
  std::ofstream f(path, std::ios::app);
  f << "{\"key\":\"" << key << "\",\"variant\":" << c.variant << ",\"us\":[";
  for (size_t i = 0; i < c.us.size(); ++i) f << (i ? "," : "") << c.us[i];
  f << "]}\n";
}

}  // namespace

int tune_lookup(const std::string& key) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_file();
  if (!g_enabled) return 0;
  auto it = g_cache.find(key);
  return it == g_cache.end() ? -1 : it->second.variant;
}

int tune_pick(const std::string& key, int nvar, const std::function<void(int)>& run, hipStream_t s) {
  const int known = tune_lookup(key);
  if (known >= 0) return std::min(known, nvar - 1);
  Choice c;
  c.us.assign(nvar, 0.0);
  hipEvent_t a, b;
  AWG_HIP(hipEventCreate(&a));
  AWG_HIP(hipEventCreate(&b));
  try {
    for (int v = 0; v < nvar; ++v) {
      run(v);   // untimed
      std::vector<double> t(3);
      for (int r = 0; r < 3; ++r) {
        AWG_HIP(hipEventRecord(a, s));
        run(v);
        AWG_HIP(hipEventRecord(b, s));
        AWG_HIP(hipEventSynchronize(b));
        float ms = 0.f;
        AWG_HIP(hipEventElapsedTime(&ms, a, b));
        t[r] = 1e3 * ms;
      }
      std::sort(t.begin(), t.end());
      c.us[v] = t[1];
    }
  } catch (...) {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    throw;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  c.variant = (int)(std::min_element(c.us.begin(), c.us.end()) - c.us.begin());
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache[key] = c;
  append_file(key, c);
  return c.variant;
}

void tune_enable(bool on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_enabled = on;
}

std::string tune_json() {
  std::lock_guard<std::mutex> lk(g_mu);
  std::ostringstream o;
  o.precision(6);
  o << "{";
  bool first = true;
  for (auto& kv : g_cache) {
    o << (first ? "" : ",") << "\"" << kv.first << "\":{\"variant\":" << kv.second.variant << ",\"us\":[";
    for (size_t i = 0; i < kv.second.us.size(); ++i) o << (i ? "," : "") << kv.second.us[i];
    o << "]}";
    first = false;
  }
  o << "}";
  return o.str();
}

}  // namespace awg
