// Tile-size autotuner: times each candidate configuration of a launch once
// (HIP events on the context's stream, after one warm-up run) and keeps the
// fastest per key, in memory and in a small JSON cache file.
//
// Key: a string naming the kernel family, the device, the HIP version, the
// precision and the shape bucket.  Environment:
//   GPBO_AUTOTUNE=0          use the first candidate (the static heuristic)
//   GPBO_AUTOTUNE_CACHE=path cache file (default $HOME/.cache/gpbo_autotune.json)
// A missing, unreadable or corrupt cache file is ignored; a cache entry whose
// value is not among the current candidates is ignored.
#include <cstdio>
#include <cstdlib>
#include <filesystem>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "gpbo_internal.h"

namespace gpbo {

namespace {

std::mutex g_mu;
std::map<std::string, int> g_best;
bool g_loaded = false;

std::string cache_path() {
  if (const char* p = std::getenv("GPBO_AUTOTUNE_CACHE")) return p;
  if (const char* h = std::getenv("HOME")) return std::string(h) + "/.cache/gpbo_autotune.json";
  return "";
}

// Lines of the form  "key": value  (other lines are skipped).
void load_cache() {
  g_loaded = true;
  const std::string path = cache_path();
  if (path.empty()) return;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t a = line.find('"');
    const size_t b = a == std::string::npos ? a : line.find('"', a + 1);
    const size_t colon = b == std::string::npos ? b : line.find(':', b + 1);
    if (colon == std::string::npos) continue;
    char* end = nullptr;
    const long v = std::strtol(line.c_str() + colon + 1, &end, 10);
    if (end == line.c_str() + colon + 1) continue;
    g_best[line.substr(a + 1, b - a - 1)] = (int)v;
  }
}

void save_cache() {
  const std::string path = cache_path();
  if (path.empty()) return;
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos && slash > 0) {
    // create the directory chain with mkdir(2); the library starts no process
    std::error_code ec;
    std::filesystem::create_directories(path.substr(0, slash), ec);
  }
  const std::string tmp = path + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) return;
    f << "{\n";
    size_t i = 0;
    for (auto& kv : g_best) f << "  \"" << kv.first << "\": " << kv.second << (++i < g_best.size() ? ",\n" : "\n");
    f << "}\n";
  }
  std::rename(tmp.c_str(), path.c_str());
}

}  // namespace

int autotune_pick(Ctx* c, const std::string& key, const std::vector<int>& cands,
                  const std::function<void(int)>& run) {
  if (cands.empty()) return 0;
  if (cands.size() == 1) return cands[0];
  const char* env = std::getenv("GPBO_AUTOTUNE");
  if (env && env[0] == '0') return cands[0];
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_loaded) load_cache();
    auto it = g_best.find(key);
    if (it != g_best.end())
      for (int v : cands)
        if (v == it->second) return v;
  }
  hipStream_t s = c->stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return cands[0];
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return cands[0];
  }
  int best = cands[0];
  float best_ms = 1e30f;
  for (int v : cands) {
    run(v);  // warm-up
    (void)hipEventRecord(e0, s);
    run(v);
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) continue;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms < best_ms) {
      best_ms = ms;
      best = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> lk(g_mu);
  g_best[key] = best;
  save_cache();
  return best;
}

}  // namespace gpbo
