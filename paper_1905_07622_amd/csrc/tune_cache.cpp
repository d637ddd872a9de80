// Tile cache of the autotuner: one JSON file of records
//   {"key": "<arch>|hip<version>|<fp64|mixed>|<box|cubic|tet6>|<single|batch>|<px>x<py>x<pz>",
//    "tile": [tx, ty, tz], "best_us": t, "rule_us": t0, "candidates": n}
// one record per line inside {"femheat_tune": 1, "entries": [ ... ]}.  The
// key names what the launch shape depends on: the GPU architecture, the HIP
// runtime, the precision of the hot gather, the element class, whether the
// simulation runs alone or as a member of a batch, and the node grid.
// Readers take the last record of a key; writers rewrite the whole file
// through a temporary file and a rename, under a process-wide lock.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "tune.hpp"

namespace femheat {
namespace {

std::mutex g_cache_mu;

struct Record {
  int tile[3] = {0, 0, 0};
  double best_us = 0.0, rule_us = 0.0;
  int candidates = 0;
};

// Parses the records of a cache file (unknown lines are skipped).
std::map<std::string, Record> read_all(const char* path) {
  std::map<std::string, Record> out;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    const size_t k = line.find("\"key\": \"");
    if (k == std::string::npos) continue;
    const size_t k0 = k + 8, k1 = line.find('"', k0);
    if (k1 == std::string::npos) continue;
    Record r;
    const size_t t = line.find("\"tile\": [", k1);
    if (t == std::string::npos) continue;
    if (std::sscanf(line.c_str() + t + 9, "%d, %d, %d", &r.tile[0], &r.tile[1], &r.tile[2]) != 3) continue;
    const size_t b = line.find("\"best_us\": ", k1);
    if (b != std::string::npos) std::sscanf(line.c_str() + b + 11, "%lf", &r.best_us);
    const size_t u = line.find("\"rule_us\": ", k1);
    if (u != std::string::npos) std::sscanf(line.c_str() + u + 11, "%lf", &r.rule_us);
    const size_t c = line.find("\"candidates\": ", k1);
    if (c != std::string::npos) std::sscanf(line.c_str() + c + 14, "%d", &r.candidates);
    if (r.tile[0] > 0 && r.tile[1] > 0 && r.tile[2] > 0) out[line.substr(k0, k1 - k0)] = r;
  }
  return out;
}

}  // namespace

std::string tune_key(int device, bool mixed, int kind, bool batched, int px, int py, int pz) {
  static std::mutex mu;
  static std::map<int, std::string> arch;
  std::string a;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = arch.find(device);
    if (it == arch.end()) {
      hipDeviceProp_t p{};
      std::string name = "unknown";
      if (hipGetDeviceProperties(&p, device) == hipSuccess) {
        name = p.gcnArchName;
        const size_t colon = name.find(':');
        if (colon != std::string::npos) name = name.substr(0, colon);  // drop target features
      } else {
        (void)hipGetLastError();
      }
      it = arch.emplace(device, name).first;
    }
    a = it->second;
  }
  int ver = 0;
  if (hipRuntimeGetVersion(&ver) != hipSuccess) (void)hipGetLastError();
  std::ostringstream k;
  k << a << "|hip" << ver << "|" << (mixed ? "mixed" : "fp64") << "|" << (kind == 2 ? "tet6" : kind == 1 ? "cubic" : "box") << "|"
    << (batched ? "batch" : "single") << "|" << px << "x" << py << "x" << pz;
  return k.str();
}

bool tune_lookup(const char* path, const std::string& key, int tile[3]) {
  if (!path || !*path) return false;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  const auto all = read_all(path);
  auto it = all.find(key);
  if (it == all.end()) return false;
  for (int d = 0; d < 3; ++d) tile[d] = it->second.tile[d];
  return true;
}

bool tune_store(const char* path, const std::string& key, const int tile[3], double best_us, double rule_us,
                int candidates) {
  if (!path || !*path) return false;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto all = read_all(path);
  Record r;
  for (int d = 0; d < 3; ++d) r.tile[d] = tile[d];
  r.best_us = best_us;
  r.rule_us = rule_us;
  r.candidates = candidates;
  all[key] = r;
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream out(tmp, std::ios::trunc);
    if (!out) return false;
    out << "{\"femheat_tune\": 1, \"entries\": [\n";
    size_t i = 0;
    for (const auto& kv : all) {
      const Record& e = kv.second;
      char buf[160];
      std::snprintf(buf, sizeof(buf), "\"tile\": [%d, %d, %d], \"best_us\": %.3f, \"rule_us\": %.3f, \"candidates\": %d}",
                    e.tile[0], e.tile[1], e.tile[2], e.best_us, e.rule_us, e.candidates);
      out << "{\"key\": \"" << kv.first << "\", " << buf << (++i < all.size() ? ",\n" : "\n");
    }
    out << "]}\n";
    if (!out) return false;
  }
  return std::rename(tmp.c_str(), path) == 0;
}

}  // namespace femheat
