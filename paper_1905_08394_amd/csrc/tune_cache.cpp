// Tile choices of the autotuner kept across processes: a small JSON object in
// the file named by PSIM_TUNE_CACHE, one member per (device architecture,
// precision, interior-site contraction shape) holding the tile candidate
// psim_tune measured fastest and its time.  psim_tune merges its results into
// the file (written whole to a temporary file, then renamed); psim_plan reads
// it and starts from the stored choices.  Without PSIM_TUNE_CACHE nothing is
// read or written.
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <sstream>
#include <string>

#include <hip/hip_runtime_api.h>

#include "psim_internal.hpp"

namespace psim {

namespace {

const char* cache_path() {
  const char* p = std::getenv("PSIM_TUNE_CACHE");
  return (p && p[0]) ? p : nullptr;
}

const char* prec_name(int prec) {
  switch (prec) {
    case PSIM_FP64: return "fp64";
    case PSIM_FP32_4M: return "fp32_4m";
    case PSIM_FP32_3M: return "fp32_3m";
    case PSIM_BF16X3: return "bf16x3";
    default: return "unknown";
  }
}

// Members of the object, one per line as tune_cache_store writes them:
//   "key": {"cfg": 2, "ms": 83.75},
std::map<std::string, std::pair<int, double>> read_all(const char* path) {
  std::map<std::string, std::pair<int, double>> out;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t a = line.find('"');
    if (a == std::string::npos) continue;
    const size_t b = line.find('"', a + 1);
    const size_t c = line.find("\"cfg\":");
    const size_t d = line.find("\"ms\":");
    if (b == std::string::npos || c == std::string::npos || c < b) continue;
    const int cfg = std::atoi(line.c_str() + c + 6);
    const double ms = d == std::string::npos ? 0.0 : std::atof(line.c_str() + d + 5);
    out[line.substr(a + 1, b - a - 1)] = {cfg, ms};
  }
  return out;
}

}  // namespace

std::string device_arch(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string name = prop.gcnArchName;
  const size_t colon = name.find(':');
  return colon == std::string::npos ? name : name.substr(0, colon);
}

std::string tune_key(const std::string& arch, int prec, int64_t M, int64_t K1, int64_t K2, int64_t N, int64_t Bz,
                     bool split) {
  std::ostringstream k;
  k << arch << "|" << prec_name(prec) << (split ? "_split" : "") << "|M=" << M << "|K1=" << K1 << "|K2=" << K2
    << "|N=" << N << "|Bz=" << Bz;
  return k.str();
}

bool tune_cache_lookup(const std::string& key, int* cfg) {
  const char* path = cache_path();
  if (!path) return false;
  const auto all = read_all(path);
  const auto it = all.find(key);
  if (it == all.end()) return false;
  *cfg = it->second.first;
  return true;
}

void tune_cache_store(const std::map<std::string, std::pair<int, double>>& entries) {
  const char* path = cache_path();
  if (!path || entries.empty()) return;
  auto all = read_all(path);
  for (const auto& kv : entries) all[kv.first] = kv.second;
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) fail(PSIM_EINVAL, std::string("cannot write the tune cache ") + tmp);
    f << "{\n";
    size_t i = 0;
    for (const auto& kv : all) {
      char ms[64];
      std::snprintf(ms, sizeof ms, "%.6g", kv.second.second);
      f << "  \"" << kv.first << "\": {\"cfg\": " << kv.second.first << ", \"ms\": " << ms << "}"
        << (++i < all.size() ? "," : "") << "\n";
    }
    f << "}\n";
  }
  if (std::rename(tmp.c_str(), path) != 0) fail(PSIM_EINVAL, std::string("cannot replace the tune cache ") + path);
}

}  // namespace psim
