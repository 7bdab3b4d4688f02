// Measured workgroup-tile choices of the batched GEMM.  A launch is keyed by
// its element types, transposition flags, shape (m, n, k) and the log2
// buckets of its output count and of its tasks per output; tiles.txt (next
// to the library, or the file named by H2_TILE_TABLE) maps keys to tile ids,
// written by the package's tuner from timed runs of whole products.  Keys
// not in the table keep the shape heuristic of launch_bgemm.
//
// Tuning hooks (environment, read once): H2_TILE_FORCE=<id> makes every
// launch use that tile; H2_TILE_LOG=<file> appends "key tile ms" per launch
// (each launch then synchronises to be timed by itself).
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <unordered_map>

#include "internal.h"

namespace h2 {
namespace {

std::once_flag g_once;
std::unordered_map<std::string, int> g_table;
int g_force = -1;
std::string g_log_path;
std::mutex g_log_mu;

int lg2(long long v) {
  int r = 0;
  while (v > 1) {
    v >>= 1;
    ++r;
  }
  return r;
}

void init() {
  if (const char* f = std::getenv("H2_TILE_FORCE")) g_force = std::atoi(f);
  if (const char* f = std::getenv("H2_TILE_LOG")) g_log_path = f;
  std::string path;
  if (const char* f = std::getenv("H2_TILE_TABLE")) {
    path = f;
  } else {
    Dl_info info;
    if (dladdr((void*)&init, &info) && info.dli_fname) {
      path = info.dli_fname;
      const size_t slash = path.rfind('/');
      path = (slash == std::string::npos ? std::string(".") : path.substr(0, slash)) + "/tiles.txt";
    }
  }
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    if (line.empty() || line[0] == '#') continue;
    std::istringstream ss(line);
    std::string key, f;
    int vals[11], tile = -1, i = 0;
    for (; i < 11 && (ss >> vals[i]); ++i) {
    }
    if (i != 11 || !(ss >> tile) || tile < 0 || tile >= h2k::kTileCount) continue;
    for (int v : vals) key += std::to_string(v) + " ";
    g_table[key] = tile;
  }
}

}  // namespace

std::string tile_key(int tsize, int af32, int bf32, int triple, int tA, int tB, int m, int n, int k,
                     int nout, long long ntask) {
  const long long per = nout > 0 ? ntask / nout : 0;
  std::string key;
  for (long long v : {(long long)tsize, (long long)af32, (long long)bf32, (long long)triple,
                      (long long)tA, (long long)tB, (long long)m, (long long)n, (long long)k,
                      (long long)lg2(nout), (long long)lg2(per > 0 ? per : 1)})
    key += std::to_string(v) + " ";
  return key;
}

int tile_for(const std::string& key) {
  std::call_once(g_once, init);
  if (g_force >= 0 && g_force < h2k::kTileCount) return g_force;
  auto it = g_table.find(key);
  return it == g_table.end() ? -1 : it->second;
}

bool tile_logging() {
  std::call_once(g_once, init);
  return !g_log_path.empty();
}

void tile_log(const std::string& key, int tile, float ms) {
  std::lock_guard<std::mutex> lk(g_log_mu);
  FILE* f = std::fopen(g_log_path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "%s%d %.5f\n", key.c_str(), tile, ms);
  std::fclose(f);
}

}  // namespace h2
