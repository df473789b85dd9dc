// GEMM autotuner: for one dense GEMM step, times every valid (tile edge,
// K-split count) variant on the step's own device buffers and keeps the
// fastest.  Results are cached per process by (dtype, M, N, K, form, split
// capacity) and, when a database path is given, in a plain text file
// ("tnrcs-gemm dtype M N K form cap tile split occ ms" per line; occ is the
// variant of the FP16/BF16 128-row kernels: 1 or 2 waves per SIMD of the
// 128x128 kernel, 3 the ping-pong 256x128 kernel; 0 elsewhere).
// The same file holds the kernel-class choices of whole steps
// ("tnrcs-class dtype key class ms"), which the plan builder times itself.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "kernels.h"
#include "tune.h"

namespace tnrcs {
namespace {

using Key = std::tuple<int, int64_t, int64_t, int64_t, int, int>;  // dtype, M, N, K, form, cap

struct Choice {
  int tile = 0;
  int split = 1;
  int occ = 0;
  float ms = 0.f;
};

std::mutex g_mu;
std::map<Key, Choice> g_cache;
std::map<std::string, std::set<Key>> g_db_keys;  // keys present in each database file
std::map<std::pair<int, std::string>, int> g_class;  // (dtype, step key) -> kernel class
std::map<std::string, std::set<std::pair<int, std::string>>> g_db_class;

void load_db(const std::string& path) {
  if (g_db_keys.count(path)) return;
  std::set<Key>& have = g_db_keys[path];
  std::set<std::pair<int, std::string>>& have_c = g_db_class[path];
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return;
  char line[4096], tag[32], key[4000];
  while (std::fgets(line, sizeof line, f)) {
    int dt, form, cap, tile, split, occ, cls;
    long long M, N, K;
    float ms;
    if (std::sscanf(line, "%31s", tag) != 1) continue;
    const std::string t(tag);
    if (t == "tnrcs-gemm" && std::sscanf(line, "%31s %d %lld %lld %lld %d %d %d %d %d %f", tag, &dt, &M, &N, &K, &form,
                                         &cap, &tile, &split, &occ, &ms) == 11) {
      const Key k{dt, M, N, K, form, cap};
      g_cache[k] = Choice{tile, split, occ, ms};
      have.insert(k);
    } else if (t == "tnrcs-class" && std::sscanf(line, "%31s %d %3999s %d %f", tag, &dt, key, &cls, &ms) == 5) {
      g_class[{dt, std::string(key)}] = cls;
      have_c.insert({dt, std::string(key)});
    }
  }
  std::fclose(f);
}

void append_db(const std::string& path, const Key& k, const Choice& c) {
  if (!g_db_keys[path].insert(k).second) return;
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "tnrcs-gemm %d %lld %lld %lld %d %d %d %d %d %.5f\n", std::get<0>(k), (long long)std::get<1>(k),
               (long long)std::get<2>(k), (long long)std::get<3>(k), std::get<4>(k), std::get<5>(k), c.tile, c.split,
               c.occ, c.ms);
  std::fclose(f);
}

}  // namespace

int tune_gemm(int dtype, GemmOp& g, const void* a, const void* b, void* c, float2* w, float* slot, const char* db,
              std::string& err) {
  const Key key{dtype, g.M, g.N, g.K, g.form, g.split_max};
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (db) load_db(db);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      if (db) append_db(db, key, it->second);  // a shape tuned earlier in this process
      g.tile = it->second.tile;
      g.split_k = it->second.split;
      g.occ = it->second.occ;
      return TN_OK;
    }
  }
  const bool fits128 = g.M % 128 == 0 && g.N % 128 == 0;
  struct V {
    int tile, split, occ;
  };
  std::vector<V> variants;
  for (int sp = 1; sp <= std::max(g.split_max, 1); sp *= 2) {
    if (sp > 1 && (!w || g.K % (16 * sp) != 0)) continue;
    for (int tile : {64, 128}) {
      if (tile == 128 && !fits128) continue;
      if (dtype != TN_DTYPE_C64 && tile == 128) {
        variants.push_back({tile, sp, 1});
        variants.push_back({tile, sp, 2});
        // the ping-pong 256x128 kernel (4M form only)
        if (g.form == TN_GEMM_4M && g.M % 256 == 0 && (g.K / sp) % 32 == 0) variants.push_back({tile, sp, 3});
      } else {
        variants.push_back({tile, sp, 0});
      }
    }
  }
  auto launch = [&](const V& v) -> hipError_t {
    float2* work = v.split > 1 ? w : nullptr;
    if (dtype == TN_DTYPE_C64)
      return launch_gemm_c64((const float2*)a, (const float2*)b, (float2*)c, g.M, g.N, g.K, 1, g.form, nullptr, work,
                             v.split, v.tile);
    return launch_gemm_half(dtype, a, b, c, g.M, g.N, g.K, 1, g.form, nullptr, work, v.split, 1.f, slot, v.tile,
                            v.occ);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    err = "tuner: event create failed";
    if (e0) hipEventDestroy(e0);
    return TN_E_HIP;
  }
  Choice best;
  best.ms = INFINITY;
  int rc = TN_OK;
  for (const V& v : variants) {
    float t1 = 0.f, tr = 0.f;
    hipError_t e = hipEventRecord(e0, nullptr);
    if (e == hipSuccess) e = launch(v);
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&t1, e0, e1);
    // repeat to about 2 ms of work (at most 20 runs)
    const int reps = std::max(1, std::min(20, (int)std::ceil(2.0 / std::max(t1, 1e-3f))));
    if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch(v);
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&tr, e0, e1);
    if (e != hipSuccess) {
      err = std::string("tuner: ") + hipGetErrorString(e);
      rc = TN_E_HIP;
      break;
    }
    const float ms = tr / reps;
    if (ms < best.ms) best = Choice{v.tile, v.split, v.occ, ms};
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  if (variants.empty()) return TN_OK;
  g.tile = best.tile;
  g.split_k = best.split;
  g.occ = best.occ;
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache[key] = best;
  if (db) append_db(db, key, best);
  return TN_OK;
}

bool class_lookup(int dtype, const std::string& key, const char* db, int* cls) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (db) load_db(db);
  auto it = g_class.find({dtype, key});
  if (it == g_class.end()) return false;
  *cls = it->second;
  if (db && g_db_class[db].insert({dtype, key}).second) {  // chosen earlier in this process
    if (FILE* f = std::fopen(db, "a")) {
      std::fprintf(f, "tnrcs-class %d %s %d %.5f\n", dtype, key.c_str(), *cls, 0.f);
      std::fclose(f);
    }
  }
  return true;
}

void class_store(int dtype, const std::string& key, const char* db, int cls, float ms) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_class[{dtype, key}] = cls;
  if (!db) return;
  load_db(db);
  if (!g_db_class[db].insert({dtype, key}).second) return;
  if (FILE* f = std::fopen(db, "a")) {
    std::fprintf(f, "tnrcs-class %d %s %d %.5f\n", dtype, key.c_str(), cls, ms);
    std::fclose(f);
  }
}

}  // namespace tnrcs
