// Autotuner of single sgemm launches: times the compiled tiles of one
// precision on a problem and caches the fastest (HPVM report, Sec. 3.4
// leaves tile sizes to autotuning tools).  Host code only.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include <unistd.h>

#include "device_common.hpp"
#include "hpvm_sgemm.h"
#include "internal.hpp"

#ifndef HPVM_TARGET_ARCH
#define HPVM_TARGET_ARCH "gfx950"
#endif

namespace hpvm {
namespace {

struct Choice {
  hpvm_tile tile;  // fastest tile overall
  float ms;
  hpvm_tile fused;  // fastest tile that needs no workspace
  float fused_ms;
};

using Key = std::tuple<int32_t, int64_t, int64_t, int64_t, int32_t>;  // prec, m|cls, n|cls, k|cls, is_class

std::mutex g_mu;
std::map<Key, Choice> g_cache;

int32_t clog2(int64_t v) {
  int32_t c = 0;
  while ((int64_t(1) << c) < v) ++c;
  return c;
}

Key exact_key(int32_t prec, int64_t m, int64_t n, int64_t k) { return Key{prec, m, n, k, 0}; }
Key class_key(int32_t prec, int64_t m, int64_t n, int64_t k) {
  return Key{prec, clog2(m), clog2(n), clog2(k), 1};
}

bool in_menu(int32_t prec, const hpvm_tile& t) { return find_menu_entry(prec, t) != nullptr; }

bool needs_workspace(int32_t prec, const hpvm_tile& t) {
  const MfmaEntry* e = find_menu_entry(prec, t);
  return e && e->launch_staged;
}

void record(int32_t prec, int64_t m, int64_t n, int64_t k, const Choice& c) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache[exact_key(prec, m, n, k)] = c;
  g_cache[class_key(prec, m, n, k)] = c;
}

// A choice from one tile: its no-workspace fallback is menu entry 0 unless
// the tile itself needs none.
Choice single_choice(int32_t prec, const hpvm_tile& t, float ms) {
  Choice c{t, ms, t, ms};
  if (needs_workspace(prec, t)) {
    c.fused = menu_entry_at(prec, 0)->tile;
    c.fused_ms = -1.0f;
  }
  return c;
}

// What a saved entry is valid for: the GPU architecture (the current
// device's, without its feature suffix, else the one this library is
// compiled for) and the HIP runtime version in use (else the one it was
// built against).  Timings taken on another architecture or runtime say
// nothing about this one, so loading skips entries with another tag.
std::string cache_tag() {
  std::string arch = HPVM_TARGET_ARCH;
  int count = 0, dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDeviceCount(&count) == hipSuccess && count > 0 && hipGetDevice(&dev) == hipSuccess &&
      hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.gcnArchName[0]) {
    arch.assign(prop.gcnArchName, strnlen(prop.gcnArchName, sizeof prop.gcnArchName));
    arch = arch.substr(0, arch.find(':'));
  }
  (void)hipGetLastError();  // a host without a device leaves an error behind
  int runtime = 0;
  if (hipRuntimeGetVersion(&runtime) != hipSuccess || runtime <= 0) runtime = HIP_VERSION;
  (void)hipGetLastError();
  char buf[96];
  std::snprintf(buf, sizeof buf, "%s hip%d", arch.c_str(), runtime);
  return buf;
}

// The cache as text, one entry per line (see hpvm_autotune_save), written
// to a file of its own and renamed over `path`, so that a reader (or another
// process saving the same cache) never sees a half-written file.
bool save_file(const char* path) {
  const std::string tmp = std::string(path) + ".tmp" + std::to_string((long long)getpid());
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  const std::string tag = cache_tag();
  std::fprintf(f,
               "# hpvm_sgemm autotune cache v3: arch runtime | prec m n k | best tile (m n k leaf_m leaf_n "
               "stages) ms | best tile without workspace, ms\n");
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto& kv : g_cache) {
      if (std::get<4>(kv.first)) continue;  // class entries are rebuilt on load
      const hpvm_tile& t = kv.second.tile;
      const hpvm_tile& u = kv.second.fused;
      std::fprintf(f, "%s %d %lld %lld %lld %d %d %d %d %d %d %.6f %d %d %d %d %d %d %.6f\n", tag.c_str(),
                   std::get<0>(kv.first),
                   (long long)std::get<1>(kv.first), (long long)std::get<2>(kv.first),
                   (long long)std::get<3>(kv.first), t.tile_m, t.tile_n, t.tile_k, t.leaf_m, t.leaf_n, t.stages,
                   kv.second.ms, u.tile_m, u.tile_n, u.tile_k, u.leaf_m, u.leaf_n, u.stages, kv.second.fused_ms);
    }
  }
  const bool written = !std::ferror(f);
  if (std::fclose(f) != 0 || !written || std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return false;
  }
  return true;
}

// Merges a saved cache: entries timed on another architecture or runtime,
// and entries whose tiles this library does not hold, are skipped.
bool load_file(const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  const std::string tag = cache_tag();
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#') continue;
    char arch[64], runtime[32];
    int prec;
    long long m, n, k;
    hpvm_tile t, u;
    float ms, ums;
    if (std::sscanf(line, "%63s %31s %d %lld %lld %lld %d %d %d %d %d %d %f %d %d %d %d %d %d %f", arch, runtime,
                    &prec, &m, &n, &k, &t.tile_m, &t.tile_n, &t.tile_k, &t.leaf_m, &t.leaf_n, &t.stages, &ms,
                    &u.tile_m, &u.tile_n, &u.tile_k, &u.leaf_m, &u.leaf_n, &u.stages, &ums) != 20)
      continue;
    if (tag != std::string(arch) + " " + runtime) continue;  // timed on another device or runtime
    if (m < 0 || n < 0 || k < 0 || !in_menu(prec, t) || !in_menu(prec, u) || needs_workspace(prec, u)) continue;
    record(prec, m, n, k, Choice{t, ms, u, ums});
  }
  std::fclose(f);
  return true;
}

// HPVM_AUTOTUNE_CACHE names a file the cache persists in across processes:
// merged in at the library's first use of the cache (a missing file is an
// empty cache), written back after every tuning or record.
const char* env_path() {
  const char* p = std::getenv("HPVM_AUTOTUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

void env_cache() {
  static std::once_flag once;
  std::call_once(once, [] {
    if (const char* p = env_path()) (void)load_file(p);
  });
}

void env_save() {
  if (const char* p = env_path()) (void)save_file(p);
}

}  // namespace

// Used by hpvm_sgemm / hpvm_sgemm_ws when no tile is given: 2 exact, 1
// class, 0 none.
int tuned_tile(int32_t prec, int64_t m, int64_t n, int64_t k, bool allow_workspace, hpvm_tile* out) {
  env_cache();
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_cache.find(exact_key(prec, m, n, k));
  int found = 2;
  if (it == g_cache.end()) {
    it = g_cache.find(class_key(prec, m, n, k));
    found = 1;
  }
  if (it == g_cache.end()) return 0;
  *out = allow_workspace ? it->second.tile : it->second.fused;
  return found;
}

}  // namespace hpvm

using namespace hpvm;

extern "C" {

int hpvm_autotune(int64_t m, int64_t n, int64_t k, int32_t prec, const float* A, int64_t lda, const float* B,
                  int64_t ldb, float* C_scratch, int64_t ldc, void* workspace, int64_t workspace_bytes, int32_t reps,
                  void* stream, hpvm_tile* best, float* best_ms) {
  bool reads_ab = false;
  int rc = check_gemm_args("", m, n, k, 1.0f, A, lda, B, ldb, 0.0f, C_scratch, ldc, &reads_ab);
  if (rc != HPVM_OK) return rc;
  const int count = menu_size(prec);
  if (count == 0) return set_error(HPVM_INVALID_ARG, "argument 4: unknown precision %d", prec);
  if (workspace_bytes < 0 || (workspace_bytes > 0 && !workspace))
    return set_error(HPVM_INVALID_ARG, "argument 11/12: bad workspace");
  if (reps < 1) return set_error(HPVM_INVALID_ARG, "argument 13: reps = %d < 1", reps);
  if (!reads_ab) return set_error(HPVM_INVALID_ARG, "nothing to time: m, n and k must be positive");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  auto run = [&](const MfmaEntry* me) {
    return hpvm_sgemm_ws(m, n, k, 1.0f, A, lda, B, ldb, 0.0f, C_scratch, ldc, prec, &me->tile, workspace,
                         workspace_bytes, stream);
  };
  // Two interleaved rounds over the menu; each tile keeps its faster round,
  // so a clock ramp or a one-off stall does not decide the choice.  Tiles
  // needing more workspace than given are skipped.
  std::vector<float> best_of(count, -1.0f);
  for (int round = 0; round < 2 && e == hipSuccess && rc == HPVM_OK; ++round) {
    for (int i = 0; i < count && e == hipSuccess; ++i) {
      const MfmaEntry* me = menu_entry_at(prec, i);
      if (entry_workspace_bytes(me, m, n, k) > workspace_bytes) continue;
      if (me->launch_staged && !staged_k_ok(k)) continue;
      rc = run(me);
      if (rc != HPVM_OK) break;
      e = hipEventRecord(e0, s);
      for (int r = 0; r < reps && e == hipSuccess && rc == HPVM_OK; ++r) rc = run(me);
      if (rc != HPVM_OK) break;
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess && (best_of[i] < 0.0f || ms < best_of[i])) best_of[i] = ms;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc != HPVM_OK) return rc;
  if (e != hipSuccess) return hip_error(e, "autotune timing");
  // The fallback without a workspace is the fastest entry that ran without
  // one: neither staged nor split into contraction slices.
  auto used_workspace = [&](const MfmaEntry* me) {
    const int64_t split = entry_split_bytes(me, m, n, k);
    return me->launch_staged ||
           (split > 0 && workspace && (uintptr_t)workspace % 16 == 0 && workspace_bytes >= split);
  };
  int bi = -1, bf = -1;
  for (int i = 0; i < count; ++i) {
    if (best_of[i] < 0.0f) continue;
    if (bi < 0 || best_of[i] < best_of[bi]) bi = i;
    if (!used_workspace(menu_entry_at(prec, i)) && (bf < 0 || best_of[i] < best_of[bf])) bf = i;
  }
  if (bi < 0 || bf < 0) return set_error(HPVM_INVALID_ARG, "no tile could be timed");
  Choice c{menu_entry_at(prec, bi)->tile, best_of[bi] / (float)reps, menu_entry_at(prec, bf)->tile,
           best_of[bf] / (float)reps};
  env_cache();
  record(prec, m, n, k, c);
  env_save();
  if (best) *best = c.tile;
  if (best_ms) *best_ms = c.ms;
  return clear_error();
}

int hpvm_autotune_lookup(int64_t m, int64_t n, int64_t k, int32_t prec, hpvm_tile* tile, int32_t* found) {
  if (m < 0 || n < 0 || k < 0) return set_error(HPVM_INVALID_ARG, "sizes must be >= 0");
  const MfmaEntry* menu;
  if (mfma_menu(prec, &menu) == 0) return set_error(HPVM_INVALID_ARG, "argument 4: unknown precision %d", prec);
  if (!tile || !found) return set_error(HPVM_INVALID_ARG, "NULL output");
  *found = tuned_tile(prec, m, n, k, true, tile);
  if (*found == 0) *tile = menu[0].tile;
  return clear_error();
}

int hpvm_autotune_record(int64_t m, int64_t n, int64_t k, int32_t prec, const hpvm_tile* tile, float ms) {
  if (m < 0 || n < 0 || k < 0) return set_error(HPVM_INVALID_ARG, "sizes must be >= 0");
  if (!tile) return set_error(HPVM_INVALID_ARG, "argument 5: tile is NULL");
  if (!in_menu(prec, *tile)) return set_error(HPVM_UNSUPPORTED, "argument 5: tile not compiled for precision %d", prec);
  env_cache();
  record(prec, m, n, k, single_choice(prec, *tile, ms));
  env_save();
  return clear_error();
}

int hpvm_autotune_clear(void) {
  env_cache();  // a cache file merged later would bring the entries back
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache.clear();
  return clear_error();
}

int hpvm_autotune_save(const char* path) {
  if (!path) return set_error(HPVM_INVALID_ARG, "argument 1: path is NULL");
  if (!save_file(path)) return set_error(HPVM_INVALID_ARG, "cannot write %s", path);
  return clear_error();
}

int hpvm_autotune_load(const char* path) {
  if (!path) return set_error(HPVM_INVALID_ARG, "argument 1: path is NULL");
  env_cache();
  if (!load_file(path)) return set_error(HPVM_INVALID_ARG, "cannot open %s", path);
  return clear_error();
}

}  // extern "C"
