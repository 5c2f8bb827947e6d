// C-ABI layer of the sgemm dataflow-graph library: argument checks, the
// Allocation-size function, structural queries and the root launch.
//
// This file plays the role of the host code the paper's GPU backend emits
// (HPVM report, Sec. 6.3): it unpacks the root node's arguments, computes the
// Allocation node's size before the launch, sets the launch geometry from the
// SgemmInternal / SgemmLeaf instance counts, and enqueues the kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "device_common.hpp"
#include "hpvm_sgemm.h"
#include "internal.hpp"

namespace hpvm {

namespace {
thread_local char g_error[512] = "";
}

int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_error, sizeof g_error, fmt, ap);
  va_end(ap);
  return code;
}

int clear_error() {
  g_error[0] = '\0';
  return HPVM_OK;
}

const char* last_error_text() { return g_error; }

int hip_error(hipError_t e, const char* what) {
  return set_error(HPVM_HIP_ERROR, "%s: %s", what, hipGetErrorString(e));
}

// HPVM_FAULT_INJECT=<site> makes the named step report a HIP failure after
// the argument checks, so that error propagation can be exercised without a
// GPU.  Sites: launch, wait, capture.
bool fault_injected(const char* site) {
  const char* v = std::getenv("HPVM_FAULT_INJECT");
  return v && std::strcmp(v, site) == 0;
}

void matrix_extent(const void* p, int64_t rows, int64_t cols, int64_t ld, uintptr_t* lo, uintptr_t* hi) {
  *lo = (uintptr_t)p;
  *hi = (uintptr_t)p + (uintptr_t)(((rows - 1) * ld + cols) * (int64_t)sizeof(float));
}

int check_gemm_args(const char* what, int64_t m, int64_t n, int64_t k, float alpha, const float* A,
                    int64_t lda, const float* B, int64_t ldb, float beta, const float* C,
                    int64_t ldc, bool* reads_ab) {
  (void)beta;
  if (m < 0) return set_error(HPVM_INVALID_ARG, "%sargument 1: m = %lld < 0", what, (long long)m);
  if (n < 0) return set_error(HPVM_INVALID_ARG, "%sargument 2: n = %lld < 0", what, (long long)n);
  if (k < 0) return set_error(HPVM_INVALID_ARG, "%sargument 3: k = %lld < 0", what, (long long)k);
  if (m > INT32_MAX || n > INT32_MAX || k > INT32_MAX)
    return set_error(HPVM_UNSUPPORTED, "%ssizes above 2^31 - 1 are not supported", what);
  const bool empty = (m == 0 || n == 0);
  *reads_ab = !empty && k > 0 && alpha != 0.0f;
  if (*reads_ab && !A) return set_error(HPVM_INVALID_ARG, "%sargument 5: A is NULL", what);
  if (lda < (k > 1 ? k : 1))
    return set_error(HPVM_INVALID_ARG, "%sargument 6: lda = %lld < max(1, k)", what, (long long)lda);
  if (*reads_ab && !B) return set_error(HPVM_INVALID_ARG, "%sargument 7: B is NULL", what);
  if (ldb < (n > 1 ? n : 1))
    return set_error(HPVM_INVALID_ARG, "%sargument 8: ldb = %lld < max(1, n)", what, (long long)ldb);
  if (!empty && !C) return set_error(HPVM_INVALID_ARG, "%sargument 10: C is NULL", what);
  if (ldc < (n > 1 ? n : 1))
    return set_error(HPVM_INVALID_ARG, "%sargument 11: ldc = %lld < max(1, n)", what, (long long)ldc);
  if (*reads_ab) {
    uintptr_t c0, c1, x0, x1;
    matrix_extent(C, m, n, ldc, &c0, &c1);
    matrix_extent(A, m, k, lda, &x0, &x1);
    const bool oa = c0 < x1 && x0 < c1;
    matrix_extent(B, k, n, ldb, &x0, &x1);
    const bool ob = c0 < x1 && x0 < c1;
    if (oa || ob) return set_error(HPVM_INVALID_ARG, "%sargument 10: C overlaps A or B", what);
  }
  return HPVM_OK;
}

}  // namespace hpvm

namespace {

using hpvm::set_error;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return set_error(code, "%s", buf);
}

int ok() { return hpvm::clear_error(); }

int hip_fail(hipError_t e, const char* what) { return hpvm::hip_error(e, what); }

bool inject(const char* site) { return hpvm::fault_injected(site); }

bool valid_prec(int32_t prec) {
  return prec == HPVM_PREC_FP32 || prec == HPVM_PREC_BF16 || prec == HPVM_PREC_BF16X3;
}

bool is_literal(const hpvm_tile& t) { return t.leaf_m == 1 && t.leaf_n == 1; }

// Literal lowering: tile_n x tile_m lanes (block_x = tile_n, block_y =
// tile_m), a whole number of wavefronts, at most 1024 lanes; the staged B
// slab is tile_m deep and one buffer.  The untiled one-level graph has the
// same lanes, tile_k = 0 and stages = 0 (no Allocation node).
bool is_flat(const hpvm_tile& t) { return t.stages == 0 && t.tile_k == 0; }
bool literal_ok(const hpvm_tile& t) {
  const int64_t lanes = (int64_t)t.tile_m * t.tile_n;
  return t.tile_m > 0 && t.tile_n > 0 && lanes >= hpvm::kWave && lanes <= 1024 &&
         lanes % hpvm::kWave == 0 && ((t.tile_k == t.tile_m && t.stages == 1) || is_flat(t));
}

const hpvm::MfmaEntry* find_entry(int32_t prec, const hpvm_tile* tile) {
  if (!tile) return hpvm::menu_entry_at(prec, 0);
  return hpvm::find_menu_entry(prec, *tile);
}

// Resolves the lowering for (prec, tile); *entry is null for the literal one.
int resolve(int32_t prec, const hpvm_tile* tile, const hpvm::MfmaEntry** entry, int argno) {
  *entry = nullptr;
  if (tile && is_literal(*tile)) {
    if (prec != HPVM_PREC_FP32)
      return fail(HPVM_UNSUPPORTED, "argument %d: the literal lowering (leaf 1x1) is FP32 only", argno);
    if (!literal_ok(*tile))
      return fail(HPVM_UNSUPPORTED,
                  "argument %d: literal tile %dx%d (k %d, stages %d) needs 64..1024 lanes in whole "
                  "wavefronts, and tile_k == tile_m with one stage, or tile_k = 0 with none (untiled)",
                  argno, tile->tile_m, tile->tile_n, tile->tile_k, tile->stages);
    return HPVM_OK;
  }
  *entry = find_entry(prec, tile);
  if (!*entry) {
    if (tile)
      return fail(HPVM_UNSUPPORTED, "argument %d: tile %dx%dx%d leaf %dx%d stages %d is not compiled for precision %d",
                  argno, tile->tile_m, tile->tile_n, tile->tile_k, tile->leaf_m, tile->leaf_n,
                  tile->stages, prec);
    return fail(HPVM_UNSUPPORTED, "no compiled tile for precision %d", prec);
  }
  return HPVM_OK;
}

// Built-in choice for tile == NULL when the autotuner has no entry and no
// workspace lowering applies, for problems the menu's entry 0 would leave
// CUs idle on.  FP32: entry 0 (256 x 256 DMA-fed tiles) when it gives at
// least 256 tiles (one per CU of a 256-CU part), else the DMA-fed
// 128 x 128 x 32 tile when that does (2048^3: 0.128 ms against 0.166 for the
// best register-staged tile and 0.457 for 64 tiles of 256 x 256), else the
// 64 x 64 x 16 tile (at 1024 x 1024 x 4096, 64 tiles of 128 x 128 ran at 28
// TFLOP/s and 256 of 64 x 64 at 75).  BF16 and bf16x3: entry 0 (the
// DMA-fed 256 x 256 tile) when it gives at least 256 tiles, else the
// DMA-fed 128 x 128 tile when that does, else the register-staged
// 64 x 64 x 32 tile (1024^3 BF16: 0.020 ms against 0.064 for 256 x 256).
// Returns false for entry 0.
int64_t tiles_of(const hpvm_tile& t, int64_t m, int64_t n) {
  return ((m + t.tile_m - 1) / t.tile_m) * ((n + t.tile_n - 1) / t.tile_n);
}
const hpvm::MfmaEntry* f32_mid_entry() {
  return hpvm::find_menu_entry(HPVM_PREC_FP32, hpvm_tile{128, 128, 32, 32, 128, 2});
}
}  // namespace

namespace hpvm {
bool default_small_tile(int32_t prec, int64_t m, int64_t n, hpvm_tile* out) {
  const hpvm::MfmaEntry* e0 = hpvm::menu_entry_at(prec, 0);
  if (!e0) return false;
  if (prec == HPVM_PREC_FP32) {
    const hpvm::MfmaEntry* mid = f32_mid_entry();
    const hpvm::MfmaEntry* small = hpvm::find_menu_entry(prec, hpvm_tile{64, 64, 16, 32, 32, 2});
    if (!mid || !small || tiles_of(e0->tile, m, n) >= 256) return false;
    *out = tiles_of(mid->tile, m, n) >= 256 ? mid->tile : small->tile;
    return true;
  }
  // BF16 / bf16x3: the DMA-fed 128 x 128 tile when it covers the CUs
  // (2048^3 BF16: 0.055 ms against 0.084 for 64 tiles of 256 x 256), else
  // the register-staged 64 x 64 x 32 tile.
  const hpvm::MfmaEntry* mid = hpvm::find_menu_entry(prec, hpvm_tile{128, 128, 32, 64, 64, 4});
  const hpvm::MfmaEntry* small = hpvm::find_menu_entry(prec, hpvm_tile{64, 64, 32, 32, 32, 2});
  if (!small || !mid || tiles_of(e0->tile, m, n) >= 256) return false;
  *out = tiles_of(mid->tile, m, n) >= 256 ? mid->tile : small->tile;
  return true;
}
}  // namespace hpvm

namespace {

// The DMA-fed entry whose split contraction needs the fewest partial sums
// (the deepest slices; the first in menu order on a tie), or null.
const hpvm::MfmaEntry* fewest_slices(int32_t prec, int64_t m, int64_t n, int64_t k, int64_t* bytes) {
  const hpvm::MfmaEntry* best = nullptr;
  int64_t best_bytes = 0;
  for (int i = 0; i < hpvm::menu_size(prec); ++i) {
    const hpvm::MfmaEntry* e = hpvm::menu_entry_at(prec, i);
    const int64_t b = hpvm::entry_split_bytes(e, m, n, k);
    if (b > 0 && (!best || b < best_bytes)) {
      best = e;
      best_bytes = b;
    }
  }
  *bytes = best_bytes;
  return best;
}

// Built-in choice of hpvm_sgemm_ws (and of hpvm_sgemm_workspace_bytes) for
// tile == NULL when the autotuner has no entry: products that even 128 x 128
// tiles would not cover the CUs with (BF16 and bf16x3: with k >= 2048) take
// the DMA-fed entry that splits the contraction into the deepest slices,
// provided `ws_bytes` (the caller's workspace; -1 = as much as needed)
// holds its partial sums (BF16 512 x 512 x 4096: 0.035 ms against 0.095 on
// 64 x 64 tiles, 1024 x 1024 x 4096: 0.047 against 0.069 staged); other
// BF16 products of at least 2^31 multiply-adds take the first staged tile,
// whose conversion pass is then a small share of the time (or, when that
// gives fewer than 256 tiles, the 128 x 128 x 64 tile with 64 x 32 leaves);
// bf16x3 products the same only when 256 x 256 tiles would not cover the
// CUs (or k or n does not suit the DMA-fed tile).  Returns false when
// neither applies (hpvm_sgemm's choice then): a split tile run as one
// launch would be the slowest choice there is (64 tiles of 128 x 128 at
// 1024 x 1024 x 4096 FP32: 28 TFLOP/s against 75 for hpvm_sgemm's 64 x 64
// tiles).
bool default_ws_tile(int32_t prec, int64_t m, int64_t n, int64_t k, int64_t ws_bytes, hpvm_tile* out) {
  // The split contraction, only when even 128 x 128 tiles would not cover
  // the CUs (BF16 / bf16x3: and k >= 2048; at 1024^3 the 64 x 64 tiles were
  // as fast, 0.031 ms against 0.033), on the entry with the deepest slices.
  const hpvm::MfmaEntry* mid =
      prec == HPVM_PREC_FP32 ? f32_mid_entry() : hpvm::find_menu_entry(prec, hpvm_tile{128, 128, 32, 64, 64, 4});
  if (mid && tiles_of(mid->tile, m, n) < 256 && (prec == HPVM_PREC_FP32 || k >= 2048)) {
    int64_t need = 0;
    const hpvm::MfmaEntry* best = fewest_slices(prec, m, n, k, &need);
    if (best && (ws_bytes < 0 || ws_bytes >= need)) {
      *out = best->tile;
      return true;
    }
  }
  if (prec != HPVM_PREC_BF16 && prec != HPVM_PREC_BF16X3) return false;
  if ((double)m * (double)n * (double)k < 2147483648.0 || !hpvm::staged_k_ok(k)) return false;
  const hpvm::MfmaEntry* staged = nullptr;
  if (hpvm::staged_menu(prec, &staged) == 0) return false;
  // Fewer than 256 of the first tile leave CUs idle: eight waves of 64 x 32
  // on 128 x 128 tiles then ran 1.8-3x faster (2048^3 BF16: 0.039 ms
  // against 0.070; at 4096^3 the first tile stays ahead, 0.150 against 0.159).
  const hpvm::MfmaEntry* small = hpvm::find_menu_entry(prec, hpvm_tile{128, 128, 64, 64, 32, 3});
  const bool big = tiles_of(staged[0].tile, m, n) >= 256;
  // bf16x3 products that the DMA-fed 256 x 256 tile (menu entry 0) covers
  // run faster on it, converting in the GEMM's own fragment reads (8192^3:
  // 2.71 ms against 2.82 staged, 4096^3: 0.353 against 0.366), so they take
  // no workspace.
  const hpvm::MfmaEntry* e0 = hpvm::menu_entry_at(prec, 0);
  if (prec == HPVM_PREC_BF16X3 && e0 && tiles_of(e0->tile, m, n) >= 256 && k % e0->tile.tile_k == 0 && n % 4 == 0)
    return false;
  const hpvm_tile pick = big || !small ? staged[0].tile : small->tile;
  // A workspace too small for the planes: the choice without one.
  if (ws_bytes >= 0 && ws_bytes < hpvm::staged_workspace_bytes(prec, m, n, k)) return false;
  *out = pick;
  return true;
}

// The tile a call with tile == NULL runs.  ws_ok: the call has a workspace
// argument (hpvm_sgemm_ws); ws_bytes: its size, or -1 for "as much as the
// choice needs" (hpvm_sgemm_workspace_bytes asks which tile that is).  In
// order: the autotuned winner (with a workspace the overall one, unless it
// splits the contraction and the workspace cannot hold the partial sums:
// then the winner that needs none), the built-in workspace choice, the
// built-in small-problem choice; false = the menu's entry 0.
int describe_impl(int64_t m, int64_t n, int64_t k, int32_t prec, const hpvm_tile* tile, bool ws_ok,
                  int64_t ws_bytes, hpvm_dfg* out);

bool choose_tile(int32_t prec, int64_t m, int64_t n, int64_t k, bool ws_ok, int64_t ws_bytes, hpvm_tile* out) {
  if (hpvm::tuned_tile(prec, m, n, k, ws_ok, out)) {
    if (!ws_ok || ws_bytes < 0) return true;
    const hpvm::MfmaEntry* e = hpvm::find_menu_entry(prec, *out);
    const int64_t need = std::max(hpvm::entry_split_bytes(e, m, n, k), hpvm::entry_workspace_bytes(e, m, n, k));
    if (need == 0 || ws_bytes >= need) return true;
    return hpvm::tuned_tile(prec, m, n, k, false, out) != 0;
  }
  if (ws_ok && default_ws_tile(prec, m, n, k, ws_bytes, out)) return true;
  return hpvm::default_small_tile(prec, m, n, out);
}

}  // namespace

extern "C" {

const char* hpvm_status_string(int status) {
  switch (status) {
    case HPVM_OK: return "HPVM_OK";
    case HPVM_INVALID_ARG: return "HPVM_INVALID_ARG";
    case HPVM_UNSUPPORTED: return "HPVM_UNSUPPORTED";
    case HPVM_HIP_ERROR: return "HPVM_HIP_ERROR";
    case HPVM_WORKSPACE_TOO_SMALL: return "HPVM_WORKSPACE_TOO_SMALL";
    case HPVM_BAD_HANDLE: return "HPVM_BAD_HANDLE";
    case HPVM_QUEUE_FULL: return "HPVM_QUEUE_FULL";
    case HPVM_TIMEOUT: return "HPVM_TIMEOUT";
    case HPVM_STREAM_ENDED: return "HPVM_STREAM_ENDED";
    default: return "HPVM_UNKNOWN_STATUS";
  }
}

const char* hpvm_last_error(void) { return hpvm::last_error_text(); }

int hpvm_alloc_bytes(const hpvm_tile* tile, int32_t prec, int64_t* bytes) {
  if (!tile) return fail(HPVM_INVALID_ARG, "argument 1: tile is NULL");
  if (!valid_prec(prec)) return fail(HPVM_INVALID_ARG, "argument 2: unknown precision %d", prec);
  if (!bytes) return fail(HPVM_INVALID_ARG, "argument 3: bytes is NULL");
  const hpvm::MfmaEntry* e;
  int rc = resolve(prec, tile, &e, 1);
  if (rc != HPVM_OK) return rc;
  *bytes = e ? e->lds_bytes : is_flat(*tile) ? 0 : hpvm::literal_alloc_bytes(tile->tile_n, tile->tile_m);
  return ok();
}

int hpvm_tile_menu(int32_t prec, hpvm_tile* out, int32_t capacity, int32_t* count) {
  if (!valid_prec(prec)) return fail(HPVM_INVALID_ARG, "argument 1: unknown precision %d", prec);
  if (capacity < 0 || (capacity > 0 && !out))
    return fail(HPVM_INVALID_ARG, "argument 3: bad capacity or NULL output");
  if (!count) return fail(HPVM_INVALID_ARG, "argument 4: count is NULL");
  const int n = hpvm::menu_size(prec);
  for (int i = 0; i < n && i < capacity; ++i) out[i] = hpvm::menu_entry_at(prec, i)->tile;
  *count = n;
  return ok();
}

int hpvm_describe(int64_t m, int64_t n, int64_t k, int32_t prec, const hpvm_tile* tile, hpvm_dfg* out) {
  if (m < 0) return fail(HPVM_INVALID_ARG, "argument 1: m = %lld < 0", (long long)m);
  if (n < 0) return fail(HPVM_INVALID_ARG, "argument 2: n = %lld < 0", (long long)n);
  if (k < 0) return fail(HPVM_INVALID_ARG, "argument 3: k = %lld < 0", (long long)k);
  if (!valid_prec(prec)) return fail(HPVM_INVALID_ARG, "argument 4: unknown precision %d", prec);
  if (!out) return fail(HPVM_INVALID_ARG, "argument 6: out is NULL");
  return describe_impl(m, n, k, prec, tile, false, 0, out);
}

int hpvm_describe_ws(int64_t m, int64_t n, int64_t k, int32_t prec, const hpvm_tile* tile,
                     int64_t workspace_bytes, hpvm_dfg* out) {
  if (m < 0) return fail(HPVM_INVALID_ARG, "argument 1: m = %lld < 0", (long long)m);
  if (n < 0) return fail(HPVM_INVALID_ARG, "argument 2: n = %lld < 0", (long long)n);
  if (k < 0) return fail(HPVM_INVALID_ARG, "argument 3: k = %lld < 0", (long long)k);
  if (!valid_prec(prec)) return fail(HPVM_INVALID_ARG, "argument 4: unknown precision %d", prec);
  if (workspace_bytes < 0)
    return fail(HPVM_INVALID_ARG, "argument 6: workspace_bytes = %lld < 0", (long long)workspace_bytes);
  if (!out) return fail(HPVM_INVALID_ARG, "argument 7: out is NULL");
  return describe_impl(m, n, k, prec, tile, true, workspace_bytes, out);
}

}  // extern "C"

namespace {

int describe_impl(int64_t m, int64_t n, int64_t k, int32_t prec, const hpvm_tile* tile, bool ws_ok,
                  int64_t ws_bytes, hpvm_dfg* out) {
  hpvm_tile chosen;
  if (!tile && choose_tile(prec, m, n, k, ws_ok, ws_bytes, &chosen)) tile = &chosen;
  const hpvm::MfmaEntry* e;
  int rc = resolve(prec, tile, &e, 5);
  if (rc != HPVM_OK) return rc;
  const hpvm_tile t = e ? e->tile : *tile;
  std::memset(out, 0, sizeof *out);
  out->root_instances = 1;
  out->splits = 1;
  out->tile = t;
  const int64_t split = ws_ok ? hpvm::entry_split_bytes(e, m, n, k) : 0;
  if (split > 0 && ws_bytes >= split && m > 0 && n > 0 && k > 0)
    out->splits = (int32_t)(split / (m * n * (int64_t)sizeof(float)));
  out->grid_x = (int32_t)((n + t.tile_n - 1) / t.tile_n);
  out->grid_y = (int32_t)((m + t.tile_m - 1) / t.tile_m);
  out->k_slabs = t.tile_k > 0 ? (int32_t)((k + t.tile_k - 1) / t.tile_k) : 0;
  if (e) {
    out->block_x = e->threads;
    out->block_y = 1;
    out->waves = e->threads / hpvm::kWave;
    out->alloc_bytes = e->lds_bytes;
    if (e->launch_staged)
      out->lowering = prec == HPVM_PREC_BF16 ? hpvm::kStagedBf16 : hpvm::kStagedBf16x3;
    else
      out->lowering = prec == HPVM_PREC_FP32 ? hpvm::kMfmaF32
                      : prec == HPVM_PREC_BF16 ? hpvm::kMfmaBf16
                                                : hpvm::kMfmaBf16x3;
  } else {
    out->block_x = t.tile_n;
    out->block_y = t.tile_m;
    out->waves = t.tile_m * t.tile_n / hpvm::kWave;
    out->alloc_bytes = is_flat(t) ? 0 : hpvm::literal_alloc_bytes(t.tile_n, t.tile_m);
    out->lowering = is_flat(t) ? hpvm::kFlat : hpvm::kLiteral;
    if (is_flat(t)) out->k_slabs = 0;
  }
  return ok();
}

}  // namespace

extern "C" {

// The sgemm graph of Sec. 6.1: SgemmRoot (0) creates a 2-D SgemmInternal (1)
// and binds its inputs 0..13 through; SgemmInternal creates Allocation (2)
// and a 2-D SgemmLeaf (3), wires Allocation's outputs 0 and 1 (pointer,
// bytes) to the leaf's inputs 12 and 13 with all-to-all replication (one
// Allocation instance feeds every leaf instance), binds its own inputs 0..11
// to the leaf's 0..11 and its inputs 12, 13 (block_x, block_y) to
// Allocation's 0, 1.
int hpvm_dfg_edges(hpvm_edge* out, int32_t capacity, int32_t* count) {
  if (capacity < 0 || (capacity > 0 && !out))
    return fail(HPVM_INVALID_ARG, "argument 2: bad capacity or NULL output");
  if (!count) return fail(HPVM_INVALID_ARG, "argument 3: count is NULL");
  hpvm_edge table[64];
  int n = 0;
  table[n++] = hpvm_edge{0, 2, 3, 0, 12, 1};
  table[n++] = hpvm_edge{0, 2, 3, 1, 13, 1};
  for (int port = 0; port < 12; ++port) table[n++] = hpvm_edge{1, 1, 3, port, port, 0};
  table[n++] = hpvm_edge{1, 1, 2, 12, 0, 0};
  table[n++] = hpvm_edge{1, 1, 2, 13, 1, 0};
  for (int port = 0; port < 14; ++port) table[n++] = hpvm_edge{1, 0, 1, port, port, 0};
  for (int i = 0; i < n && i < capacity; ++i) out[i] = table[i];
  *count = n;
  return ok();
}

}  // extern "C"

namespace {

// hpvm_sgemm and hpvm_sgemm_ws: `ws_ok` tells whether a workspace argument
// exists (it is argument 14/15 of hpvm_sgemm_ws).
int sgemm_impl(int64_t m, int64_t n, int64_t k, float alpha, const float* A, int64_t lda, const float* B,
               int64_t ldb, float beta, float* C, int64_t ldc, int32_t prec, const hpvm_tile* tile, bool ws_ok,
               void* workspace, int64_t workspace_bytes, void* stream) {
  // Checks in argument order; nothing below touches the device until all pass.
  bool reads_ab = false;
  int rc = hpvm::check_gemm_args("", m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, &reads_ab);
  if (rc != HPVM_OK) return rc;
  if (!valid_prec(prec)) return fail(HPVM_INVALID_ARG, "argument 12: unknown precision %d", prec);
  hpvm_tile tuned;
  if (!tile && choose_tile(prec, m, n, k, ws_ok, workspace ? workspace_bytes : 0, &tuned)) tile = &tuned;
  const hpvm::MfmaEntry* entry;
  rc = resolve(prec, tile, &entry, 13);
  if (rc != HPVM_OK) return rc;
  const int64_t need = hpvm::entry_workspace_bytes(entry, m, n, k);
  if (need > 0 && reads_ab) {
    if (!hpvm::staged_k_ok(k))
      return fail(HPVM_UNSUPPORTED, "argument 13: k = %lld is too deep for a tile with stages = 3", (long long)k);
    if (!ws_ok)
      return fail(HPVM_UNSUPPORTED, "argument 13: tile with stages = 3 needs a workspace (use hpvm_sgemm_ws)");
    if (!workspace) return fail(HPVM_INVALID_ARG, "argument 14: workspace is NULL");
    if ((uintptr_t)workspace % 16) return fail(HPVM_INVALID_ARG, "argument 14: workspace is not 16-byte aligned");
    if (workspace_bytes < need)
      return fail(HPVM_WORKSPACE_TOO_SMALL, "argument 15: workspace has %lld bytes, needs %lld",
                  (long long)workspace_bytes, (long long)need);
  }
  const bool empty = (m == 0 || n == 0);
  if (empty) return ok();
  if (inject("launch")) return fail(HPVM_HIP_ERROR, "injected launch failure (HPVM_FAULT_INJECT)");

  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e;
  if (!reads_ab) {
    e = hpvm::launch_scale(C, ldc, m, n, beta, s);
    return e == hipSuccess ? ok() : hip_fail(e, "scale launch");
  }
  hpvm::GemmArgs a{};
  a.A = A;
  a.B = B;
  a.C = C;
  a.lda = lda;
  a.ldb = ldb;
  a.ldc = ldc;
  a.m = (int32_t)m;
  a.n = (int32_t)n;
  a.k = (int32_t)k;
  a.alpha = alpha;
  a.beta = beta;
  a.vec_a = hpvm::vec16(A, lda);
  a.vec_b = hpvm::vec16(B, ldb);
  const int64_t split = ws_ok ? hpvm::entry_split_bytes(entry, m, n, k) : 0;
  if (entry && entry->launch_staged)
    e = entry->launch_staged(a, workspace, s);
  else if (split > 0 && workspace && (uintptr_t)workspace % 16 == 0 && workspace_bytes >= split)
    e = entry->launch_split(a, workspace, s);
  else if (entry)
    e = entry->launch(a, false, false, s);
  else if (is_flat(*tile))
    e = hpvm::launch_flat(a, tile->tile_n, tile->tile_m, s);
  else
    e = hpvm::launch_literal(a, tile->tile_n, tile->tile_m, s);
  return e == hipSuccess ? ok() : hip_fail(e, "sgemm launch");
}

}  // namespace

extern "C" {

int hpvm_sgemm(int64_t m, int64_t n, int64_t k, float alpha, const float* A, int64_t lda, const float* B,
               int64_t ldb, float beta, float* C, int64_t ldc, int32_t prec, const hpvm_tile* tile, void* stream) {
  return sgemm_impl(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, prec, tile, false, nullptr, 0, stream);
}

int hpvm_sgemm_ws(int64_t m, int64_t n, int64_t k, float alpha, const float* A, int64_t lda, const float* B,
                  int64_t ldb, float beta, float* C, int64_t ldc, int32_t prec, const hpvm_tile* tile,
                  void* workspace, int64_t workspace_bytes, void* stream) {
  return sgemm_impl(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, prec, tile, true, workspace, workspace_bytes,
                    stream);
}

int hpvm_sgemm_workspace_bytes(int64_t m, int64_t n, int64_t k, int32_t prec, const hpvm_tile* tile,
                               int64_t* bytes) {
  if (m < 0 || n < 0 || k < 0) return fail(HPVM_INVALID_ARG, "sizes must be >= 0");
  if (!valid_prec(prec)) return fail(HPVM_INVALID_ARG, "argument 4: unknown precision %d", prec);
  if (!bytes) return fail(HPVM_INVALID_ARG, "argument 6: bytes is NULL");
  hpvm_tile tuned;
  if (!tile && choose_tile(prec, m, n, k, true, -1, &tuned)) tile = &tuned;
  const hpvm::MfmaEntry* entry;
  int rc = resolve(prec, tile, &entry, 5);
  if (rc != HPVM_OK) return rc;
  *bytes = std::max(hpvm::entry_workspace_bytes(entry, m, n, k), hpvm::entry_split_bytes(entry, m, n, k));
  return ok();
}

int hpvm_launch_root(const hpvm_root_in* r, void* stream) {
  if (!r) return fail(HPVM_INVALID_ARG, "argument 1: args is NULL");
  if (r->block_x <= 0 || r->block_y <= 0 || r->grid_x < 0 || r->grid_y < 0)
    return fail(HPVM_INVALID_ARG, "block and grid counts must be positive");
  const int64_t lanes = (int64_t)r->block_x * r->block_y;
  if (lanes > 1024 || lanes % hpvm::kWave)
    return fail(HPVM_UNSUPPORTED, "block_x * block_y = %lld must be a multiple of 64, at most 1024",
                (long long)lanes);
  const int64_t m = (int64_t)r->grid_y * r->block_y;
  const int64_t n = (int64_t)r->grid_x * r->block_x;
  const int64_t k = r->k;
  if (k < 0) return fail(HPVM_INVALID_ARG, "k = %lld < 0", (long long)k);
  // The byte extents stand in for the sizes the paper's runtime copies.
  const int64_t f = (int64_t)sizeof(float);
  if (m > 0 && n > 0) {
    if (k > 0 && r->alpha != 0.0f) {
      if (r->lda < (k > 1 ? k : 1) || r->bytesA < ((m - 1) * r->lda + k) * f)
        return fail(HPVM_INVALID_ARG, "bytesA / lda too small for %lld x %lld", (long long)m, (long long)k);
      if (r->ldb < (n > 1 ? n : 1) || r->bytesB < ((k - 1) * r->ldb + n) * f)
        return fail(HPVM_INVALID_ARG, "bytesB / ldb too small for %lld x %lld", (long long)k, (long long)n);
    }
    if (r->ldc < (n > 1 ? n : 1) || r->bytesC < ((m - 1) * r->ldc + n) * f)
      return fail(HPVM_INVALID_ARG, "bytesC / ldc too small for %lld x %lld", (long long)m, (long long)n);
  }
  hpvm_tile t{r->block_y, r->block_x, r->block_y, 1, 1, 1};
  return hpvm_sgemm(m, n, k, r->alpha, r->A, r->lda > 0 ? r->lda : 1, r->B, r->ldb > 0 ? r->ldb : 1,
                    r->beta, r->C, r->ldc > 0 ? r->ldc : 1, HPVM_PREC_FP32, &t, stream);
}

int hpvm_wait(void* stream) {
  if (inject("wait")) return fail(HPVM_HIP_ERROR, "injected wait failure (HPVM_FAULT_INJECT)");
  hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? ok() : hip_fail(e, "stream synchronize");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// hpvm_sgemm_noalloc: hpvm_sgemm_ws whose workspace is a fixed array of
// device memory that the library's code object carries, so that the call
// itself allocates nothing.  Each device that loads the library holds its
// own copy of the array (at its own address) until the process ends.
// ---------------------------------------------------------------------------
namespace {

// Device-side storage.  On the host this name is only a stand-in for the
// symbol: its device address, per device, comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[HPVM_NOALLOC_SCRATCH_BYTES];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_at[kScratchDevices] = {};

// The current device's copy of the array, looked up once per device with
// that device current.
int scratch_of_current_device(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kScratchDevices)
    return fail(HPVM_UNSUPPORTED, "device %d: the no-allocation entry point supports devices 0..%d", dev,
                kScratchDevices - 1);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_at[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p || (uintptr_t)p % 256) return fail(HPVM_HIP_ERROR, "scratch symbol has no usable device address");
    g_scratch_at[dev] = p;
  }
  *out = g_scratch_at[dev];
  return HPVM_OK;
}

}  // namespace

extern "C" int hpvm_sgemm_noalloc(int64_t m, int64_t n, int64_t k, float alpha, const float* A, int64_t lda,
                                  const float* B, int64_t ldb, float beta, float* C, int64_t ldc, int32_t prec,
                                  const hpvm_tile* tile, void* stream) {
  // Checks in argument order, then the lowering hpvm_sgemm_ws would run with
  // a workspace of HPVM_NOALLOC_SCRATCH_BYTES; nothing touches the device
  // before all of them pass.
  bool reads_ab = false;
  int rc = hpvm::check_gemm_args("", m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, &reads_ab);
  if (rc != HPVM_OK) return rc;
  if (!valid_prec(prec)) return fail(HPVM_INVALID_ARG, "argument 12: unknown precision %d", prec);
  const int64_t cap = HPVM_NOALLOC_SCRATCH_BYTES;
  hpvm_tile chosen;
  const hpvm_tile* t = tile;
  if (!t && choose_tile(prec, m, n, k, true, cap, &chosen)) t = &chosen;
  const hpvm::MfmaEntry* entry;
  rc = resolve(prec, t, &entry, 13);
  if (rc != HPVM_OK) return rc;
  const int64_t need = hpvm::entry_workspace_bytes(entry, m, n, k);
  if (need > cap && reads_ab && m > 0 && n > 0)
    return fail(HPVM_WORKSPACE_TOO_SMALL,
                "argument 13: this tile needs %lld bytes of scratch; the no-allocation entry point has %lld "
                "(use hpvm_sgemm_ws with a workspace of that size)",
                (long long)need, (long long)cap);
  void* ws = nullptr;
  if (reads_ab && m > 0 && n > 0 && (need > 0 || hpvm::entry_split_bytes(entry, m, n, k) > 0)) {
    if (inject("launch")) return fail(HPVM_HIP_ERROR, "injected launch failure (HPVM_FAULT_INJECT)");
    rc = scratch_of_current_device(&ws);
    if (rc != HPVM_OK) return rc;
  }
  return sgemm_impl(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, prec, t, true, ws, ws ? cap : 0, stream);
}
