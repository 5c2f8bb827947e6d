// Memory tracker for host-resident arrays (HPVM report, Sec. 2.3 "Performance
// features"; the runtime calls of Sec. 6.3).
//
// The tracker records, per tracked host region, where the latest copy of the
// data lives (host, device, or both) and keeps the region's device copy.  A
// launch on tracked host arrays copies an argument to the device only when
// the device copy is stale and the node reads it (`in` / `inout`), and after
// the launch marks its outputs (`out` / `inout`) as living on the device
// only.  The host asks for a region with request_mem, which copies it back
// only when the latest copy is on the device.  This is how redundant copies
// between address spaces are avoided when successive nodes reuse data.
//
// Device copies are allocated and freed stream-ordered on the caller's
// stream, so the tracker never waits for the whole device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <mutex>

#include "hpvm_sgemm.h"
#include "internal.hpp"

namespace hpvm {
namespace {

struct Region {
  int64_t bytes = 0;
  void* dev = nullptr;       // device copy (allocated on first use)
  hipStream_t owner = nullptr;  // stream the device copy was allocated on
  bool on_host = true;       // host copy is current
  bool on_device = false;    // device copy is current
};

std::mutex g_mu;
std::map<uintptr_t, Region> g_regions;  // keyed by host start address
hpvm_tracker_stats g_stats{};

// The region holding [p, p + bytes), or nullptr.
Region* find_region(const void* p, int64_t bytes, uintptr_t* start) {
  const uintptr_t a = (uintptr_t)p;
  auto it = g_regions.upper_bound(a);
  if (it == g_regions.begin()) return nullptr;
  --it;
  if (a < it->first || a + (uintptr_t)bytes > it->first + (uintptr_t)it->second.bytes) return nullptr;
  if (start) *start = it->first;
  return &it->second;
}

// Makes the device copy of region r current (copying only when it is stale
// and `read` is set) and returns its device address for host address p.
hipError_t to_device(Region& r, uintptr_t start, const void* p, bool read, hipStream_t s, void** dptr) {
  hipError_t e = hipSuccess;
  if (!r.dev) {
    // HPVM_FAULT_INJECT=alloc: the device copy's allocation fails.
    e = fault_injected("alloc") ? hipErrorOutOfMemory : hipMallocAsync(&r.dev, (size_t)r.bytes, s);
    if (e != hipSuccess) {
      r.dev = nullptr;
      return e;
    }
    r.owner = s;
    r.on_device = false;
  }
  if (read && !r.on_device) {
    e = hipMemcpyAsync(r.dev, (const void*)start, (size_t)r.bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    g_stats.h2d_bytes += r.bytes;
    g_stats.h2d_copies += 1;
    r.on_device = true;
  }
  *dptr = (char*)r.dev + ((uintptr_t)p - start);
  return hipSuccess;
}

}  // namespace
}  // namespace hpvm

using namespace hpvm;

extern "C" {

int hpvm_track_mem(void* ptr, int64_t bytes) {
  if (!ptr) return set_error(HPVM_INVALID_ARG, "argument 1: ptr is NULL");
  if (bytes <= 0) return set_error(HPVM_INVALID_ARG, "argument 2: bytes = %lld <= 0", (long long)bytes);
  std::lock_guard<std::mutex> lk(g_mu);
  const uintptr_t a = (uintptr_t)ptr;
  auto next = g_regions.lower_bound(a);
  if (next != g_regions.end() && next->first < a + (uintptr_t)bytes)
    return set_error(HPVM_INVALID_ARG, "argument 1: region overlaps a tracked region");
  if (next != g_regions.begin()) {
    auto prev = std::prev(next);
    if (prev->first + (uintptr_t)prev->second.bytes > a)
      return set_error(HPVM_INVALID_ARG, "argument 1: region overlaps a tracked region");
  }
  Region r;
  r.bytes = bytes;
  g_regions[a] = r;
  return clear_error();
}

int hpvm_request_mem(void* ptr, int64_t bytes, void* stream) {
  if (!ptr) return set_error(HPVM_INVALID_ARG, "argument 1: ptr is NULL");
  if (bytes < 0) return set_error(HPVM_INVALID_ARG, "argument 2: bytes = %lld < 0", (long long)bytes);
  std::lock_guard<std::mutex> lk(g_mu);
  uintptr_t start = 0;
  Region* r = find_region(ptr, bytes, &start);
  if (!r) return set_error(HPVM_INVALID_ARG, "argument 1: [ptr, ptr + bytes) is not inside a tracked region");
  if (r->on_host) return clear_error();
  if (fault_injected("launch")) return set_error(HPVM_HIP_ERROR, "injected copy failure (HPVM_FAULT_INJECT)");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync((void*)start, r->dev, (size_t)r->bytes, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_error(e, "request_mem copy");
  g_stats.d2h_bytes += r->bytes;
  g_stats.d2h_copies += 1;
  r->on_host = true;
  return clear_error();
}

int hpvm_untrack_mem(void* ptr, void* stream) {
  if (!ptr) return set_error(HPVM_INVALID_ARG, "argument 1: ptr is NULL");
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_regions.find((uintptr_t)ptr);
  if (it == g_regions.end()) return set_error(HPVM_INVALID_ARG, "argument 1: ptr does not start a tracked region");
  if (it->second.dev) {
    // Ordered after the work already queued on `stream` and on the stream
    // the copy was made on.
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (it->second.owner != s) {
      hipEvent_t ev;
      e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventRecord(ev, it->second.owner);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, ev, 0);
      if (e == hipSuccess) e = hipEventDestroy(ev);
    }
    if (e == hipSuccess) e = hipFreeAsync(it->second.dev, s);
    if (e != hipSuccess) return hip_error(e, "untrack_mem");
  }
  g_regions.erase(it);
  return clear_error();
}

int hpvm_tracked_state(const void* ptr, hpvm_tracked* out) {
  if (!ptr) return set_error(HPVM_INVALID_ARG, "argument 1: ptr is NULL");
  if (!out) return set_error(HPVM_INVALID_ARG, "argument 2: out is NULL");
  std::lock_guard<std::mutex> lk(g_mu);
  uintptr_t start = 0;
  Region* r = find_region(ptr, 1, &start);
  if (!r) return set_error(HPVM_INVALID_ARG, "argument 1: ptr is not inside a tracked region");
  out->start = (void*)start;
  out->bytes = r->bytes;
  out->device = r->dev;
  out->on_host = r->on_host ? 1 : 0;
  out->on_device = r->on_device ? 1 : 0;
  return clear_error();
}

int hpvm_tracker_counters(hpvm_tracker_stats* out) {
  if (!out) return set_error(HPVM_INVALID_ARG, "argument 1: out is NULL");
  std::lock_guard<std::mutex> lk(g_mu);
  *out = g_stats;
  out->regions = (int64_t)g_regions.size();
  return clear_error();
}

int hpvm_sgemm_tracked(int64_t m, int64_t n, int64_t k, float alpha, const float* A, int64_t lda, const float* B,
                       int64_t ldb, float beta, float* C, int64_t ldc, int32_t prec, const hpvm_tile* tile,
                       void* stream) {
  bool reads_ab = false;
  int rc = check_gemm_args("", m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, &reads_ab);
  if (rc != HPVM_OK) return rc;
  if (m == 0 || n == 0) return clear_error();
  std::lock_guard<std::mutex> lk(g_mu);
  const int64_t ab = (m - 1) * lda + (reads_ab ? k : 1);
  const int64_t bb = (k > 0 ? (k - 1) * ldb + n : 1);
  const int64_t cb = (m - 1) * ldc + n;
  uintptr_t sa = 0, sb = 0, sc = 0;
  Region* ra = reads_ab ? find_region(A, ab * 4, &sa) : nullptr;
  Region* rb = reads_ab ? find_region(B, bb * 4, &sb) : nullptr;
  Region* rcg = find_region(C, cb * 4, &sc);
  if (reads_ab && !ra) return set_error(HPVM_INVALID_ARG, "argument 5: A is not inside a tracked region");
  if (reads_ab && !rb) return set_error(HPVM_INVALID_ARG, "argument 7: B is not inside a tracked region");
  if (!rcg) return set_error(HPVM_INVALID_ARG, "argument 10: C is not inside a tracked region");
  if (fault_injected("launch")) return set_error(HPVM_HIP_ERROR, "injected launch failure (HPVM_FAULT_INJECT)");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  void *da = nullptr, *db = nullptr, *dc = nullptr;
  hipError_t e = hipSuccess;
  // A and B are `in`: copied when their device copy is stale.  C is `in
  // out`; its initial data may be skipped only when the node overwrites the
  // whole region (beta == 0, no gaps between rows, region == C's extent) --
  // otherwise the unwritten rest of a stale device copy would come back.
  const bool c_overwritten = beta == 0.0f && ldc == n && sc == (uintptr_t)C && rcg->bytes == cb * 4;
  if (reads_ab) e = to_device(*ra, sa, A, true, s, &da);
  if (e == hipSuccess && reads_ab) e = to_device(*rb, sb, B, true, s, &db);
  if (e == hipSuccess) e = to_device(*rcg, sc, C, !c_overwritten, s, &dc);
  if (e != hipSuccess) return hip_error(e, "tracked copy");
  rc = hpvm_sgemm(m, n, k, alpha, (const float*)da, lda, (const float*)db, ldb, beta, (float*)dc, ldc, prec, tile,
                  stream);
  if (rc != HPVM_OK) return rc;
  rcg->on_device = true;
  rcg->on_host = false;  // the latest C is on the device now
  g_stats.launches += 1;
  return clear_error();
}

}  // extern "C"
