// Streaming sgemm graph: llvm.hpvm.launch with Stream = 1, then push / pop
// (HPVM report, Table 1 and Sec. 2.3 for the intrinsics, Sec. 3.5 for the
// persistent nodes a streaming graph needs).
//
// A streaming graph stays alive after its launch: every argument pack pushed
// into it is one more sgemm for its nodes to process, and pop returns the
// outputs in push order.  On the GPU the persistent node is one resident
// kernel.  Argument packs go into a ring of slots in pinned, coherent host
// memory; the host publishes each with a release store of the ring's tail.
// The resident workgroups take tickets from a device counter; the tiles of
// item i are tickets [first_i, end_i), handed out in push order.  At push
// the host also writes, for every ticket of the item, the item's slot into a
// ticket map (a window of kTicketWindow words, each tagged with its ticket),
// so a workgroup finds the item that holds its ticket with one read of host
// memory and then reads the item's argument pack with a second.  The workgroup that finishes an item's last tile raises the item's
// completion flag in host memory, which pop waits on.
//
// Every wait in the kernel is bounded: a workgroup with nothing to do leaves
// when the host has closed the stream, when another workgroup has ended it,
// or when it has been idle for the configured limit (it then ends the stream
// for all).  The host side never waits without a time limit either.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <thread>
#include <unordered_set>
#include <vector>

#include "device_common.hpp"
#include "hpvm_sgemm.h"
#include "internal.hpp"
#include "mfma_f32.hpp"
#include "persistent.hpp"

namespace hpvm {

// Ticket map entries: tickets in flight (from the oldest unpopped item's
// first ticket to the next ticket) never exceed this, so an entry is not
// rewritten while a workgroup may still look it up.
constexpr uint64_t kTicketWindow = 1ull << 18;

// One argument pack as the kernel reads it (host memory).
struct alignas(128) StreamSlot {
  uint64_t seq;    // sequence number of the item held
  uint64_t first;  // first ticket of the item
  uint64_t end;    // one past its last ticket
  const float* A;
  const float* B;
  float* C;
  int64_t lda, ldb, ldc;
  int32_t m, n, k;
  float alpha, beta;
  int32_t shape, tiles_n, vec_a, vec_b;
};

// Control words (host memory).  done[] follows the struct.
struct alignas(128) StreamCtl {
  uint64_t tail;    // items pushed (host writes, kernel reads)
  uint32_t closed;  // host: no more pushes; drain and leave
  uint32_t status;  // kernel: 0 running, else why it ended the stream
};
constexpr uint32_t kStreamIdle = 2;     // nothing pushed for the idle limit
constexpr uint32_t kStreamBadSlot = 3;  // a ticket map word named a slot past the ring


__device__ __forceinline__ uint64_t ld_acquire(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint32_t ld_acquire32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// What thread 0 tells the workgroup after a ticket lookup.
struct StreamTask {
  GemmArgs p;
  int32_t exit;
  int32_t slot;
  int32_t local;  // tile index inside the item
  int32_t shape, tiles_n;
  uint32_t tiles;
  uint64_t seq;
};

// Ticket map entry, one word written with a release store: the ticket + 1
// in the high bits (0 = never written) and the slot of the item holding the
// ticket in the low kSlotBits, so the tag and the slot arrive in one read.
struct TicketEntry {
  uint64_t word;
};
constexpr int kSlotBits = 12;
constexpr uint64_t kSlotMask = (1ull << kSlotBits) - 1;

// Thread 0: find the item that holds ticket t.  Returns false when the
// workgroup must leave.  The idle clock restarts whenever the tail moves:
// a workgroup whose ticket lies ahead of the pushed items is waiting, but
// the stream is not idle.
__device__ bool stream_find(StreamCtl* ctl, const StreamSlot* slots, const TicketEntry* tmap, int cap,
                            uint64_t t, uint64_t idle_ticks, StreamTask* task) {
  const TicketEntry* e = tmap + (t & (kTicketWindow - 1));
  const uint64_t want = (t + 1) << kSlotBits;
  uint64_t last_tail = ~0ull;  // read with the other control words when polling
  uint64_t since = wall_clock64();
  int backoff = 1;
  uint32_t polls = 0;
  for (;;) {
    const uint64_t w = ld_acquire(&e->word);
    if ((w & ~kSlotMask) == want) {
      // The item holding t stays in its slot until this tile is done, and
      // the acquire above orders these plain loads after the host's writes
      // of the slot, which is read as eight 16-byte loads issued together.
      const int s = (int)(w & kSlotMask);
      if (s >= cap) {  // never written so by the host: end the stream rather than read past the ring
        __hip_atomic_store(&ctl->status, kStreamBadSlot, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        return false;
      }
      StreamSlot slot;
      {
        const u32x4* src = reinterpret_cast<const u32x4*>(slots + s);
        u32x4 v[sizeof(StreamSlot) / 16];
#pragma unroll
        for (int i = 0; i < (int)(sizeof(StreamSlot) / 16); ++i) v[i] = src[i];
        __builtin_memcpy(&slot, v, sizeof slot);
      }
      const StreamSlot* q = &slot;
      GemmArgs& p = task->p;
      p.A = q->A;
      p.B = q->B;
      p.C = q->C;
      p.lda = q->lda;
      p.ldb = q->ldb;
      p.ldc = q->ldc;
      p.m = q->m;
      p.n = q->n;
      p.k = q->k;
      p.alpha = q->alpha;
      p.beta = q->beta;
      p.vec_a = q->vec_a;
      p.vec_b = q->vec_b;
      p.tiles_m = 0;
      p.tiles_n = 0;
      task->shape = q->shape;
      task->tiles_n = q->tiles_n;
      task->exit = 0;
      task->slot = s;
      task->local = (int32_t)(t - q->first);
      task->tiles = (uint32_t)(q->end - q->first);
      task->seq = q->seq;
      return true;
    }
    // Nothing pushed for this ticket yet: the entry is polled every time,
    // the control words every 8th time.
    if ((++polls & 7) != 0) {
      for (int i = 0; i < backoff; ++i) __builtin_amdgcn_s_sleep(127);
      continue;
    }
    if (ld_acquire32(&ctl->closed)) {
      // A push before the close is visible now: look once more.
      if ((ld_acquire(&e->word) & ~kSlotMask) == want) continue;
      return false;
    }
    if (ld_acquire32(&ctl->status) != 0) return false;
    const uint64_t tail = ld_acquire(&ctl->tail);
    if (tail != last_tail) {
      last_tail = tail;
      since = wall_clock64();
      backoff = 1;
    } else if (wall_clock64() - since > idle_ticks) {
      __hip_atomic_store(&ctl->status, kStreamIdle, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
      return false;
    }
    for (int i = 0; i < backoff; ++i) __builtin_amdgcn_s_sleep(127);
    backoff = backoff < 8 ? 2 * backoff : 8;
  }
}

// Workgroup-uniform copies (scalar registers) of values thread 0 put in LDS.
__device__ __forceinline__ int32_t uni(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ float uni(float x) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x))); }
__device__ __forceinline__ int64_t uni(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <class T>
__device__ __forceinline__ T* uni(T* x) { return (T*)uni((int64_t)x); }

__global__ void __launch_bounds__(kGroupedThreads) __attribute__((amdgpu_waves_per_eu(3)))
    sgemm_stream_f32(StreamCtl* ctl, const StreamSlot* slots, const TicketEntry* tmap, uint64_t* done,
                     int32_t cap, unsigned long long* ticket, uint32_t* pending, uint64_t idle_ticks) {
  extern __shared__ __align__(16) float lds[];
  __shared__ StreamTask task;
  for (;;) {
    if (threadIdx.x == 0) {
      const uint64_t t = atomicAdd(ticket, 1ull);
      if (!stream_find(ctl, slots, tmap, cap, t, idle_ticks, &task)) task.exit = 1;
    }
    __syncthreads();
    if (task.exit) break;
    GemmArgs p;
    p.A = uni(task.p.A);
    p.B = uni(task.p.B);
    p.C = uni(task.p.C);
    p.lda = uni(task.p.lda);
    p.ldb = uni(task.p.ldb);
    p.ldc = uni(task.p.ldc);
    p.m = uni(task.p.m);
    p.n = uni(task.p.n);
    p.k = uni(task.p.k);
    p.alpha = uni(task.p.alpha);
    p.beta = uni(task.p.beta);
    p.vec_a = uni(task.p.vec_a);
    p.vec_b = uni(task.p.vec_b);
    p.tiles_m = 0;
    p.tiles_n = 0;
    run_shape_tile(uni(task.shape), p, uni(task.tiles_n), uni(task.local), lds);
    // The tile's C stores: complete within the workgroup, then one
    // device-scope release (a write-back of this XCD's L2) by thread 0
    // before it counts the tile; the barrier carries the other lanes'
    // stores into that release.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const uint32_t old = atomicAdd(pending + task.slot, 1u);
      if (old + 1 == task.tiles) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        atomicExch(pending + task.slot, 0u);  // ready for the slot's next item
        __hip_atomic_store(done + task.slot, task.seq + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
    __syncthreads();
  }
}

namespace {

constexpr uint64_t kStreamMagic = 0x48505653474d4d53ull;  // "HPVSGMMS"
constexpr int kMaxCapacity = 4096;
static_assert(kMaxCapacity <= (1 << kSlotBits), "a slot index must fit the ticket map's slot bits");
constexpr int kMaxIdleMs = 60000;
constexpr int kMaxGridPerCu = 2;  // resident workgroups per CU (see hpvm_stream_open)
constexpr int kMaxCus = 256;      // CUs of the largest gfx950 part

struct Stream {
  uint64_t magic = kStreamMagic;
  std::mutex mu;
  int32_t capacity = 0, grid = 0, idle_ms = 0;
  // host memory shared with the kernel
  char* host = nullptr;
  int64_t host_size = 0;
  StreamCtl* ctl = nullptr;
  StreamSlot* slots = nullptr;
  uint64_t* done = nullptr;
  TicketEntry* tmap = nullptr;
  // device counters
  void* dev = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t finished = nullptr;
  // host bookkeeping
  uint64_t pushed = 0, popped = 0, next_ticket = 0;
  std::vector<uint64_t> first_ticket;  // per slot: first ticket of its item
  int64_t tiles = 0;
  bool ended = false;     // the kernel has exited
  hipError_t exit_error = hipSuccess;
};

std::mutex g_mu;
std::unordered_set<const void*> g_streams;
bool g_atexit = false;
// Pinned host blocks of closed streams, kept for reuse: freeing pinned
// memory can wait for the whole device, including other streams' kernels.
std::vector<std::pair<int64_t, char*>> g_host_pool;

char* pool_take(int64_t bytes, int64_t* size) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (size_t i = 0; i < g_host_pool.size(); ++i)
    if (g_host_pool[i].first >= bytes) {
      char* p = g_host_pool[i].second;
      *size = g_host_pool[i].first;
      g_host_pool.erase(g_host_pool.begin() + (long)i);
      return p;
    }
  return nullptr;
}

void pool_give(int64_t bytes, char* p) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_host_pool.push_back({bytes, p});
}

Stream* live_stream(const void* h) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!h || !g_streams.count(h)) return nullptr;
  Stream* s = (Stream*)h;
  return s->magic == kStreamMagic ? s : nullptr;
}

void host_store(uint64_t* p, uint64_t v) { __atomic_store_n(p, v, __ATOMIC_RELEASE); }
uint64_t host_load(const uint64_t* p) { return __atomic_load_n(p, __ATOMIC_ACQUIRE); }
uint32_t host_load32(const uint32_t* p) { return __atomic_load_n(p, __ATOMIC_ACQUIRE); }

// Non-blocking check whether the kernel has exited.
bool kernel_exited(Stream* s) {
  if (s->ended) return true;
  hipError_t e = hipEventQuery(s->finished);
  if (e == hipErrorNotReady) return false;
  s->ended = true;
  s->exit_error = e;
  return true;
}

// Frees a stream whose kernel has exited (or never started).  Device memory
// is stream-ordered, so nothing here waits for other streams' kernels.
void release(Stream* s) {
  if (s->dev) (void)hipFreeAsync(s->dev, s->stream);
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  if (s->finished) (void)hipEventDestroy(s->finished);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  if (s->host) pool_give(s->host_size, s->host);
  s->magic = 0;
  delete s;
}

int64_t done_bytes(int cap) { return ((int64_t)cap * 8 + 127) / 128 * 128; }

int64_t host_bytes(int cap) {
  return (int64_t)sizeof(StreamCtl) + (int64_t)cap * (int64_t)sizeof(StreamSlot) + done_bytes(cap) +
         (int64_t)kTicketWindow * (int64_t)sizeof(TicketEntry);
}

// Waits (bounded) for the kernel to exit after `closed` is set.
bool wait_exit(Stream* s, int32_t timeout_ms) {
  const auto until = std::chrono::steady_clock::now() + std::chrono::milliseconds(timeout_ms);
  while (!kernel_exited(s)) {
    if (std::chrono::steady_clock::now() >= until) return false;
    std::this_thread::sleep_for(std::chrono::microseconds(200));
  }
  return true;
}

// At process exit: tell every live stream's kernel to leave and give it a
// bounded time to do so, so no workgroup still reads host memory that the
// process is about to release.
void close_all_at_exit() {
  std::lock_guard<std::mutex> lk(g_mu);
  for (const void* h : g_streams) {
    Stream* s = (Stream*)h;
    __atomic_store_n(&s->ctl->closed, 1u, __ATOMIC_RELEASE);
    (void)wait_exit(s, s->idle_ms + 1000);
  }
}

bool overlaps(const void* a, int64_t ra, int64_t ca, int64_t lda, const void* b, int64_t rb, int64_t cb,
              int64_t ldb) {
  if (!a || !b || ra == 0 || ca == 0 || rb == 0 || cb == 0) return false;
  uintptr_t a0, a1, b0, b1;
  matrix_extent((const float*)a, ra, ca, lda, &a0, &a1);
  matrix_extent((const float*)b, rb, cb, ldb, &b0, &b1);
  return a0 < b1 && b0 < a1;
}

}  // namespace
}  // namespace hpvm

using namespace hpvm;

extern "C" {

int hpvm_stream_open(const hpvm_stream_config* cfg, void** handle) {
  if (!cfg) return set_error(HPVM_INVALID_ARG, "argument 1: config is NULL");
  if (cfg->capacity < 1 || cfg->capacity > kMaxCapacity)
    return set_error(HPVM_INVALID_ARG, "argument 1: capacity = %d not in [1, %d]", cfg->capacity, kMaxCapacity);
  // Two resident workgroups per CU at most: a third takes every SIMD's
  // registers, so no wave of another kernel (a copy's blit kernel included)
  // could start while the stream is open; such work would wait until the
  // stream idles out.  512 = two per CU of a 256-CU gfx950 part; the
  // device's own CU count is checked again below.
  if (cfg->grid < 0 || cfg->grid > kMaxGridPerCu * kMaxCus)
    return set_error(HPVM_INVALID_ARG, "argument 1: grid = %d not in [0, %d] (at most %d workgroups per CU)",
                     cfg->grid, kMaxGridPerCu * kMaxCus, kMaxGridPerCu);
  if (cfg->idle_ms < 1 || cfg->idle_ms > kMaxIdleMs)
    return set_error(HPVM_INVALID_ARG, "argument 1: idle_ms = %d not in [1, %d]", cfg->idle_ms, kMaxIdleMs);
  if (!handle) return set_error(HPVM_INVALID_ARG, "argument 2: handle is NULL");
  *handle = nullptr;
  if (fault_injected("launch")) return set_error(HPVM_HIP_ERROR, "injected launch failure (HPVM_FAULT_INJECT)");

  Stream* s = new (std::nothrow) Stream();
  if (!s) return set_error(HPVM_INVALID_ARG, "out of host memory");
  s->capacity = cfg->capacity;
  s->idle_ms = cfg->idle_ms;
  int dev = 0, cus = 0, rate_khz = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev);
  if (e == hipSuccess && rate_khz <= 0) e = hipErrorInvalidValue;
  if (e == hipSuccess && cfg->grid > kMaxGridPerCu * std::max(cus, 1)) {
    delete s;
    return set_error(HPVM_INVALID_ARG, "argument 1: grid = %d is more than %d workgroups per CU on %d CUs",
                     cfg->grid, kMaxGridPerCu, cus);
  }
  s->grid = cfg->grid > 0 ? cfg->grid : kMaxGridPerCu * std::max(cus, 1);
  const int64_t hb = host_bytes(s->capacity);
  if (e == hipSuccess) {
    s->host = pool_take(hb, &s->host_size);  // a block of at least hb bytes
    if (!s->host) {
      e = hipHostMalloc((void**)&s->host, (size_t)hb, hipHostMallocCoherent | hipHostMallocMapped);
      if (e == hipSuccess) s->host_size = hb;
      else s->host = nullptr;
    }
  }
  if (e == hipSuccess) {
    std::memset(s->host, 0, (size_t)hb);
    s->ctl = (StreamCtl*)s->host;
    s->slots = (StreamSlot*)(s->host + sizeof(StreamCtl));
    s->done = (uint64_t*)(s->host + sizeof(StreamCtl) + (size_t)s->capacity * sizeof(StreamSlot));
    s->tmap = (TicketEntry*)((char*)s->done + done_bytes(s->capacity));
    s->first_ticket.assign((size_t)s->capacity, 0);
  }
  const size_t db = 256 + (size_t)s->capacity * 4;
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->finished, hipEventDisableTiming);
  // HPVM_FAULT_INJECT=alloc: the device counters' allocation fails (the
  // host ring, stream and event exist by then and are released below).
  if (e == hipSuccess) e = fault_injected("alloc") ? hipErrorOutOfMemory : hipMallocAsync(&s->dev, db, s->stream);
  if (e == hipSuccess) e = hipMemsetAsync(s->dev, 0, db, s->stream);  // ordered before the kernel
  StreamCtl* dctl = nullptr;
  StreamSlot* dslots = nullptr;
  uint64_t* ddone = nullptr;
  TicketEntry* dtmap = nullptr;
  if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&dtmap, s->tmap, 0);
  if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&dctl, s->ctl, 0);
  if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&dslots, s->slots, 0);
  if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&ddone, s->done, 0);
  if (e == hipSuccess) {
    unsigned long long* ticket = (unsigned long long*)s->dev;
    uint32_t* pending = (uint32_t*)((char*)s->dev + 256);
    int32_t cap = s->capacity;
    uint64_t idle_ticks = (uint64_t)s->idle_ms * (uint64_t)rate_khz;
    void* kargs[] = {&dctl, &dslots, &dtmap, &ddone, &cap, &ticket, &pending, &idle_ticks};
    e = hipLaunchKernel(reinterpret_cast<const void*>(&sgemm_stream_f32), dim3(s->grid), dim3(kGroupedThreads),
                        kargs, (size_t)kGroupedLds, s->stream);
  }
  if (e == hipSuccess) e = hipEventRecord(s->finished, s->stream);
  if (e != hipSuccess) {
    // A launched kernel must not outlive its host memory: close it first.
    if (s->ctl) __atomic_store_n(&s->ctl->closed, 1u, __ATOMIC_RELEASE);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    release(s);
    return hip_error(e, "stream open");
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_streams.insert(s);
    if (!g_atexit) {
      std::atexit(close_all_at_exit);
      g_atexit = true;
    }
  }
  *handle = s;
  return clear_error();
}

int hpvm_stream_push(void* handle, const hpvm_sgemm_desc* item, int64_t* seq) {
  Stream* s = live_stream(handle);
  if (!s) return set_error(HPVM_BAD_HANDLE, "argument 1: unknown or closed stream");
  if (!item) return set_error(HPVM_INVALID_ARG, "argument 2: item is NULL");
  const hpvm_sgemm_desc& d = *item;
  bool reads_ab;
  int rc = check_gemm_args("item: ", d.m, d.n, d.k, d.alpha, d.A, d.lda, d.B, d.ldb, d.beta, d.C, d.ldc, &reads_ab);
  if (rc != HPVM_OK) return rc;
  std::lock_guard<std::mutex> lk(s->mu);
  if (host_load32(&s->ctl->status) != 0 || kernel_exited(s))
    return set_error(HPVM_STREAM_ENDED, "argument 1: the streaming kernel has ended (idle limit or error)");
  if (s->pushed - s->popped >= (uint64_t)s->capacity)
    return set_error(HPVM_QUEUE_FULL, "argument 1: all %d slots hold items not yet popped", s->capacity);
  // Items in flight run concurrently: the new one may not write what another
  // one reads or writes, nor read what another one writes.
  if (d.m > 0 && d.n > 0) {
    for (uint64_t q = s->popped; q < s->pushed; ++q) {
      const StreamSlot& o = s->slots[q % (uint64_t)s->capacity];
      if (o.m == 0 || o.n == 0) continue;
      const bool o_reads = o.k > 0 && o.alpha != 0.0f;
      bool clash = overlaps(d.C, d.m, d.n, d.ldc, o.C, o.m, o.n, o.ldc);
      if (o_reads) clash = clash || overlaps(d.C, d.m, d.n, d.ldc, o.A, o.m, o.k, o.lda) ||
                           overlaps(d.C, d.m, d.n, d.ldc, o.B, o.k, o.n, o.ldb);
      if (reads_ab) clash = clash || overlaps(d.A, d.m, d.k, d.lda, o.C, o.m, o.n, o.ldc) ||
                            overlaps(d.B, d.k, d.n, d.ldb, o.C, o.m, o.n, o.ldc);
      if (clash)
        return set_error(HPVM_INVALID_ARG, "argument 2: item overlaps in-flight item %llu; pop it first",
                         (unsigned long long)q);
    }
  }
  const uint64_t sq = s->pushed;
  const int slot = (int)(sq % (uint64_t)s->capacity);
  StreamSlot* q = s->slots + slot;
  const int shape = cost_model_shape(d.m, d.n, reads_ab ? d.k : 0, 1.0);
  const uint64_t tiles = (uint64_t)shape_tiles(d.m, d.n, shape);
  if (tiles > kTicketWindow)
    return set_error(HPVM_UNSUPPORTED, "argument 2: the item needs %llu tiles, more than the %llu a stream "
                     "can hold in flight", (unsigned long long)tiles, (unsigned long long)kTicketWindow);
  // Tickets in flight stay within the ticket map's window.
  const uint64_t oldest = s->popped < s->pushed ? s->first_ticket[s->popped % (uint64_t)s->capacity]
                                                 : s->next_ticket;
  if (s->next_ticket + tiles - oldest > kTicketWindow)
    return set_error(HPVM_QUEUE_FULL, "argument 1: the items in flight hold too many tiles; pop first");
  q->first = s->next_ticket;
  q->end = s->next_ticket + tiles;
  q->A = d.A;
  q->B = d.B;
  q->C = d.C;
  q->lda = d.lda;
  q->ldb = d.ldb;
  q->ldc = d.ldc;
  q->m = (int32_t)d.m;
  q->n = (int32_t)d.n;
  q->k = reads_ab ? (int32_t)d.k : 0;  // alpha == 0 or k == 0: C <- beta C, A and B unread
  q->alpha = d.alpha;
  q->beta = d.beta;
  q->shape = shape;
  q->tiles_n = (int32_t)((d.n + kGroupedShapes[shape].tile.tile_n - 1) / kGroupedShapes[shape].tile.tile_n);
  q->vec_a = vec16(d.A, d.lda);
  q->vec_b = vec16(d.B, d.ldb);
  q->seq = sq;
  s->first_ticket[slot] = s->next_ticket;
  for (uint64_t t = s->next_ticket; t < s->next_ticket + tiles; ++t)
    host_store(&s->tmap[t & (kTicketWindow - 1)].word, ((t + 1) << kSlotBits) | (uint64_t)slot);
  if (tiles == 0) host_store(s->done + slot, sq + 1);  // nothing for the kernel to do
  s->next_ticket += tiles;
  s->tiles += (int64_t)tiles;
  s->pushed = sq + 1;
  host_store(&s->ctl->tail, s->pushed);
  if (seq) *seq = (int64_t)sq;
  return clear_error();
}

int hpvm_stream_pop(void* handle, int32_t timeout_ms, int64_t* seq, float** C) {
  Stream* s = live_stream(handle);
  if (!s) return set_error(HPVM_BAD_HANDLE, "argument 1: unknown or closed stream");
  if (timeout_ms < 0) return set_error(HPVM_INVALID_ARG, "argument 2: timeout_ms = %d < 0", timeout_ms);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->popped == s->pushed) return set_error(HPVM_INVALID_ARG, "argument 1: no item in flight to pop");
  const uint64_t sq = s->popped;
  const int slot = (int)(sq % (uint64_t)s->capacity);
  // The completion flag is in coherent host memory, so polling it is a
  // cached load.  Spin (yielding) for the first 2 ms -- a sleep costs tens
  // of microseconds of timer slack per item -- then poll every 50 us.
  const auto start = std::chrono::steady_clock::now();
  const auto until = start + std::chrono::milliseconds(timeout_ms);
  const auto spin_until = start + std::chrono::milliseconds(2);
  for (uint64_t spins = 0; host_load(s->done + slot) != sq + 1; ++spins) {
    if (spins % 256 == 255 && (host_load32(&s->ctl->status) != 0 || kernel_exited(s))) {
      if (host_load(s->done + slot) == sq + 1) break;
      if (s->exit_error != hipSuccess) return hip_error(s->exit_error, "streaming kernel");
      return set_error(HPVM_STREAM_ENDED, "the streaming kernel ended before item %llu completed",
                       (unsigned long long)sq);
    }
    const auto now = std::chrono::steady_clock::now();
    if (now >= until)
      return set_error(HPVM_TIMEOUT, "item %llu not complete after %d ms", (unsigned long long)sq, timeout_ms);
    if (now < spin_until)
      std::this_thread::yield();
    else
      std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
  if (seq) *seq = (int64_t)sq;
  if (C) *C = s->slots[slot].C;
  s->popped = sq + 1;
  return clear_error();
}

int hpvm_stream_info(const void* handle, hpvm_stream_status* info) {
  Stream* s = live_stream(handle);
  if (!s) return set_error(HPVM_BAD_HANDLE, "argument 1: unknown or closed stream");
  if (!info) return set_error(HPVM_INVALID_ARG, "argument 2: info is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  info->pushed = (int64_t)s->pushed;
  info->popped = (int64_t)s->popped;
  info->tiles = s->tiles;
  info->capacity = s->capacity;
  info->grid = s->grid;
  info->idle_ms = s->idle_ms;
  info->running = kernel_exited(s) ? 0 : 1;
  info->idle_ended = host_load32(&s->ctl->status) == kStreamIdle ? 1 : 0;
  return clear_error();
}

int hpvm_stream_close(void* handle, int32_t timeout_ms) {
  Stream* s = live_stream(handle);
  if (!s) return set_error(HPVM_BAD_HANDLE, "argument 1: unknown or closed stream");
  if (timeout_ms < 0) return set_error(HPVM_INVALID_ARG, "argument 2: timeout_ms = %d < 0", timeout_ms);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    __atomic_store_n(&s->ctl->closed, 1u, __ATOMIC_RELEASE);
    if (!wait_exit(s, timeout_ms))
      return set_error(HPVM_TIMEOUT, "the streaming kernel is still draining after %d ms; close again",
                       timeout_ms);
  }
  const hipError_t e = hipStreamSynchronize(s->stream);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_streams.erase(s);
  }
  const hipError_t ke = s->exit_error;
  release(s);
  if (ke != hipSuccess) return hip_error(ke, "streaming kernel");
  if (e != hipSuccess) return hip_error(e, "stream close");
  return clear_error();
}

}  // extern "C"
