// Grouped launch: many independent sgemm graphs in one persistent kernel.
//
// Every instance of a batch is its own sgemm dataflow graph; the dynamic
// instances of SgemmInternal are independent (HPVM report, Sec. 2.1), so all
// tiles of all instances can be worked off by one set of resident
// workgroups.  The kernel keeps its workgroups alive and has them pull tiles
// from a device-side list (the persistent-node idea of Sec. 3.5), and one
// launch replaces one launch per instance (the launch-overhead argument of
// Sec. 4.2 and of the bfs result in Sec. 5.1).  Each instance carries its
// own tile shape, chosen on the host by a cost model or by the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <numeric>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "device_common.hpp"
#include "hpvm_sgemm.h"
#include "internal.hpp"
#include "mfma_f32.hpp"
#include "persistent.hpp"

namespace hpvm {

// One instance as the device sees it.
struct alignas(16) GroupDesc {
  const float* A;
  const float* B;
  float* C;
  int64_t lda, ldb, ldc;
  int32_t m, n, k;
  float alpha, beta;
  int32_t shape;       // index into kGroupedShapes
  int32_t tiles_n;     // tiles along n for that shape
  int32_t tile_start;  // first entry of this instance in the tile list
  int32_t vec_a, vec_b;
};

// Three workgroups per CU (the register budget the attribute asks for fits
// without spills; LDS allows it too).
// Persistent kernel.  Every workgroup loops: take the next tile index from
// the shared counter, find its instance and position, run that tile.  All
// workgroups leave once the list is exhausted.
__global__ void __launch_bounds__(kGroupedThreads) __attribute__((amdgpu_waves_per_eu(3)))
    sgemm_grouped_f32(const GroupDesc* __restrict__ descs, const int32_t* __restrict__ tile_inst,
                      int32_t total_tiles, int32_t* counter) {
  extern __shared__ __align__(16) float lds[];
  __shared__ int32_t next_tile;
  for (;;) {
    if (threadIdx.x == 0) next_tile = atomicAdd(counter, 1);
    __syncthreads();
    const int t = next_tile;
    __syncthreads();
    if (t >= total_tiles) break;
    const GroupDesc& d = descs[tile_inst[t]];
    GemmArgs p;
    p.A = d.A;
    p.B = d.B;
    p.C = d.C;
    p.lda = d.lda;
    p.ldb = d.ldb;
    p.ldc = d.ldc;
    p.m = d.m;
    p.n = d.n;
    p.k = d.k;
    p.alpha = d.alpha;
    p.beta = d.beta;
    p.vec_a = d.vec_a;
    p.vec_b = d.vec_b;
    run_shape_tile(d.shape, p, d.tiles_n, t - d.tile_start, lds);
  }
}

// Clears the tile counter (a kernel, so graphs hold no memset node).
__global__ void grouped_reset(int32_t* counter) {
  if (threadIdx.x == 0) *counter = 0;
}

namespace {

constexpr uint64_t kPlanMagic = 0x48505653474d4d50ull;   // "HPVSGMMP"
constexpr uint64_t kGraphMagic = 0x48505653474d4d47ull;  // "HPVSGMMG"
constexpr int64_t kDescOffset = 256;

struct Plan {
  uint64_t magic = kPlanMagic;
  uint64_t serial = 0;
  uint64_t version = 0;
  std::vector<hpvm_sgemm_desc> user;  // caller order
  std::vector<int> shape;             // per instance, caller order
  // Derived schedule:
  std::vector<GroupDesc> dev;  // longest tiles first
  std::vector<int32_t> tile_inst;
  int32_t total_tiles = 0;
  double flops = 0.0;
  int32_t grid = 0;
};

struct Graph {
  uint64_t magic = kGraphMagic;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

std::mutex g_mu;
std::unordered_set<const void*> g_plans;
std::unordered_set<const void*> g_graphs;
std::unordered_map<const void*, std::pair<uint64_t, uint64_t>> g_ws_owner;  // workspace -> plan
uint64_t g_serial = 0;

Plan* live_plan(const void* h) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!h || !g_plans.count(h)) return nullptr;
  Plan* p = (Plan*)h;
  return p->magic == kPlanMagic ? p : nullptr;
}

Graph* live_graph(const void* h) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!h || !g_graphs.count(h)) return nullptr;
  Graph* g = (Graph*)h;
  return g->magic == kGraphMagic ? g : nullptr;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

int64_t tiles_of(const hpvm_sgemm_desc& d, int shape) { return shape_tiles(d.m, d.n, shape); }

// Rebuilds the device schedule from plan->user and plan->shape.  With
// `scratch`, every instance reads and writes its own slice of scratch
// (ldc = n) instead of its C, with its own beta, so that timing runs do the
// replays' work (C read when beta != 0) without touching C.
void build_schedule(Plan* p, float* scratch) {
  const int count = (int)p->user.size();
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  auto work = [&](int i) {
    const hpvm_tile& t = kGroupedShapes[p->shape[i]].tile;
    const int64_t k = p->user[i].alpha != 0.0f ? p->user[i].k : 0;
    return (double)t.tile_m * t.tile_n * (double)(k + 32);
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
  std::vector<int64_t> scratch_off(count, 0);
  int64_t off = 0;
  for (int i = 0; i < count; ++i) {
    scratch_off[i] = off;
    off += p->user[i].m * p->user[i].n;
  }
  p->dev.clear();
  p->tile_inst.clear();
  p->flops = 0.0;
  for (int i : order) {
    const hpvm_sgemm_desc& u = p->user[i];
    p->flops += 2.0 * (double)u.m * (double)u.n * (double)u.k;
    const int64_t tiles = tiles_of(u, p->shape[i]);
    if (tiles == 0) continue;
    GroupDesc d{};
    d.A = u.A;
    d.B = u.B;
    d.C = scratch ? scratch + scratch_off[i] : u.C;
    d.lda = u.lda;
    d.ldb = u.ldb;
    d.ldc = scratch ? std::max<int64_t>(u.n, 1) : u.ldc;
    d.m = (int32_t)u.m;
    d.n = (int32_t)u.n;
    d.k = u.alpha != 0.0f ? (int32_t)u.k : 0;  // alpha == 0: A and B are not read
    d.alpha = u.alpha;
    d.beta = u.beta;
    d.shape = p->shape[i];
    d.tiles_n = (int32_t)ceil_div(u.n, kGroupedShapes[d.shape].tile.tile_n);
    d.tile_start = (int32_t)p->tile_inst.size();
    d.vec_a = vec16(u.A, u.lda);
    d.vec_b = vec16(u.B, u.ldb);
    const int32_t idx = (int32_t)p->dev.size();
    p->dev.push_back(d);
    p->tile_inst.insert(p->tile_inst.end(), (size_t)tiles, idx);
  }
  p->total_tiles = (int32_t)p->tile_inst.size();
  p->version += 1;
}

// The workspace is sized for the largest schedule any shape assignment can
// produce (every instance on the shape with the most tiles), so autotuning
// never needs a larger one.
int64_t max_tiles(const Plan* p) {
  int64_t total = 0;
  for (const auto& u : p->user) {
    int64_t most = 0;
    for (int s = 0; s < kNumGroupedShapes; ++s) most = std::max(most, tiles_of(u, s));
    total += most;
  }
  return total;
}

int64_t workspace_bytes(const Plan* p) {
  const int64_t descs = (int64_t)p->user.size() * (int64_t)sizeof(GroupDesc);
  return kDescOffset + ((descs + 15) / 16) * 16 + max_tiles(p) * 4 + 16;
}

int64_t scratch_bytes(const Plan* p) {
  int64_t e = 0;
  for (const auto& u : p->user) e += u.m * u.n;
  return e * (int64_t)sizeof(float);
}

struct WsLayout {
  int32_t* counter;
  GroupDesc* descs;
  int32_t* tile_inst;
};

WsLayout layout(const Plan* p, void* ws) {
  char* base = (char*)ws;
  const int64_t descs = (int64_t)p->user.size() * (int64_t)sizeof(GroupDesc);
  WsLayout l;
  l.counter = (int32_t*)base;
  l.descs = (GroupDesc*)(base + kDescOffset);
  l.tile_inst = (int32_t*)(base + kDescOffset + ((descs + 15) / 16) * 16);
  return l;
}

int check_workspace(const Plan* p, void* ws, int64_t bytes, int argno) {
  if (!ws) return set_error(HPVM_INVALID_ARG, "argument %d: workspace is NULL", argno);
  if ((uintptr_t)ws % 16) return set_error(HPVM_INVALID_ARG, "argument %d: workspace is not 16-byte aligned", argno);
  const int64_t need = workspace_bytes(p);
  if (bytes < need)
    return set_error(HPVM_WORKSPACE_TOO_SMALL, "argument %d: workspace has %lld bytes, the plan needs %lld",
                     argno + 1, (long long)bytes, (long long)need);
  return HPVM_OK;
}

// Copies the schedule into the workspace unless it already holds it.
hipError_t upload(Plan* p, void* ws, hipStream_t s) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_ws_owner.find(ws);
    if (it != g_ws_owner.end() && it->second == std::make_pair(p->serial, p->version)) return hipSuccess;
  }
  WsLayout l = layout(p, ws);
  hipError_t e = hipSuccess;
  if (!p->dev.empty())
    e = hipMemcpyAsync(l.descs, p->dev.data(), p->dev.size() * sizeof(GroupDesc), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !p->tile_inst.empty())
    e = hipMemcpyAsync(l.tile_inst, p->tile_inst.data(), p->tile_inst.size() * 4, hipMemcpyHostToDevice, s);
  // The host vectors may change (autotuning), so finish the copies now.
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_ws_owner[ws] = std::make_pair(p->serial, p->version);
  }
  return e;
}

hipError_t persistent_grid(Plan* p) {
  if (p->grid > 0) return hipSuccess;
  int dev = 0, cus = 0, occ = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(&sgemm_grouped_f32),
                                                     kGroupedThreads, (size_t)kGroupedLds);
  if (e != hipSuccess) return e;
  p->grid = std::max(1, cus * std::max(occ, 1));
  return hipSuccess;
}

hipError_t enqueue(Plan* p, void* ws, hipStream_t s) {
  WsLayout l = layout(p, ws);
  void* rargs[] = {&l.counter};
  hipError_t e = hipLaunchKernel(reinterpret_cast<const void*>(&grouped_reset), dim3(1), dim3(64), rargs, 0, s);
  if (e != hipSuccess || p->total_tiles == 0) return e;
  const GroupDesc* d = l.descs;
  const int32_t* ti = l.tile_inst;
  int32_t total = p->total_tiles;
  int32_t* counter = l.counter;
  void* kargs[] = {&d, &ti, &total, &counter};
  const int grid = std::min(p->grid, p->total_tiles);
  return hipLaunchKernel(reinterpret_cast<const void*>(&sgemm_grouped_f32), dim3(grid), dim3(kGroupedThreads),
                         kargs, (size_t)kGroupedLds, s);
}

int shape_of(const hpvm_tile* t) {
  for (int s = 0; s < kNumGroupedShapes; ++s) {
    const hpvm_tile& g = kGroupedShapes[s].tile;
    if (g.tile_m == t->tile_m && g.tile_n == t->tile_n && g.tile_k == t->tile_k && g.leaf_m == t->leaf_m &&
        g.leaf_n == t->leaf_n && g.stages == t->stages)
      return s;
  }
  return -1;
}

}  // namespace
}  // namespace hpvm

using namespace hpvm;

extern "C" {

int hpvm_grouped_menu(hpvm_tile* out, int32_t capacity, int32_t* count) {
  if (capacity < 0 || (capacity > 0 && !out))
    return set_error(HPVM_INVALID_ARG, "argument 2: bad capacity or NULL output");
  if (!count) return set_error(HPVM_INVALID_ARG, "argument 3: count is NULL");
  for (int i = 0; i < kNumGroupedShapes && i < capacity; ++i) out[i] = kGroupedShapes[i].tile;
  *count = kNumGroupedShapes;
  return clear_error();
}

int hpvm_grouped_plan_create(int32_t count, const hpvm_sgemm_desc* descs, int32_t prec, const hpvm_tile* tile,
                             void** plan) {
  if (count < 0) return set_error(HPVM_INVALID_ARG, "argument 1: count = %d < 0", count);
  if (count > 0 && !descs) return set_error(HPVM_INVALID_ARG, "argument 2: descs is NULL");
  if (prec != HPVM_PREC_FP32)
    return set_error(HPVM_UNSUPPORTED, "argument 3: the grouped kernel is FP32 only (got %d)", prec);
  int fixed = -1;
  if (tile) {
    fixed = shape_of(tile);
    if (fixed < 0)
      return set_error(HPVM_UNSUPPORTED, "argument 4: tile %dx%dx%d leaf %dx%d is not in the grouped menu",
                       tile->tile_m, tile->tile_n, tile->tile_k, tile->leaf_m, tile->leaf_n);
  }
  if (!plan) return set_error(HPVM_INVALID_ARG, "argument 5: plan is NULL");
  *plan = nullptr;
  for (int32_t i = 0; i < count; ++i) {
    const hpvm_sgemm_desc& d = descs[i];
    char what[48];
    snprintf(what, sizeof what, "instance %d: ", i);
    bool reads_ab;
    int rc = check_gemm_args(what, d.m, d.n, d.k, d.alpha, d.A, d.lda, d.B, d.ldb, d.beta, d.C, d.ldc, &reads_ab);
    if (rc != HPVM_OK) return rc;
  }
  // No two instances may write overlapping memory.
  std::vector<std::pair<uintptr_t, std::pair<uintptr_t, int>>> spans;
  for (int32_t i = 0; i < count; ++i) {
    const hpvm_sgemm_desc& d = descs[i];
    if (d.m == 0 || d.n == 0) continue;
    uintptr_t lo, hi;
    matrix_extent(d.C, d.m, d.n, d.ldc, &lo, &hi);
    spans.push_back({lo, {hi, i}});
  }
  std::sort(spans.begin(), spans.end());
  for (size_t i = 1; i < spans.size(); ++i)
    if (spans[i].first < spans[i - 1].second.first)
      return set_error(HPVM_INVALID_ARG, "instances %d and %d write overlapping C ranges",
                       spans[i - 1].second.second, spans[i].second.second);
  Plan* p = new (std::nothrow) Plan();
  if (!p) return set_error(HPVM_INVALID_ARG, "out of host memory");
  p->user.assign(descs, descs + count);
  p->shape.resize(count);
  for (int32_t i = 0; i < count; ++i)
    p->shape[i] = fixed >= 0 ? fixed : cost_model_shape(descs[i].m, descs[i].n, descs[i].k, 1.0);
  build_schedule(p, nullptr);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    p->serial = ++g_serial;
    g_plans.insert(p);
  }
  *plan = p;
  return clear_error();
}

int hpvm_grouped_plan_info(const void* plan, hpvm_grouped_info* info) {
  const Plan* p = live_plan(plan);
  if (!p) return set_error(HPVM_BAD_HANDLE, "argument 1: unknown or destroyed plan");
  if (!info) return set_error(HPVM_INVALID_ARG, "argument 2: info is NULL");
  info->count = (int32_t)p->user.size();
  info->total_tiles = p->total_tiles;
  info->grid = p->grid ? std::min(p->grid, p->total_tiles) : 0;
  bool used[kNumGroupedShapes] = {false, false, false, false};
  for (int s : p->shape) used[s] = true;
  info->shapes_used = (int32_t)std::count(used, used + kNumGroupedShapes, true);
  info->workspace_bytes = workspace_bytes(p);
  info->scratch_bytes = scratch_bytes(p);
  info->flops = p->flops;
  return clear_error();
}

int hpvm_grouped_instance_tile(const void* plan, int32_t index, hpvm_tile* tile) {
  const Plan* p = live_plan(plan);
  if (!p) return set_error(HPVM_BAD_HANDLE, "argument 1: unknown or destroyed plan");
  if (index < 0 || index >= (int32_t)p->user.size())
    return set_error(HPVM_INVALID_ARG, "argument 2: index %d out of range", index);
  if (!tile) return set_error(HPVM_INVALID_ARG, "argument 3: tile is NULL");
  *tile = kGroupedShapes[p->shape[index]].tile;
  return clear_error();
}

int hpvm_grouped_workspace_bytes(const void* plan, int64_t* bytes) {
  const Plan* p = live_plan(plan);
  if (!p) return set_error(HPVM_BAD_HANDLE, "argument 1: unknown or destroyed plan");
  if (!bytes) return set_error(HPVM_INVALID_ARG, "argument 2: bytes is NULL");
  *bytes = workspace_bytes(p);
  return clear_error();
}

int hpvm_grouped_run(void* plan, void* workspace, int64_t workspace_bytes_, void* stream) {
  Plan* p = live_plan(plan);
  if (!p) return set_error(HPVM_BAD_HANDLE, "argument 1: unknown or destroyed plan");
  int rc = check_workspace(p, workspace, workspace_bytes_, 2);
  if (rc != HPVM_OK) return rc;
  if (fault_injected("launch")) return set_error(HPVM_HIP_ERROR, "injected launch failure (HPVM_FAULT_INJECT)");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = persistent_grid(p);
  if (e == hipSuccess) e = upload(p, workspace, s);
  if (e == hipSuccess) e = enqueue(p, workspace, s);
  return e == hipSuccess ? clear_error() : hip_error(e, "grouped launch");
}

int hpvm_grouped_capture(void* plan, void* workspace, int64_t workspace_bytes_, void* stream, void** graph) {
  Plan* p = live_plan(plan);
  if (!p) return set_error(HPVM_BAD_HANDLE, "argument 1: unknown or destroyed plan");
  int rc = check_workspace(p, workspace, workspace_bytes_, 2);
  if (rc != HPVM_OK) return rc;
  if (!graph) return set_error(HPVM_INVALID_ARG, "argument 5: graph is NULL");
  *graph = nullptr;
  if (fault_injected("capture")) return set_error(HPVM_HIP_ERROR, "injected capture failure (HPVM_FAULT_INJECT)");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = persistent_grid(p);
  if (e == hipSuccess) e = upload(p, workspace, s);
  if (e != hipSuccess) return hip_error(e, "grouped capture (upload)");

  Graph* g = new (std::nothrow) Graph();
  if (!g) return set_error(HPVM_INVALID_ARG, "out of host memory");
  WsLayout l = layout(p, workspace);
  e = hipGraphCreate(&g->graph, 0);
  hipGraphNode_t reset_node = nullptr, run_node = nullptr;
  if (e == hipSuccess) {
    void* rargs[] = {&l.counter};
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void*>(&grouped_reset);
    kp.gridDim = dim3(1);
    kp.blockDim = dim3(64);
    kp.sharedMemBytes = 0;
    kp.kernelParams = rargs;
    kp.extra = nullptr;
    e = hipGraphAddKernelNode(&reset_node, g->graph, nullptr, 0, &kp);
  }
  if (e == hipSuccess && p->total_tiles > 0) {
    const GroupDesc* d = l.descs;
    const int32_t* ti = l.tile_inst;
    int32_t total = p->total_tiles;
    int32_t* counter = l.counter;
    void* kargs[] = {&d, &ti, &total, &counter};
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void*>(&sgemm_grouped_f32);
    kp.gridDim = dim3(std::min(p->grid, p->total_tiles));
    kp.blockDim = dim3(kGroupedThreads);
    kp.sharedMemBytes = (unsigned)kGroupedLds;
    kp.kernelParams = kargs;
    kp.extra = nullptr;
    e = hipGraphAddKernelNode(&run_node, g->graph, &reset_node, 1, &kp);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return hip_error(e, "grouped capture");
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_graphs.insert(g);
  }
  *graph = g;
  return clear_error();
}

int hpvm_graph_launch(void* graph, void* stream) {
  Graph* g = live_graph(graph);
  if (!g) return set_error(HPVM_BAD_HANDLE, "argument 1: unknown or destroyed graph");
  if (fault_injected("launch")) return set_error(HPVM_HIP_ERROR, "injected launch failure (HPVM_FAULT_INJECT)");
  hipError_t e = hipGraphLaunch(g->exec, reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? clear_error() : hip_error(e, "graph launch");
}

int hpvm_graph_destroy(void* graph) {
  Graph* g = live_graph(graph);
  if (!g) return set_error(HPVM_BAD_HANDLE, "argument 1: unknown or destroyed graph");
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_graphs.erase(g);
  }
  hipError_t e1 = g->exec ? hipGraphExecDestroy(g->exec) : hipSuccess;
  hipError_t e2 = g->graph ? hipGraphDestroy(g->graph) : hipSuccess;
  g->magic = 0;
  delete g;
  if (e1 != hipSuccess) return hip_error(e1, "graph destroy");
  if (e2 != hipSuccess) return hip_error(e2, "graph destroy");
  return clear_error();
}

int hpvm_grouped_plan_destroy(void* plan) {
  Plan* p = live_plan(plan);
  if (!p) return set_error(HPVM_BAD_HANDLE, "argument 1: unknown or destroyed plan");
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_plans.erase(p);
    for (auto it = g_ws_owner.begin(); it != g_ws_owner.end();)
      it = (it->second.first == p->serial) ? g_ws_owner.erase(it) : std::next(it);
  }
  p->magic = 0;
  delete p;
  return clear_error();
}

int hpvm_grouped_autotune(void* plan, void* workspace, int64_t workspace_bytes_, float* scratch,
                          int64_t scratch_bytes_, int32_t reps, void* stream, float* best_ms) {
  Plan* p = live_plan(plan);
  if (!p) return set_error(HPVM_BAD_HANDLE, "argument 1: unknown or destroyed plan");
  int rc = check_workspace(p, workspace, workspace_bytes_, 2);
  if (rc != HPVM_OK) return rc;
  const int64_t need = scratch_bytes(p);
  if (need > 0 && !scratch) return set_error(HPVM_INVALID_ARG, "argument 4: scratch is NULL");
  if (scratch_bytes_ < need)
    return set_error(HPVM_WORKSPACE_TOO_SMALL, "argument 5: scratch has %lld bytes, the plan needs %lld",
                     (long long)scratch_bytes_, (long long)need);
  if (reps < 1) return set_error(HPVM_INVALID_ARG, "argument 6: reps = %d < 1", reps);
  if (!best_ms) return set_error(HPVM_INVALID_ARG, "argument 8: best_ms is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // The timing runs read the scratch as C: clear it first (a fill kernel,
  // so the values read are finite and the same every time).
  if (need > 0) {
    hipError_t ze = launch_scale(scratch, 1, 1, need / (int64_t)sizeof(float), 0.0f, s);
    if (ze != hipSuccess) return hip_error(ze, "grouped autotune (clear scratch)");
  }

  // Candidates: one shape for all instances, and the cost model at several
  // weights of the per-shape cost factors and of the per-tile overhead
  // (each distinct assignment timed once).
  std::vector<std::vector<int>> cands;
  for (int sh = 0; sh < kNumGroupedShapes; ++sh) cands.emplace_back(p->user.size(), sh);
  for (double overhead : {0.0, 32.0, 64.0, 128.0, 256.0})
    for (double lambda : {0.0, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0}) {
      std::vector<int> c(p->user.size());
      for (size_t i = 0; i < p->user.size(); ++i)
        c[i] = cost_model_shape(p->user[i].m, p->user[i].n, p->user[i].k, lambda, overhead);
      if (std::find(cands.begin(), cands.end(), c) == cands.end()) cands.push_back(std::move(c));
    }
  const std::vector<int> original = p->shape;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipError_t e = hipEventCreate(&ev0);
  if (e == hipSuccess) e = hipEventCreate(&ev1);
  if (e == hipSuccess) e = persistent_grid(p);
  float best = -1.0f;
  size_t best_c = 0;
  for (size_t c = 0; c < cands.size() && e == hipSuccess; ++c) {
    p->shape = cands[c];
    build_schedule(p, scratch);
    e = upload(p, workspace, s);
    if (e == hipSuccess) e = enqueue(p, workspace, s);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(ev0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = enqueue(p, workspace, s);
    if (e == hipSuccess) e = hipEventRecord(ev1, s);
    if (e == hipSuccess) e = hipEventSynchronize(ev1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
    if (e == hipSuccess && (best < 0.0f || ms < best)) {
      best = ms;
      best_c = c;
    }
  }
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  p->shape = (e == hipSuccess) ? cands[best_c] : original;
  build_schedule(p, nullptr);
  if (e != hipSuccess) return hip_error(e, "grouped autotune");
  *best_ms = best / (float)reps;
  return clear_error();
}

}  // extern "C"
