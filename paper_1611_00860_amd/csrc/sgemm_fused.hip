// Node fusion on the sgemm dataflow graph (HPVM report, Sec. 4.1 and 4.2).
//
// Sec. 4.1 defines the merge primitives and Sec. 4.2 applies them to fuse
// kernels: fewer launches, and better temporal locality when the fused
// nodes reuse data.  Two merges of the sgemm leaf are lowered here:
//
//  * MergeDependentNodes(sgemm leaf, consumer leaf): the consumer reads,
//    over a 1-1 edge, the element its producer instance wrote.  The merged
//    node replaces the edge by a register: each output element goes through
//    the consumer's function in the epilogue, so the sgemm result is never
//    written out and read back.
//
//  * MergeIndependentNodes on two sgemm leaves with the same dimensions
//    whose parents (SgemmInternal) share input A; the merge of their two
//    Allocation nodes (MergeAllocComputeGraphs) gives one LDS allocation
//    holding one A slab and both B slabs.  Each merged workgroup computes a
//    TM x TN tile of C1 and the same tile of C2 from a single staged A tile.
//
// Independent sgemms that share nothing merge into one launch through the
// grouped persistent kernel instead.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "device_common.hpp"
#include "hpvm_sgemm.h"
#include "internal.hpp"
#include "mfma_f32.hpp"
#include "mfma_f32_dma.hpp"

namespace hpvm {

// ---------------------------------------------------------------------------
// MergeDependentNodes: sgemm leaf + one-to-one consumer leaf.
// ---------------------------------------------------------------------------
struct ConsumerArgs {
  float* D;
  int64_t ldd;
  const float* bias;  // one value per column (BIAS ops)
  float lo, hi;       // CLAMP
  int32_t op;
};

// D <- consumer(alpha * acc + beta * C), element-wise, masked at the edges.
// C is read-only here (beta == 0 never reads it); D may be C itself.  As in
// store_c, each group of 4 rows loads its C values before its stores.
template <int OP, int BM, int BN>
__device__ __forceinline__ void store_consumed(const GemmArgs& p, const ConsumerArgs& c,
                                               const f32x16 (&acc)[BM][BN], int row0, int col0, int lane) {
  constexpr bool kBias = OP == HPVM_CONSUMER_BIAS || OP == HPVM_CONSUMER_BIAS_RELU;
  const bool read_c = p.beta != 0.0f;
#pragma unroll
  for (int bi = 0; bi < BM; ++bi)
#pragma unroll
    for (int bj = 0; bj < BN; ++bj) {
      const int j = col0 + 32 * bj + acc_col(lane);
      if (j >= p.n) continue;
      const float b = kBias ? c.bias[j] : 0.0f;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        float cin[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int i = row0 + 32 * bi + acc_row(4 * g + t, lane);
          cin[t] = (read_c && i < p.m) ? p.C[(int64_t)i * p.ldc + j] : 0.0f;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int i = row0 + 32 * bi + acc_row(4 * g + t, lane);
          if (i < p.m) {
            float v = p.alpha * acc[bi][bj][4 * g + t];
            if (read_c) v = fmaf(p.beta, cin[t], v);
            c.D[(int64_t)i * c.ldd + j] = consume<OP>(v, b, c.lo, c.hi);
          }
        }
      }
    }
}

template <int TM, int TN, int TK, int WM, int WN>
__global__ void __launch_bounds__((TM / WM) * (TN / WN) * kWave)
    sgemm_consumer_f32(GemmArgs p, ConsumerArgs c) {
  extern __shared__ __align__(16) float lds[];
  int tm, tn;
  tile_coords(p.tiles_m, p.tiles_n, blockIdx.x, tm, tn);
  f32x16 acc[WM / 32][WN / 32];
  f32_mainloop<TM, TN, TK, WM, WN, false, false>(p, tm * TM, tn * TN, lds, acc);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int row0 = tm * TM + (wave / (TN / WN)) * WM, col0 = tn * TN + (wave % (TN / WN)) * WN;
  constexpr int BM = WM / 32, BN = WN / 32;
  switch (c.op) {
    case HPVM_CONSUMER_RELU: store_consumed<HPVM_CONSUMER_RELU, BM, BN>(p, c, acc, row0, col0, lane); break;
    case HPVM_CONSUMER_BIAS: store_consumed<HPVM_CONSUMER_BIAS, BM, BN>(p, c, acc, row0, col0, lane); break;
    case HPVM_CONSUMER_BIAS_RELU:
      store_consumed<HPVM_CONSUMER_BIAS_RELU, BM, BN>(p, c, acc, row0, col0, lane);
      break;
    case HPVM_CONSUMER_CLAMP: store_consumed<HPVM_CONSUMER_CLAMP, BM, BN>(p, c, acc, row0, col0, lane); break;
    default: store_consumed<HPVM_CONSUMER_NONE, BM, BN>(p, c, acc, row0, col0, lane); break;
  }
}

// ---------------------------------------------------------------------------
// MergeIndependentNodes with a shared A: one A slab, two B slabs per stage.
// The B stage holds B1's TN columns followed by B2's TN columns; waves whose
// columns fall in the first half produce C1, the others C2.  Per wave the
// MFMA sequence is that of the single-output kernel with the same wave tile.
// ---------------------------------------------------------------------------
template <int TM, int TN, int TK, int WM, int WN>
struct PairTile {
  static constexpr int TN2 = 2 * TN;
  static constexpr int kWavesN = TN2 / WN;
  static constexpr int NT = (TM / WM) * kWavesN * kWave;
  static constexpr int BM = WM / 32, BN = WN / 32;
  using OpA = F32Operand<TM, TK, true>;
  using OpB = F32Operand<TN2, TK, false>;
  static constexpr int64_t kLdsBytes = 2 * (OpA::kFloats + OpB::kFloats) * (int64_t)sizeof(float);
  static_assert(TN % WN == 0, "a wave's columns must lie in one output");
  static_assert(TK % 8 == 0, "K slab must hold whole groups of 8");
};

template <int TM, int TN, int TK, int WM, int WN>
__device__ __forceinline__ bool pair_interior(const GemmArgs& p1, const GemmArgs& p2, int m0, int n0) {
  return p1.vec_a && p1.vec_b && p2.vec_b && m0 + TM <= p1.m && n0 + TN <= p1.n && p1.k > 0 && p1.k % TK == 0;
}

template <int TM, int TN, int TK, int WM, int WN, bool MASKED>
__device__ __forceinline__ void pair_mainloop_impl(const GemmArgs& p1, const GemmArgs& p2, int m0, int n0,
                                                   float* lds, f32x16 (&acc)[WM / 32][WN / 32]) {
  using T = PairTile<TM, TN, TK, WM, WN>;
  using OpA = typename T::OpA;
  using OpB = typename T::OpB;
  constexpr int NT = T::NT, BM = T::BM, BN = T::BN;
  float* As0 = lds;
  float* As1 = lds + OpA::kFloats;
  float* Bs0 = lds + 2 * OpA::kFloats;
  float* Bs1 = Bs0 + OpB::kFloats;

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid / kWave;
  const int wm0 = (wave / T::kWavesN) * WM, wn0 = (wave % T::kWavesN) * WN;

  GlobalTile<TM, TK, NT> ga;
  GlobalTile<TK, TN, NT> gb1, gb2;
  auto fetch = [&](int k0) {
    const float* base;
    int rl, cl;
    slab_a<false>(p1, m0, k0, base, rl, cl);
    ga.template load<MASKED>(base, p1.lda, rl, cl, p1.vec_a, tid);
    slab_b<false>(p1, n0, k0, base, rl, cl);
    gb1.template load<MASKED>(base, p1.ldb, rl, cl, p1.vec_b, tid);
    slab_b<false>(p2, n0, k0, base, rl, cl);
    gb2.template load<MASKED>(base, p2.ldb, rl, cl, p2.vec_b, tid);
  };
  auto stage = [&](float* As, float* Bs) {
    ga.template store_f32<OpA::kStride>(As, tid);
    gb1.template store_f32<OpB::kStride>(Bs, tid);
    gb2.template store_f32<OpB::kStride>(Bs + TN, tid);
  };

  zero_acc(acc);
  const int slabs = (p1.k + TK - 1) / TK;
  fetch(0);
  stage(As0, Bs0);
  __syncthreads();

  for (int s = 0; s < slabs; ++s) {
    const float* As = (s & 1) ? As1 : As0;
    const float* Bs = (s & 1) ? Bs1 : Bs0;
    const bool more = s + 1 < slabs;
    if (more) fetch((s + 1) * TK);
#pragma unroll
    for (int kg = 0; kg < TK / 8; ++kg) {
      f32x4 a[BM], b[BN];
#pragma unroll
      for (int bi = 0; bi < BM; ++bi) a[bi] = OpA::frag(As, wm0 + 32 * bi, kg, lane);
#pragma unroll
      for (int bj = 0; bj < BN; ++bj) b[bj] = OpB::frag(Bs, wn0 + 32 * bj, kg, lane);
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int bi = 0; bi < BM; ++bi)
#pragma unroll
          for (int bj = 0; bj < BN; ++bj)
            acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[bi][t], b[bj][t], acc[bi][bj], 0, 0, 0);
    }
    if (more) stage((s & 1) ? As0 : As1, (s & 1) ? Bs0 : Bs1);
    __syncthreads();
  }
}

template <int TM, int TN, int TK, int WM, int WN>
__global__ void __launch_bounds__((TM / WM) * (2 * TN / WN) * kWave)
    sgemm_pair_f32(GemmArgs p1, GemmArgs p2) {
  using T = PairTile<TM, TN, TK, WM, WN>;
  extern __shared__ __align__(16) float lds[];
  int tm, tn;
  tile_coords(p1.tiles_m, p1.tiles_n, blockIdx.x, tm, tn);
  const int m0 = tm * TM, n0 = tn * TN;
  f32x16 acc[T::BM][T::BN];
  if (pair_interior<TM, TN, TK, WM, WN>(p1, p2, m0, n0))
    pair_mainloop_impl<TM, TN, TK, WM, WN, false>(p1, p2, m0, n0, lds, acc);
  else
    pair_mainloop_impl<TM, TN, TK, WM, WN, true>(p1, p2, m0, n0, lds, acc);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int row0 = m0 + (wave / T::kWavesN) * WM;
  const int col = (wave % T::kWavesN) * WN;
  if (col < TN)
    store_c<T::BM, T::BN>(p1, acc, row0, n0 + col, lane);
  else
    store_c<T::BM, T::BN>(p2, acc, row0, n0 + col - TN, lane);
}

// ---------------------------------------------------------------------------
// Menus and launches.
// ---------------------------------------------------------------------------
template <typename Kernel>
static hipError_t allow_lds_fused(Kernel* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

struct FusedEntry {
  hpvm_tile tile;
  int32_t threads;
  int64_t lds_bytes;
  hipError_t (*consumer)(const GemmArgs&, const ConsumerArgs&, hipStream_t) = nullptr;
  hipError_t (*pair)(const GemmArgs&, const GemmArgs&, hipStream_t) = nullptr;
  // Pair with the contraction split into slices (DMA-fed pair tiles): the
  // workspace bytes that let an m x n x k pair run split (0 when the entry
  // would not split it), and that launch.
  int64_t (*pair_split_bytes)(int64_t m, int64_t n, int64_t k) = nullptr;
  hipError_t (*pair_split)(const GemmArgs&, const GemmArgs&, void* workspace, hipStream_t) = nullptr;
};

template <int TM, int TN, int TK, int WM, int WN>
struct ConsumerConfig {
  static constexpr int kThreads = (TM / WM) * (TN / WN) * kWave;
  static constexpr int64_t kLds = F32Tile<TM, TN, TK, WM, WN, false, false>::kLdsBytes;
  static hipError_t launch(const GemmArgs& args, const ConsumerArgs& c, hipStream_t s) {
    GemmArgs a = args;
    ConsumerArgs cc = c;
    a.tiles_m = (a.m + TM - 1) / TM;
    a.tiles_n = (a.n + TN - 1) / TN;
    void* kargs[] = {&a, &cc};
    auto fn = &sgemm_consumer_f32<TM, TN, TK, WM, WN>;
    hipError_t e = allow_lds_fused(fn, (size_t)kLds);
    if (e != hipSuccess) return e;
    return hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3((unsigned)(a.tiles_m * a.tiles_n)),
                           dim3(kThreads), kargs, (size_t)kLds, s);
  }
};

template <int TM, int TN, int TK, int WM, int WN>
struct PairConfig {
  using T = PairTile<TM, TN, TK, WM, WN>;
  static constexpr int kThreads = T::NT;
  static constexpr int64_t kLds = T::kLdsBytes;
  static hipError_t launch(const GemmArgs& a1, const GemmArgs& a2, hipStream_t s) {
    GemmArgs p1 = a1, p2 = a2;
    p1.tiles_m = p2.tiles_m = (p1.m + TM - 1) / TM;
    p1.tiles_n = p2.tiles_n = (p1.n + TN - 1) / TN;
    void* kargs[] = {&p1, &p2};
    auto fn = &sgemm_pair_f32<TM, TN, TK, WM, WN>;
    hipError_t e = allow_lds_fused(fn, (size_t)kLds);
    if (e != hipSuccess) return e;
    return hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3((unsigned)(p1.tiles_m * p1.tiles_n)),
                           dim3(kThreads), kargs, (size_t)kLds, s);
  }
};

// Aligned problems of at least one tile each way (edge tiles moved inward)
// of the consumer on the DMA-fed loop (the consumer applied in its
// epilogue); any other problem on the 128 x 128 x 16 tile.
template <int TM, int TN, int TK, int WM, int NST>
struct ConsumerDmaConfig {
  using S = F32DmaShape<TM, TN, TK, WM, 128, false, false, NST>;
  static constexpr int kThreads = S::NW * kWave;
  template <int OP>
  static hipError_t run(const GemmArgs& a, const F32DmaOut& o, hipStream_t s) {
    auto* fn = f32_dma_fits<TM, TN, TK>(a, o.D, o.ldd, 1)
                   ? &sgemm_f32_dma<TM, TN, TK, WM, 128, false, false, NST, kDmaConsume, OP>
                   : &sgemm_f32_dma<TM, TN, TK, WM, 128, false, false, NST, kDmaConsume, OP, false, true>;
    hipError_t e = allow_lds_fused(fn, (size_t)S::kLdsBytes);
    if (e != hipSuccess) return e;
    GemmArgs a1 = a, a2 = a;
    F32DmaOut oo = o;
    void* kargs[] = {&a1, &a2, &oo};
    return hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3((unsigned)(a.tiles_m * a.tiles_n)),
                           dim3(kThreads), kargs, (size_t)S::kLdsBytes, s);
  }
  static hipError_t launch(const GemmArgs& args, const ConsumerArgs& c, hipStream_t s) {
    const bool c_ok = args.beta == 0.0f || (args.ldc % 4 == 0 && (reinterpret_cast<uintptr_t>(args.C) & 15) == 0);
    if (!c_ok || !f32_dma_fits_edges<TM, TN, TK>(args, c.D, c.ldd))
      return ConsumerConfig<128, 128, 16, 64, 64>::launch(args, c, s);
    GemmArgs a = args;
    a.tiles_m = (a.m + TM - 1) / TM;
    a.tiles_n = (a.n + TN - 1) / TN;
    F32DmaOut o{};
    o.splits = 1;
    o.D = c.D;
    o.ldd = c.ldd;
    o.bias = c.bias;
    o.lo = c.lo;
    o.hi = c.hi;
    switch (c.op) {
      case HPVM_CONSUMER_RELU: return run<HPVM_CONSUMER_RELU>(a, o, s);
      case HPVM_CONSUMER_BIAS: return run<HPVM_CONSUMER_BIAS>(a, o, s);
      case HPVM_CONSUMER_BIAS_RELU: return run<HPVM_CONSUMER_BIAS_RELU>(a, o, s);
      case HPVM_CONSUMER_CLAMP: return run<HPVM_CONSUMER_CLAMP>(a, o, s);
      default: return run<HPVM_CONSUMER_NONE>(a, o, s);
    }
  }
};

// Aligned problems of at least one tile each way (edge tiles moved inward)
// of the pair on the DMA-fed loop: per stage one A slab and both B slabs
// (B1's tile, then B2's); any other problem on the 128 x 128 x 16 pair tile.
template <int TM, int TN, int TK, int WM, int NST>
struct PairDmaConfig {
  using S = F32DmaShape<TM, TN, TK, WM, 128, false, false, NST, true>;
  static constexpr int kThreads = S::NW * kWave;
  static hipError_t launch(const GemmArgs& a1, const GemmArgs& a2, hipStream_t s) {
    const bool ok = f32_dma_fits_edges<TM, TN, TK>(a1, a1.C, a1.ldc) && a2.vec_b && a2.ldc % 4 == 0 &&
                    (reinterpret_cast<uintptr_t>(a2.C) & 15) == 0;
    if (!ok) return PairConfig<128, 128, 16, 64, 64>::launch(a1, a2, s);
    GemmArgs p1 = a1, p2 = a2;
    p1.tiles_m = p2.tiles_m = (p1.m + TM - 1) / TM;
    p1.tiles_n = p2.tiles_n = (p1.n + TN - 1) / TN;
    F32DmaOut o{};
    o.splits = 1;
    void* kargs[] = {&p1, &p2, &o};
    auto* fn = f32_dma_fits<TM, TN, TK>(a1, a1.C, a1.ldc, 1)
                   ? &sgemm_f32_dma<TM, TN, TK, WM, 128, false, false, NST, kDmaUpdate, 0, true>
                   : &sgemm_f32_dma<TM, TN, TK, WM, 128, false, false, NST, kDmaUpdate, 0, true, true>;
    hipError_t e = allow_lds_fused(fn, (size_t)S::kLdsBytes);
    if (e != hipSuccess) return e;
    return hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3((unsigned)(p1.tiles_m * p1.tiles_n)),
                           dim3(kThreads), kargs, (size_t)S::kLdsBytes, s);
  }
  // Split contraction (the rule of the single launch's split): each
  // workgroup computes one tile of both outputs over one slice, writing raw
  // partial sums [slice][m][n] of output 1 and then of output 2 to the
  // workspace; then each output is formed from its slices, in order.
  static int splits(int64_t m, int64_t n, int64_t k) {
    if (m <= 0 || n <= 0 || k <= 0 || m % TM || n % TN || k % TK) return 1;
    return dma_split_count((m / TM) * (n / TN), k, TK);
  }
  static int64_t split_bytes(int64_t m, int64_t n, int64_t k) {
    const int sp = splits(m, n, k);
    return sp > 1 ? 2 * (int64_t)sp * m * n * (int64_t)sizeof(float) : 0;
  }
  static hipError_t launch_split(const GemmArgs& a1, const GemmArgs& a2, void* workspace, hipStream_t s) {
    const int sp = splits(a1.m, a1.n, a1.k);
    float* part1 = static_cast<float*>(workspace);
    float* part2 = part1 + (int64_t)sp * a1.m * a1.n;
    GemmArgs b2 = a2;
    b2.vec_a = a1.vec_a;
    if (sp <= 1 || !f32_dma_fits<TM, TN, TK>(a1, part1, a1.n, sp) || !f32_dma_fits<TM, TN, TK>(a1, a1.C, a1.ldc, sp) ||
        !f32_dma_fits<TM, TN, TK>(b2, a2.C, a2.ldc, sp))
      return launch(a1, a2, s);
    GemmArgs p1 = a1, p2 = a2;
    p1.C = part1;
    p2.C = part2;
    p1.ldc = p2.ldc = a1.n;
    p1.beta = p2.beta = 0.0f;
    p1.tiles_m = p2.tiles_m = a1.m / TM;
    p1.tiles_n = p2.tiles_n = a1.n / TN;
    F32DmaOut o{};
    o.splits = sp;
    void* kargs[] = {&p1, &p2, &o};
    auto* fn = &sgemm_f32_dma<TM, TN, TK, WM, 128, false, false, NST, kDmaSplit, 0, true>;
    hipError_t e = allow_lds_fused(fn, (size_t)S::kLdsBytes);
    if (e != hipSuccess) return e;
    e = hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3((unsigned)(p1.tiles_m * p1.tiles_n * sp)),
                        dim3(kThreads), kargs, (size_t)S::kLdsBytes, s);
    if (e == hipSuccess) e = launch_split_finish(part1, sp, a1.m, a1.n, a1.alpha, a1.beta, a1.C, a1.ldc, s);
    if (e == hipSuccess) e = launch_split_finish(part2, sp, a2.m, a2.n, a2.alpha, a2.beta, a2.C, a2.ldc, s);
    return e;
  }
};

#define HPVM_CONSUMER_DMA_ENTRY(TM, TN, TK, WM, NST)                                                 \
  {{TM, TN, TK, WM, 128, NST}, ConsumerDmaConfig<TM, TN, TK, WM, NST>::kThreads,                       \
   ConsumerDmaConfig<TM, TN, TK, WM, NST>::S::kLdsBytes, &ConsumerDmaConfig<TM, TN, TK, WM, NST>::launch, nullptr}
#define HPVM_PAIR_DMA_ENTRY(TM, TN, TK, WM, NST)                                                     \
  {{TM, TN, TK, WM, 128, NST}, PairDmaConfig<TM, TN, TK, WM, NST>::kThreads,                           \
   PairDmaConfig<TM, TN, TK, WM, NST>::S::kLdsBytes, nullptr, &PairDmaConfig<TM, TN, TK, WM, NST>::launch, \
   &PairDmaConfig<TM, TN, TK, WM, NST>::split_bytes, &PairDmaConfig<TM, TN, TK, WM, NST>::launch_split}
#define HPVM_CONSUMER_ENTRY(TM, TN, TK, WM, WN)                                                   \
  {{TM, TN, TK, WM, WN, 2}, ConsumerConfig<TM, TN, TK, WM, WN>::kThreads,                           \
   ConsumerConfig<TM, TN, TK, WM, WN>::kLds, &ConsumerConfig<TM, TN, TK, WM, WN>::launch, nullptr}
#define HPVM_PAIR_ENTRY(TM, TN, TK, WM, WN)                                                       \
  {{TM, TN, TK, WM, WN, 2}, PairConfig<TM, TN, TK, WM, WN>::kThreads, PairConfig<TM, TN, TK, WM, WN>::kLds, \
   nullptr, &PairConfig<TM, TN, TK, WM, WN>::launch}

// The consumer kernel takes the tiles of the FP32 single-launch menu, in its
// order, so the autotuner's choice for a shape carries over.
static const FusedEntry kConsumerMenu[] = {
    HPVM_CONSUMER_DMA_ENTRY(256, 256, 32, 64, 2),
    HPVM_CONSUMER_ENTRY(128, 128, 16, 64, 64), HPVM_CONSUMER_ENTRY(256, 128, 16, 128, 64),
    HPVM_CONSUMER_ENTRY(128, 128, 32, 64, 64), HPVM_CONSUMER_ENTRY(64, 64, 16, 32, 32),
    HPVM_CONSUMER_ENTRY(128, 64, 16, 64, 32), HPVM_CONSUMER_ENTRY(64, 128, 16, 32, 64),
    HPVM_CONSUMER_DMA_ENTRY(256, 256, 16, 64, 4),
    HPVM_CONSUMER_DMA_ENTRY(128, 256, 32, 32, 2),
    HPVM_CONSUMER_DMA_ENTRY(128, 128, 32, 32, 2),
};
// Pair tiles: tile_m x tile_n of each output; 8, 8, 4 and 8 waves.  The
// first DMA-fed entry's two stages of one A slab and two B slabs take all
// 160 KB of LDS; the last (96 KB) is the one that splits the contraction of
// pairs whose tiles would not cover the CUs.
static const FusedEntry kPairMenu[] = {
    HPVM_PAIR_DMA_ENTRY(128, 256, 32, 64, 2),
    HPVM_PAIR_ENTRY(128, 128, 16, 64, 64),
    HPVM_PAIR_ENTRY(64, 64, 16, 32, 64),
    HPVM_PAIR_DMA_ENTRY(128, 128, 32, 32, 2),
};
constexpr int kNumConsumer = (int)(sizeof(kConsumerMenu) / sizeof(kConsumerMenu[0]));
constexpr int kNumPair = (int)(sizeof(kPairMenu) / sizeof(kPairMenu[0]));

const FusedEntry* find_fused(const FusedEntry* menu, int count, const hpvm_tile& t) {
  for (int i = 0; i < count; ++i)
    if (same_tile(menu[i].tile, t)) return &menu[i];
  return nullptr;
}

bool ranges_meet(const float* a, int64_t ra, int64_t ca, int64_t lda, const float* b, int64_t rb, int64_t cb,
                 int64_t ldb) {
  if (!a || !b || ra == 0 || ca == 0 || rb == 0 || cb == 0) return false;
  uintptr_t a0, a1, b0, b1;
  matrix_extent(a, ra, ca, lda, &a0, &a1);
  matrix_extent(b, rb, cb, ldb, &b0, &b1);
  return a0 < b1 && b0 < a1;
}

}  // namespace hpvm

using namespace hpvm;

extern "C" {

int hpvm_fusion_menu(int32_t which, hpvm_tile* out, int32_t capacity, int32_t* count) {
  if (which != HPVM_FUSION_CONSUMER && which != HPVM_FUSION_PAIR)
    return set_error(HPVM_INVALID_ARG, "argument 1: unknown fusion %d", which);
  if (capacity < 0 || (capacity > 0 && !out))
    return set_error(HPVM_INVALID_ARG, "argument 3: bad capacity or NULL output");
  if (!count) return set_error(HPVM_INVALID_ARG, "argument 4: count is NULL");
  const FusedEntry* menu = which == HPVM_FUSION_CONSUMER ? kConsumerMenu : kPairMenu;
  const int n = which == HPVM_FUSION_CONSUMER ? kNumConsumer : kNumPair;
  for (int i = 0; i < n && i < capacity; ++i) out[i] = menu[i].tile;
  *count = n;
  return clear_error();
}

int hpvm_sgemm_consumer(int64_t m, int64_t n, int64_t k, float alpha, const float* A, int64_t lda, const float* B,
                        int64_t ldb, float beta, const float* C, int64_t ldc, const hpvm_consumer* consumer,
                        float* D, int64_t ldd, const hpvm_tile* tile, void* stream) {
  if (m < 0) return set_error(HPVM_INVALID_ARG, "argument 1: m = %lld < 0", (long long)m);
  if (n < 0) return set_error(HPVM_INVALID_ARG, "argument 2: n = %lld < 0", (long long)n);
  if (k < 0) return set_error(HPVM_INVALID_ARG, "argument 3: k = %lld < 0", (long long)k);
  if (m > INT32_MAX || n > INT32_MAX || k > INT32_MAX)
    return set_error(HPVM_UNSUPPORTED, "sizes above 2^31 - 1 are not supported");
  const bool empty = m == 0 || n == 0;
  const bool reads_ab = !empty && k > 0 && alpha != 0.0f;
  const bool reads_c = !empty && beta != 0.0f;
  if (reads_ab && !A) return set_error(HPVM_INVALID_ARG, "argument 5: A is NULL");
  if (lda < std::max<int64_t>(k, 1)) return set_error(HPVM_INVALID_ARG, "argument 6: lda = %lld < max(1, k)", (long long)lda);
  if (reads_ab && !B) return set_error(HPVM_INVALID_ARG, "argument 7: B is NULL");
  if (ldb < std::max<int64_t>(n, 1)) return set_error(HPVM_INVALID_ARG, "argument 8: ldb = %lld < max(1, n)", (long long)ldb);
  if (reads_c && !C) return set_error(HPVM_INVALID_ARG, "argument 10: C is NULL (beta != 0)");
  if (ldc < std::max<int64_t>(n, 1)) return set_error(HPVM_INVALID_ARG, "argument 11: ldc = %lld < max(1, n)", (long long)ldc);
  if (!consumer) return set_error(HPVM_INVALID_ARG, "argument 12: consumer is NULL");
  const int op = consumer->op;
  if (op < HPVM_CONSUMER_NONE || op > HPVM_CONSUMER_CLAMP)
    return set_error(HPVM_INVALID_ARG, "argument 12: unknown consumer op %d", op);
  const bool uses_bias = op == HPVM_CONSUMER_BIAS || op == HPVM_CONSUMER_BIAS_RELU;
  if (!empty && uses_bias && !consumer->bias) return set_error(HPVM_INVALID_ARG, "argument 12: bias is NULL");
  if (op == HPVM_CONSUMER_CLAMP && !(consumer->lo <= consumer->hi))
    return set_error(HPVM_INVALID_ARG, "argument 12: clamp needs lo <= hi");
  if (!empty && !D) return set_error(HPVM_INVALID_ARG, "argument 13: D is NULL");
  if (ldd < std::max<int64_t>(n, 1)) return set_error(HPVM_INVALID_ARG, "argument 14: ldd = %lld < max(1, n)", (long long)ldd);
  if (reads_ab && (ranges_meet(D, m, n, ldd, A, m, k, lda) || ranges_meet(D, m, n, ldd, B, k, n, ldb)))
    return set_error(HPVM_INVALID_ARG, "argument 13: D overlaps A or B");
  if (reads_c && !(D == C && ldd == ldc) && ranges_meet(D, m, n, ldd, C, m, n, ldc))
    return set_error(HPVM_INVALID_ARG, "argument 13: D overlaps C without being C itself");
  if (uses_bias && ranges_meet(D, m, n, ldd, consumer->bias, 1, n, n))
    return set_error(HPVM_INVALID_ARG, "argument 13: D overlaps the bias vector");
  hpvm_tile t = kConsumerMenu[0].tile;
  if (tile) {
    t = *tile;
  } else {
    hpvm_tile tuned;
    if (tuned_tile(HPVM_PREC_FP32, m, n, k, false, &tuned) && find_fused(kConsumerMenu, kNumConsumer, tuned))
      t = tuned;
    else if (default_small_tile(HPVM_PREC_FP32, m, n, &tuned))
      t = tuned;  // the single launch's choice for problems entry 0 leaves CUs idle on
  }
  const FusedEntry* e = find_fused(kConsumerMenu, kNumConsumer, t);
  if (!e)
    return set_error(HPVM_UNSUPPORTED, "argument 15: tile %dx%dx%d leaf %dx%d is not in the consumer menu",
                     t.tile_m, t.tile_n, t.tile_k, t.leaf_m, t.leaf_n);
  if (empty) return clear_error();
  if (fault_injected("launch")) return set_error(HPVM_HIP_ERROR, "injected launch failure (HPVM_FAULT_INJECT)");
  GemmArgs g{};
  g.A = A;
  g.B = B;
  g.C = const_cast<float*>(C);  // read only: the consumer store writes D
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.m = (int32_t)m;
  g.n = (int32_t)n;
  g.k = reads_ab ? (int32_t)k : 0;  // k == 0 or alpha == 0: A and B are not read
  g.alpha = alpha;
  g.beta = beta;
  g.vec_a = vec16(A, lda);
  g.vec_b = vec16(B, ldb);
  ConsumerArgs c{};
  c.D = D;
  c.ldd = ldd;
  c.bias = consumer->bias;
  c.lo = consumer->lo;
  c.hi = consumer->hi;
  c.op = op;
  const hipError_t he = e->consumer(g, c, reinterpret_cast<hipStream_t>(stream));
  return he == hipSuccess ? clear_error() : hip_error(he, "consumer launch");
}

}  // extern "C"

namespace {

// The pair tile that splits the contraction when a pair's tiles would not
// cover the CUs.
const FusedEntry* pair_split_entry() { return find_fused(kPairMenu, kNumPair, hpvm_tile{128, 128, 32, 32, 128, 2}); }

// Built-in choice: the largest tile per output that still gives a tile per
// CU of a 256-CU part -- the DMA-fed 128 x 256, else (with a workspace
// argument that holds its partial sums; -1 = as much as needed) the
// DMA-fed 128 x 128 in contraction slices, else 128 x 128, else 64 x 64.
hpvm_tile pair_choice(int64_t m, int64_t n, int64_t k, bool ws_ok, int64_t ws_bytes) {
  auto tiles = [&](const hpvm_tile& u) { return ((m + u.tile_m - 1) / u.tile_m) * ((n + u.tile_n - 1) / u.tile_n); };
  if (tiles(kPairMenu[0].tile) >= 256) return kPairMenu[0].tile;
  const FusedEntry* sp = pair_split_entry();
  if (ws_ok && sp) {
    const int64_t need = sp->pair_split_bytes(m, n, k);
    if (need > 0 && (ws_bytes < 0 || ws_bytes >= need)) return sp->tile;
  }
  return tiles(kPairMenu[1].tile) >= 256 ? kPairMenu[1].tile : kPairMenu[2].tile;
}

int pair_impl(int64_t m, int64_t n, int64_t k, const float* A, int64_t lda, float alpha1, const float* B1,
              int64_t ldb1, float beta1, float* C1, int64_t ldc1, float alpha2, const float* B2, int64_t ldb2,
              float beta2, float* C2, int64_t ldc2, const hpvm_tile* tile, bool ws_ok, void* workspace,
              int64_t workspace_bytes, void* stream) {
  bool r1, r2;
  int rc = check_gemm_args("output 1: ", m, n, k, alpha1, A, lda, B1, ldb1, beta1, C1, ldc1, &r1);
  if (rc != HPVM_OK) return rc;
  rc = check_gemm_args("output 2: ", m, n, k, alpha2, A, lda, B2, ldb2, beta2, C2, ldc2, &r2);
  if (rc != HPVM_OK) return rc;
  const bool empty = m == 0 || n == 0;
  if (!empty && ranges_meet(C1, m, n, ldc1, C2, m, n, ldc2))
    return set_error(HPVM_INVALID_ARG, "arguments 10 and 16: C1 and C2 overlap");
  if (r2 && ranges_meet(C1, m, n, ldc1, B2, k, n, ldb2))
    return set_error(HPVM_INVALID_ARG, "argument 10: C1 overlaps B2");
  if (r1 && ranges_meet(C2, m, n, ldc2, B1, k, n, ldb1))
    return set_error(HPVM_INVALID_ARG, "argument 16: C2 overlaps B1");
  const hpvm_tile t = tile ? *tile : pair_choice(m, n, k, ws_ok, workspace ? workspace_bytes : 0);
  const FusedEntry* e = find_fused(kPairMenu, kNumPair, t);
  if (!e)
    return set_error(HPVM_UNSUPPORTED, "argument 18: tile %dx%dx%d leaf %dx%d is not in the pair menu", t.tile_m,
                     t.tile_n, t.tile_k, t.leaf_m, t.leaf_n);
  if (ws_ok && workspace && (uintptr_t)workspace % 16)
    return set_error(HPVM_INVALID_ARG, "argument 19: workspace is not 16-byte aligned");
  if (empty) return clear_error();
  if (!r1 || !r2) {
    // A scale-only output (k == 0 or alpha == 0) reads neither A nor its B:
    // nothing is shared, so each output goes through the single launch.
    rc = hpvm_sgemm(m, n, k, alpha1, A, lda, B1, ldb1, beta1, C1, ldc1, HPVM_PREC_FP32, nullptr, stream);
    if (rc != HPVM_OK) return rc;
    return hpvm_sgemm(m, n, k, alpha2, A, lda, B2, ldb2, beta2, C2, ldc2, HPVM_PREC_FP32, nullptr, stream);
  }
  if (fault_injected("launch")) return set_error(HPVM_HIP_ERROR, "injected launch failure (HPVM_FAULT_INJECT)");
  GemmArgs g1{}, g2{};
  g1.A = g2.A = A;
  g1.lda = g2.lda = lda;
  g1.m = g2.m = (int32_t)m;
  g1.n = g2.n = (int32_t)n;
  g1.k = g2.k = (int32_t)k;
  g1.vec_a = g2.vec_a = vec16(A, lda);
  g1.B = B1;
  g1.ldb = ldb1;
  g1.C = C1;
  g1.ldc = ldc1;
  g1.alpha = alpha1;
  g1.beta = beta1;
  g1.vec_b = vec16(B1, ldb1);
  g2.B = B2;
  g2.ldb = ldb2;
  g2.C = C2;
  g2.ldc = ldc2;
  g2.alpha = alpha2;
  g2.beta = beta2;
  g2.vec_b = vec16(B2, ldb2);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t need = e->pair_split_bytes ? e->pair_split_bytes(m, n, k) : 0;
  const hipError_t he = (ws_ok && need > 0 && workspace && workspace_bytes >= need)
                            ? e->pair_split(g1, g2, workspace, s)
                            : e->pair(g1, g2, s);
  return he == hipSuccess ? clear_error() : hip_error(he, "pair launch");
}

}  // namespace

extern "C" {

int hpvm_sgemm_pair(int64_t m, int64_t n, int64_t k, const float* A, int64_t lda, float alpha1, const float* B1,
                    int64_t ldb1, float beta1, float* C1, int64_t ldc1, float alpha2, const float* B2, int64_t ldb2,
                    float beta2, float* C2, int64_t ldc2, const hpvm_tile* tile, void* stream) {
  return pair_impl(m, n, k, A, lda, alpha1, B1, ldb1, beta1, C1, ldc1, alpha2, B2, ldb2, beta2, C2, ldc2, tile,
                   false, nullptr, 0, stream);
}

int hpvm_sgemm_pair_ws(int64_t m, int64_t n, int64_t k, const float* A, int64_t lda, float alpha1, const float* B1,
                       int64_t ldb1, float beta1, float* C1, int64_t ldc1, float alpha2, const float* B2,
                       int64_t ldb2, float beta2, float* C2, int64_t ldc2, const hpvm_tile* tile, void* workspace,
                       int64_t workspace_bytes, void* stream) {
  if (workspace_bytes < 0)
    return set_error(HPVM_INVALID_ARG, "argument 20: workspace_bytes = %lld < 0", (long long)workspace_bytes);
  return pair_impl(m, n, k, A, lda, alpha1, B1, ldb1, beta1, C1, ldc1, alpha2, B2, ldb2, beta2, C2, ldc2, tile,
                   true, workspace, workspace_bytes, stream);
}

int hpvm_sgemm_pair_workspace_bytes(int64_t m, int64_t n, int64_t k, const hpvm_tile* tile, int64_t* bytes) {
  if (m < 0 || n < 0 || k < 0) return set_error(HPVM_INVALID_ARG, "sizes must be >= 0");
  if (!bytes) return set_error(HPVM_INVALID_ARG, "argument 5: bytes is NULL");
  const hpvm_tile t = tile ? *tile : pair_choice(m, n, k, true, -1);
  const FusedEntry* e = find_fused(kPairMenu, kNumPair, t);
  if (!e)
    return set_error(HPVM_UNSUPPORTED, "argument 4: tile %dx%dx%d leaf %dx%d is not in the pair menu", t.tile_m,
                     t.tile_n, t.tile_k, t.leaf_m, t.leaf_n);
  *bytes = e->pair_split_bytes ? e->pair_split_bytes(m, n, k) : 0;
  return clear_error();
}

}  // extern "C"
