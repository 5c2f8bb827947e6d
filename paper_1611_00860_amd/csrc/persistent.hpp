// Pieces shared by the two persistent lowerings of the sgemm graph: grouped
// batches (many graphs, one launch) and the streaming graph (argument packs
// pushed while the kernel runs).
//
// Both keep a fixed set of resident workgroups that pull SgemmInternal
// instances (tiles) from a device-side counter -- the persistent-node form
// of Sec. 3.5 -- and both let every sgemm carry its own tile shape, chosen
// from a menu whose shapes share one workgroup size and one LDS size so a
// single kernel can run any of them.
#pragma once

#include <cmath>
#include <cstdint>

#include "device_common.hpp"
#include "host_common.hpp"
#include "hpvm_sgemm.h"
#include "mfma_f32.hpp"
#include "mfma_f32_dma.hpp"

namespace hpvm {

struct GroupedShape {
  hpvm_tile tile;
  double cost_per_flop;  // relative cost of a useful flop, for the cost model
};

// The shapes a persistent kernel can run: all use 256 lanes (4 waves).
// Relative costs per useful flop, from the grouped autotuner's timings of
// batches of 512 sgemms with log-uniform sizes: the 128 x 128 tiles,
// DMA-fed for most instances, run well ahead of the register-staged smaller
// ones (factors of 1.12 and 1.35 gave 9626 tiles and 1.32 ms where the tuned
// assignments, these factors or their squares, gave 8762 or 8398 tiles and
// 1.20-1.22 ms).
static const GroupedShape kGroupedShapes[] = {
    {{128, 128, 16, 64, 64, 2}, 1.00},
    {{128, 64, 16, 64, 32, 2}, 1.25},
    {{64, 128, 16, 32, 64, 2}, 1.25},
    {{64, 64, 16, 32, 32, 2}, 1.82},
};
constexpr int kNumGroupedShapes = 4;
constexpr int kGroupedThreads = 256;
constexpr int64_t kGroupedLds = F32Tile<128, 128, 16, 64, 64, false, false>::kLdsBytes;
static_assert(F32Tile<128, 64, 16, 64, 32, false, false>::kLdsBytes <= kGroupedLds, "LDS");
static_assert(F32Tile<64, 128, 16, 32, 64, false, false>::kLdsBytes <= kGroupedLds, "LDS");
static_assert(F32Tile<64, 64, 16, 32, 32, false, false>::kLdsBytes <= kGroupedLds, "LDS");

template <int TM, int TN, int TK, int WM, int WN>
__device__ __forceinline__ void grouped_tile(const GemmArgs& p, int tm, int tn, float* lds) {
  static_assert(F32Tile<TM, TN, TK, WM, WN, false, false>::NT == kGroupedThreads, "256 lanes");
  f32x16 acc[WM / 32][WN / 32];
  f32_mainloop<TM, TN, TK, WM, WN, false, false>(p, tm * TM, tn * TN, lds, acc);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  store_c<WM / 32, WN / 32>(p, acc, tm * TM + (wave / (TN / WN)) * WM,
                            tn * TN + (wave % (TN / WN)) * WN, lane);
}

// 128 x 128 tiles of instances at least 128 x 128 with k a multiple of 16,
// n a multiple of 4 and rows 16-byte aligned take the DMA-fed loop (edge
// tiles moved inward, mfma_f32_dma.hpp): four waves of 32 x 128, 16-deep
// slabs in two 16 KB stages.
using GroupedDma = F32DmaShape<128, 128, 16, 32, 128, false, false, 2>;
static_assert(GroupedDma::NW * kWave == kGroupedThreads && GroupedDma::kLdsBytes <= kGroupedLds, "DMA tile fits");

__device__ __forceinline__ bool grouped_dma_ok(const GemmArgs& p) {
  return p.vec_a && p.vec_b && p.k > 0 && p.k % 16 == 0 && p.m >= 128 && p.n >= 128 && p.n % 4 == 0 &&
         p.ldc % 4 == 0 && (reinterpret_cast<uintptr_t>(p.C) & 15) == 0;
}

// Runs tile `local` (row-major over the instance's tile grid) of one sgemm
// with menu shape `shape`.  Uniform across the workgroup.
__device__ __forceinline__ void run_shape_tile(int shape, const GemmArgs& p, int tiles_n, int local,
                                               float* lds) {
  const int tm = local / tiles_n, tn = local - (local / tiles_n) * tiles_n;
  switch (shape) {
    case 0:
      if (grouped_dma_ok(p)) {
        F32DmaOut o{};
        o.splits = 1;
        f32_dma_tile<128, 128, 16, 32, 128, false, false, 2, kDmaUpdate, 0, false, true>(
            p, p, o, tm, tn, 0, reinterpret_cast<char*>(lds));
      } else {
        grouped_tile<128, 128, 16, 64, 64>(p, tm, tn, lds);
      }
      break;
    case 1: grouped_tile<128, 64, 16, 64, 32>(p, tm, tn, lds); break;
    case 2: grouped_tile<64, 128, 16, 32, 64>(p, tm, tn, lds); break;
    default: grouped_tile<64, 64, 16, 32, 32>(p, tm, tn, lds); break;
  }
}

// Host side ---------------------------------------------------------------

inline int64_t shape_tiles(int64_t m, int64_t n, int shape) {
  if (m == 0 || n == 0) return 0;
  const hpvm_tile& t = kGroupedShapes[shape].tile;
  return ((m + t.tile_m - 1) / t.tile_m) * ((n + t.tile_n - 1) / t.tile_n);
}

// Cost model: padded flops of the tiles an instance needs (each tile k + 32
// deep, for its epilogue), weighted by the shape's relative cost per flop
// raised to `lambda`, plus `overhead` steps of k of a 128 x 128 tile per tile
// whatever its shape (the latency of a tile's start and end, which favours
// fewer, larger tiles for shallow instances).
inline int cost_model_shape(int64_t m, int64_t n, int64_t k, double lambda, double overhead = 0.0) {
  int best = 0;
  double best_cost = 0.0;
  for (int s = 0; s < kNumGroupedShapes; ++s) {
    const hpvm_tile& t = kGroupedShapes[s].tile;
    const double per_tile = (double)t.tile_m * t.tile_n * (double)((k > 0 ? k : 0) + 32);
    const double cost = (double)shape_tiles(m, n, s) *
                        (per_tile * std::pow(kGroupedShapes[s].cost_per_flop, lambda) + overhead * 128.0 * 128.0);
    if (s == 0 || cost < best_cost) {
      best = s;
      best_cost = cost;
    }
  }
  return best;
}

}  // namespace hpvm
