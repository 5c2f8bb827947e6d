// Device-side building blocks shared by the sgemm lowerings (gfx950 only).
//
// The hierarchy of the sgemm dataflow graph (HPVM report, Sec. 3.4 and 6.1)
// maps onto CDNA4 as: one SgemmInternal instance = one workgroup tile of C,
// the Allocation node = the LDS staging buffers of that workgroup, and the
// SgemmLeaf instances = lanes whose outputs sit in MFMA accumulators.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hpvm {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// Arguments of one sgemm as every kernel sees them.  A is addressed as
// element (i, p) = A[i * lda + p], or A[p * lda + i] when a_trans; B as
// (p, j) = B[p * ldb + j], or B[j * ldb + p] when b_trans (the backward pass
// needs the transposed forms; the forward entry point is row-major only).
struct GemmArgs {
  const float* A;
  const float* B;
  float* C;
  int64_t lda, ldb, ldc;
  int32_t m, n, k;
  float alpha, beta;
  int32_t vec_a, vec_b;  // 16-byte vector loads allowed for this operand
  int32_t tiles_m, tiles_n;
};

// True when the TM x TN tile at (m0, n0) and every K-slab of depth TK lie
// inside the matrices and both operands allow 16-byte loads: the main loop
// then needs no per-element checks.  k == 0 (which the persistent kernels
// pass for alpha == 0) is never interior: the masked loads then read no
// memory at all, so A and B may be NULL.  Uniform across the workgroup.
template <int TM, int TN, int TK>
__device__ __forceinline__ bool interior_tile(const GemmArgs& p, int m0, int n0) {
  return p.vec_a && p.vec_b && m0 + TM <= p.m && n0 + TN <= p.n && p.k > 0 && p.k % TK == 0;
}

// --------------------------------------------------------------------------
// Tile of a row-major global matrix -> registers -> LDS.
// R x Cc elements starting at `base` (already offset to the tile corner);
// rows >= rlim or columns >= clim read as zero (edge tiles, K tail).
// Each thread moves U float4 units; consecutive threads take consecutive
// units along a row, so a wavefront reads whole 128-byte row segments.
// --------------------------------------------------------------------------
template <int R, int Cc, int NT>
struct GlobalTile {
  static_assert(Cc % 4 == 0, "tile width must be a multiple of 4");
  static constexpr int kUnitsPerRow = Cc / 4;
  static constexpr int kUnits = R * kUnitsPerRow;
  static_assert(kUnits % NT == 0, "tile must split evenly over the workgroup");
  static constexpr int U = kUnits / NT;

  f32x4 v[U];

  // MASKED = false: the caller guarantees the whole tile is inside the
  // matrix and 16-byte aligned, so every unit is one unconditional vector
  // load (no divergent branches between the loads of a slab).
  template <bool MASKED>
  __device__ __forceinline__ void load(const float* __restrict__ base, int64_t ld, int rlim, int clim,
                                       bool vec, int tid) {
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int u = tid + j * NT;
      const int r = u / kUnitsPerRow;
      const int c = (u % kUnitsPerRow) * 4;
      const float* p = base + (int64_t)r * ld + c;
      if constexpr (!MASKED) {
        v[j] = *reinterpret_cast<const f32x4*>(p);
      } else if (vec && r < rlim && c + 4 <= clim) {
        v[j] = *reinterpret_cast<const f32x4*>(p);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[j][e] = (r < rlim && c + e < clim) ? p[e] : 0.0f;
      }
    }
  }

  // FP32 staging with the global layout kept: LDS row stride S floats.
  template <int S>
  __device__ __forceinline__ void store_f32(float* lds, int tid) const {
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int u = tid + j * NT;
      const int r = u / kUnitsPerRow;
      const int c = (u % kUnitsPerRow) * 4;
      *reinterpret_cast<f32x4*>(lds + r * S + c) = v[j];
    }
  }
};

// ---------------------------------------------------------------------------
// Tile order.  Workgroup w is placed on XCD (w mod 8); renumber so that each
// XCD works through one contiguous run of tiles, then walk that run in
// groups of kGroupM tile-rows so that concurrently resident tiles share
// A row-panels and B column-panels.
// ---------------------------------------------------------------------------
constexpr int kXcds = 8;
constexpr int kGroupM = 8;

__device__ __forceinline__ void tile_coords(int tiles_m, int tiles_n, int w, int& tm, int& tn) {
  const int total = tiles_m * tiles_n;
  const int q = total / kXcds, rem = total % kXcds;
  const int x = w % kXcds;
  const int t = x * q + (x < rem ? x : rem) + w / kXcds;
  const int per_group = kGroupM * tiles_n;
  const int group = t / per_group;
  const int first_m = group * kGroupM;
  const int gsize = (tiles_m - first_m) < kGroupM ? (tiles_m - first_m) : kGroupM;
  const int in_group = t - group * per_group;
  tm = first_m + in_group % gsize;
  tn = in_group / gsize;
}

// Sum over a wavefront with a fixed butterfly.
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Sum over the workgroup; the result is valid in thread 0.  `red` holds one
// float per wavefront.  Ends with every thread past a barrier.
__device__ __forceinline__ float block_sum(float v, float* red) {
  v = wave_sum(v);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  float t = 0.0f;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += red[w];
  __syncthreads();
  return t;
}

}  // namespace hpvm
