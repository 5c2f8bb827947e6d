// FP32 MFMA main loop of one SgemmInternal instance (one workgroup tile).
//
// Hierarchy (HPVM report, Sec. 3.4: leaf instances form one tile, the parent's
// instances the grid of tiles, allocation-node memory goes to the scratchpad):
//   SgemmInternal instance -> one workgroup owning a TM x TN tile of C;
//   Allocation node        -> two LDS stages, each a TM x TK slab of A and a
//                             TK x TN slab of B, filled from HBM with
//                             coalesced 16-byte loads while the other stage
//                             feeds the matrix cores;
//   SgemmLeaf instances    -> the TM x TN outputs, held as MFMA accumulators:
//                             each 64-lane wavefront owns a WM x WN sub-tile,
//                             i.e. (WM/32) x (WN/32) blocks of 32 x 32.
#pragma once

#include "device_common.hpp"

namespace hpvm {

// ---------------------------------------------------------------------------
// FP32 operand staging.  KC: rows are m (or n) indices with k contiguous,
// row stride TK + 4 floats; otherwise rows are k indices with m (or n)
// contiguous, row stride MN + 8 floats.  Both keep the global layout, so no
// transposition happens on the way into LDS; the paddings spread one
// fragment read over all LDS banks.
//
// v_mfma_f32_32x32x2f32 takes, in lane l, A(row l%32, k-slot l/32) and
// B(k-slot l/32, col l%32).  Within a group of 8 k values the slot h of
// step t is k = 4h + t, so a k-contiguous operand is read with one 16-byte
// LDS read per group and an m/n-contiguous one with four 4-byte reads.
// ---------------------------------------------------------------------------
template <int MN, int TK, bool KC>
struct F32Operand {
  static constexpr int kRows = KC ? MN : TK;
  static constexpr int kCols = KC ? TK : MN;
  static constexpr int kStride = KC ? TK + 4 : MN + 8;
  static constexpr int kFloats = kRows * kStride;

  __device__ __forceinline__ static f32x4 frag(const float* lds, int mn0, int kg, int lane) {
    const int r32 = lane & 31, h = lane >> 5;
    if constexpr (KC) {
      return *reinterpret_cast<const f32x4*>(lds + (mn0 + r32) * kStride + kg * 8 + 4 * h);
    } else {
      const float* q = lds + (kg * 8 + 4 * h) * kStride + mn0 + r32;
      f32x4 v;
      v[0] = q[0];
      v[1] = q[kStride];
      v[2] = q[2 * kStride];
      v[3] = q[3 * kStride];
      return v;
    }
  }
};

// Global-memory corner of the slab at k0 for each operand form.
template <bool AT>
__device__ __forceinline__ void slab_a(const GemmArgs& p, int m0, int k0, const float*& base,
                                       int& rlim, int& clim) {
  if constexpr (!AT) {
    base = p.A + (int64_t)m0 * p.lda + k0;
    rlim = p.m - m0;
    clim = p.k - k0;
  } else {
    base = p.A + (int64_t)k0 * p.lda + m0;
    rlim = p.k - k0;
    clim = p.m - m0;
  }
}
template <bool BT>
__device__ __forceinline__ void slab_b(const GemmArgs& p, int n0, int k0, const float*& base,
                                       int& rlim, int& clim) {
  if constexpr (!BT) {
    base = p.B + (int64_t)k0 * p.ldb + n0;
    rlim = p.k - k0;
    clim = p.n - n0;
  } else {
    base = p.B + (int64_t)n0 * p.ldb + k0;
    rlim = p.n - n0;
    clim = p.k - k0;
  }
}

// Row and column of accumulator register r of lane `lane` in a 32 x 32
// block: output (i, j) lives in lane j + 32 * ((i / 4) % 2), register
// (i % 4) + 4 * (i / 8).
__device__ __forceinline__ int acc_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }
__device__ __forceinline__ int acc_col(int lane) { return lane & 31; }

// Epilogue: C <- alpha * acc + beta * C, element-wise, masked at the edges.
// beta == 0 never reads C.  The 16 accumulators of a lane in a 32 x 32
// block cover 4 groups of 4 consecutive rows; each group's 4 loads of C are
// issued before its 4 stores.  (A load placed after a store to C could not
// be moved above it -- the addresses may alias as far as the compiler
// knows -- so element by element every load would wait for its own memory
// round trip; four at a time keeps the address registers few enough not
// to cost occupancy.)
template <int BM, int BN>
__device__ __forceinline__ void store_c(const GemmArgs& p, const f32x16 (&acc)[BM][BN], int row0,
                                        int col0, int lane) {
  const bool read_c = p.beta != 0.0f;
#pragma unroll
  for (int bi = 0; bi < BM; ++bi)
#pragma unroll
    for (int bj = 0; bj < BN; ++bj) {
      const int j = col0 + 32 * bj + acc_col(lane);
      if (j >= p.n) continue;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        float c[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int i = row0 + 32 * bi + acc_row(4 * g + t, lane);
          c[t] = (read_c && i < p.m) ? p.C[(int64_t)i * p.ldc + j] : 0.0f;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int i = row0 + 32 * bi + acc_row(4 * g + t, lane);
          if (i < p.m) {
            float v = p.alpha * acc[bi][bj][4 * g + t];
            if (read_c) v = fmaf(p.beta, c[t], v);
            p.C[(int64_t)i * p.ldc + j] = v;
          }
        }
      }
    }
}

template <int BM, int BN>
__device__ __forceinline__ void zero_acc(f32x16 (&acc)[BM][BN]) {
#pragma unroll
  for (int bi = 0; bi < BM; ++bi)
#pragma unroll
    for (int bj = 0; bj < BN; ++bj)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[bi][bj][r] = 0.0f;
}

// Shape constants of an FP32 MFMA tile.
template <int TM, int TN, int TK, int WM, int WN, bool AT, bool BT>
struct F32Tile {
  static constexpr int kWavesN = TN / WN;
  static constexpr int NT = (TM / WM) * kWavesN * kWave;
  static constexpr int BM = WM / 32, BN = WN / 32;
  using OpA = F32Operand<TM, TK, !AT>;
  using OpB = F32Operand<TN, TK, BT>;
  static constexpr int64_t kLdsBytes = 2 * (OpA::kFloats + OpB::kFloats) * (int64_t)sizeof(float);
  static_assert(TK % 8 == 0, "K slab must hold whole groups of 8");
};

template <int TM, int TN, int TK, int WM, int WN, bool AT, bool BT, bool MASKED>
__device__ __forceinline__ void f32_mainloop_impl(
    const GemmArgs& p, int m0, int n0, float* lds, f32x16 (&acc)[WM / 32][WN / 32]) {
  using T = F32Tile<TM, TN, TK, WM, WN, AT, BT>;
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

  GlobalTile<OpA::kRows, OpA::kCols, NT> ga;
  GlobalTile<OpB::kRows, OpB::kCols, NT> gb;
  auto fetch = [&](int k0) {
    const float* base;
    int rl, cl;
    slab_a<AT>(p, m0, k0, base, rl, cl);
    ga.template load<MASKED>(base, p.lda, rl, cl, p.vec_a, tid);
    slab_b<BT>(p, n0, k0, base, rl, cl);
    gb.template load<MASKED>(base, p.ldb, rl, cl, p.vec_b, tid);
  };

  zero_acc(acc);
  const int slabs = (p.k + TK - 1) / TK;
  fetch(0);
  ga.template store_f32<OpA::kStride>(As0, tid);
  gb.template store_f32<OpB::kStride>(Bs0, tid);
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
    if (more) {
      ga.template store_f32<OpA::kStride>((s & 1) ? As0 : As1, tid);
      gb.template store_f32<OpB::kStride>((s & 1) ? Bs0 : Bs1, tid);
    }
    __syncthreads();
  }
}

// Accumulates the TM x TN tile at (m0, n0) of op(A) op(B) into acc.  Ends
// with a barrier, so the caller may reuse `lds` right away.  Interior tiles
// take the unmasked loop.
template <int TM, int TN, int TK, int WM, int WN, bool AT, bool BT>
__device__ __forceinline__ void f32_mainloop(const GemmArgs& p, int m0, int n0, float* lds,
                                             f32x16 (&acc)[WM / 32][WN / 32]) {
  if (interior_tile<TM, TN, TK>(p, m0, n0))
    f32_mainloop_impl<TM, TN, TK, WM, WN, AT, BT, false>(p, m0, n0, lds, acc);
  else
    f32_mainloop_impl<TM, TN, TK, WM, WN, AT, BT, true>(p, m0, n0, lds, acc);
}

}  // namespace hpvm
