// BF16 / bf16x3 MFMA main loop of one SgemmInternal instance.
//
// Same hierarchy as the FP32 main loop (one workgroup per SgemmInternal
// instance, the Allocation node as two LDS stages, SgemmLeaf outputs as MFMA
// accumulators); the products are bf16 x bf16 on v_mfma_f32_32x32x16_bf16
// with FP32 accumulation.
#pragma once

#include <type_traits>

#include "device_common.hpp"
#include "mfma_f32.hpp"

namespace hpvm {

// ---------------------------------------------------------------------------
// BF16 / bf16x3 operand staging.  The conversion from the FP32 storage is
// fused into the HBM -> LDS copy: each element is rounded (nearest-even, the
// hardware conversion) once per workgroup as it enters LDS.  With X3 the
// element is also split, hi = bf16(x), lo = bf16(x - hi), into two tiles.
//
// v_mfma_f32_32x32x16_bf16 takes, in lane l, eight consecutive k of row
// l%32 of A (k = 8(l/32) .. 8(l/32)+7) and the same eight k of column l%32
// of B.  Both operands are therefore kept k-contiguous in LDS: row r (an m
// or n index) holds TK bf16 values plus 16 bytes of padding, so one
// fragment is one 16-byte LDS read and a wavefront's reads cover all banks.
// ---------------------------------------------------------------------------
template <int TK>
struct Bf16Rows {
  static constexpr int kRowBytes = 2 * TK + 16;
};

__device__ __forceinline__ uint32_t pack_bf16(float lo_k, float hi_k) {
  bf16x2 v;
  v[0] = (__bf16)lo_k;
  v[1] = (__bf16)hi_k;
  return __builtin_bit_cast(uint32_t, v);
}

// hi/lo split of two values packed as bf16 pairs.
__device__ __forceinline__ void split_bf16(float a, float b, uint32_t& hi, uint32_t& lo) {
  bf16x2 h;
  h[0] = (__bf16)a;
  h[1] = (__bf16)b;
  const float ha = (float)h[0], hb = (float)h[1];
  bf16x2 l;
  l[0] = (__bf16)(a - ha);
  l[1] = (__bf16)(b - hb);
  hi = __builtin_bit_cast(uint32_t, h);
  lo = __builtin_bit_cast(uint32_t, l);
}

// Source k-contiguous (rows = m or n, columns = k): unit = 8 consecutive k.
template <int MN, int TK, int NT>
struct KcTile {
  static constexpr int kUnitsPerRow = TK / 8;
  static constexpr int kUnits = MN * kUnitsPerRow;
  static_assert(kUnits % NT == 0, "tile must split evenly over the workgroup");
  static constexpr int U = kUnits / NT;
  f32x4 v[U][2];

  template <bool MASKED>
  __device__ __forceinline__ void load(const float* __restrict__ base, int64_t ld, int rlim,
                                       int clim, bool vec, int tid) {
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int u = tid + j * NT;
      const int r = u / kUnitsPerRow;
      const int c = (u % kUnitsPerRow) * 8;
      const float* p = base + (int64_t)r * ld + c;
      if (!MASKED || (vec && r < rlim && c + 8 <= clim)) {
        v[j][0] = *reinterpret_cast<const f32x4*>(p);
        v[j][1] = *reinterpret_cast<const f32x4*>(p + 4);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[j][e >> 2][e & 3] = (r < rlim && c + e < clim) ? p[e] : 0.0f;
      }
    }
  }

  template <bool X3>
  __device__ __forceinline__ void store(char* hi, char* lo, int tid) const {
    constexpr int RB = Bf16Rows<TK>::kRowBytes;
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int u = tid + j * NT;
      const int r = u / kUnitsPerRow;
      const int c = (u % kUnitsPerRow) * 8;
      u32x4 h, l;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float a = v[j][q >> 1][(q & 1) * 2], b = v[j][q >> 1][(q & 1) * 2 + 1];
        if constexpr (X3) {
          uint32_t hh, ll;
          split_bf16(a, b, hh, ll);
          h[q] = hh;
          l[q] = ll;
        } else {
          h[q] = pack_bf16(a, b);
        }
      }
      *reinterpret_cast<u32x4*>(hi + r * RB + 2 * c) = h;
      if constexpr (X3) *reinterpret_cast<u32x4*>(lo + r * RB + 2 * c) = l;
    }
  }
};

// Source m/n-contiguous (rows = k, columns = m or n): unit = two k rows by
// four columns, stored transposed as four (k, k+1) bf16 pairs.  Consecutive
// threads take consecutive k pairs, which keeps the 4-byte LDS writes on
// distinct banks.
template <int MN, int TK, int NT>
struct MnTile {
  static constexpr int kPairs = TK / 2;
  static constexpr int kUnits = kPairs * (MN / 4);
  static_assert(kUnits % NT == 0, "tile must split evenly over the workgroup");
  static constexpr int U = kUnits / NT;
  f32x4 v[U][2];

  template <bool MASKED>
  __device__ __forceinline__ void load(const float* __restrict__ base, int64_t ld, int rlim,
                                       int clim, bool vec, int tid) {
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int u = tid + j * NT;
      const int kp = u % kPairs;
      const int c = (u / kPairs) * 4;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = 2 * kp + h;
        const float* p = base + (int64_t)r * ld + c;
        if (!MASKED || (vec && r < rlim && c + 4 <= clim)) {
          v[j][h] = *reinterpret_cast<const f32x4*>(p);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) v[j][h][e] = (r < rlim && c + e < clim) ? p[e] : 0.0f;
        }
      }
    }
  }

  template <bool X3>
  __device__ __forceinline__ void store(char* hi, char* lo, int tid) const {
    constexpr int RB = Bf16Rows<TK>::kRowBytes;
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int u = tid + j * NT;
      const int kp = u % kPairs;
      const int c = (u / kPairs) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int off = (c + e) * RB + 4 * kp;
        if constexpr (X3) {
          uint32_t hh, ll;
          split_bf16(v[j][0][e], v[j][1][e], hh, ll);
          *reinterpret_cast<uint32_t*>(hi + off) = hh;
          *reinterpret_cast<uint32_t*>(lo + off) = ll;
        } else {
          *reinterpret_cast<uint32_t*>(hi + off) = pack_bf16(v[j][0][e], v[j][1][e]);
        }
      }
    }
  }
};

template <bool KC, int MN, int TK, int NT>
using Bf16Tile = typename std::conditional<KC, KcTile<MN, TK, NT>, MnTile<MN, TK, NT>>::type;

__device__ __forceinline__ bf16x8 frag_bf16(const char* lds, int row, int kstep, int lane, int rb) {
  return *reinterpret_cast<const bf16x8*>(lds + (row + (lane & 31)) * rb + kstep * 32 + 16 * (lane >> 5));
}

// Shape constants of a BF16 / bf16x3 MFMA tile.
template <int TM, int TN, int TK, int WM, int WN, bool X3>
struct Bf16TileShape {
  static constexpr int kWavesN = TN / WN;
  static constexpr int NT = (TM / WM) * kWavesN * kWave;
  static constexpr int BM = WM / 32, BN = WN / 32;
  static constexpr int RB = Bf16Rows<TK>::kRowBytes;
  static constexpr int kPlanes = X3 ? 2 : 1;
  static constexpr int kABytes = TM * RB, kBBytes = TN * RB;
  static constexpr int kStageBytes = kPlanes * (kABytes + kBBytes);
  static constexpr int64_t kLdsBytes = 2 * (int64_t)kStageBytes;
  static_assert(TK % 16 == 0, "K slab must hold whole MFMA steps of 16");
};

// The MFMAs of one LDS stage: TK/16 steps of 16 k over the wave's
// (WM/32) x (WN/32) blocks.  a_lo / b_lo are read only with X3.  With
// PIPE, the fragments of step ks + 1 are read from LDS before the MFMAs of
// step ks are issued (two fragment buffers), so LDS latency overlaps the
// matrix-core work instead of preceding it.
template <int TK, int BM, int BN, bool X3, bool PIPE = false>
__device__ __forceinline__ void bf16_stage_mfma(const char* a_hi, const char* a_lo, const char* b_hi,
                                                const char* b_lo, int wm0, int wn0, int lane,
                                                f32x16 (&acc)[BM][BN]) {
  constexpr int RB = Bf16Rows<TK>::kRowBytes;
  constexpr int KS = TK / 16;
  constexpr int NB = PIPE ? 2 : 1;
  bf16x8 ah[NB][BM], bh[NB][BN], al[NB][X3 ? BM : 1], bl[NB][X3 ? BN : 1];
  auto read = [&](int buf, int ks) {
#pragma unroll
    for (int bi = 0; bi < BM; ++bi) ah[buf][bi] = frag_bf16(a_hi, wm0 + 32 * bi, ks, lane, RB);
#pragma unroll
    for (int bj = 0; bj < BN; ++bj) bh[buf][bj] = frag_bf16(b_hi, wn0 + 32 * bj, ks, lane, RB);
    if constexpr (X3) {
#pragma unroll
      for (int bi = 0; bi < BM; ++bi) al[buf][bi] = frag_bf16(a_lo, wm0 + 32 * bi, ks, lane, RB);
#pragma unroll
      for (int bj = 0; bj < BN; ++bj) bl[buf][bj] = frag_bf16(b_lo, wn0 + 32 * bj, ks, lane, RB);
    }
  };
  auto mfma = [&](int buf) {
    if constexpr (X3) {
#pragma unroll
      for (int bi = 0; bi < BM; ++bi)
#pragma unroll
        for (int bj = 0; bj < BN; ++bj) {
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[buf][bi], bh[buf][bj], acc[bi][bj], 0, 0, 0);
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[buf][bi], bl[buf][bj], acc[bi][bj], 0, 0, 0);
        }
    }
#pragma unroll
    for (int bi = 0; bi < BM; ++bi)
#pragma unroll
      for (int bj = 0; bj < BN; ++bj)
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[buf][bi], bh[buf][bj], acc[bi][bj], 0, 0, 0);
  };
  if constexpr (PIPE) {
    read(0, 0);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      if (ks + 1 < KS) read((ks + 1) & 1, ks + 1);
      __builtin_amdgcn_sched_barrier(0);
      mfma(ks & 1);
    }
  } else {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      read(0, ks);
      mfma(0);
    }
  }
}

// Accumulates the TM x TN tile at (m0, n0) of op(A) op(B) into acc with
// bf16 products (X3: lo*hi + hi*lo + hi*hi).  Ends with a barrier.
template <int TM, int TN, int TK, int WM, int WN, bool AT, bool BT, bool X3, bool MASKED>
__device__ __forceinline__ void bf16_mainloop_impl(const GemmArgs& p, int m0, int n0, char* smem,
                                                   f32x16 (&acc)[WM / 32][WN / 32]) {
  using T = Bf16TileShape<TM, TN, TK, WM, WN, X3>;
  constexpr int NT = T::NT, BM = T::BM, BN = T::BN;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid / kWave;
  const int wm0 = (wave / T::kWavesN) * WM, wn0 = (wave % T::kWavesN) * WN;

  // stage layout: [A hi][A lo][B hi][B lo] (lo planes only with X3)
  auto a_hi = [&](int st) { return smem + st * T::kStageBytes; };
  auto a_lo = [&](int st) { return smem + st * T::kStageBytes + T::kABytes; };
  auto b_hi = [&](int st) { return smem + st * T::kStageBytes + T::kPlanes * T::kABytes; };
  auto b_lo = [&](int st) { return smem + st * T::kStageBytes + T::kPlanes * T::kABytes + T::kBBytes; };

  Bf16Tile<!AT, TM, TK, NT> ga;
  Bf16Tile<BT, TN, TK, NT> gb;
  auto fetch = [&](int k0) {
    const float* base;
    int rl, cl;
    slab_a<AT>(p, m0, k0, base, rl, cl);
    ga.template load<MASKED>(base, p.lda, rl, cl, p.vec_a, tid);
    slab_b<BT>(p, n0, k0, base, rl, cl);
    gb.template load<MASKED>(base, p.ldb, rl, cl, p.vec_b, tid);
  };
  auto stash = [&](int st) {
    ga.template store<X3>(a_hi(st), a_lo(st), tid);
    gb.template store<X3>(b_hi(st), b_lo(st), tid);
  };

  zero_acc(acc);
  const int slabs = (p.k + TK - 1) / TK;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int s = 0; s < slabs; ++s) {
    const int st = s & 1;
    const bool more = s + 1 < slabs;
    if (more) fetch((s + 1) * TK);
    bf16_stage_mfma<TK, BM, BN, X3>(a_hi(st), a_lo(st), b_hi(st), b_lo(st), wm0, wn0, lane, acc);
    if (more) stash(st ^ 1);
    __syncthreads();
  }
}

template <int TM, int TN, int TK, int WM, int WN, bool AT, bool BT, bool X3>
__device__ __forceinline__ void bf16_mainloop(const GemmArgs& p, int m0, int n0, char* smem,
                                              f32x16 (&acc)[WM / 32][WN / 32]) {
  if (interior_tile<TM, TN, TK>(p, m0, n0))
    bf16_mainloop_impl<TM, TN, TK, WM, WN, AT, BT, X3, false>(p, m0, n0, smem, acc);
  else
    bf16_mainloop_impl<TM, TN, TK, WM, WN, AT, BT, X3, true>(p, m0, n0, smem, acc);
}

}  // namespace hpvm
