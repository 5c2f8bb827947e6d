// BF16 / bf16x3 products on FP32 storage, fed by DMA (gfx950).
//
// The Allocation node is the FP32 DMA-fed loop's (mfma_f32_dma.hpp): a ring
// of NST LDS stages that FP32 K-slabs of A and B reach straight from HBM
// (global_load_lds_dwordx4), in the same KC / MN layouts.  The rounding to
// bfloat16 happens between LDS and the matrix cores: each wave reads the
// FP32 values of its MFMA fragments and converts them in registers
// (v_cvt_pk_bf16_f32, round to nearest even) right before
// v_mfma_f32_32x32x16_bf16, so the conversion costs no pass over HBM and no
// LDS space beyond the FP32 slabs.  bf16x3 splits each value there too:
// hi = bf16(x), lo = bf16(x - hi), x - hi being exact in FP32.
//
// v_mfma_f32_32x32x16_bf16 takes, in lane l, eight consecutive k of row
// l % 32 of A (k = 8 (l / 32) + j for slot j) and the same eight k of
// column l % 32 of B.  Within a slab, 16-k step s gives slot j of lane half
// h the value at k = 16 s + 8 h + j:
//   KC operand (k contiguous): the 16-byte chunks 4 s + 2 h and 4 s + 2 h + 1
//     of the lane's row, read from the SwizzledRows layout;
//   MN operand (m or n contiguous): eight reads, one per slot, of V adjacent
//     values at that slot's k; component t goes to accumulator block t, which
//     owns every V-th row or column (as in the FP32 loop).
// The slots hold k in natural order, as in the lowerings over bfloat16
// planes, and bf16x3 issues lo*hi, hi*lo, then hi*hi per block pair as they
// do, so every lowering of a precision sums the same products in the same
// order.
#pragma once

#include <type_traits>

#include "mfma_f32_dma.hpp"

namespace hpvm {

// Byte offset of 16-byte chunk c of this lane's row within a 32-row block
// of a KC stage whose rows are RB bytes (the SwizzledRows layouts).
template <int RB>
__device__ __forceinline__ int kc_chunk_off(int lane, int c);
template <>
__device__ __forceinline__ int kc_chunk_off<128>(int lane, int c) {
  const int r = lane & 31;
  return (r ^ ((r >> 3) & 1)) * 128 + ((c ^ (r & 7)) << 4);
}
template <>
__device__ __forceinline__ int kc_chunk_off<64>(int lane, int c) {
  const int l = lane & 31;
  const int g = ((l >> 1) & 3) ^ ((l >> 3) & 1);
  return (l >> 1) * 128 + (((((l & 1) << 2) | c) ^ g) << 4);
}

// One operand side of the BF16 product: the FP32 stage layout and DMA of
// F32DmaOperand, with fragment reads by 16-k steps.
template <bool KC, int R, int W, int TK>
struct Bf16SrcOperand : F32DmaOperand<KC, R, W, TK> {
  using Base = F32DmaOperand<KC, R, W, TK>;
  using Frag = typename Base::Frag;
  static constexpr int V = Base::V, kBlocks = Base::kBlocks;
  static constexpr int kRowBytes = 4 * TK;
  static constexpr int kReads = KC ? 2 * kBlocks : 8;  // 16-byte (KC) or V-float (MN) reads per step
  using Raw = typename std::conditional<KC, f32x4, Frag>::type;

  // KC: byte offset of chunk e of step s within the lane's 32-row block.
  __device__ static int chunk(int lane, int s, int e) {
    return kc_chunk_off<kRowBytes>(lane, 4 * s + 2 * (lane >> 5) + e);
  }
  // The FP32 values of step s's fragments from stage `st`; w0 = the wave's
  // first row (KC) or value (MN) on this side; koff = chunk(lane, s, 0..1).
  __device__ static void read(Raw (&r)[kReads], const char* st, int s, int w0, int lane, const int (&koff)[2]) {
    if constexpr (KC) {
#pragma unroll
      for (int b = 0; b < kBlocks; ++b)
#pragma unroll
        for (int e = 0; e < 2; ++e)
          r[2 * b + e] = *reinterpret_cast<const Raw*>(st + (w0 + 32 * b) * kRowBytes + koff[e]);
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j)
        r[j] = *reinterpret_cast<const Raw*>(st + (16 * s + 8 * (lane >> 5) + j) * R * 4 + (w0 + V * (lane & 31)) * 4);
    }
  }
  // Slot j of block b.
  __device__ static float value(const Raw (&r)[kReads], int b, int j) {
    if constexpr (KC) return r[2 * b + (j >> 2)][j & 3];
    else return r[j][b];
  }
};

template <int TM, int TN, int TK, int WM, int WN, bool AT, bool BT, int NST>
struct Bf16SrcShape : F32DmaShape<TM, TN, TK, WM, WN, AT, BT, NST> {
  using OA = Bf16SrcOperand<!AT, TM, WM, TK>;
  using OB = Bf16SrcOperand<BT, TN, WN, TK>;
  static constexpr int KS = TK / 16;  // MFMA steps per slab
};

// Two values rounded to bfloat16, packed (a in the low half).
__device__ __forceinline__ uint32_t bf16_pair(float a, float b) {
  bf16x2 v;
  v[0] = (__bf16)a;
  v[1] = (__bf16)b;
  return __builtin_bit_cast(uint32_t, v);
}
// The lo parts of a pair whose packed hi parts are `hi`: bf16(x - hi), the
// FP32 value of a bfloat16 being its bits in the upper half.
__device__ __forceinline__ uint32_t bf16_lo_pair(float a, float b, uint32_t hi) {
  const float ha = __builtin_bit_cast(float, hi << 16);
  const float hb = __builtin_bit_cast(float, hi & 0xffff0000u);
  return bf16_pair(a - ha, b - hb);
}

// One tile (tm, tn) of contraction slice z with BF16 (X3: bf16x3) products
// on the FP32 DMA-fed loop, by the whole workgroup, Allocation at smem
// (S::kLdsBytes).  MODE: kDmaUpdate or kDmaSplit.  CVB: buffers of
// converted fragments (2: a step's successor is converted into the other
// one; 1 saves the registers of a second set).  Ends with every transfer
// drained and the workgroup past a barrier.
template <int TM, int TN, int TK, int WM, int WN, bool AT, bool BT, int NST, bool X3, int MODE, bool EDGES, int CVB>
__device__ __forceinline__ void bf16src_dma_tile(const GemmArgs& p, const F32DmaOut& o, int tm, int tn, int z,
                                                 char* smem) {
  using S = Bf16SrcShape<TM, TN, TK, WM, WN, AT, BT, NST>;
  using OA = typename S::OA;
  using OB = typename S::OB;
  constexpr int NA = OA::kBlocks, NB = OB::kBlocks, KS = S::KS, P = X3 ? 2 : 1;
  static_assert(MODE == kDmaUpdate || MODE == kDmaSplit, "update or split");

  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int wm0 = (wave / S::NWN) * WM, wn0 = (wave % S::NWN) * WN;
  const int splits = MODE == kDmaSplit ? o.splits : 1;
  const int64_t m_own = (int64_t)tm * TM, n_own = (int64_t)tn * TN;
  const int64_t m0 = EDGES && m_own + TM > p.m ? p.m - TM : m_own;
  const int64_t n0 = EDGES && n_own + TN > p.n ? p.n - TN : n_own;
  const int slabs_all = p.k / TK;
  const int per = (slabs_all + splits - 1) / splits;
  const int sbeg = z * per, slabs = (slabs_all - sbeg < per ? slabs_all - sbeg : per);
  const uint32_t lds0 = lds_addr(smem);

  const int64_t lda4 = p.lda * 4, ldb4 = p.ldb * 4;
  const char* abase = reinterpret_cast<const char*>(p.A);
  const char* bbase = reinterpret_cast<const char*>(p.B);
  const uint32_t aoff[2] = {OA::lane_off(lane, 0, lda4), OA::lane_off(lane, 1, lda4)};
  const uint32_t boff[2] = {OB::lane_off(lane, 0, ldb4), OB::lane_off(lane, 1, ldb4)};
  // This wave's DMA sources at the slice's first slab (uniform pointers)
  // and the byte step from one slab to the next: a KC operand advances
  // along its rows, an MN operand by TK rows.
  const char* asrc[S::QA];
  const char* bsrc[S::QB];
#pragma unroll
  for (int j = 0; j < S::QA; ++j) asrc[j] = abase + OA::base(wave * S::QA + j, m0, (int64_t)sbeg * TK, p.lda) * 4;
#pragma unroll
  for (int j = 0; j < S::QB; ++j) bsrc[j] = bbase + OB::base(wave * S::QB + j, n0, (int64_t)sbeg * TK, p.ldb) * 4;
  const int64_t astep = (AT ? p.lda : 1) * (int64_t)TK * 4, bstep = (BT ? 1 : p.ldb) * (int64_t)TK * 4;
  auto dma_slab = [&](int slab, int st) {
    const uint32_t la = lds0 + st * S::kStage + wave * S::QA * 1024;
    const uint32_t lb = lds0 + st * S::kStage + OA::kBytes + wave * S::QB * 1024;
    const int64_t ao = slab * astep, bo = slab * bstep;
#pragma unroll
    for (int j = 0; j < S::QA; ++j) dma16(la + j * 1024, asrc[j] + ao, aoff[j & 1]);
#pragma unroll
    for (int j = 0; j < S::QB; ++j) dma16(lb + j * 1024, bsrc[j] + bo, boff[(wave * S::QB + j) & 1]);
  };

  int akoff[KS][2], bkoff[KS][2];
#pragma unroll
  for (int s = 0; s < KS; ++s)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      akoff[s][e] = OA::chunk(lane, s, e);
      bkoff[s][e] = OB::chunk(lane, s, e);
    }

  f32x16 acc[NA][NB];
  zero_acc(acc);
  typename OA::Raw ra[OA::kReads];
  typename OB::Raw rb[OB::kReads];
  // Converted fragments, [buffer][hi, lo][block], as 4 packed bf16 pairs.
  // With one buffer, a step's conversion overwrites fragments the step's
  // MFMAs have already read (the hardware reads an MFMA's sources as it
  // issues it), so it follows them.
  u32x4 ca[CVB][P][NA], cb[CVB][P][NB];
  auto read = [&](const char* st, int s) {
    OB::read(rb, st + OA::kBytes, s, wn0, lane, bkoff[s]);
    OA::read(ra, st, s, wm0, lane, akoff[s]);
  };
  // Pair p of the next step's values (B's blocks first, then A's) into
  // fragment buffer buf.
  constexpr int kPairs = 4 * (NA + NB);
  auto convert_pair = [&](int buf, int p) {
    const bool bside = p < 4 * NB;
    const int blk = bside ? p / 4 : p / 4 - NB, q = p % 4;
    const float x = bside ? OB::value(rb, blk, 2 * q) : OA::value(ra, blk, 2 * q);
    const float y = bside ? OB::value(rb, blk, 2 * q + 1) : OA::value(ra, blk, 2 * q + 1);
    const uint32_t h = bf16_pair(x, y);
    (bside ? cb[buf][0][blk] : ca[buf][0][blk])[q] = h;
    if constexpr (X3) (bside ? cb[buf][1][blk] : ca[buf][1][blk])[q] = bf16_lo_pair(x, y, h);
  };
  auto convert = [&](int buf) {
#pragma unroll
    for (int p = 0; p < kPairs; ++p) convert_pair(buf % CVB, p);
  };
  // MFMA i of a step: with X3 first lo*hi and hi*lo of every block pair,
  // then hi*hi of every pair (each accumulator sees lo*hi, hi*lo, hi*hi).
  constexpr int kMfmas = (X3 ? 3 : 1) * NA * NB;
  auto mfma_i = [&](int buf, int i) {
    auto op = [](const u32x4& v) { return __builtin_bit_cast(bf16x8, v); };
    if (X3 && i < 2 * NA * NB) {
      const int a = i / (2 * NB), b = (i / 2) % NB, w = i & 1;
      acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(op(ca[buf][w ? 0 : P - 1][a]), op(cb[buf][w ? P - 1 : 0][b]),
                                                          acc[a][b], 0, 0, 0);
    } else {
      const int j = X3 ? i - 2 * NA * NB : i, a = j / NB, b = j % NB;
      acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(op(ca[buf][0][a]), op(cb[buf][0][b]), acc[a][b], 0, 0, 0);
    }
  };
  // One step's MFMAs on buffer b2 % CVB, then the next step's conversion
  // (its fragments were read before the MFMAs) into the next buffer.
  auto mfma_convert = [&](int b2) {
#pragma unroll
    for (int i = 0; i < kMfmas; ++i) mfma_i(b2 % CVB, i);
#pragma unroll
    for (int p = 0; p < kPairs; ++p) convert_pair((b2 + 1) % CVB, p);
  };

  if (slabs > 0) {
#pragma unroll
    for (int i = 0; i < NST - 1; ++i) dma_slab(i < slabs ? i : slabs - 1, i);
    dma_wait_barrier<(NST - 2) * S::Q>();
    read(smem, 0);
    dma_slab(NST - 1 < slabs ? NST - 1 : slabs - 1, NST - 1);
    convert(0);
  }
  // Step u of slab s uses fragment buffer (P0 + u) & 1, P0 the parity of
  // the steps before the slab; with an odd number of steps per slab the
  // parity alternates, so slabs are taken in pairs.
  int st = 0;
  auto slab = [&](int s, auto parity) {
    constexpr int P0 = decltype(parity)::value;
    const char* cur = smem + st * S::kStage;
#pragma unroll
    for (int u = 0; u + 1 < KS; ++u) {
      read(cur, u + 1);
      mfma_convert((P0 + u) & 1);
    }
    // Slab s + 1 has landed everywhere and slab s is no longer read:
    // request slab s + NST into its stage (the last slab again past the
    // end, which keeps the wait counts exact), read slab s + 1's first step
    // and convert it under the last step's MFMAs.
    const int nst = st + 1 == NST ? 0 : st + 1;
    dma_wait_barrier<(NST - 2) * S::Q>();
    read(smem + nst * S::kStage, 0);
    dma_slab(s + NST < slabs ? s + NST : slabs - 1, st);
    mfma_convert((P0 + KS - 1) & 1);
    st = nst;
  };
  if constexpr (KS % 2 == 0) {
    for (int s = 0; s < slabs; ++s) slab(s, std::integral_constant<int, 0>{});
  } else {
    int s = 0;
    for (; s + 1 < slabs; s += 2) {
      slab(s, std::integral_constant<int, 0>{});
      slab(s + 1, std::integral_constant<int, 1>{});
    }
    if (s < slabs) slab(s, std::integral_constant<int, 0>{});
  }
  // No transfer may still be writing LDS when the workgroup ends.
  dma_wait_barrier<0>();
  dma_epilogue<OA, OB, BT, MODE, 0, EDGES>(p, o, acc, m0, n0, m_own, n_own, wm0, wn0, lane, z);
}

// One launch: a workgroup per tile and contraction slice, XCD-aware order.
// Converted-fragment buffers: two when the wave tile leaves room for them.
template <int WM, int WN, bool X3>
constexpr int kBf16SrcCvb = (WM * WN >= 128 * 128 || !X3) ? 2 : 1;

template <int TM, int TN, int TK, int WM, int WN, bool AT, bool BT, int NST, bool X3, int MODE, bool EDGES = false>
__global__ void __launch_bounds__((Bf16SrcShape<TM, TN, TK, WM, WN, AT, BT, NST>::NW * kWave))
    __attribute__((amdgpu_waves_per_eu(1, (Bf16SrcShape<TM, TN, TK, WM, WN, AT, BT, NST>::kMaxWaves))))
    sgemm_bf16src_dma(GemmArgs p, F32DmaOut o) {
  extern __shared__ __align__(16) char smem[];
  const int tiles = p.tiles_m * p.tiles_n;
  const int z = blockIdx.x / tiles;
  int tm, tn;
  tile_coords(p.tiles_m, p.tiles_n, blockIdx.x - z * tiles, tm, tn);
  bf16src_dma_tile<TM, TN, TK, WM, WN, AT, BT, NST, X3, MODE, EDGES, kBf16SrcCvb<WM, WN, X3>>(p, o, tm, tn, z, smem);
}

}  // namespace hpvm
