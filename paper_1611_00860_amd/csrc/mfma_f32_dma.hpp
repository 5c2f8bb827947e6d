// DMA-fed FP32 MFMA loop of one SgemmInternal instance (gfx950).
//
// The Allocation node is a ring of NST LDS stages filled straight from HBM
// (global_load_lds_dwordx4, lds_dma.hpp): slab s + NST - 1 is requested
// while slab s feeds the matrix cores, so no register holds a slab in
// transit and the freed registers keep two sets of MFMA fragments -- an
// 8-k group's fragments are read while the previous group's MFMAs run.
// One barrier per slab, placed before the last group's MFMAs so that the
// next slab's first fragments are read under them.
//
// v_mfma_f32_32x32x2f32 takes, in lane l, A(row l % 32, slot l / 32) and
// B(slot l / 32, column l % 32); within an 8-k group, slot h of step p is
// k = 4h + p.  Each operand comes in one of two forms:
//   KC (k contiguous in HBM: A as m x k, or B read transposed from n x k):
//     a stage holds the tile's rows, TK floats each, in the SwizzledRows
//     layout; a wave covers its rows as blocks of 32, and a fragment is one
//     16-byte read of the four k of slot h of one row (component p = step p).
//   MN (m or n contiguous: B as k x n, or A read transposed from k x m):
//     a stage holds the slab's TK rows of the tile as in HBM; a wave covers
//     32 V consecutive m (or n) as V phases, and a fragment is one read of V
//     adjacent values at the k of step p (component t = phase t, which owns
//     the values t, t + V, t + 2V, ...).
// With EDGES, m and n need not be multiples of the tile when they are at
// least one tile (and n a multiple of 4): a tile that would cross the edge
// is moved inward to end at it, so every load stays inside the matrices,
// and it stores only the rows and columns it owns (those of its place in
// the tile grid); the rows and columns it overlaps belong to the
// neighbouring tile, which computes them the same way.  Without EDGES the
// problem is whole tiles and the epilogue has no masks.  k must be a
// multiple of the slab (the caller checks; other problems take the masked
// loop of mfma_f32.hpp).
#pragma once

#include "device_common.hpp"
#include "hpvm_sgemm.h"
#include "lds_dma.hpp"
#include "mfma_f32.hpp"

namespace hpvm {

template <int V>
struct VecF;
template <>
struct VecF<2> {
  typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct VecF<4> {
  typedef float type __attribute__((ext_vector_type(4)));
};

// R: the tile's extent on this side (TM or TN); W: a wave's extent.
template <bool KC, int R, int W, int TK>
struct F32DmaOperand {
  static constexpr int kBytes = R * TK * 4;       // one stage
  static constexpr int V = KC ? 4 : W / 32;        // floats per fragment read
  static constexpr int kBlocks = KC ? W / 32 : V;  // accumulator blocks on this side
  static constexpr int kFrags = KC ? W / 32 : 4;   // fragment reads per 8-k group
  static constexpr int kDma = kBytes / 1024;       // DMA instructions per stage
  using Rows = SwizzledRows<4 * TK>;
  static constexpr int kRowsPerDma = KC ? Rows::kRowsPerDma : (256 / R > 0 ? 256 / R : 1);
  static constexpr int kDmaPerRow = KC ? 1 : (R / 256 > 0 ? R / 256 : 1);
  using Frag = typename VecF<V>::type;
  static_assert(kDma * 1024 == kBytes, "whole DMA instructions per stage");
  static_assert(KC ? (W % 32 == 0) : (V == 2 || V == 4), "wave extent");

  // Per-lane source offset of instruction q (its parity for KC).
  __device__ static uint32_t lane_off(int lane, int q, int64_t ldb) {
    if constexpr (KC) {
      return Rows::src(lane, q & 1, ldb);
    } else {
      constexpr int lanes_per_row = 64 / kRowsPerDma;
      return (uint32_t)((lane / lanes_per_row) * ldb + (lane % lanes_per_row) * 16);
    }
  }
  // Global float offset of instruction q's first chunk, slab at k0, tile
  // corner r0 on this side, leading dimension ld (floats).
  __device__ static int64_t base(int q, int64_t r0, int64_t k0, int64_t ld) {
    if constexpr (KC)
      return (r0 + (int64_t)q * kRowsPerDma) * ld + k0;
    else
      return (k0 + (int64_t)(q / kDmaPerRow) * kRowsPerDma) * ld + r0 + (q % kDmaPerRow) * 256;
  }
  // Fragment j (block for KC, step for MN) of group g; w0 = the wave's
  // first row (KC) or value (MN) within the tile.
  __device__ static Frag frag(const char* st, int j, int g, int w0, int lane, int foff) {
    if constexpr (KC)
      return *reinterpret_cast<const Frag*>(st + (w0 + 32 * j) * 4 * TK + foff);
    else
      return *reinterpret_cast<const Frag*>(st + (8 * g + 4 * (lane >> 5) + j) * R * 4 + (w0 + V * (lane & 31)) * 4);
  }
  // Operand of MFMA step p for block b.
  __device__ static float pick(const Frag (&f)[kFrags], int b, int p) {
    if constexpr (KC) return f[b][p];
    else return f[p][b];
  }
  // Row (A side) or column (B side) of accumulator block b's element at
  // in-block index x (0..31) for a wave starting at w0.
  __device__ static int index(int b, int x, int w0) { return KC ? w0 + 32 * b + x : w0 + V * x + b; }
};

// PAIR: two B operands (B1, B2) share A, MergeIndependentNodes with a
// merged Allocation: the B stage holds B1's tile and then B2's, and the
// waves covering the second TN columns produce the second output.
template <int TM, int TN, int TK, int WM, int WN, bool AT, bool BT, int NST, bool PAIR = false>
struct F32DmaShape {
  using OA = F32DmaOperand<!AT, TM, WM, TK>;
  using OB = F32DmaOperand<BT, TN, WN, TK>;
  static constexpr int kOuts = PAIR ? 2 : 1;
  static constexpr int NWN = kOuts * TN / WN, NW = (TM / WM) * NWN;
  static constexpr int kBBytes = kOuts * OB::kBytes;
  static constexpr int kStage = OA::kBytes + kBBytes;
  static constexpr int64_t kLdsBytes = (int64_t)NST * kStage;
  static constexpr int QA = OA::kDma / NW, QB = kOuts * OB::kDma / NW, Q = QA + QB;
  static constexpr int kMaxWaves = (163840 / (NST * kStage)) * NW / 4;
  static_assert(TM % WM == 0 && TN % WN == 0, "wave tiles");
  static_assert(QA * NW == OA::kDma && QB * NW == kOuts * OB::kDma, "DMA instructions split evenly over the waves");
  static_assert(!PAIR || (!AT && !BT), "the pair reads A and both B as stored");
  static_assert((AT || QA % 2 == 0) && (!BT || QB % 2 == 0), "swizzled row groups: a wave starts at an even one");
  static_assert(TK % 16 == 0, "a slab holds an even number of 8-k groups");
  static_assert((NST - 2) * Q < 64, "vmcnt range");
};

// The consumer of MergeDependentNodes, applied to each output element.
template <int OP>
__device__ __forceinline__ float consume(float v, float b, float lo, float hi) {
  if constexpr (OP == HPVM_CONSUMER_RELU) return v > 0.0f ? v : 0.0f;
  if constexpr (OP == HPVM_CONSUMER_BIAS) return v + b;
  if constexpr (OP == HPVM_CONSUMER_BIAS_RELU) {
    const float w = v + b;
    return w > 0.0f ? w : 0.0f;
  }
  if constexpr (OP == HPVM_CONSUMER_CLAMP) return v < lo ? lo : (v > hi ? hi : v);
  return v;
}

// Where the DMA-fed loop's results go.
enum F32DmaMode {
  kDmaUpdate = 0,   // C <- alpha acc + beta C (beta == 0 never reads C)
  kDmaSplit = 1,    // raw accumulators of contraction slice z to C + z m ldc
  kDmaConsume = 2,  // D <- consumer(alpha acc + beta C); C only read
};
struct F32DmaOut {
  int32_t splits;     // contraction slices (kDmaSplit), else 1
  int32_t reserved;
  float* D;           // kDmaConsume: output and its leading dimension
  int64_t ldd;
  const float* bias;  // one value per column (BIAS ops)
  float lo, hi;       // CLAMP
};

// Epilogue of the DMA-fed loops: tile outputs from the accumulators (of
// FP32 or BF16 MFMAs; both use the 32 x 32 block layout of acc_row /
// acc_col).  q: the sgemm whose output this wave holds; m0, n0: the corner
// the tile was computed from; m_own, n_own: its place in the tile grid
// (EDGES stores only the outputs it owns); z: contraction slice (kDmaSplit).
template <typename OA, typename OB, bool BT, int MODE, int OP, bool EDGES, int NA, int NB>
__device__ __forceinline__ void dma_epilogue(const GemmArgs& q, const F32DmaOut& o, const f32x16 (&acc)[NA][NB],
                                             int64_t m0, int64_t n0, int64_t m_own, int64_t n_own, int wm0,
                                             int wn0, int lane, int z) {
  const float* cin = q.C + (MODE == kDmaSplit ? (int64_t)z * q.m * q.ldc : 0);
  float* out = MODE == kDmaConsume ? o.D : q.C + (MODE == kDmaSplit ? (int64_t)z * q.m * q.ldc : 0);
  const int64_t ldo = MODE == kDmaConsume ? o.ldd : q.ldc;
  const float alpha = MODE == kDmaSplit ? 1.0f : q.alpha;
  const bool read_c = MODE != kDmaSplit && q.beta != 0.0f;
  constexpr bool kBias = OP == HPVM_CONSUMER_BIAS || OP == HPVM_CONSUMER_BIAS_RELU;
  const int I = lane & 31;
  if constexpr (!BT) {
    // The NB blocks give a lane NB adjacent outputs of a row: one vector
    // access per row.  A group of 4 rows loads its C values first.
    using VB = typename OB::Frag;
    const int64_t col = n0 + OB::index(0, I, wn0);
    const bool col_own = !EDGES || col >= n_own;  // the lane's NB columns are owned together (n % 4 == 0)
    VB bias{};
    if constexpr (MODE == kDmaConsume && kBias) {
#pragma unroll
      for (int b = 0; b < NB; ++b) bias[b] = o.bias[col + b];
    }
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        VB c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t i = m0 + OA::index(a, acc_row(4 * g + u, lane), wm0);
          if (read_c && col_own && (!EDGES || i >= m_own)) c[u] = *reinterpret_cast<const VB*>(cin + i * q.ldc + col);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t i = m0 + OA::index(a, acc_row(4 * g + u, lane), wm0);
          VB v;
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            v[b] = alpha * acc[a][b][4 * g + u];
            if (read_c) v[b] = fmaf(q.beta, c[u][b], v[b]);
            if constexpr (MODE == kDmaConsume) v[b] = consume<OP>(v[b], bias[b], o.lo, o.hi);
          }
          if (col_own && (!EDGES || i >= m_own)) *reinterpret_cast<VB*>(out + i * ldo + col) = v;
        }
      }
  } else {
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int64_t col = n0 + OB::index(b, I, wn0);
          float c[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int64_t i = m0 + OA::index(a, acc_row(4 * g + u, lane), wm0);
            c[u] = (read_c && (!EDGES || (col >= n_own && i >= m_own))) ? cin[i * q.ldc + col] : 0.0f;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int64_t i = m0 + OA::index(a, acc_row(4 * g + u, lane), wm0);
            float v = alpha * acc[a][b][4 * g + u];
            if (read_c) v = fmaf(q.beta, c[u], v);
            if (!EDGES || (col >= n_own && i >= m_own)) out[i * ldo + col] = v;
          }
        }
  }
}

// One tile (tm, tn) of contraction slice z on the DMA-fed loop, by the
// whole workgroup (S::NW waves), with the Allocation at smem (S::kLdsBytes).
// p: the sgemm (for PAIR, output 1); p2: PAIR's output 2 (B2, C2, alpha2,
// beta2; the rest as p), ignored otherwise.  Ends with every transfer
// drained and the workgroup past a barrier, so smem may be reused at once.
template <int TM, int TN, int TK, int WM, int WN, bool AT, bool BT, int NST, int MODE, int OP = 0,
          bool PAIR = false, bool EDGES = false>
__device__ __forceinline__ void f32_dma_tile(const GemmArgs& p, const GemmArgs& p2, const F32DmaOut& o, int tm,
                                             int tn, int z, char* smem) {
  using S = F32DmaShape<TM, TN, TK, WM, WN, AT, BT, NST, PAIR>;
  using OA = typename S::OA;
  using OB = typename S::OB;
  constexpr int NA = OA::kBlocks, NB = OB::kBlocks, KG = TK / 8;
  static_assert(MODE != kDmaConsume || !BT, "the consumer epilogue stores rows of adjacent outputs");

  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int wm0 = (wave / S::NWN) * WM, wcol = (wave % S::NWN) * WN;
  const int half = PAIR ? wcol / TN : 0;  // which output this wave's columns belong to
  const int wn0 = wcol - half * TN;
  const int splits = MODE == kDmaSplit ? o.splits : 1;
  // The tile's own corner, and the corner it computes from: with EDGES, a
  // tile that would cross the edge is moved inward; without, every tile is
  // whole and the two are the same (no masks in the epilogue).
  const int64_t m_own = (int64_t)tm * TM, n_own = (int64_t)tn * TN;
  const int64_t m0 = EDGES && m_own + TM > p.m ? p.m - TM : m_own;
  const int64_t n0 = EDGES && n_own + TN > p.n ? p.n - TN : n_own;
  const int slabs_all = p.k / TK;
  const int per = (slabs_all + splits - 1) / splits;
  const int sbeg = z * per, slabs = (slabs_all - sbeg < per ? slabs_all - sbeg : per);
  const uint32_t lds0 = lds_addr(smem);

  const int64_t lda4 = p.lda * 4, ldb4 = p.ldb * 4, ldb24 = p2.ldb * 4;
  const char* abase = reinterpret_cast<const char*>(p.A);
  const uint32_t aoff[2] = {OA::lane_off(lane, 0, lda4), OA::lane_off(lane, 1, lda4)};
  const uint32_t boff[2][2] = {{OB::lane_off(lane, 0, ldb4), OB::lane_off(lane, 1, ldb4)},
                               {OB::lane_off(lane, 0, ldb24), OB::lane_off(lane, 1, ldb24)}};
  auto dma_slab = [&](int slab, int st) {
    const int64_t k0 = (int64_t)(sbeg + slab) * TK;
    const uint32_t la = lds0 + st * S::kStage + wave * S::QA * 1024;
    const uint32_t lb = lds0 + st * S::kStage + OA::kBytes + wave * S::QB * 1024;
#pragma unroll
    for (int j = 0; j < S::QA; ++j)
      dma16(la + j * 1024, abase + OA::base(wave * S::QA + j, m0, k0, p.lda) * 4, aoff[j & 1]);
#pragma unroll
    for (int j = 0; j < S::QB; ++j) {
      const int q = wave * S::QB + j, h = PAIR ? q / OB::kDma : 0, qq = q - h * OB::kDma;
      const GemmArgs& pb = h ? p2 : p;
      dma16(lb + j * 1024, reinterpret_cast<const char*>(pb.B) + OB::base(qq, n0, k0, pb.ldb) * 4, boff[h][qq & 1]);
    }
  };

  int foff[KG];
#pragma unroll
  for (int g = 0; g < KG; ++g) foff[g] = OA::Rows::frag(lane, g);
  const int bstage = OA::kBytes + half * OB::kBytes;

  f32x16 acc[NA][NB];
  zero_acc(acc);
  typename OA::Frag fa[2][OA::kFrags];
  typename OB::Frag fb[2][OB::kFrags];
  auto read = [&](int buf, const char* st, int g) {
#pragma unroll
    for (int j = 0; j < OB::kFrags; ++j) fb[buf][j] = OB::frag(st + bstage, j, g, wn0, lane, foff[g]);
#pragma unroll
    for (int j = 0; j < OA::kFrags; ++j) fa[buf][j] = OA::frag(st, j, g, wm0, lane, foff[g]);
  };
  auto mfma = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(OA::pick(fa[buf], a, q), OB::pick(fb[buf], b, q),
                                                           acc[a][b], 0, 0, 0);
  };

  if (slabs > 0) {
#pragma unroll
    for (int i = 0; i < NST - 1; ++i) dma_slab(i < slabs ? i : slabs - 1, i);
    dma_wait_barrier<(NST - 2) * S::Q>();
    read(0, smem, 0);
    dma_slab(NST - 1 < slabs ? NST - 1 : slabs - 1, NST - 1);
  }
  int st = 0;
  for (int s = 0; s < slabs; ++s) {
    const char* cur = smem + st * S::kStage;
#pragma unroll
    for (int g = 0; g + 1 < KG; ++g) {
      read((g + 1) & 1, cur, g + 1);
      __builtin_amdgcn_sched_barrier(0);
      mfma(g & 1);
    }
    // Slab s + 1 has landed everywhere and slab s is no longer read:
    // request slab s + NST into its stage (the last slab again past the
    // end, which keeps the wait counts exact) and read slab s + 1's first
    // group under the last group's MFMAs.
    const int nst = st + 1 == NST ? 0 : st + 1;
    dma_wait_barrier<(NST - 2) * S::Q>();
    read(0, smem + nst * S::kStage, 0);
    dma_slab(s + NST < slabs ? s + NST : slabs - 1, st);
    __builtin_amdgcn_sched_barrier(0);
    mfma(1);
    st = nst;
  }
  // No transfer may still be writing LDS when the workgroup ends.
  dma_wait_barrier<0>();

  dma_epilogue<OA, OB, BT, MODE, OP, EDGES>(half ? p2 : p, o, acc, m0, n0, m_own, n_own, wm0, wn0, lane, z);
}

// One launch: a workgroup per tile and contraction slice (slice-major, so
// co-resident workgroups share a slice), XCD-aware tile order.
template <int TM, int TN, int TK, int WM, int WN, bool AT, bool BT, int NST, int MODE, int OP = 0,
          bool PAIR = false, bool EDGES = false>
__global__ void __launch_bounds__((F32DmaShape<TM, TN, TK, WM, WN, AT, BT, NST, PAIR>::NW * kWave))
    __attribute__((amdgpu_waves_per_eu(1, (F32DmaShape<TM, TN, TK, WM, WN, AT, BT, NST, PAIR>::kMaxWaves))))
    sgemm_f32_dma(GemmArgs p, GemmArgs p2, F32DmaOut o) {
  extern __shared__ __align__(16) char smem[];
  const int tiles = p.tiles_m * p.tiles_n;
  const int z = blockIdx.x / tiles;
  int tm, tn;
  tile_coords(p.tiles_m, p.tiles_n, blockIdx.x - z * tiles, tm, tn);
  f32_dma_tile<TM, TN, TK, WM, WN, AT, BT, NST, MODE, OP, PAIR, EDGES>(p, p2, o, tm, tn, z, smem);
}

// True when the DMA-fed loop covers the problem in whole tiles: m, n and k
// multiples of the tile (k of splits * TK), every operand and the output
// 16-byte aligned with leading dimensions that are multiples of 4.
template <int TM, int TN, int TK>
inline bool f32_dma_fits(const GemmArgs& a, const void* out, int64_t ldo, int splits) {
  return a.vec_a && a.vec_b && a.m > 0 && a.n > 0 && a.k > 0 && a.m % TM == 0 && a.n % TN == 0 &&
         a.k % (TK * splits) == 0 && ldo % 4 == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0;
}

// True when the DMA-fed loop covers the problem with edge tiles moved
// inward (see the top of this file): at least one tile each way, n a
// multiple of 4, k a multiple of the slab, alignment as f32_dma_fits.
template <int TM, int TN, int TK>
inline bool f32_dma_fits_edges(const GemmArgs& a, const void* out, int64_t ldo) {
  return a.vec_a && a.vec_b && a.m >= TM && a.n >= TN && a.n % 4 == 0 && a.k > 0 && a.k % TK == 0 &&
         ldo % 4 == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0;
}

}  // namespace hpvm
