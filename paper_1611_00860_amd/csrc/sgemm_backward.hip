// Backward pass of the sgemm node: C_out = alpha A B + beta C_in.
//
// dA = alpha G B^T reuses the MFMA main loop with B read in transposed form
// and folds the scalar gradient dalpha = <A, G B^T> into its epilogue (A is
// read once more, tile by tile, where dA is written).  dB = alpha A^T G is a
// plain launch of the main loop with A read in transposed form.  One
// element-wise pass writes dC_in = beta G and the partial sums of
// dbeta = <G, C_in>; a single workgroup then reduces the partials.  Every
// reduction is FP32 with a fixed order, so results repeat bit for bit.
//
// FP32 whole-tile problems can instead run both GEMMs on the DMA-fed loop
// (mfma_f32_dma.hpp) with the contraction split into slices: dA and dB have
// few outputs next to their long contractions (m x k and k x n against n and
// m), so big tiles alone would leave most CUs idle.  Each slice writes its
// raw partial tile to the workspace; one pass then sums the slices in order,
// scales by alpha and forms dalpha's partials.  When both gradients are
// wanted, their slices run in one launch and their sums with grad_c in
// another.
//
// Staged (BF16, bf16x3) entries convert everything first, in one launch: a
// single pass over G writes its bfloat16 planes for both products together
// with dC_in and dbeta's partials, beside B's and A's conversions; both
// products then run in one launch when the entry has the paired kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "device_common.hpp"
#include "hpvm_sgemm.h"
#include "internal.hpp"
#include "mfma_bf16.hpp"
#include "mfma_bf16_dma.hpp"
#include "mfma_f32.hpp"
#include "mfma_f32_dma.hpp"

namespace hpvm {

// dA tile: acc = (G B^T) tile; dA = alpha acc; partial = sum A .* acc.
// p: A = G (m x n_g), B = B (read transposed), m = m, n = k, k = n.
template <int TM, int TN, int TK, int WM, int WN, int PREC>
__global__ void __launch_bounds__((TM / WM) * (TN / WN) * kWave)
    sgemm_grad_a(GemmArgs p, const float* __restrict__ Aorig, int64_t lda, float* __restrict__ partial) {
  extern __shared__ __align__(16) char smem[];
  int tm, tn;
  tile_coords(p.tiles_m, p.tiles_n, blockIdx.x, tm, tn);
  constexpr int BM = WM / 32, BN = WN / 32;
  f32x16 acc[BM][BN];
  if constexpr (PREC == HPVM_PREC_FP32)
    f32_mainloop<TM, TN, TK, WM, WN, false, true>(p, tm * TM, tn * TN, reinterpret_cast<float*>(smem), acc);
  else
    bf16_mainloop<TM, TN, TK, WM, WN, false, true, PREC == HPVM_PREC_BF16X3>(p, tm * TM, tn * TN, smem, acc);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int row0 = tm * TM + (wave / (TN / WN)) * WM;
  const int col0 = tn * TN + (wave % (TN / WN)) * WN;
  // Each group of 4 rows loads its elements of A before storing its dA
  // values (a load after a possibly aliasing store would wait for a full
  // memory round trip, element by element).
  float part = 0.0f;
#pragma unroll
  for (int bi = 0; bi < BM; ++bi)
#pragma unroll
    for (int bj = 0; bj < BN; ++bj) {
      const int j = col0 + 32 * bj + acc_col(lane);
      if (j >= p.n) continue;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        float a[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int i = row0 + 32 * bi + acc_row(4 * g + t, lane);
          a[t] = i < p.m ? Aorig[(int64_t)i * lda + j] : 0.0f;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int i = row0 + 32 * bi + acc_row(4 * g + t, lane);
          if (i < p.m) {
            const float v = acc[bi][bj][4 * g + t];
            if (p.C) p.C[(int64_t)i * p.ldc + j] = p.alpha * v;
            part = fmaf(a[t], v, part);
          }
        }
      }
    }
  const float s = block_sum(part, reinterpret_cast<float*>(smem));
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

constexpr int kElemThreads = 256;
constexpr int kElemBlocks = 1024;

// dC_in = beta G (zeros when beta == 0) and per-block partials of <G, C_in>
// (Cin is read only for partial).  Rows are dealt to the job's blocks in
// turn; a block's threads walk a row in 16-byte units when every matrix it
// touches allows them (vec), one element at a time otherwise.  The
// element-to-thread assignment depends only on m, n and the block count, so
// the partials repeat bit for bit.
struct GradCJob {
  const float* G;
  int64_t ldg;
  const float* Cin;
  int64_t ldci;
  float* dCin;
  int64_t lddci, m, n;
  float beta;
  float* partial;
  int32_t vec;
  int64_t blocks;
};

__device__ __forceinline__ void grad_c_block(const GradCJob& jb, int64_t block, float* red) {
  const float* __restrict__ G = jb.G;
  const float* __restrict__ Cin = jb.Cin;
  float* __restrict__ dCin = jb.dCin;
  float* __restrict__ partial = jb.partial;
  const int64_t ldg = jb.ldg, ldci = jb.ldci, lddci = jb.lddci, m = jb.m, n = jb.n;
  const float beta = jb.beta;
  float part = 0.0f;
  const int64_t n4 = jb.vec ? n / 4 : 0;
  for (int64_t i = block; i < m; i += jb.blocks) {
    const float* g = G + i * ldg;
    const float* c = partial ? Cin + i * ldci : nullptr;
    float* d = dCin ? dCin + i * lddci : nullptr;
    int64_t q = threadIdx.x;
    // Four units per step, all loads ahead of the stores so that they overlap;
    // the sum still takes this thread's units in ascending order.
    for (; q + 3 * (int64_t)blockDim.x < n4; q += 4 * (int64_t)blockDim.x) {
      f32x4 gv[4], cv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        gv[u] = reinterpret_cast<const f32x4*>(g)[q + u * blockDim.x];
        if (c) cv[u] = reinterpret_cast<const f32x4*>(c)[q + u * blockDim.x];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (d)
          reinterpret_cast<f32x4*>(d)[q + u * blockDim.x] =
              (beta == 0.0f) ? f32x4{0.0f, 0.0f, 0.0f, 0.0f} : beta * gv[u];
        if (c) {
          part = fmaf(gv[u][0], cv[u][0], part);
          part = fmaf(gv[u][1], cv[u][1], part);
          part = fmaf(gv[u][2], cv[u][2], part);
          part = fmaf(gv[u][3], cv[u][3], part);
        }
      }
    }
    for (; q < n4; q += blockDim.x) {
      const f32x4 gv = reinterpret_cast<const f32x4*>(g)[q];
      if (d) reinterpret_cast<f32x4*>(d)[q] = (beta == 0.0f) ? f32x4{0.0f, 0.0f, 0.0f, 0.0f} : beta * gv;
      if (c) {
        const f32x4 cv = reinterpret_cast<const f32x4*>(c)[q];
        part = fmaf(gv[0], cv[0], part);
        part = fmaf(gv[1], cv[1], part);
        part = fmaf(gv[2], cv[2], part);
        part = fmaf(gv[3], cv[3], part);
      }
    }
    for (int64_t j = 4 * n4 + threadIdx.x; j < n; j += blockDim.x) {
      const float gv = g[j];
      if (d) d[j] = (beta == 0.0f) ? 0.0f : beta * gv;
      if (c) part = fmaf(gv, c[j], part);
    }
  }
  if (!partial) return;
  const float s = block_sum(part, red);
  if (threadIdx.x == 0) partial[block] = s;
}

__global__ void __launch_bounds__(kElemThreads) sgemm_grad_c(GradCJob j) {
  __shared__ float red[kElemThreads / kWave];
  grad_c_block(j, blockIdx.x, red);
}

// Final fixed-order reduction of both partial arrays.
__global__ void __launch_bounds__(kElemThreads)
    sgemm_grad_finish(const float* __restrict__ pa, int32_t na, const float* __restrict__ pb, int32_t nb,
                      float* dalpha, float* dbeta) {
  __shared__ float red[kElemThreads / kWave];
  // Each thread adds its partials in ascending order, loading four ahead.
  auto strided = [](const float* p, int count) {
    float s = 0.0f;
    int t = threadIdx.x;
    for (; t + 3 * (int)blockDim.x < count; t += 4 * (int)blockDim.x) {
      float v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = p[t + u * blockDim.x];
#pragma unroll
      for (int u = 0; u < 4; ++u) s += v[u];
    }
    for (; t < count; t += blockDim.x) s += p[t];
    return s;
  };
  const float a = strided(pa, na), b = strided(pb, nb);
  const float sa = block_sum(a, red);
  const float sb = block_sum(b, red);
  if (threadIdx.x == 0) {
    if (dalpha) *dalpha = sa;
    if (dbeta) *dbeta = sb;
  }
}

// Sum of one gradient's slice partials part[z] (rows x cols, contiguous), in
// slice order: v = part[0] + part[1] + ...; out <- alpha v when out is
// given; with aorig, this block's partial of <aorig, v> into dpart.  Float4
// units are dealt to the job's threads in turn, so everything repeats bit
// for bit.  cols, ldo and ldao are multiples of 4 and the arrays 16-byte
// aligned.
struct SumJob {
  const float* part;
  int32_t splits;
  int64_t rows, cols;
  float alpha;
  float* out;
  int64_t ldo;
  const float* aorig;
  int64_t ldao;
  float* dpart;
  int64_t blocks;
};

__device__ __forceinline__ void split_sum_block(const SumJob& jb, int64_t block, float* red) {
  const float* __restrict__ part = jb.part;
  float* __restrict__ out = jb.out;
  const float* __restrict__ aorig = jb.aorig;
  const int64_t cols = jb.cols, c4 = cols / 4, units = jb.rows * c4, plane = jb.rows * cols;
  const int64_t stride = jb.blocks * blockDim.x;
  float sum = 0.0f;
  for (int64_t u = block * blockDim.x + threadIdx.x; u < units; u += stride) {
    const int64_t i = u / c4, j = (u - i * c4) * 4;
    f32x4 v = *reinterpret_cast<const f32x4*>(part + i * cols + j);
    for (int z = 1; z < jb.splits; ++z) v += *reinterpret_cast<const f32x4*>(part + z * plane + i * cols + j);
    if (out) *reinterpret_cast<f32x4*>(out + i * jb.ldo + j) = jb.alpha * v;
    if (jb.dpart) {
      const f32x4 a = *reinterpret_cast<const f32x4*>(aorig + i * jb.ldao + j);
      sum = fmaf(a[0], v[0], sum);
      sum = fmaf(a[1], v[1], sum);
      sum = fmaf(a[2], v[2], sum);
      sum = fmaf(a[3], v[3], sum);
    }
  }
  if (!jb.dpart) return;
  const float t = block_sum(sum, red);
  if (threadIdx.x == 0) jb.dpart[block] = t;
}

__global__ void __launch_bounds__(kElemThreads) sgemm_split_sum(SumJob j) {
  __shared__ float red[kElemThreads / kWave];
  split_sum_block(j, blockIdx.x, red);
}

// The element-wise passes after both gradients' slices: dA's slice sum,
// dB's, and grad_c, in one launch of three block ranges (a range with no
// blocks is absent) so that the passes overlap.
__global__ void __launch_bounds__(kElemThreads) sgemm_grad_tail(SumJob a, SumJob b, GradCJob c) {
  __shared__ float red[kElemThreads / kWave];
  int64_t blk = blockIdx.x;
  if (blk < a.blocks) {
    split_sum_block(a, blk, red);
    return;
  }
  blk -= a.blocks;
  if (blk < b.blocks) split_sum_block(b, blk, red);
  else grad_c_block(c, blk - b.blocks, red);
}

namespace {

// One candidate tile of the backward.  Fused entries run dA through
// sgemm_grad_a and dB through the fused menu entry's launch; staged entries
// run both through the staged lowering (one conversion launch into the
// workspace, with the transposition of each operand folded into it).
struct BwdEntry {
  hpvm_tile tile;
  int32_t prec;
  int32_t threads;
  int64_t lds;
  void (*grad_a)(GemmArgs, const float*, int64_t, float*);  // null for staged entries
  bool dma = false;  // split-contraction DMA-fed entry
  // DMA entries: the entry for what the DMA-fed loop does not cover (FP32:
  // the passes that are not whole aligned tiles; BF16: the whole call).
  int fallback = 1;
};

template <int TM, int TN, int TK, int WM, int WN, int PREC>
constexpr BwdEntry fused_entry() {
  constexpr int64_t lds = PREC == HPVM_PREC_FP32
                              ? F32Tile<TM, TN, TK, WM, WN, false, true>::kLdsBytes
                              : Bf16TileShape<TM, TN, TK, WM, WN, PREC == HPVM_PREC_BF16X3>::kLdsBytes;
  return BwdEntry{{TM, TN, TK, WM, WN, 2}, PREC, (TM / WM) * (TN / WN) * kWave, lds,
                  &sgemm_grad_a<TM, TN, TK, WM, WN, PREC>};
}
constexpr BwdEntry staged_entry(int tm, int tn, int tk, int wm, int wn, int prec) {
  return BwdEntry{{tm, tn, tk, wm, wn, 3}, prec, 0, 0, nullptr};
}

// The DMA-fed FP32 backward: 256 x 256 x 32 tiles of 8 waves (64 x 128 each),
// two LDS stages.  dA reads G (k contiguous) and B transposed (k
// contiguous); dB reads A transposed (m contiguous, two adjacent rows per
// fragment) and G (n contiguous, four adjacent columns).
constexpr int kDmaTile = 256, kDmaK = 32, kDmaWM = 64, kDmaWN = 128, kDmaStages = 2;
using DmaA = F32DmaShape<kDmaTile, kDmaTile, kDmaK, kDmaWM, kDmaWN, false, true, kDmaStages>;
using DmaB = F32DmaShape<kDmaTile, kDmaTile, kDmaK, kDmaWM, kDmaWN, true, false, kDmaStages>;
constexpr BwdEntry dma_entry() {
  BwdEntry e{{kDmaTile, kDmaTile, kDmaK, kDmaWM, kDmaWN, kDmaStages}, HPVM_PREC_FP32, DmaA::NW * kWave,
             DmaA::kLdsBytes > DmaB::kLdsBytes ? DmaA::kLdsBytes : DmaB::kLdsBytes,
             &sgemm_grad_a<128, 128, 32, 64, 64, HPVM_PREC_FP32>};
  e.dma = true;
  return e;
}
// The same tiles with BF16 products converted from the FP32 slabs in the
// fragment reads (mfma_bf16_dma.hpp): no conversion pass at all.  A call it
// does not cover in whole aligned tiles takes the staged entry `fallback`.
using Bf16DmaA = Bf16SrcShape<kDmaTile, kDmaTile, kDmaK, kDmaWM, kDmaWN, false, true, kDmaStages>;
using Bf16DmaB = Bf16SrcShape<kDmaTile, kDmaTile, kDmaK, kDmaWM, kDmaWN, true, false, kDmaStages>;
constexpr BwdEntry bf16_dma_entry(int fallback) {
  BwdEntry e{{kDmaTile, kDmaTile, kDmaK, kDmaWM, kDmaWN, kDmaStages}, HPVM_PREC_BF16, Bf16DmaA::NW * kWave,
             Bf16DmaA::kLdsBytes > Bf16DmaB::kLdsBytes ? Bf16DmaA::kLdsBytes : Bf16DmaB::kLdsBytes, nullptr};
  e.dma = true;
  e.fallback = fallback;
  return e;
}

// Per precision, in the order the built-in choice tries them.  kBwd[1] is
// the DMA entry's fallback for problems that are not whole tiles.
constexpr BwdEntry kBwd[] = {
    dma_entry(),
    fused_entry<128, 128, 32, 64, 64, HPVM_PREC_FP32>(),
    fused_entry<128, 128, 16, 64, 64, HPVM_PREC_FP32>(),
    fused_entry<128, 64, 16, 64, 32, HPVM_PREC_FP32>(),
    fused_entry<64, 128, 16, 32, 64, HPVM_PREC_FP32>(),
    fused_entry<64, 64, 16, 32, 32, HPVM_PREC_FP32>(),
    bf16_dma_entry(7),
    staged_entry(128, 128, 64, 64, 32, HPVM_PREC_BF16),
    staged_entry(128, 128, 64, 64, 64, HPVM_PREC_BF16),
    staged_entry(256, 256, 64, 128, 64, HPVM_PREC_BF16),
    staged_entry(256, 128, 64, 128, 64, HPVM_PREC_BF16),
    fused_entry<128, 128, 32, 64, 64, HPVM_PREC_BF16>(),
    fused_entry<64, 64, 32, 32, 32, HPVM_PREC_BF16>(),
    staged_entry(256, 256, 32, 128, 64, HPVM_PREC_BF16X3),
    staged_entry(128, 128, 64, 64, 32, HPVM_PREC_BF16X3),
    staged_entry(128, 128, 64, 64, 64, HPVM_PREC_BF16X3),
    staged_entry(256, 128, 32, 128, 64, HPVM_PREC_BF16X3),
    fused_entry<128, 128, 32, 64, 64, HPVM_PREC_BF16X3>(),
    fused_entry<64, 64, 32, 32, 32, HPVM_PREC_BF16X3>(),
};
constexpr int kNumBwd = sizeof(kBwd) / sizeof(kBwd[0]);
static_assert(kBwd[6].dma && kBwd[6].prec == HPVM_PREC_BF16 && !kBwd[7].grad_a && kBwd[7].prec == HPVM_PREC_BF16,
              "the BF16 DMA entry falls back to the staged entry after it");

int64_t tiles_for(const hpvm_tile& t, int64_t rows, int64_t cols) {
  return ((rows + t.tile_m - 1) / t.tile_m) * ((cols + t.tile_n - 1) / t.tile_n);
}

const BwdEntry* find_bwd(int32_t prec, const hpvm_tile& t) {
  for (int i = 0; i < kNumBwd; ++i)
    if (kBwd[i].prec == prec && same_tile(kBwd[i].tile, t)) return &kBwd[i];
  return nullptr;
}

constexpr int64_t kTargetTiles = 256;

// Contraction slices for a DMA-fed gradient with `tiles` output tiles:
// doubled while the workgroups would not cover 256 CUs, each slice staying a
// whole number of slabs and at least 256 deep.  0 when the gradient is not
// whole tiles (by size; alignment is checked at launch).
int dma_splits(int64_t rows, int64_t cols, int64_t contraction) {
  if (rows <= 0 || cols <= 0 || contraction <= 0 || rows % kDmaTile || cols % kDmaTile ||
      contraction % kDmaK)
    return 0;
  const int64_t tiles = (rows / kDmaTile) * (cols / kDmaTile);
  int s = 1;
  while (s < 16 && tiles * s < kTargetTiles && contraction % (2 * s * kDmaK) == 0 && contraction / (2 * s) >= 256)
    s *= 2;
  return s;
}

// Slices per gradient when both gradients run in one launch (both whole
// tiles): doubled while the two together would not cover 256 CUs, under the
// same conditions as dma_splits on both contractions.  0 otherwise.
int pair_splits(int64_t m, int64_t n, int64_t k) {
  if (!dma_splits(m, k, n) || !dma_splits(k, n, m)) return 0;
  const int64_t tiles = (m / kDmaTile) * (k / kDmaTile) + (k / kDmaTile) * (n / kDmaTile);
  int s = 1;
  while (s < 16 && tiles * s < kTargetTiles && n % (2 * s * kDmaK) == 0 && n / (2 * s) >= 256 &&
         m % (2 * s * kDmaK) == 0 && m / (2 * s) >= 256)
    s *= 2;
  return s;
}

struct DmaPlan {
  int sa = 0, sb = 0;  // slices of dA (m x k over n) and dB (k x n over m); 0 = not DMA-fed
  int sp = 0;          // slices of each when both run in one launch
};
DmaPlan dma_plan(const BwdEntry* e, int64_t m, int64_t n, int64_t k) {
  DmaPlan d;
  if (e->dma) {
    d.sa = dma_splits(m, k, n);
    d.sb = dma_splits(k, n, m);
    d.sp = pair_splits(m, n, k);
  }
  return d;
}
int64_t split_sum_blocks(int64_t rows, int64_t cols) {
  return std::max<int64_t>(1, std::min<int64_t>(kElemBlocks, (rows * cols / 4 + kElemThreads - 1) / kElemThreads));
}

// Built-in choice: the DMA entry when dA is whole tiles, else the first
// entry giving at least one tile per CU of a 256-CU part, else the one
// giving the most tiles -- counting dA's tiles, plus dB's for a staged entry
// that runs both products in one launch.
int64_t launch_tiles(const BwdEntry& e, int64_t m, int64_t n, int64_t k) {
  int64_t tiles = tiles_for(e.tile, m, k);
  if (!e.grad_a) {
    const MfmaEntry* me = find_menu_entry(e.prec, e.tile);
    if (me && me->launch_staged_pair) tiles += tiles_for(e.tile, k, n);
  }
  return tiles;
}

const BwdEntry* pick(int32_t prec, int64_t m, int64_t n, int64_t k) {
  hpvm_tile tuned;
  if (tuned_backward_tile(prec, m, n, k, &tuned)) {
    const BwdEntry* e = find_bwd(prec, tuned);
    if (e) return e;
  }
  const BwdEntry* most = nullptr;
  const bool staged_ok = staged_k_ok(n) && staged_k_ok(m);  // the dA and dB contractions
  for (int i = 0; i < kNumBwd; ++i) {
    if (kBwd[i].prec != prec) continue;
    if (kBwd[i].dma) {
      // FP32 only: the BF16 DMA entry reads FP32 slabs where the staged
      // products read bfloat16 planes, twice the bytes (4096 x 4096 x 1024:
      // 0.181 ms against 0.131 for the staged 128 x 128 x 64 tile).
      if (prec == HPVM_PREC_FP32 && dma_splits(m, k, n)) return &kBwd[i];
      continue;
    }
    if (!kBwd[i].grad_a && !staged_ok) continue;
    const int64_t tiles = launch_tiles(kBwd[i], m, n, k);
    if (tiles >= kTargetTiles) return &kBwd[i];
    if (!most || tiles > launch_tiles(*most, m, n, k)) most = &kBwd[i];
  }
  return most;
}

int64_t elem_blocks(int64_t m, int64_t n) {
  return std::max<int64_t>(1, std::min<int64_t>(kElemBlocks, (m * n + kElemThreads - 1) / kElemThreads));
}

// Workspace: [dA partials][element-wise partials][staging region], each
// 256-byte aligned.  A DMA entry's dA and dB passes run one after the other
// on the stream and share the region; a staged entry keeps the planes of
// both products there at once, since one pass over G writes G's planes for
// both (each plane pair hi, lo adjacent):
//   [G: round256(m) x round64(n)][G^T: round256(n) x round64(m)]
//   [B: round256(k) x round64(n)][A^T: round256(k) x round64(m)]
struct BwdLayout {
  int64_t na, nb, ng;  // dalpha partials, grad_c partials, partials of the pass over G
  int64_t pb_off, stage_off, total;
};

// bfloat16 planes of a staged backward (see BwdLayout) from the staging
// region: ga = the dA product's (G, B), gb = the dB product's (A^T, G^T).
struct BwdPlanes {
  uint16_t *gh, *gl, *th, *tl, *bh, *bl, *ah, *al;
};
int64_t bwd_plane_elems(int64_t m, int64_t n, int64_t k, int64_t* g, int64_t* gt, int64_t* b, int64_t* a) {
  *g = staged_rows_pad(m) * staged_k_pad(n);
  *gt = staged_rows_pad(n) * staged_k_pad(m);
  *b = staged_rows_pad(k) * staged_k_pad(n);
  *a = staged_rows_pad(k) * staged_k_pad(m);
  return *g + *gt + *b + *a;
}
BwdPlanes bwd_planes(int32_t prec, void* stage, int64_t m, int64_t n, int64_t k) {
  const bool x3 = prec == HPVM_PREC_BF16X3;
  int64_t g, gt, b, a;
  bwd_plane_elems(m, n, k, &g, &gt, &b, &a);
  uint16_t* p = reinterpret_cast<uint16_t*>(stage);
  BwdPlanes P;
  auto take = [&](int64_t elems, uint16_t** hi, uint16_t** lo) {
    *hi = p;
    p += elems;
    *lo = x3 ? p : nullptr;
    if (x3) p += elems;
  };
  take(g, &P.gh, &P.gl);
  take(gt, &P.th, &P.tl);
  take(b, &P.bh, &P.bl);
  take(a, &P.ah, &P.al);
  return P;
}

// A DMA entry sizes for all of its paths: the slice partials (dA's and dB's
// passes share the region when they run one after the other and split it
// when they run in one launch) and the larger of its dalpha partial counts.
BwdLayout bwd_layout(const BwdEntry* e, int64_t m, int64_t n, int64_t k) {
  auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
  BwdLayout L;
  L.na = (m > 0 && k > 0) ? tiles_for(e->dma ? kBwd[e->fallback].tile : e->tile, m, k) : 0;
  const DmaPlan d = dma_plan(e, m, n, k);
  if (d.sa) L.na = std::max(L.na, split_sum_blocks(m, k));
  L.nb = elem_blocks(m, n);
  L.ng = (!e->grad_a && !e->dma && m > 0 && n > 0) ? stage_gradient_blocks(m, n) : 0;
  L.pb_off = up(L.na * 4);
  L.stage_off = L.pb_off + up(std::max(L.nb, L.ng) * 4);
  int64_t stage = 0;
  if (!e->grad_a && !e->dma) {
    int64_t g, gt, b, a;
    stage = (e->prec == HPVM_PREC_BF16X3 ? 2 : 1) * 2 * bwd_plane_elems(m, n, k, &g, &gt, &b, &a);
  }
  if (e->dma) stage = 4 * std::max<int64_t>(std::max<int64_t>(d.sa * m * k, d.sb * k * n), d.sp * (m * k + k * n));
  L.total = L.stage_off + stage;
  // A call the BF16 DMA entry does not cover takes its fallback entry, in
  // the same workspace.
  if (e->dma && e->prec != HPVM_PREC_FP32) L.total = std::max(L.total, bwd_layout(&kBwd[e->fallback], m, n, k).total);
  return L;
}

// One gradient on the DMA-fed loop: `splits` contraction slices write their
// partial tiles to part ([splits][a.m][a.n]), then sgemm_split_sum adds
// them, writes out = alpha * sum (when out is given) and dalpha's partials
// (when aorig is given).
template <int PREC, bool AT, bool BT>
hipError_t launch_split(const GemmArgs& args, int splits, float* part, float* out, int64_t ldo, const float* aorig,
                        int64_t ldao, float* dpart, hipStream_t s) {
  using S = F32DmaShape<kDmaTile, kDmaTile, kDmaK, kDmaWM, kDmaWN, AT, BT, kDmaStages>;
  const void* fn = PREC == HPVM_PREC_FP32
                       ? reinterpret_cast<const void*>(
                             &sgemm_f32_dma<kDmaTile, kDmaTile, kDmaK, kDmaWM, kDmaWN, AT, BT, kDmaStages, kDmaSplit>)
                       : reinterpret_cast<const void*>(&sgemm_bf16src_dma<kDmaTile, kDmaTile, kDmaK, kDmaWM, kDmaWN,
                                                                          AT, BT, kDmaStages, false, kDmaSplit>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)S::kLdsBytes);
  if (e != hipSuccess) return e;
  GemmArgs a = args;
  a.C = part;
  a.ldc = a.n;
  a.tiles_m = a.m / kDmaTile;
  a.tiles_n = a.n / kDmaTile;
  GemmArgs unused = a;
  F32DmaOut o{};
  o.splits = splits;
  int32_t sp = splits;
  void* kargs_f32[] = {&a, &unused, &o};
  void* kargs_bf16[] = {&a, &o};
  e = hipLaunchKernel(fn, dim3((unsigned)(a.tiles_m * a.tiles_n * splits)), dim3(S::NW * kWave),
                      PREC == HPVM_PREC_FP32 ? kargs_f32 : kargs_bf16, (size_t)S::kLdsBytes, s);
  if (e != hipSuccess || (!out && !dpart)) return e;
  SumJob j{part, sp, a.m, a.n, args.alpha, out, ldo, aorig, ldao, dpart, split_sum_blocks(a.m, a.n)};
  void* sargs[] = {&j};
  return hipLaunchKernel(reinterpret_cast<const void*>(&sgemm_split_sum), dim3((unsigned)j.blocks),
                         dim3(kElemThreads), sargs, 0, s);
}

// Both gradients' contraction slices in one launch: the first
// tiles(pa) * oa.splits workgroups run dA's (G, B transposed), the rest dB's
// (A transposed, G), each writing raw slice partials like launch_split.
constexpr int64_t kDmaPairLds = DmaA::kLdsBytes > DmaB::kLdsBytes ? DmaA::kLdsBytes : DmaB::kLdsBytes;
constexpr int kDmaPairWaves = DmaA::kMaxWaves < DmaB::kMaxWaves ? DmaA::kMaxWaves : DmaB::kMaxWaves;
static_assert(DmaA::NW == DmaB::NW, "one workgroup size");

__global__ void __launch_bounds__(DmaA::NW * kWave) __attribute__((amdgpu_waves_per_eu(1, kDmaPairWaves)))
    sgemm_grad_pair_dma(GemmArgs pa, F32DmaOut oa, GemmArgs pb, F32DmaOut ob) {
  extern __shared__ __align__(16) char smem[];
  const int ta = pa.tiles_m * pa.tiles_n, na = ta * oa.splits;
  int t = blockIdx.x, tm, tn;
  if (t < na) {
    const int z = t / ta;
    tile_coords(pa.tiles_m, pa.tiles_n, t - z * ta, tm, tn);
    f32_dma_tile<kDmaTile, kDmaTile, kDmaK, kDmaWM, kDmaWN, false, true, kDmaStages, kDmaSplit>(pa, pa, oa, tm, tn,
                                                                                               z, smem);
  } else {
    t -= na;
    const int tb = pb.tiles_m * pb.tiles_n, z = t / tb;
    tile_coords(pb.tiles_m, pb.tiles_n, t - z * tb, tm, tn);
    f32_dma_tile<kDmaTile, kDmaTile, kDmaK, kDmaWM, kDmaWN, true, false, kDmaStages, kDmaSplit>(pb, pb, ob, tm, tn,
                                                                                               z, smem);
  }
}

// The same with BF16 products (the FP32 slabs converted in the fragment
// reads).
constexpr int64_t kBf16DmaPairLds = Bf16DmaA::kLdsBytes > Bf16DmaB::kLdsBytes ? Bf16DmaA::kLdsBytes
                                                                                : Bf16DmaB::kLdsBytes;
constexpr int kBf16DmaPairWaves = Bf16DmaA::kMaxWaves < Bf16DmaB::kMaxWaves ? Bf16DmaA::kMaxWaves
                                                                             : Bf16DmaB::kMaxWaves;
static_assert(Bf16DmaA::NW == DmaA::NW && Bf16DmaB::NW == DmaA::NW, "one workgroup size");

__global__ void __launch_bounds__(Bf16DmaA::NW * kWave) __attribute__((amdgpu_waves_per_eu(1, kBf16DmaPairWaves)))
    sgemm_grad_pair_bf16src(GemmArgs pa, F32DmaOut oa, GemmArgs pb, F32DmaOut ob) {
  extern __shared__ __align__(16) char smem[];
  const int ta = pa.tiles_m * pa.tiles_n, na = ta * oa.splits;
  int t = blockIdx.x, tm, tn;
  if (t < na) {
    const int z = t / ta;
    tile_coords(pa.tiles_m, pa.tiles_n, t - z * ta, tm, tn);
    bf16src_dma_tile<kDmaTile, kDmaTile, kDmaK, kDmaWM, kDmaWN, false, true, kDmaStages, false, kDmaSplit, false,
                     kBf16SrcCvb<kDmaWM, kDmaWN, false>>(pa, oa, tm, tn, z, smem);
  } else {
    t -= na;
    const int tb = pb.tiles_m * pb.tiles_n, z = t / tb;
    tile_coords(pb.tiles_m, pb.tiles_n, t - z * tb, tm, tn);
    bf16src_dma_tile<kDmaTile, kDmaTile, kDmaK, kDmaWM, kDmaWN, true, false, kDmaStages, false, kDmaSplit, false,
                     kBf16SrcCvb<kDmaWM, kDmaWN, false>>(pb, ob, tm, tn, z, smem);
  }
}

// dA and dB with `splits` slices each in one launch (partials [splits][m][k]
// at part_a, [splits][k][n] at part_b), then one launch of both slice sums
// and the grad_c job gc (absent when gc.blocks == 0).
hipError_t launch_split_pair(int32_t prec, const GemmArgs& ga, const GemmArgs& gb, int splits, float* part_a,
                             float* part_b, float* dA, int64_t ldda, float* dB, int64_t lddb, const float* aorig,
                             int64_t ldao, float* dpart, GradCJob gc, hipStream_t s) {
  const bool f32 = prec == HPVM_PREC_FP32;
  const void* fn = f32 ? reinterpret_cast<const void*>(&sgemm_grad_pair_dma)
                       : reinterpret_cast<const void*>(&sgemm_grad_pair_bf16src);
  const int64_t lds = f32 ? kDmaPairLds : kBf16DmaPairLds;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  GemmArgs a = ga, b = gb;
  a.C = part_a;
  a.ldc = a.n;
  a.tiles_m = a.m / kDmaTile;
  a.tiles_n = a.n / kDmaTile;
  b.C = part_b;
  b.ldc = b.n;
  b.tiles_m = b.m / kDmaTile;
  b.tiles_n = b.n / kDmaTile;
  F32DmaOut oa{}, ob{};
  oa.splits = ob.splits = splits;
  void* kargs[] = {&a, &oa, &b, &ob};
  const int64_t wgs = ((int64_t)a.tiles_m * a.tiles_n + (int64_t)b.tiles_m * b.tiles_n) * splits;
  e = hipLaunchKernel(fn, dim3((unsigned)wgs), dim3(DmaA::NW * kWave), kargs, (size_t)lds, s);
  if (e != hipSuccess) return e;
  SumJob ja{part_a, splits, a.m, a.n, ga.alpha, dA, ldda, aorig, ldao, dpart,
            (dA || dpart) ? split_sum_blocks(a.m, a.n) : 0};
  SumJob jb{part_b, splits, b.m, b.n, gb.alpha, dB, lddb, nullptr, 0, nullptr, split_sum_blocks(b.m, b.n)};
  void* targs[] = {&ja, &jb, &gc};
  return hipLaunchKernel(reinterpret_cast<const void*>(&sgemm_grad_tail),
                         dim3((unsigned)(ja.blocks + jb.blocks + gc.blocks)), dim3(kElemThreads), targs, 0, s);
}

std::mutex g_tune_mu;
std::map<std::tuple<int32_t, int64_t, int64_t, int64_t>, hpvm_tile> g_tuned;

int resolve_bwd(int32_t prec, const hpvm_tile* tile, int64_t m, int64_t n, int64_t k, const BwdEntry** out,
                int argno) {
  if (prec < HPVM_PREC_FP32 || prec > HPVM_PREC_BF16X3)
    return set_error(HPVM_INVALID_ARG, "argument %d: unknown precision %d", argno - 1, prec);
  *out = tile ? find_bwd(prec, *tile) : pick(prec, m, n, k);
  if (!*out)
    return set_error(HPVM_UNSUPPORTED, "argument %d: tile not in the backward menu for precision %d", argno,
                     prec);
  if (!(*out)->grad_a && !(*out)->dma && !(staged_k_ok(n) && staged_k_ok(m)))
    return set_error(HPVM_UNSUPPORTED, "argument %d: m or n too deep a contraction for a staged tile", argno);
  return HPVM_OK;
}

}  // namespace

int tuned_backward_tile(int32_t prec, int64_t m, int64_t n, int64_t k, hpvm_tile* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(std::make_tuple(prec, m, n, k));
  if (it == g_tuned.end()) return 0;
  *out = it->second;
  return 1;
}

void record_backward_tile(int32_t prec, int64_t m, int64_t n, int64_t k, const hpvm_tile& t) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[std::make_tuple(prec, m, n, k)] = t;
}

}  // namespace hpvm

using namespace hpvm;

extern "C" {

int hpvm_sgemm_backward_menu(int32_t prec, hpvm_tile* out, int32_t capacity, int32_t* count) {
  if (prec < HPVM_PREC_FP32 || prec > HPVM_PREC_BF16X3)
    return set_error(HPVM_INVALID_ARG, "argument 1: unknown precision %d", prec);
  if (capacity < 0 || (capacity > 0 && !out))
    return set_error(HPVM_INVALID_ARG, "argument 3: bad capacity or NULL output");
  if (!count) return set_error(HPVM_INVALID_ARG, "argument 4: count is NULL");
  int n = 0;
  for (int i = 0; i < kNumBwd; ++i) {
    if (kBwd[i].prec != prec) continue;
    if (n < capacity) out[n] = kBwd[i].tile;
    ++n;
  }
  *count = n;
  return clear_error();
}

int hpvm_sgemm_backward_workspace_bytes(int64_t m, int64_t n, int64_t k, int32_t prec, const hpvm_tile* tile,
                                        int64_t* bytes) {
  if (m < 0 || n < 0 || k < 0) return set_error(HPVM_INVALID_ARG, "sizes must be >= 0");
  const BwdEntry* e;
  int rc = resolve_bwd(prec, tile, m, n, k, &e, 5);
  if (rc != HPVM_OK) return rc;
  if (!bytes) return set_error(HPVM_INVALID_ARG, "argument 6: bytes is NULL");
  *bytes = bwd_layout(e, m, n, k).total;
  return clear_error();
}

int hpvm_sgemm_backward(int64_t m, int64_t n, int64_t k, float alpha, float beta, const float* A, int64_t lda,
                        const float* B, int64_t ldb, const float* C_in, int64_t ldci, const float* G, int64_t ldg,
                        float* dA, int64_t ldda, float* dB, int64_t lddb, float* dC_in, int64_t lddci,
                        float* dalpha, float* dbeta, int32_t prec, const hpvm_tile* tile, void* workspace,
                        int64_t workspace_bytes, void* stream) {
  if (m < 0) return set_error(HPVM_INVALID_ARG, "argument 1: m = %lld < 0", (long long)m);
  if (n < 0) return set_error(HPVM_INVALID_ARG, "argument 2: n = %lld < 0", (long long)n);
  if (k < 0) return set_error(HPVM_INVALID_ARG, "argument 3: k = %lld < 0", (long long)k);
  if (m > INT32_MAX || n > INT32_MAX || k > INT32_MAX)
    return set_error(HPVM_UNSUPPORTED, "sizes above 2^31 - 1 are not supported");
  const bool mn = m > 0 && n > 0, mk = m > 0 && k > 0, kn = k > 0 && n > 0;
  const bool want_a = dA != nullptr || dalpha != nullptr;  // dalpha rides on dA's pass
  const bool run_a = want_a && mk && n > 0;
  const bool run_b = dB && kn && m > 0;
  if ((run_a || run_b) && !A) return set_error(HPVM_INVALID_ARG, "argument 6: A is NULL");
  if (lda < std::max<int64_t>(1, k)) return set_error(HPVM_INVALID_ARG, "argument 7: lda < max(1, k)");
  if (run_a && !B) return set_error(HPVM_INVALID_ARG, "argument 8: B is NULL");
  if (ldb < std::max<int64_t>(1, n)) return set_error(HPVM_INVALID_ARG, "argument 9: ldb < max(1, n)");
  if (dbeta && mn && !C_in) return set_error(HPVM_INVALID_ARG, "argument 10: C_in is NULL");
  if (ldci < std::max<int64_t>(1, n)) return set_error(HPVM_INVALID_ARG, "argument 11: ldci < max(1, n)");
  if (mn && !G && (want_a || dB || dC_in || dbeta)) return set_error(HPVM_INVALID_ARG, "argument 12: G is NULL");
  if (ldg < std::max<int64_t>(1, n)) return set_error(HPVM_INVALID_ARG, "argument 13: ldg < max(1, n)");
  if (ldda < std::max<int64_t>(1, k)) return set_error(HPVM_INVALID_ARG, "argument 15: ldda < max(1, k)");
  if (lddb < std::max<int64_t>(1, n)) return set_error(HPVM_INVALID_ARG, "argument 17: lddb < max(1, n)");
  if (lddci < std::max<int64_t>(1, n)) return set_error(HPVM_INVALID_ARG, "argument 19: lddci < max(1, n)");
  const BwdEntry* cfg;
  int rc = resolve_bwd(prec, tile, m, n, k, &cfg, 23);
  if (rc != HPVM_OK) return rc;
  // The BF16 DMA entry runs a call only when every pass it makes is whole,
  // aligned tiles; otherwise the whole call takes its staged fallback (the
  // workspace it asks for covers that entry too).
  const BwdLayout L0 = bwd_layout(cfg, m, n, k);
  if (cfg->dma && prec != HPVM_PREC_FP32) {
    const DmaPlan d = dma_plan(cfg, m, n, k);
    const bool ok_a = !run_a || (d.sa && vec16(G, ldg) && vec16(B, ldb) && (!dA || vec16(dA, ldda)) &&
                                 (!dalpha || vec16(A, lda)));
    const bool ok_b = !run_b || (d.sb && vec16(A, lda) && vec16(G, ldg) && vec16(dB, lddb));
    if (!ok_a || !ok_b) cfg = &kBwd[cfg->fallback];
  }
  BwdLayout L = bwd_layout(cfg, m, n, k);
  L.total = L0.total;
  const bool staged = cfg->grad_a == nullptr && !cfg->dma;
  const DmaPlan plan = dma_plan(cfg, m, n, k);
  const bool need_ws = dalpha || dbeta || (staged && (run_a || run_b)) || (cfg->dma && (run_a || run_b));
  if (need_ws && !workspace) return set_error(HPVM_INVALID_ARG, "argument 24: workspace is NULL");
  if (need_ws && workspace_bytes < L.total)
    return set_error(HPVM_WORKSPACE_TOO_SMALL, "argument 25: workspace has %lld bytes, needs %lld",
                     (long long)workspace_bytes, (long long)L.total);
  if (workspace && (uintptr_t)workspace % 16)
    return set_error(HPVM_INVALID_ARG, "argument 24: workspace is not 16-byte aligned");
  if (fault_injected("launch")) return set_error(HPVM_HIP_ERROR, "injected launch failure (HPVM_FAULT_INJECT)");

  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* ws = reinterpret_cast<char*>(workspace);
  float* pa = ws ? reinterpret_cast<float*>(ws) : nullptr;
  float* pb = ws ? reinterpret_cast<float*>(ws + L.pb_off) : nullptr;
  void* stage = ws ? ws + L.stage_off : nullptr;
  // A DMA entry runs a pass it does not cover in whole, aligned tiles on
  // its fallback entry.
  const BwdEntry* fb = cfg->dma ? &kBwd[cfg->fallback] : cfg;
  const MfmaEntry* me = find_menu_entry(prec, fb->tile);
  const bool dma_a = plan.sa && vec16(G, ldg) && vec16(B, ldb) && (!dA || vec16(dA, ldda)) &&
                     (!dalpha || vec16(A, lda));
  const bool dma_b = plan.sb && vec16(A, lda) && vec16(G, ldg) && vec16(dB, lddb);
  hipError_t e = hipSuccess;
  int64_t na = L.na;

  // dC_in and dbeta's partials: an element-wise pass over G (and C_in),
  // launched on its own below unless a launch already carries it.
  const bool grad_c = mn && (dC_in || dbeta);
  GradCJob gc{G, ldg, C_in, ldci, dC_in, lddci, m, n, beta, dbeta ? pb : nullptr,
              vec16(G, ldg) && (!dC_in || vec16(dC_in, lddci)) && (!dbeta || vec16(C_in, ldci)), 0};
  if (grad_c) gc.blocks = L.nb;
  bool gc_done = false;

  // Staged entries: one launch converts everything the products read — one
  // pass over G (its planes for both products, dC_in and dbeta's partials),
  // B for dA and A transposed for dB.
  BwdPlanes P{};
  bool g_pass = false;
  // Both staged products in one launch when the entry has the kernel: each
  // gives too few tiles to fill the CUs twice over on its own.
  const bool pair = staged && run_a && run_b && me && me->launch_staged_pair;
  // Likewise the DMA entry's slices of both gradients, when both are whole
  // tiles and aligned.
  const bool dma_pair = cfg->dma && run_a && run_b && dma_a && dma_b && plan.sp > 0;
  GemmArgs a_pair{};
  if (staged && (run_a || run_b)) {
    if (!me || !me->launch_staged_planes) return hip_error(hipErrorInvalidValue, "backward staged entry");
    P = bwd_planes(prec, stage, m, n, k);
    BackwardStaging st{};
    st.G = G;
    st.ldg = ldg;
    st.Cin = dbeta ? C_in : nullptr;
    st.ldci = ldci;
    st.dCin = dC_in;
    st.lddci = lddci;
    st.m = m;
    st.n = n;
    st.k = k;
    st.beta = beta;
    st.partial = dbeta ? pb : nullptr;
    st.vec_g = vec16(G, ldg) && (!dC_in || vec16(dC_in, lddci)) && (!dbeta || vec16(C_in, ldci));
    if (run_a) {
      st.gh = P.gh;
      st.gl = P.gl;
      st.B = B;
      st.ldb = ldb;
      st.bh = P.bh;
      st.bl = P.bl;
      st.vec_b = vec16(B, ldb);
    }
    if (run_b) {
      st.th = P.th;
      st.tl = P.tl;
      st.A = A;
      st.lda = lda;
      st.ah = P.ah;
      st.al = P.al;
      st.vec_a = vec16(A, lda);
    }
    e = stage_backward(prec, st, s);
    if (e != hipSuccess) return hip_error(e, "backward staging launch");
    g_pass = gc_done = true;
  }

  // dA (and dalpha's partials): contraction over n.
  if (want_a && mk && n == 0) {
    if (dA) e = launch_scale(dA, ldda, m, k, 0.0f, s);
    na = 0;
  } else if (run_a) {
    GemmArgs a{};
    a.A = G;
    a.lda = ldg;
    a.B = B;
    a.ldb = ldb;
    a.C = dA;
    a.ldc = ldda;
    a.m = (int32_t)m;
    a.n = (int32_t)k;
    a.k = (int32_t)n;
    a.alpha = alpha;
    a.beta = 0.0f;
    a.vec_a = vec16(G, ldg);
    a.vec_b = vec16(B, ldb);
    a.tiles_m = (a.m + fb->tile.tile_m - 1) / fb->tile.tile_m;
    a.tiles_n = (a.n + fb->tile.tile_n - 1) / fb->tile.tile_n;
    if (dma_a) {
      if (dma_pair)
        a_pair = a;  // launched with dB below
      else
        e = prec == HPVM_PREC_FP32
                ? launch_split<HPVM_PREC_FP32, false, true>(a, plan.sa, reinterpret_cast<float*>(stage), dA, ldda,
                                                            dalpha ? A : nullptr, lda, dalpha ? pa : nullptr, s)
                : launch_split<HPVM_PREC_BF16, false, true>(a, plan.sa, reinterpret_cast<float*>(stage), dA, ldda,
                                                            dalpha ? A : nullptr, lda, dalpha ? pa : nullptr, s);
      na = dalpha ? split_sum_blocks(m, k) : 0;
    } else if (staged) {
      if (pair)
        a_pair = a;  // launched with dB below
      else
        e = me->launch_staged_planes(a, StagedPlanes{P.gh, P.gl, P.bh, P.bl}, A, lda, dalpha ? pa : nullptr, s);
    } else if (dalpha) {
      // Fused pass: dA (when requested) and the per-tile partials of dalpha.
      if (fb->lds > 65536)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(fb->grad_a),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)fb->lds);
      if (e == hipSuccess) {
        const float* Ao = A;
        int64_t ldao = lda;
        float* part = pa;
        void* kargs[] = {&a, &Ao, &ldao, &part};
        e = hipLaunchKernel(reinterpret_cast<const void*>(fb->grad_a), dim3((unsigned)(a.tiles_m * a.tiles_n)),
                            dim3(fb->threads), kargs, (size_t)fb->lds, s);
      }
      na = a.tiles_m * a.tiles_n;
    } else {
      e = me ? me->launch(a, false, true, s) : hipErrorInvalidValue;
    }
  } else {
    na = 0;
  }
  if (e != hipSuccess) return hip_error(e, "backward dA launch");

  // dB: contraction over m.
  if (dB && kn && m == 0) {
    e = launch_scale(dB, lddb, k, n, 0.0f, s);
  } else if (run_b) {
    GemmArgs b{};
    b.A = A;
    b.lda = lda;
    b.B = G;
    b.ldb = ldg;
    b.C = dB;
    b.ldc = lddb;
    b.m = (int32_t)k;
    b.n = (int32_t)n;
    b.k = (int32_t)m;
    b.alpha = alpha;
    b.beta = 0.0f;
    b.vec_a = vec16(A, lda);
    b.vec_b = vec16(G, ldg);
    if (dma_pair) {
      e = launch_split_pair(prec, a_pair, b, plan.sp, reinterpret_cast<float*>(stage),
                            reinterpret_cast<float*>(stage) + plan.sp * m * k, dA, ldda, dB, lddb,
                            dalpha ? A : nullptr, lda, dalpha ? pa : nullptr, gc, s);
      gc_done = true;
    }
    else if (dma_b)
      e = prec == HPVM_PREC_FP32
              ? launch_split<HPVM_PREC_FP32, true, false>(b, plan.sb, reinterpret_cast<float*>(stage), dB, lddb,
                                                          nullptr, 0, nullptr, s)
              : launch_split<HPVM_PREC_BF16, true, false>(b, plan.sb, reinterpret_cast<float*>(stage), dB, lddb,
                                                          nullptr, 0, nullptr, s);
    else if (!me) e = hipErrorInvalidValue;
    else if (staged && pair)
      e = me->launch_staged_pair(a_pair, StagedPlanes{P.gh, P.gl, P.bh, P.bl}, A, lda, dalpha ? pa : nullptr, b,
                                 StagedPlanes{P.ah, P.al, P.th, P.tl}, s);
    else if (staged)
      e = me->launch_staged_planes(b, StagedPlanes{P.ah, P.al, P.th, P.tl}, nullptr, 0, nullptr, s);
    else e = me->launch(b, true, false, s);
  }
  if (e != hipSuccess) return hip_error(e, "backward dB launch");

  if (grad_c && !gc_done) {
    void* kargs[] = {&gc};
    e = hipLaunchKernel(reinterpret_cast<const void*>(&sgemm_grad_c), dim3((unsigned)gc.blocks), dim3(kElemThreads),
                        kargs, 0, s);
  }
  if (e != hipSuccess) return hip_error(e, "backward dC_in launch");

  if (dalpha || dbeta) {
    const float* pa_ = pa;
    const float* pb_ = pb;
    int32_t na_ = (int32_t)(dalpha ? na : 0);
    int32_t nb_ = (int32_t)((dbeta && mn) ? (g_pass ? L.ng : L.nb) : 0);
    void* kargs[] = {&pa_, &na_, &pb_, &nb_, &dalpha, &dbeta};
    e = hipLaunchKernel(reinterpret_cast<const void*>(&sgemm_grad_finish), dim3(1), dim3(kElemThreads), kargs, 0, s);
  }
  if (e != hipSuccess) return hip_error(e, "backward reduction launch");
  return clear_error();
}

int hpvm_autotune_backward(int64_t m, int64_t n, int64_t k, int32_t prec, const float* A, int64_t lda,
                           const float* B, int64_t ldb, const float* G, int64_t ldg, float* dA, int64_t ldda,
                           float* dB, int64_t lddb, void* workspace, int64_t workspace_bytes, int32_t reps,
                           void* stream, hpvm_tile* best, float* best_ms) {
  if (m <= 0 || n <= 0 || k <= 0) return set_error(HPVM_INVALID_ARG, "m, n and k must be positive");
  if (prec < HPVM_PREC_FP32 || prec > HPVM_PREC_BF16X3)
    return set_error(HPVM_INVALID_ARG, "argument 4: unknown precision %d", prec);
  if (reps < 1) return set_error(HPVM_INVALID_ARG, "argument 17: reps = %d < 1", reps);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float best_t = -1.0f;
  const BwdEntry* best_e = nullptr;
  int rc = HPVM_OK;
  // dA, dB and dalpha: the outputs whose GEMMs the tile decides.
  float* dalpha = nullptr;
  for (int round = 0; round < 2 && e == hipSuccess && rc == HPVM_OK; ++round) {
    for (int i = 0; i < kNumBwd && e == hipSuccess; ++i) {
      const BwdEntry* c = &kBwd[i];
      if (c->prec != prec) continue;
      if (!c->grad_a && !(staged_k_ok(n) && staged_k_ok(m))) continue;
      const BwdLayout L = bwd_layout(c, m, n, k);
      if (L.total + 256 > workspace_bytes) continue;
      // the last 256 bytes of the workspace hold dalpha
      dalpha = reinterpret_cast<float*>(reinterpret_cast<char*>(workspace) + workspace_bytes - 256);
      auto run = [&]() {
        return hpvm_sgemm_backward(m, n, k, 1.0f, 0.0f, A, lda, B, ldb, nullptr, std::max<int64_t>(n, 1), G, ldg,
                                   dA, ldda, dB, lddb, nullptr, std::max<int64_t>(n, 1), dalpha, nullptr, prec,
                                   &c->tile, workspace, workspace_bytes - 256, stream);
      };
      rc = run();
      if (rc != HPVM_OK) break;
      e = hipEventRecord(e0, s);
      for (int r = 0; r < reps && e == hipSuccess && rc == HPVM_OK; ++r) rc = run();
      if (rc != HPVM_OK) break;
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess && (best_t < 0.0f || ms < best_t)) {
        best_t = ms;
        best_e = c;
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc != HPVM_OK) return rc;
  if (e != hipSuccess) return hip_error(e, "backward autotune timing");
  if (!best_e) return set_error(HPVM_WORKSPACE_TOO_SMALL, "no backward tile fits the workspace");
  record_backward_tile(prec, m, n, k, best_e->tile);
  if (best) *best = best_e->tile;
  if (best_ms) *best_ms = best_t / (float)reps;
  return clear_error();
}

}  // extern "C"
