// Single-launch MFMA lowerings of the sgemm dataflow graph for CDNA4 (gfx950):
// one kernel launch per SgemmRoot instance, one workgroup per SgemmInternal
// instance (the main loops live in mfma_f32.hpp and mfma_bf16.hpp).
//
// The dynamic instances of SgemmInternal are independent (HPVM report,
// Sec. 2.1), so the tiles may run in any order; the order chosen keeps the
// tiles in flight on one XCD close together so that they share its L2.
#include "device_common.hpp"
#include "internal.hpp"
#include "lds_dma.hpp"
#include "mfma_bf16.hpp"
#include "mfma_f32.hpp"

namespace hpvm {

// Waves per SIMD the register allocation must leave room for.  The
// 128 x 128 x 16 tile fits four resident workgroups per CU without spills
// (with its 38 KB of LDS each), so 4096^3 runs its 1024 tiles in one wave
// of workgroups instead of 768 and then 256; the other tiles keep the
// compiler's choice (forcing them spills).
template <int TM, int TN, int TK>
constexpr int kF32MinWaves = (TM == 128 && TN == 128 && TK == 16) ? 4 : 1;

// FP32 kernel: v_mfma_f32_32x32x2f32, FP32 operands and accumulation.
template <int TM, int TN, int TK, int WM, int WN, bool AT, bool BT>
__global__ void __launch_bounds__((TM / WM) * (TN / WN) * kWave)
    __attribute__((amdgpu_waves_per_eu(kF32MinWaves<TM, TN, TK>))) sgemm_mfma_f32(GemmArgs p) {
  extern __shared__ __align__(16) float lds[];
  int tm, tn;
  tile_coords(p.tiles_m, p.tiles_n, blockIdx.x, tm, tn);
  f32x16 acc[WM / 32][WN / 32];
  f32_mainloop<TM, TN, TK, WM, WN, AT, BT>(p, tm * TM, tn * TN, lds, acc);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  store_c<WM / 32, WN / 32>(p, acc, tm * TM + (wave / (TN / WN)) * WM,
                            tn * TN + (wave % (TN / WN)) * WN, lane);
}

// BF16 kernel (X3 = false) and bf16x3 kernel (X3 = true).
template <int TM, int TN, int TK, int WM, int WN, bool AT, bool BT, bool X3>
__global__ void __launch_bounds__((TM / WM) * (TN / WN) * kWave)
    sgemm_mfma_bf16(GemmArgs p) {
  extern __shared__ __align__(16) char smem[];
  int tm, tn;
  tile_coords(p.tiles_m, p.tiles_n, blockIdx.x, tm, tn);
  f32x16 acc[WM / 32][WN / 32];
  bf16_mainloop<TM, TN, TK, WM, WN, AT, BT, X3>(p, tm * TM, tn * TN, smem, acc);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  store_c<WM / 32, WN / 32>(p, acc, tm * TM + (wave / (TN / WN)) * WM,
                            tn * TN + (wave % (TN / WN)) * WN, lane);
}

// ---------------------------------------------------------------------------
// DMA-fed FP32 kernel for whole tiles: K-slabs of A (m x k, k contiguous) and
// B (k x n, n contiguous) go from HBM straight into NST LDS stages, so no
// register holds a slab in transit and the fragments of the next 8-k group
// are read while the current group's MFMAs run.
//
// Each wave owns WM x 128 outputs.  v_mfma_f32_32x32x2f32 takes, in lane l,
// A(row l % 32, slot l / 32) and B(slot l / 32, column l % 32); within an
// 8-k group, slot h of step p is k = 4h + p.  A lane reads its A row's four
// k of slot h with one 16-byte read, and its B row 4h + p's four
// consecutive columns 4(l % 32) .. 4(l % 32) + 3 with another; component t
// of that B read feeds accumulator block t, so block t holds the columns
// 4j + t of the wave's 128 and a lane's four blocks give it four adjacent
// outputs of a row (one 16-byte store).  A rows in LDS are swizzled
// (SwizzledRows); B rows are kept as in HBM (a fragment read is 512
// contiguous bytes per half-wave).
// ---------------------------------------------------------------------------
template <int TM, int TN, int TK, int WM, int NST>
struct F32DmaShape {
  static constexpr int WN = 128, NWN = TN / WN, NW = (TM / WM) * NWN, BM = WM / 32;
  static constexpr int ARB = 4 * TK;                 // bytes of an A row in LDS
  static constexpr int kABytes = TM * ARB, kBBytes = TK * TN * 4, kStage = kABytes + kBBytes;
  static constexpr int64_t kLdsBytes = (int64_t)NST * kStage;
  static constexpr int QA = kABytes / 1024 / NW, QB = kBBytes / 1024 / NW, Q = QA + QB;
  static constexpr int kMaxWaves = (163840 / (NST * kStage)) * NW / 4;
  static_assert(TN % WN == 0 && TM % WM == 0 && WM % 32 == 0, "wave tiles");
  static_assert(QA * NW * 1024 == kABytes && QB * NW * 1024 == kBBytes && QA % 2 == 0, "even DMA split");
  static_assert((TN * 4) % 1024 == 0 || 1024 % (TN * 4) == 0, "B rows tile a DMA instruction");
  static_assert((NST - 2) * Q < 64, "vmcnt range");
};

template <int TM, int TN, int TK, int WM, int NST>
__global__ void __launch_bounds__((F32DmaShape<TM, TN, TK, WM, NST>::NW * kWave))
    __attribute__((amdgpu_waves_per_eu(1, (F32DmaShape<TM, TN, TK, WM, NST>::kMaxWaves))))
    sgemm_f32_dma(GemmArgs p) {
  using S = F32DmaShape<TM, TN, TK, WM, NST>;
  using LayA = SwizzledRows<S::ARB>;
  constexpr int BM = S::BM, QA = S::QA, QB = S::QB, KG = TK / 8;
  static_assert(KG % 2 == 0, "a slab's last group uses fragment buffer 1, the next slab's first buffer 0");
  extern __shared__ __align__(16) char smem[];

  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int wm0 = (wave / S::NWN) * WM, wn0 = (wave % S::NWN) * S::WN;
  int tm, tn;
  tile_coords(p.tiles_m, p.tiles_n, blockIdx.x, tm, tn);
  const int64_t m0 = (int64_t)tm * TM, n0 = (int64_t)tn * TN;
  const uint32_t lds0 = lds_addr(smem);

  // DMA sources.  A: this wave fills row slots [wave*QA*RA, (wave+1)*QA*RA)
  // of the A stage (RA rows per instruction; instruction j's group parity
  // is j's, QA being even).  B: kilobytes [wave*QB, (wave+1)*QB) of the B
  // stage, which holds the slab's TK rows of TN floats as in HBM.
  constexpr int RA = LayA::kRowsPerDma;
  const int64_t arow = p.lda * 4, brow = p.ldb * 4;
  const char* asrc = reinterpret_cast<const char*>(p.A) + (m0 + (int64_t)wave * QA * RA) * arow;
  const uint32_t aoff[2] = {LayA::src(lane, 0, arow), LayA::src(lane, 1, arow)};
  constexpr int kBRowsPerDma = 1024 / (TN * 4) > 0 ? 1024 / (TN * 4) : 1;
  constexpr int kDmaPerBRow = (TN * 4) / 1024 > 0 ? (TN * 4) / 1024 : 1;
  const uint32_t boff = (uint32_t)((lane / (64 / kBRowsPerDma)) * brow + (lane % (64 / kBRowsPerDma)) * 16);
  auto dma_slab = [&](int slab, int st) {
    const int64_t k0b = (int64_t)slab * TK * 4;
    const uint32_t la = lds0 + st * S::kStage + wave * QA * 1024;
#pragma unroll
    for (int j = 0; j < QA; ++j) dma16(la + j * 1024, asrc + j * RA * arow + k0b, aoff[j & 1]);
    const uint32_t lb = lds0 + st * S::kStage + S::kABytes + wave * QB * 1024;
#pragma unroll
    for (int j = 0; j < QB; ++j) {
      const int q = wave * QB + j;  // B-stage kilobyte q
      const int64_t row = (int64_t)slab * TK + (q / kDmaPerBRow) * kBRowsPerDma;
      const int64_t col = n0 + (q % kDmaPerBRow) * 256;
      dma16(lb + j * 1024, reinterpret_cast<const char*>(p.B) + row * brow + col * 4, boff);
    }
  };

  int afr[KG];
#pragma unroll
  for (int g = 0; g < KG; ++g) afr[g] = LayA::frag(lane, g);
  const int bcol = (wn0 + 4 * (lane & 31)) * 4, bhalf = (lane >> 5) * 4;

  f32x16 acc[BM][4];
  zero_acc(acc);
  f32x4 fa[2][BM], fb[2][4];
  auto read = [&](int buf, const char* st, int g) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      fb[buf][q] = *reinterpret_cast<const f32x4*>(st + S::kABytes + (8 * g + bhalf + q) * (TN * 4) + bcol);
#pragma unroll
    for (int bi = 0; bi < BM; ++bi)
      fa[buf][bi] = *reinterpret_cast<const f32x4*>(st + (wm0 + 32 * bi) * S::ARB + afr[g]);
  };
  auto mfma = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int bi = 0; bi < BM; ++bi)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          acc[bi][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[buf][bi][q], fb[buf][q][t], acc[bi][t], 0, 0, 0);
  };

  const int slabs = p.k / TK;
#pragma unroll
  for (int i = 0; i < NST - 1; ++i) dma_slab(i < slabs ? i : slabs - 1, i);
  dma_wait_barrier<(NST - 2) * S::Q>();
  read(0, smem, 0);
  dma_slab(NST - 1 < slabs ? NST - 1 : slabs - 1, NST - 1);
  int st = 0;
  for (int s = 0; s < slabs; ++s) {
    const char* cur = smem + st * S::kStage;
#pragma unroll
    for (int g = 0; g + 1 < KG; ++g) {
      read((g + 1) & 1, cur, g + 1);
      __builtin_amdgcn_sched_barrier(0);
      mfma(g & 1);
    }
    // Slab s + 1 has landed everywhere and nobody reads slab s any more:
    // refill its stage with slab s + NST and read slab s + 1's first group
    // under the last group's MFMAs.
    const int nst = st + 1 == NST ? 0 : st + 1;
    dma_wait_barrier<(NST - 2) * S::Q>();
    read(0, smem + nst * S::kStage, 0);
    dma_slab(s + NST < slabs ? s + NST : slabs - 1, st);
    __builtin_amdgcn_sched_barrier(0);
    mfma(1);
    st = nst;
  }
  dma_wait_barrier<0>();

  // Epilogue: four adjacent outputs of a row per lane and register.
  const int64_t row0 = m0 + wm0, col = n0 + wn0 + 4 * (lane & 31);
  const bool read_c = p.beta != 0.0f;
#pragma unroll
  for (int bi = 0; bi < BM; ++bi)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      f32x4 c[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t i = row0 + 32 * bi + acc_row(4 * g + u, lane);
        c[u] = read_c ? *reinterpret_cast<const f32x4*>(p.C + i * p.ldc + col) : f32x4{0, 0, 0, 0};
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t i = row0 + 32 * bi + acc_row(4 * g + u, lane);
        f32x4 v;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          v[t] = p.alpha * acc[bi][t][4 * g + u];
          if (read_c) v[t] = fmaf(p.beta, c[u][t], v[t]);
        }
        *reinterpret_cast<f32x4*>(p.C + i * p.ldc + col) = v;
      }
    }
}

// Dynamic LDS beyond 64 KiB must be enabled per kernel before its launch.
template <typename Kernel>
static hipError_t allow_lds(Kernel* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int TM, int TN, int TK, int WM, int WN>
struct F32Config {
  static constexpr int kThreads = (TM / WM) * (TN / WN) * kWave;
  // LDS bytes for the given operand forms (the Allocation node's size).
  static constexpr int64_t lds(bool at, bool bt) {
    return at ? F32Tile<TM, TN, TK, WM, WN, true, false>::kLdsBytes
              : bt ? F32Tile<TM, TN, TK, WM, WN, false, true>::kLdsBytes
                   : F32Tile<TM, TN, TK, WM, WN, false, false>::kLdsBytes;
  }
  static hipError_t launch(const GemmArgs& args, bool at, bool bt, hipStream_t s) {
    GemmArgs a = args;
    a.tiles_m = (a.m + TM - 1) / TM;
    a.tiles_n = (a.n + TN - 1) / TN;
    const dim3 grid((unsigned)(a.tiles_m * a.tiles_n));
    void* kargs[] = {&a};
    void (*fn)(GemmArgs);
    if (!at && !bt) fn = &sgemm_mfma_f32<TM, TN, TK, WM, WN, false, false>;
    else if (at && !bt) fn = &sgemm_mfma_f32<TM, TN, TK, WM, WN, true, false>;
    else if (!at && bt) fn = &sgemm_mfma_f32<TM, TN, TK, WM, WN, false, true>;
    else return hipErrorInvalidValue;
    const size_t bytes = (size_t)lds(at, bt);
    hipError_t e = allow_lds(fn, bytes);
    if (e != hipSuccess) return e;
    return hipLaunchKernel(reinterpret_cast<const void*>(fn), grid, dim3(kThreads), kargs, bytes, s);
  }
};


template <int TM, int TN, int TK, int WM, int WN, bool X3>
struct Bf16Config {
  static constexpr int kThreads = (TM / WM) * (TN / WN) * kWave;
  static constexpr int64_t lds(bool, bool) { return Bf16TileShape<TM, TN, TK, WM, WN, X3>::kLdsBytes; }
  static hipError_t launch(const GemmArgs& args, bool at, bool bt, hipStream_t s) {
    GemmArgs a = args;
    a.tiles_m = (a.m + TM - 1) / TM;
    a.tiles_n = (a.n + TN - 1) / TN;
    const dim3 grid((unsigned)(a.tiles_m * a.tiles_n));
    void* kargs[] = {&a};
    void (*fn)(GemmArgs);
    if (!at && !bt) fn = &sgemm_mfma_bf16<TM, TN, TK, WM, WN, false, false, X3>;
    else if (at && !bt) fn = &sgemm_mfma_bf16<TM, TN, TK, WM, WN, true, false, X3>;
    else if (!at && bt) fn = &sgemm_mfma_bf16<TM, TN, TK, WM, WN, false, true, X3>;
    else return hipErrorInvalidValue;
    const size_t bytes = (size_t)lds(at, bt);
    hipError_t e = allow_lds(fn, bytes);
    if (e != hipSuccess) return e;
    return hipLaunchKernel(reinterpret_cast<const void*>(fn), grid, dim3(kThreads), kargs, bytes, s);
  }
};

#define HPVM_F32_ENTRY(TM, TN, TK, WM, WN)                                               \
  {{TM, TN, TK, WM, WN, 2}, HPVM_PREC_FP32, F32Config<TM, TN, TK, WM, WN>::kThreads,     \
   F32Config<TM, TN, TK, WM, WN>::lds(false, false), &F32Config<TM, TN, TK, WM, WN>::launch}

// Whole-tile FP32 problems (m, n, k multiples of the tile, every row
// 16-byte aligned, no transposed operand) take the DMA-fed kernel; any
// other problem the general 128 x 128 x 16 kernel.
template <int TM, int TN, int TK, int WM, int NST>
struct F32DmaConfig {
  using S = F32DmaShape<TM, TN, TK, WM, NST>;
  static constexpr int kThreads = S::NW * kWave;
  static bool fits(const GemmArgs& a, bool at, bool bt) {
    return !at && !bt && a.vec_a && a.vec_b && a.m % TM == 0 && a.n % TN == 0 && a.k > 0 && a.k % TK == 0 &&
           a.ldc % 4 == 0 && (reinterpret_cast<uintptr_t>(a.C) & 15) == 0;
  }
  static hipError_t launch(const GemmArgs& args, bool at, bool bt, hipStream_t s) {
    if (!fits(args, at, bt)) return F32Config<128, 128, 16, 64, 64>::launch(args, at, bt, s);
    GemmArgs a = args;
    a.tiles_m = a.m / TM;
    a.tiles_n = a.n / TN;
    void* kargs[] = {&a};
    auto* fn = &sgemm_f32_dma<TM, TN, TK, WM, NST>;
    hipError_t e = allow_lds(fn, (size_t)S::kLdsBytes);
    if (e != hipSuccess) return e;
    return hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3((unsigned)(a.tiles_m * a.tiles_n)),
                           dim3(kThreads), kargs, (size_t)S::kLdsBytes, s);
  }
};

#define HPVM_F32_DMA_ENTRY(TM, TN, TK, WM, NST)                                                   \
  {{TM, TN, TK, WM, 128, NST}, HPVM_PREC_FP32, F32DmaConfig<TM, TN, TK, WM, NST>::kThreads,       \
   F32DmaShape<TM, TN, TK, WM, NST>::kLdsBytes, &F32DmaConfig<TM, TN, TK, WM, NST>::launch}

// Entry 0 is the default: DMA-fed for whole-tile problems, otherwise the
// 128 x 128 x 16 tile.
static const MfmaEntry kF32Menu[] = {
    HPVM_F32_DMA_ENTRY(256, 256, 32, 64, 2),
    HPVM_F32_ENTRY(128, 128, 16, 64, 64),
    HPVM_F32_ENTRY(256, 128, 16, 128, 64),
    HPVM_F32_ENTRY(128, 128, 32, 64, 64),
    HPVM_F32_ENTRY(64, 64, 16, 32, 32),
    HPVM_F32_ENTRY(128, 64, 16, 64, 32),
    HPVM_F32_ENTRY(64, 128, 16, 32, 64),
    HPVM_F32_DMA_ENTRY(256, 256, 16, 64, 4),
    HPVM_F32_DMA_ENTRY(128, 256, 32, 32, 2),
};

#define HPVM_BF16_ENTRY(PREC, X3, TM, TN, TK, WM, WN)                                    \
  {{TM, TN, TK, WM, WN, 2}, PREC, Bf16Config<TM, TN, TK, WM, WN, X3>::kThreads,           \
   Bf16Config<TM, TN, TK, WM, WN, X3>::lds(false, false), &Bf16Config<TM, TN, TK, WM, WN, X3>::launch}

static const MfmaEntry kBf16Menu[] = {
    HPVM_BF16_ENTRY(HPVM_PREC_BF16, false, 256, 256, 32, 128, 64),
    HPVM_BF16_ENTRY(HPVM_PREC_BF16, false, 256, 128, 32, 128, 64),
    HPVM_BF16_ENTRY(HPVM_PREC_BF16, false, 128, 128, 32, 64, 64),
    HPVM_BF16_ENTRY(HPVM_PREC_BF16, false, 128, 128, 64, 64, 64),
    HPVM_BF16_ENTRY(HPVM_PREC_BF16, false, 64, 64, 32, 32, 32),
};

static const MfmaEntry kBf16x3Menu[] = {
    HPVM_BF16_ENTRY(HPVM_PREC_BF16X3, true, 256, 256, 32, 128, 64),
    HPVM_BF16_ENTRY(HPVM_PREC_BF16X3, true, 256, 128, 32, 128, 64),
    HPVM_BF16_ENTRY(HPVM_PREC_BF16X3, true, 128, 128, 32, 64, 64),
    HPVM_BF16_ENTRY(HPVM_PREC_BF16X3, true, 64, 64, 32, 32, 32),
};

int mfma_menu(int32_t prec, const MfmaEntry** entries) {
  if (prec == HPVM_PREC_FP32) {
    *entries = kF32Menu;
    return (int)(sizeof(kF32Menu) / sizeof(kF32Menu[0]));
  }
  if (prec == HPVM_PREC_BF16) {
    *entries = kBf16Menu;
    return (int)(sizeof(kBf16Menu) / sizeof(kBf16Menu[0]));
  }
  if (prec == HPVM_PREC_BF16X3) {
    *entries = kBf16x3Menu;
    return (int)(sizeof(kBf16x3Menu) / sizeof(kBf16x3Menu[0]));
  }
  *entries = nullptr;
  return 0;
}

}  // namespace hpvm
