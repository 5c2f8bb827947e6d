// Single-launch MFMA lowerings of the sgemm dataflow graph for CDNA4 (gfx950):
// one kernel launch per SgemmRoot instance, one workgroup per SgemmInternal
// instance (the main loops live in mfma_f32.hpp and mfma_bf16.hpp).
//
// The dynamic instances of SgemmInternal are independent (HPVM report,
// Sec. 2.1), so the tiles may run in any order; the order chosen keeps the
// tiles in flight on one XCD close together so that they share its L2.
#include <algorithm>

#include "device_common.hpp"
#include "internal.hpp"
#include "mfma_f32_dma.hpp"
#include "mfma_bf16.hpp"
#include "mfma_bf16_dma.hpp"
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

// FP32 problems of at least one tile each way with k a multiple of the
// slab, n a multiple of 4, every row 16-byte aligned and no transposed
// operand take the DMA-fed loop (mfma_f32_dma.hpp; edge tiles moved inward)
// with 128-wide wave tiles; any other problem the general 128 x 128 x 16
// tile.
// C <- alpha * (slice 0 + ... + slice splits-1) + beta * C, the slices
// summed in order, from partial sums [splits][m][n]; beta == 0 never reads
// C.  Four adjacent outputs per lane (n, ldc multiples of 4, C 16-byte
// aligned).
constexpr int kSplitThreads = 256;
__global__ void __launch_bounds__(kSplitThreads)
    sgemm_split_finish(const float* __restrict__ part, int32_t splits, int64_t m, int64_t n, float alpha,
                       float beta, float* __restrict__ C, int64_t ldc) {
  const int64_t c4 = n / 4, units = m * c4, plane = m * n;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < units; u += stride) {
    const int64_t i = u / c4, j = (u - i * c4) * 4;
    f32x4 v = *reinterpret_cast<const f32x4*>(part + i * n + j);
    for (int z = 1; z < splits; ++z) v += *reinterpret_cast<const f32x4*>(part + z * plane + i * n + j);
    f32x4* c = reinterpret_cast<f32x4*>(C + i * ldc + j);
    if (beta != 0.0f) {
      const f32x4 old = *c;
#pragma unroll
      for (int t = 0; t < 4; ++t) v[t] = fmaf(beta, old[t], alpha * v[t]);
    } else {
      v = alpha * v;
    }
    *c = v;
  }
}

hipError_t launch_split_finish(const float* part, int32_t splits, int64_t m, int64_t n, float alpha, float beta,
                               float* C, int64_t ldc, hipStream_t s) {
  const int64_t units = m * n / 4;
  const unsigned blocks = (unsigned)std::min<int64_t>(2048, (units + kSplitThreads - 1) / kSplitThreads);
  void* fargs[] = {&part, &splits, &m, &n, &alpha, &beta, &C, &ldc};
  return hipLaunchKernel(reinterpret_cast<const void*>(&sgemm_split_finish), dim3(blocks), dim3(kSplitThreads),
                         fargs, 0, s);
}

template <int TM, int TN, int TK, int WM, int NST>
struct F32DmaConfig {
  using S = F32DmaShape<TM, TN, TK, WM, 128, false, false, NST>;
  static constexpr int kThreads = S::NW * kWave;
  static hipError_t launch(const GemmArgs& args, bool at, bool bt, hipStream_t s) {
    if (at || bt || !f32_dma_fits_edges<TM, TN, TK>(args, args.C, args.ldc))
      return F32Config<128, 128, 16, 64, 64>::launch(args, at, bt, s);
    GemmArgs a = args;
    a.tiles_m = (a.m + TM - 1) / TM;
    a.tiles_n = (a.n + TN - 1) / TN;
    GemmArgs unused = a;
    F32DmaOut o{};
    o.splits = 1;
    void* kargs[] = {&a, &unused, &o};
    // Whole tiles take the kernel without edge masks.
    auto* fn = f32_dma_fits<TM, TN, TK>(args, args.C, args.ldc, 1)
                   ? &sgemm_f32_dma<TM, TN, TK, WM, 128, false, false, NST, kDmaUpdate>
                   : &sgemm_f32_dma<TM, TN, TK, WM, 128, false, false, NST, kDmaUpdate, 0, false, true>;
    hipError_t e = allow_lds(fn, (size_t)S::kLdsBytes);
    if (e != hipSuccess) return e;
    return hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3((unsigned)(a.tiles_m * a.tiles_n)),
                           dim3(kThreads), kargs, (size_t)S::kLdsBytes, s);
  }
  // Contraction slices for a whole-tile problem whose tiles would not cover
  // 256 CUs: doubled while they would not, each slice a whole number of
  // slabs and at least 256 deep, at most 16; 1 (no split) when the slices
  // still would not cover them.
  static int splits(int64_t m, int64_t n, int64_t k) {
    if (m <= 0 || n <= 0 || k <= 0 || m % TM || n % TN || k % TK) return 1;
    return dma_split_count((m / TM) * (n / TN), k, TK);
  }
  static int64_t split_bytes(int64_t m, int64_t n, int64_t k) {
    const int sp = splits(m, n, k);
    return sp > 1 ? (int64_t)sp * m * n * (int64_t)sizeof(float) : 0;
  }
  // The slices write raw partial tiles to `workspace` (split_bytes of it,
  // 16-byte aligned), then sgemm_split_finish forms C.  Problems the split
  // does not cover (operands or C not 16-byte units) take launch().
  static hipError_t launch_split(const GemmArgs& args, void* workspace, hipStream_t s) {
    const int sp = splits(args.m, args.n, args.k);
    float* part = static_cast<float*>(workspace);
    if (sp <= 1 || !f32_dma_fits<TM, TN, TK>(args, part, args.n, sp) ||
        !f32_dma_fits<TM, TN, TK>(args, args.C, args.ldc, sp))
      return launch(args, false, false, s);
    GemmArgs a = args;
    a.C = part;
    a.ldc = a.n;
    a.beta = 0.0f;
    a.tiles_m = a.m / TM;
    a.tiles_n = a.n / TN;
    GemmArgs unused = a;
    F32DmaOut o{};
    o.splits = sp;
    void* kargs[] = {&a, &unused, &o};
    auto* fn = &sgemm_f32_dma<TM, TN, TK, WM, 128, false, false, NST, kDmaSplit>;
    hipError_t e = allow_lds(fn, (size_t)S::kLdsBytes);
    if (e != hipSuccess) return e;
    e = hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3((unsigned)(a.tiles_m * a.tiles_n * sp)),
                        dim3(kThreads), kargs, (size_t)S::kLdsBytes, s);
    if (e != hipSuccess) return e;
    return launch_split_finish(part, sp, args.m, args.n, args.alpha, args.beta, args.C, args.ldc, s);
  }
};

#define HPVM_F32_DMA_ENTRY(TM, TN, TK, WM, NST)                                                   \
  {{TM, TN, TK, WM, 128, NST},                                                                    \
   HPVM_PREC_FP32,                                                                                \
   F32DmaConfig<TM, TN, TK, WM, NST>::kThreads,                                                   \
   F32DmaConfig<TM, TN, TK, WM, NST>::S::kLdsBytes,                                               \
   &F32DmaConfig<TM, TN, TK, WM, NST>::launch,                                                    \
   nullptr,                                                                                       \
   nullptr,                                                                                       \
   nullptr,                                                                                       \
   &F32DmaConfig<TM, TN, TK, WM, NST>::split_bytes,                                               \
   &F32DmaConfig<TM, TN, TK, WM, NST>::launch_split}

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
    HPVM_F32_DMA_ENTRY(128, 128, 32, 32, 2),
};

#define HPVM_BF16_ENTRY(PREC, X3, TM, TN, TK, WM, WN)                                    \
  {{TM, TN, TK, WM, WN, 2}, PREC, Bf16Config<TM, TN, TK, WM, WN, X3>::kThreads,           \
   Bf16Config<TM, TN, TK, WM, WN, X3>::lds(false, false), &Bf16Config<TM, TN, TK, WM, WN, X3>::launch}

// BF16 / bf16x3 products on the FP32 DMA-fed loop (mfma_bf16_dma.hpp):
// problems of at least one tile each way with k a multiple of the slab, n a
// multiple of 4 and 16-byte rows, no transposed operand (edge tiles moved
// inward as in the FP32 loop); any other problem takes the register-staged
// tile of the same size (FM x FN x 32 with FWM x FWN waves).  The split
// contraction is the FP32 entries' (same slice rule, same ordered sum).
template <int TM, int TN, int TK, int WM, int WN, int NST, bool X3, int FWM, int FWN>
struct Bf16SrcConfig {
  using S = Bf16SrcShape<TM, TN, TK, WM, WN, false, false, NST>;
  static constexpr int kThreads = S::NW * kWave;
  static hipError_t launch(const GemmArgs& args, bool at, bool bt, hipStream_t s) {
    if (at || bt || !f32_dma_fits_edges<TM, TN, TK>(args, args.C, args.ldc))
      return Bf16Config<TM, TN, 32, FWM, FWN, X3>::launch(args, at, bt, s);
    GemmArgs a = args;
    a.tiles_m = (a.m + TM - 1) / TM;
    a.tiles_n = (a.n + TN - 1) / TN;
    F32DmaOut o{};
    o.splits = 1;
    void* kargs[] = {&a, &o};
    auto* fn = f32_dma_fits<TM, TN, TK>(args, args.C, args.ldc, 1)
                   ? &sgemm_bf16src_dma<TM, TN, TK, WM, WN, false, false, NST, X3, kDmaUpdate>
                   : &sgemm_bf16src_dma<TM, TN, TK, WM, WN, false, false, NST, X3, kDmaUpdate, true>;
    hipError_t e = allow_lds(fn, (size_t)S::kLdsBytes);
    if (e != hipSuccess) return e;
    return hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3((unsigned)(a.tiles_m * a.tiles_n)),
                           dim3(kThreads), kargs, (size_t)S::kLdsBytes, s);
  }
  static int splits(int64_t m, int64_t n, int64_t k) {
    if (m <= 0 || n <= 0 || k <= 0 || m % TM || n % TN || k % TK) return 1;
    return dma_split_count((m / TM) * (n / TN), k, TK);
  }
  static int64_t split_bytes(int64_t m, int64_t n, int64_t k) {
    const int sp = splits(m, n, k);
    return sp > 1 ? (int64_t)sp * m * n * (int64_t)sizeof(float) : 0;
  }
  static hipError_t launch_split(const GemmArgs& args, void* workspace, hipStream_t s) {
    const int sp = splits(args.m, args.n, args.k);
    float* part = static_cast<float*>(workspace);
    if (sp <= 1 || !f32_dma_fits<TM, TN, TK>(args, part, args.n, sp) ||
        !f32_dma_fits<TM, TN, TK>(args, args.C, args.ldc, sp))
      return launch(args, false, false, s);
    GemmArgs a = args;
    a.C = part;
    a.ldc = a.n;
    a.beta = 0.0f;
    a.tiles_m = a.m / TM;
    a.tiles_n = a.n / TN;
    F32DmaOut o{};
    o.splits = sp;
    void* kargs[] = {&a, &o};
    auto* fn = &sgemm_bf16src_dma<TM, TN, TK, WM, WN, false, false, NST, X3, kDmaSplit>;
    hipError_t e = allow_lds(fn, (size_t)S::kLdsBytes);
    if (e != hipSuccess) return e;
    e = hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3((unsigned)(a.tiles_m * a.tiles_n * sp)),
                        dim3(kThreads), kargs, (size_t)S::kLdsBytes, s);
    if (e != hipSuccess) return e;
    return launch_split_finish(part, sp, args.m, args.n, args.alpha, args.beta, args.C, args.ldc, s);
  }
};

#define HPVM_BF16SRC_ENTRY(PREC, X3, TM, TN, TK, WM, WN, NST, FWM, FWN)                                    \
  {{TM, TN, TK, WM, WN, NST}, PREC, Bf16SrcConfig<TM, TN, TK, WM, WN, NST, X3, FWM, FWN>::kThreads,         \
   Bf16SrcConfig<TM, TN, TK, WM, WN, NST, X3, FWM, FWN>::S::kLdsBytes,                                       \
   &Bf16SrcConfig<TM, TN, TK, WM, WN, NST, X3, FWM, FWN>::launch,                                            \
   nullptr,                                                                                                   \
   nullptr,                                                                                                   \
   nullptr,                                                                                                   \
   &Bf16SrcConfig<TM, TN, TK, WM, WN, NST, X3, FWM, FWN>::split_bytes,                                       \
   &Bf16SrcConfig<TM, TN, TK, WM, WN, NST, X3, FWM, FWN>::launch_split}

// Entry 0 is the default when no tile is given: BF16 and bf16x3 on the
// DMA-fed loop, falling back to the register-staged 256 x 256 x 32 tile.
// bf16x3 takes 16-deep slabs in 4 stages first (8192^3: 2.65 ms against
// 2.87 for 32-deep slabs in 2 stages), BF16 32-deep slabs in 2 stages
// (8192^3: 1.46 ms against 1.51, 4096^3: 0.167 against 0.176; a fifth
// 16-deep stage, all 160 KB of LDS, gave 1.45).
static const MfmaEntry kBf16Menu[] = {
    HPVM_BF16SRC_ENTRY(HPVM_PREC_BF16, false, 256, 256, 32, 64, 128, 2, 128, 64),
    HPVM_BF16SRC_ENTRY(HPVM_PREC_BF16, false, 256, 256, 16, 64, 128, 4, 128, 64),
    HPVM_BF16SRC_ENTRY(HPVM_PREC_BF16, false, 128, 128, 32, 64, 64, 4, 64, 64),
    HPVM_BF16_ENTRY(HPVM_PREC_BF16, false, 256, 256, 32, 128, 64),
    HPVM_BF16_ENTRY(HPVM_PREC_BF16, false, 256, 128, 32, 128, 64),
    HPVM_BF16_ENTRY(HPVM_PREC_BF16, false, 128, 128, 32, 64, 64),
    HPVM_BF16_ENTRY(HPVM_PREC_BF16, false, 128, 128, 64, 64, 64),
    HPVM_BF16_ENTRY(HPVM_PREC_BF16, false, 64, 64, 32, 32, 32),
};

static const MfmaEntry kBf16x3Menu[] = {
    HPVM_BF16SRC_ENTRY(HPVM_PREC_BF16X3, true, 256, 256, 16, 128, 128, 4, 128, 64),
    HPVM_BF16SRC_ENTRY(HPVM_PREC_BF16X3, true, 256, 256, 32, 128, 128, 2, 128, 64),
    HPVM_BF16SRC_ENTRY(HPVM_PREC_BF16X3, true, 128, 128, 32, 64, 64, 4, 64, 64),
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
