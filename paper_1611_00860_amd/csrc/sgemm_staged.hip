// Staged BF16 / bf16x3 lowering of the sgemm dataflow graph (gfx950).
//
// The fused lowering rounds FP32 elements to bfloat16 while it copies them
// into LDS, so every workgroup streams FP32 operands: at the BF16 MFMA rate
// that is twice the bytes per product and a register budget too small to
// cover the load latency.  The staged lowering first rewrites A and B once,
// in a separate pass, as bfloat16 planes in a caller workspace:
//   A (m x k)  -> Ah[, Al]  [m_pad][k_pad], k contiguous;
//   B (k x n)  -> Bh[, Bl]  [n_pad][k_pad], k contiguous (B transposed);
// zero-padded to whole 256 x 64 blocks, with hi = bf16(x) and, for bf16x3,
// lo = bf16(x - hi).  The GEMM then moves 16-byte units with no edge checks
// and keeps two K-slabs in flight in registers ahead of the LDS stage being
// multiplied.  The hierarchy is the same as in the other lowerings: one
// workgroup per SgemmInternal instance, the Allocation node as LDS stages,
// SgemmLeaf outputs as MFMA accumulators.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.hpp"
#include "hpvm_sgemm.h"
#include "internal.hpp"
#include "mfma_bf16.hpp"
#include "mfma_f32.hpp"

namespace hpvm {

constexpr int64_t kPadMN = 256;  // multiple of every staged tile_m / tile_n
constexpr int64_t kPadK = 64;    // multiple of every staged tile_k

struct StagedLayout {
  int64_t m_pad, n_pad, k_pad;
  int planes;
  int64_t a_plane, b_plane;  // bytes of one plane
  int64_t total;
};

bool staged_k_ok(int64_t k) {
  const int64_t k_pad = (k + kPadK - 1) / kPadK * kPadK;
  return (int64_t)kPadMN * k_pad * 2 < ((int64_t)1 << 32);
}

static StagedLayout staged_layout(int32_t prec, int64_t m, int64_t n, int64_t k) {
  StagedLayout L;
  L.m_pad = (m + kPadMN - 1) / kPadMN * kPadMN;
  L.n_pad = (n + kPadMN - 1) / kPadMN * kPadMN;
  L.k_pad = (k + kPadK - 1) / kPadK * kPadK;
  L.planes = prec == HPVM_PREC_BF16X3 ? 2 : 1;
  L.a_plane = L.m_pad * L.k_pad * 2;
  L.b_plane = L.n_pad * L.k_pad * 2;
  L.total = L.planes * (L.a_plane + L.b_plane);
  return L;
}

int64_t staged_workspace_bytes(int32_t prec, int64_t m, int64_t n, int64_t k) {
  return staged_layout(prec, m, n, k).total;
}

// Rounds (and with X3 splits) one element; returns the raw bfloat16 bits.
template <bool X3>
__device__ __forceinline__ void to_bf16(float x, uint16_t& hi, uint16_t& lo) {
  const __bf16 h = (__bf16)x;
  hi = __builtin_bit_cast(uint16_t, h);
  if constexpr (X3) lo = __builtin_bit_cast(uint16_t, (__bf16)(x - (float)h));
}

// rows x cols FP32 (element (r, c) at src[r * ld + c], c is the k index)
// -> [rows_pad][cols_pad] bfloat16, zero outside rows x cols.
template <bool X3>
__global__ void __launch_bounds__(256)
    stage_rows(const float* __restrict__ src, int64_t ld, int64_t rows, int64_t cols, int64_t rows_pad,
               int64_t cols_pad, uint16_t* __restrict__ hi, uint16_t* __restrict__ lo, int32_t vec) {
  const int64_t per_row = cols_pad / 8;
  const int64_t units = rows_pad * per_row;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < units;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = u / per_row, c = (u - r * per_row) * 8;
    float v[8];
    const float* p = src + r * ld + c;
    if (vec && r < rows && c + 8 <= cols) {
      const f32x4 a = *reinterpret_cast<const f32x4*>(p);
      const f32x4 b = *reinterpret_cast<const f32x4*>(p + 4);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        v[e] = a[e];
        v[e + 4] = b[e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (r < rows && c + e < cols) ? p[e] : 0.0f;
    }
    uint16_t h[8], l[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) to_bf16<X3>(v[e], h[e], l[e]);
    u32x4 hv, lv;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      hv[q] = (uint32_t)h[2 * q] | ((uint32_t)h[2 * q + 1] << 16);
      if constexpr (X3) lv[q] = (uint32_t)l[2 * q] | ((uint32_t)l[2 * q + 1] << 16);
    }
    *reinterpret_cast<u32x4*>(hi + r * cols_pad + c) = hv;
    if constexpr (X3) *reinterpret_cast<u32x4*>(lo + r * cols_pad + c) = lv;
  }
}

// rows x cols FP32 with the k index along rows (element (r, c) at
// src[r * ld + c]) -> [cols_pad][rows_pad] bfloat16: transposed so that k is
// contiguous.  One workgroup moves a 64 x 64 block through LDS.
constexpr int kTB = 64;
template <bool X3>
__global__ void __launch_bounds__(256)
    stage_cols(const float* __restrict__ src, int64_t ld, int64_t rows, int64_t cols, int64_t rows_pad,
               uint16_t* __restrict__ hi, uint16_t* __restrict__ lo) {
  __shared__ float t[kTB][kTB + 1];
  const int64_t r0 = (int64_t)blockIdx.y * kTB, c0 = (int64_t)blockIdx.x * kTB;
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < kTB * kTB / 256; ++i) {
    const int r = i * (256 / kTB) + tid / kTB, c = tid % kTB;
    const int64_t gr = r0 + r, gc = c0 + c;
    t[r][c] = (gr < rows && gc < cols) ? src[gr * ld + gc] : 0.0f;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kTB * kTB / 8 / 256; ++j) {
    const int u = tid + j * 256;
    const int cc = u / (kTB / 8), kc = (u % (kTB / 8)) * 8;
    uint16_t h[8], l[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) to_bf16<X3>(t[kc + e][cc], h[e], l[e]);
    u32x4 hv, lv;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      hv[q] = (uint32_t)h[2 * q] | ((uint32_t)h[2 * q + 1] << 16);
      if constexpr (X3) lv[q] = (uint32_t)l[2 * q] | ((uint32_t)l[2 * q + 1] << 16);
    }
    const int64_t off = (c0 + cc) * rows_pad + r0 + kc;
    *reinterpret_cast<u32x4*>(hi + off) = hv;
    if constexpr (X3) *reinterpret_cast<u32x4*>(lo + off) = lv;
  }
}

struct StagedArgs {
  const uint16_t* ah;
  const uint16_t* al;
  const uint16_t* bh;
  const uint16_t* bl;
  int64_t kp;  // padded k: row length of every plane
  float* C;
  int64_t ldc;
  int32_t m, n, slabs, tiles_m, tiles_n;
  float alpha, beta;
  // Backward epilogue (EPI = 1): C (may be null) <- alpha acc, and
  // partial[tile] <- sum over the tile of aorig .* acc.
  const float* aorig;
  int64_t lda_orig;
  float* partial;
};

// The GEMM over staged planes.  DEPTH = 1: each K-slab is loaded into
// registers while the previous one, already in LDS, feeds the matrix cores,
// and is written to the other LDS stage after those MFMAs.  DEPTH = 2: slab j
// is loaded into register buffer j % 2 two slabs before it is written to LDS,
// so two slabs of MFMA work cover each load.  One barrier per slab either
// way.  PIPE reads the fragments of the next 16-k step ahead of the current
// MFMAs.
template <int TM, int TN, int TK, int WM, int WN, bool X3, int DEPTH, bool PIPE, int EPI>
__global__ void __launch_bounds__((TM / WM) * (TN / WN) * kWave)
    sgemm_bf16_staged(StagedArgs p) {
  using T = Bf16TileShape<TM, TN, TK, WM, WN, X3>;
  constexpr int NT = T::NT, BM = T::BM, BN = T::BN, RB = T::RB, P = T::kPlanes;
  constexpr int kUnitsPerRow = TK / 8;
  constexpr int UA = TM * kUnitsPerRow / NT, UB = TN * kUnitsPerRow / NT;
  static_assert(UA * NT == TM * kUnitsPerRow && UB * NT == TN * kUnitsPerRow, "even split");
  static_assert(DEPTH == 1 || DEPTH == 2, "prefetch depth");
  extern __shared__ __align__(16) char smem[];

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid / kWave;
  const int wm0 = (wave / T::kWavesN) * WM, wn0 = (wave % T::kWavesN) * WN;
  int tm, tn;
  tile_coords(p.tiles_m, p.tiles_n, blockIdx.x, tm, tn);
  const int64_t m0 = (int64_t)tm * TM, n0 = (int64_t)tn * TN;
  const uint16_t* aplane[2] = {p.ah + m0 * p.kp, X3 ? p.al + m0 * p.kp : nullptr};
  const uint16_t* bplane[2] = {p.bh + n0 * p.kp, X3 ? p.bl + n0 * p.kp : nullptr};

  auto a_st = [&](int st, int pl) { return smem + st * T::kStageBytes + pl * T::kABytes; };
  auto b_st = [&](int st, int pl) { return smem + st * T::kStageBytes + P * T::kABytes + pl * T::kBBytes; };

  u32x4 ra[DEPTH][P * UA], rb[DEPTH][P * UB];
  // A unit's address is a workgroup-uniform base (the plane's tile corner
  // plus the slab) and a 32-bit per-lane byte offset (planes are under
  // 4 GiB): one register per load instead of a 64-bit address.
  auto unit_off = [&](int j) {
    const int u = tid + j * NT, r = u / kUnitsPerRow, c = (u % kUnitsPerRow) * 8;
    return (uint32_t)(((int64_t)r * p.kp + c) * 2);
  };
  auto load = [&](u32x4(&a)[P * UA], u32x4(&b)[P * UB], int slab) {
    const int64_t k0 = (int64_t)slab * TK;
#pragma unroll
    for (int pl = 0; pl < P; ++pl) {
      const char* abase = reinterpret_cast<const char*>(aplane[pl] + k0);
      const char* bbase = reinterpret_cast<const char*>(bplane[pl] + k0);
#pragma unroll
      for (int j = 0; j < UA; ++j) a[pl * UA + j] = *reinterpret_cast<const u32x4*>(abase + unit_off(j));
#pragma unroll
      for (int j = 0; j < UB; ++j) b[pl * UB + j] = *reinterpret_cast<const u32x4*>(bbase + unit_off(j));
    }
  };
  auto store = [&](const u32x4(&a)[P * UA], const u32x4(&b)[P * UB], int st) {
#pragma unroll
    for (int pl = 0; pl < P; ++pl) {
#pragma unroll
      for (int j = 0; j < UA; ++j) {
        const int u = tid + j * NT, r = u / kUnitsPerRow, c = (u % kUnitsPerRow) * 8;
        *reinterpret_cast<u32x4*>(a_st(st, pl) + r * RB + 2 * c) = a[pl * UA + j];
      }
#pragma unroll
      for (int j = 0; j < UB; ++j) {
        const int u = tid + j * NT, r = u / kUnitsPerRow, c = (u % kUnitsPerRow) * 8;
        *reinterpret_cast<u32x4*>(b_st(st, pl) + r * RB + 2 * c) = b[pl * UB + j];
      }
    }
  };
  f32x16 acc[BM][BN];
  zero_acc(acc);
  auto mfma_stage = [&](int st) {
    bf16_stage_mfma<TK, BM, BN, X3, PIPE>(a_st(st, 0), a_st(st, X3 ? 1 : 0), b_st(st, 0), b_st(st, X3 ? 1 : 0),
                                          wm0, wn0, lane, acc);
  };
  const int S = p.slabs;
  if constexpr (DEPTH == 1) {
    load(ra[0], rb[0], 0);
    store(ra[0], rb[0], 0);
    __syncthreads();
    for (int s = 0; s < S; ++s) {
      const int st = s & 1;
      const bool more = s + 1 < S;
      if (more) load(ra[0], rb[0], s + 1);
      mfma_stage(st);
      if (more) store(ra[0], rb[0], st ^ 1);
      __syncthreads();
    }
  } else {
    load(ra[0], rb[0], 0);
    load(ra[1], rb[1], S > 1 ? 1 : 0);
    store(ra[0], rb[0], 0);
    __syncthreads();
    load(ra[0], rb[0], S > 2 ? 2 : S - 1);
    // One slab: multiply stage B, move slab s + 1 (register buffer B ^ 1)
    // into stage B ^ 1, refill that buffer with slab s + 3.  No branch in
    // a step: past the end the store fills a stage nobody reads and the
    // load re-reads the last slab.  The compiler's wait counting then
    // sees the same loads in flight on every path through the loop and
    // waits only for the older buffer's loads before the store, leaving
    // the newer buffer's in flight (with branches it waited for all).
    auto step = [&](auto parity, int s) {
      constexpr int B = decltype(parity)::value;
      mfma_stage(B);
      store(ra[B ^ 1], rb[B ^ 1], B ^ 1);
      load(ra[B ^ 1], rb[B ^ 1], s + 3 < S ? s + 3 : S - 1);
      __syncthreads();
    };
    int s = 0;
    for (; s + 1 < S; s += 2) {
      step(std::integral_constant<int, 0>{}, s);
      step(std::integral_constant<int, 1>{}, s + 1);
    }
    if (s < S) step(std::integral_constant<int, 0>{}, s);
  }

  if constexpr (EPI == 0) {
    GemmArgs e{};
    e.C = p.C;
    e.ldc = p.ldc;
    e.m = p.m;
    e.n = p.n;
    e.alpha = p.alpha;
    e.beta = p.beta;
    store_c<BM, BN>(e, acc, (int)m0 + wm0, (int)n0 + wn0, lane);
  } else {
    // Each group of 4 rows loads its elements of A before its dA stores.
    float part = 0.0f;
#pragma unroll
    for (int bi = 0; bi < BM; ++bi)
#pragma unroll
      for (int bj = 0; bj < BN; ++bj) {
        const int j = (int)n0 + wn0 + 32 * bj + acc_col(lane);
        if (j >= p.n) continue;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          float a[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int i = (int)m0 + wm0 + 32 * bi + acc_row(4 * g + t, lane);
            a[t] = i < p.m ? p.aorig[(int64_t)i * p.lda_orig + j] : 0.0f;
          }
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int i = (int)m0 + wm0 + 32 * bi + acc_row(4 * g + t, lane);
            if (i < p.m) {
              const float v = acc[bi][bj][4 * g + t];
              if (p.C) p.C[(int64_t)i * p.ldc + j] = p.alpha * v;
              part = fmaf(a[t], v, part);
            }
          }
        }
      }
    const float sum = block_sum(part, reinterpret_cast<float*>(smem));
    if (threadIdx.x == 0) p.partial[blockIdx.x] = sum;
  }
}

namespace {

template <typename Kernel>
hipError_t allow_lds_staged(Kernel* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

template <bool X3>
hipError_t stage_rows_launch(const float* src, int64_t ld, int64_t rows, int64_t cols, int64_t rows_pad,
                             int64_t cols_pad, uint16_t* hi, uint16_t* lo, int32_t vec, hipStream_t s) {
  const int64_t units = rows_pad * cols_pad / 8;
  const unsigned blocks = (unsigned)std::min<int64_t>((units + 255) / 256, 8192);
  void* args[] = {&src, &ld, &rows, &cols, &rows_pad, &cols_pad, &hi, &lo, &vec};
  return hipLaunchKernel(reinterpret_cast<const void*>(&stage_rows<X3>), dim3(blocks), dim3(256), args, 0, s);
}

template <bool X3>
hipError_t stage_cols_launch(const float* src, int64_t ld, int64_t rows, int64_t cols, int64_t rows_pad,
                             int64_t cols_pad, uint16_t* hi, uint16_t* lo, hipStream_t s) {
  void* args[] = {&src, &ld, &rows, &cols, &rows_pad, &hi, &lo};
  const dim3 grid((unsigned)(cols_pad / kTB), (unsigned)(rows_pad / kTB));
  return hipLaunchKernel(reinterpret_cast<const void*>(&stage_cols<X3>), grid, dim3(256), args, 0, s);
}

// Writes op(A) as [m_pad][k_pad] and op(B) as [n_pad][k_pad] planes, k
// contiguous: an operand already k-contiguous in HBM is copied row by row,
// the other is transposed through LDS.
template <bool X3>
hipError_t stage_operands(const GemmArgs& a, bool at, bool bt, const StagedLayout& L, char* ws, hipStream_t s) {
  uint16_t* ah = reinterpret_cast<uint16_t*>(ws);
  uint16_t* al = X3 ? reinterpret_cast<uint16_t*>(ws + L.a_plane) : nullptr;
  uint16_t* bh = reinterpret_cast<uint16_t*>(ws + L.planes * L.a_plane);
  uint16_t* bl = X3 ? reinterpret_cast<uint16_t*>(ws + L.planes * L.a_plane + L.b_plane) : nullptr;
  hipError_t e;
  if (!at)  // A: m x k, k contiguous
    e = stage_rows_launch<X3>(a.A, a.lda, a.m, a.k, L.m_pad, L.k_pad, ah, al, a.vec_a, s);
  else      // A stored k x m
    e = stage_cols_launch<X3>(a.A, a.lda, a.k, a.m, L.k_pad, L.m_pad, ah, al, s);
  if (e != hipSuccess) return e;
  if (!bt)  // B: k x n, n contiguous
    return stage_cols_launch<X3>(a.B, a.ldb, a.k, a.n, L.k_pad, L.n_pad, bh, bl, s);
  // B stored n x k
  return stage_rows_launch<X3>(a.B, a.ldb, a.n, a.k, L.n_pad, L.k_pad, bh, bl, a.vec_b, s);
}

template <int TM, int TN, int TK, int WM, int WN, bool X3, int DEPTH, bool PIPE>
struct StagedConfig {
  using T = Bf16TileShape<TM, TN, TK, WM, WN, X3>;
  static constexpr int kThreads = T::NT;
  static_assert(kPadMN % TM == 0 && kPadMN % TN == 0 && kPadK % TK == 0, "padding covers the tile");

  template <int EPI>
  static hipError_t run(const GemmArgs& a, bool at, bool bt, void* workspace, const float* aorig, int64_t lda_orig,
                        float* partial, hipStream_t s) {
    const int32_t prec = X3 ? HPVM_PREC_BF16X3 : HPVM_PREC_BF16;
    const StagedLayout L = staged_layout(prec, a.m, a.n, a.k);
    char* ws = reinterpret_cast<char*>(workspace);
    hipError_t e = stage_operands<X3>(a, at, bt, L, ws, s);
    if (e != hipSuccess) return e;
    StagedArgs p{};
    p.ah = reinterpret_cast<const uint16_t*>(ws);
    p.al = X3 ? reinterpret_cast<const uint16_t*>(ws + L.a_plane) : nullptr;
    p.bh = reinterpret_cast<const uint16_t*>(ws + L.planes * L.a_plane);
    p.bl = X3 ? reinterpret_cast<const uint16_t*>(ws + L.planes * L.a_plane + L.b_plane) : nullptr;
    p.kp = L.k_pad;
    p.C = a.C;
    p.ldc = a.ldc;
    p.m = a.m;
    p.n = a.n;
    p.slabs = (int32_t)(L.k_pad / TK);
    p.tiles_m = (a.m + TM - 1) / TM;
    p.tiles_n = (a.n + TN - 1) / TN;
    p.alpha = a.alpha;
    p.beta = a.beta;
    p.aorig = aorig;
    p.lda_orig = lda_orig;
    p.partial = partial;
    auto* fn = &sgemm_bf16_staged<TM, TN, TK, WM, WN, X3, DEPTH, PIPE, EPI>;
    e = allow_lds_staged(fn, (size_t)T::kLdsBytes);
    if (e != hipSuccess) return e;
    void* kargs[] = {&p};
    return hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3((unsigned)(p.tiles_m * p.tiles_n)),
                           dim3(kThreads), kargs, (size_t)T::kLdsBytes, s);
  }
  static hipError_t launch(const GemmArgs& a, void* workspace, hipStream_t s) {
    return run<0>(a, false, false, workspace, nullptr, 0, nullptr, s);
  }
  static hipError_t launch_form(const GemmArgs& a, bool at, bool bt, void* workspace, const float* aorig,
                                int64_t lda_orig, float* partial, hipStream_t s) {
    return partial ? run<1>(a, at, bt, workspace, aorig, lda_orig, partial, s)
                   : run<0>(a, at, bt, workspace, nullptr, 0, nullptr, s);
  }
};

#define HPVM_STAGED_ENTRY(PREC, X3, DEPTH, PIPE, TM, TN, TK, WM, WN)                                     \
  {{TM, TN, TK, WM, WN, 3}, PREC, StagedConfig<TM, TN, TK, WM, WN, X3, DEPTH, PIPE>::kThreads,           \
   Bf16TileShape<TM, TN, TK, WM, WN, X3>::kLdsBytes, nullptr,                                             \
   &StagedConfig<TM, TN, TK, WM, WN, X3, DEPTH, PIPE>::launch,                                           \
   &StagedConfig<TM, TN, TK, WM, WN, X3, DEPTH, PIPE>::launch_form}

const MfmaEntry kStagedMenuBf16[] = {
    HPVM_STAGED_ENTRY(HPVM_PREC_BF16, false, 2, false, 256, 256, 64, 128, 64),
    HPVM_STAGED_ENTRY(HPVM_PREC_BF16, false, 1, true, 256, 256, 32, 128, 64),
    HPVM_STAGED_ENTRY(HPVM_PREC_BF16, false, 1, true, 256, 128, 64, 128, 64),
    HPVM_STAGED_ENTRY(HPVM_PREC_BF16, false, 1, true, 128, 128, 64, 64, 64),
};
const MfmaEntry kStagedMenuBf16x3[] = {
    HPVM_STAGED_ENTRY(HPVM_PREC_BF16X3, true, 1, false, 256, 256, 32, 128, 64),
    HPVM_STAGED_ENTRY(HPVM_PREC_BF16X3, true, 1, true, 256, 128, 32, 128, 64),
    HPVM_STAGED_ENTRY(HPVM_PREC_BF16X3, true, 1, true, 128, 128, 64, 64, 64),
};

}  // namespace

int staged_menu(int32_t prec, const MfmaEntry** entries) {
  if (prec == HPVM_PREC_BF16) {
    *entries = kStagedMenuBf16;
    return (int)(sizeof(kStagedMenuBf16) / sizeof(kStagedMenuBf16[0]));
  }
  if (prec == HPVM_PREC_BF16X3) {
    *entries = kStagedMenuBf16x3;
    return (int)(sizeof(kStagedMenuBf16x3) / sizeof(kStagedMenuBf16x3[0]));
  }
  *entries = nullptr;
  return 0;
}

const MfmaEntry* menu_entry_at(int32_t prec, int index) {
  const MfmaEntry* fused;
  const MfmaEntry* staged;
  const int nf = mfma_menu(prec, &fused), ns = staged_menu(prec, &staged);
  if (index < 0) return nullptr;
  if (index < nf) return &fused[index];
  if (index < nf + ns) return &staged[index - nf];
  return nullptr;
}

int menu_size(int32_t prec) {
  const MfmaEntry* e;
  return mfma_menu(prec, &e) + staged_menu(prec, &e);
}

const MfmaEntry* find_menu_entry(int32_t prec, const hpvm_tile& t) {
  for (int i = 0, n = menu_size(prec); i < n; ++i) {
    const hpvm_tile& u = menu_entry_at(prec, i)->tile;
    if (u.tile_m == t.tile_m && u.tile_n == t.tile_n && u.tile_k == t.tile_k && u.leaf_m == t.leaf_m &&
        u.leaf_n == t.leaf_n && u.stages == t.stages)
      return menu_entry_at(prec, i);
  }
  return nullptr;
}

int64_t entry_workspace_bytes(const MfmaEntry* e, int64_t m, int64_t n, int64_t k) {
  return (e && e->launch_staged) ? staged_workspace_bytes(e->prec, m, n, k) : 0;
}

}  // namespace hpvm
