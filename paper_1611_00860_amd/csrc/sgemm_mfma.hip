// MFMA lowerings of the sgemm dataflow graph for CDNA4 (gfx950).
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
// The dynamic instances of SgemmInternal are independent (Sec. 2.1), so the
// tiles may run in any order; the order chosen keeps the tiles in flight on
// one XCD close together so that they share that XCD's L2.
#include "device_common.hpp"
#include "internal.hpp"

#include <type_traits>

namespace hpvm {

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

// Epilogue: C <- alpha * acc + beta * C, element-wise, masked at the edges.
// Output (i, j) of a 32 x 32 block lives in lane j + 32 * ((i / 4) % 2),
// register (i % 4) + 4 * (i / 8).
template <int BM, int BN>
__device__ __forceinline__ void store_c(const GemmArgs& p, const f32x16 (&acc)[BM][BN], int row0,
                                        int col0, int lane) {
  const int r32 = lane & 31, h = lane >> 5;
#pragma unroll
  for (int bi = 0; bi < BM; ++bi)
#pragma unroll
    for (int bj = 0; bj < BN; ++bj) {
      const int j = col0 + 32 * bj + r32;
      if (j >= p.n) continue;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = row0 + 32 * bi + 8 * (r >> 2) + 4 * h + (r & 3);
        if (i < p.m) {
          float* c = p.C + (int64_t)i * p.ldc + j;
          float v = p.alpha * acc[bi][bj][r];
          if (p.beta != 0.0f) v = fmaf(p.beta, *c, v);
          *c = v;
        }
      }
    }
}

// ---------------------------------------------------------------------------
// FP32 kernel: v_mfma_f32_32x32x2f32, FP32 operands and accumulation.
// ---------------------------------------------------------------------------
template <int TM, int TN, int TK, int WM, int WN, bool AT, bool BT>
__global__ void __launch_bounds__((TM / WM) * (TN / WN) * kWave)
    sgemm_mfma_f32(GemmArgs p) {
  constexpr int kWavesN = TN / WN;
  constexpr int NT = (TM / WM) * kWavesN * kWave;
  constexpr int BM = WM / 32, BN = WN / 32;
  static_assert(TK % 8 == 0, "K slab must hold whole groups of 8");
  using OpA = F32Operand<TM, TK, !AT>;
  using OpB = F32Operand<TN, TK, BT>;

  extern __shared__ __align__(16) float lds[];
  float* As0 = lds;
  float* As1 = lds + OpA::kFloats;
  float* Bs0 = lds + 2 * OpA::kFloats;
  float* Bs1 = Bs0 + OpB::kFloats;

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid / kWave;
  const int wm0 = (wave / kWavesN) * WM, wn0 = (wave % kWavesN) * WN;
  int tm, tn;
  tile_coords(p.tiles_m, p.tiles_n, blockIdx.x, tm, tn);
  const int m0 = tm * TM, n0 = tn * TN;

  GlobalTile<OpA::kRows, OpA::kCols, NT> ga;
  GlobalTile<OpB::kRows, OpB::kCols, NT> gb;
  auto fetch = [&](int k0) {
    const float* base;
    int rl, cl;
    slab_a<AT>(p, m0, k0, base, rl, cl);
    ga.load(base, p.lda, rl, cl, p.vec_a, tid);
    slab_b<BT>(p, n0, k0, base, rl, cl);
    gb.load(base, p.ldb, rl, cl, p.vec_b, tid);
  };

  f32x16 acc[BM][BN];
#pragma unroll
  for (int bi = 0; bi < BM; ++bi)
#pragma unroll
    for (int bj = 0; bj < BN; ++bj)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[bi][bj][r] = 0.0f;

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
  store_c<BM, BN>(p, acc, m0 + wm0, n0 + wn0, lane);
}

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

  __device__ __forceinline__ void load(const float* __restrict__ base, int64_t ld, int rlim,
                                       int clim, bool vec, int tid) {
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int u = tid + j * NT;
      const int r = u / kUnitsPerRow;
      const int c = (u % kUnitsPerRow) * 8;
      const float* p = base + (int64_t)r * ld + c;
      if (vec && r < rlim && c + 8 <= clim) {
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
        if (vec && r < rlim && c + 4 <= clim) {
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

// ---------------------------------------------------------------------------
// BF16 kernel (X3 = false) and bf16x3 kernel (X3 = true): FP32 storage, FP32
// accumulation; the products are bf16 x bf16 on v_mfma_f32_32x32x16_bf16.
// bf16x3 accumulates lo*hi, hi*lo and hi*hi into the same accumulator.
// ---------------------------------------------------------------------------
template <int TM, int TN, int TK, int WM, int WN, bool AT, bool BT, bool X3>
__global__ void __launch_bounds__((TM / WM) * (TN / WN) * kWave)
    sgemm_mfma_bf16(GemmArgs p) {
  constexpr int kWavesN = TN / WN;
  constexpr int NT = (TM / WM) * kWavesN * kWave;
  constexpr int BM = WM / 32, BN = WN / 32;
  constexpr int RB = Bf16Rows<TK>::kRowBytes;
  constexpr int kPlanes = X3 ? 2 : 1;
  constexpr int kABytes = TM * RB, kBBytes = TN * RB;
  constexpr int kStageBytes = kPlanes * (kABytes + kBBytes);
  static_assert(TK % 16 == 0, "K slab must hold whole MFMA steps of 16");

  extern __shared__ __align__(16) char smem[];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid / kWave;
  const int wm0 = (wave / kWavesN) * WM, wn0 = (wave % kWavesN) * WN;
  int tm, tn;
  tile_coords(p.tiles_m, p.tiles_n, blockIdx.x, tm, tn);
  const int m0 = tm * TM, n0 = tn * TN;

  // stage layout: [A hi][A lo][B hi][B lo] (lo planes only with X3)
  auto a_hi = [&](int st) { return smem + st * kStageBytes; };
  auto a_lo = [&](int st) { return smem + st * kStageBytes + kABytes; };
  auto b_hi = [&](int st) { return smem + st * kStageBytes + kPlanes * kABytes; };
  auto b_lo = [&](int st) { return smem + st * kStageBytes + kPlanes * kABytes + kBBytes; };

  Bf16Tile<!AT, TM, TK, NT> ga;
  Bf16Tile<BT, TN, TK, NT> gb;
  auto fetch = [&](int k0) {
    const float* base;
    int rl, cl;
    slab_a<AT>(p, m0, k0, base, rl, cl);
    ga.load(base, p.lda, rl, cl, p.vec_a, tid);
    slab_b<BT>(p, n0, k0, base, rl, cl);
    gb.load(base, p.ldb, rl, cl, p.vec_b, tid);
  };
  auto stash = [&](int st) {
    ga.template store<X3>(a_hi(st), a_lo(st), tid);
    gb.template store<X3>(b_hi(st), b_lo(st), tid);
  };

  f32x16 acc[BM][BN];
#pragma unroll
  for (int bi = 0; bi < BM; ++bi)
#pragma unroll
    for (int bj = 0; bj < BN; ++bj)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[bi][bj][r] = 0.0f;

  const int slabs = (p.k + TK - 1) / TK;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int s = 0; s < slabs; ++s) {
    const int st = s & 1;
    const bool more = s + 1 < slabs;
    if (more) fetch((s + 1) * TK);
#pragma unroll
    for (int ks = 0; ks < TK / 16; ++ks) {
      bf16x8 ah[BM], bh[BN];
#pragma unroll
      for (int bi = 0; bi < BM; ++bi) ah[bi] = frag_bf16(a_hi(st), wm0 + 32 * bi, ks, lane, RB);
#pragma unroll
      for (int bj = 0; bj < BN; ++bj) bh[bj] = frag_bf16(b_hi(st), wn0 + 32 * bj, ks, lane, RB);
      if constexpr (X3) {
        bf16x8 al[BM], bl[BN];
#pragma unroll
        for (int bi = 0; bi < BM; ++bi) al[bi] = frag_bf16(a_lo(st), wm0 + 32 * bi, ks, lane, RB);
#pragma unroll
        for (int bj = 0; bj < BN; ++bj) bl[bj] = frag_bf16(b_lo(st), wn0 + 32 * bj, ks, lane, RB);
#pragma unroll
        for (int bi = 0; bi < BM; ++bi)
#pragma unroll
          for (int bj = 0; bj < BN; ++bj) {
            acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[bi], bh[bj], acc[bi][bj], 0, 0, 0);
            acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[bi], bl[bj], acc[bi][bj], 0, 0, 0);
          }
      }
#pragma unroll
      for (int bi = 0; bi < BM; ++bi)
#pragma unroll
        for (int bj = 0; bj < BN; ++bj)
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[bi], bh[bj], acc[bi][bj], 0, 0, 0);
    }
    if (more) stash(st ^ 1);
    __syncthreads();
  }
  store_c<BM, BN>(p, acc, m0 + wm0, n0 + wn0, lane);
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
    const int64_t a = at ? F32Operand<TM, TK, false>::kFloats : F32Operand<TM, TK, true>::kFloats;
    const int64_t b = bt ? F32Operand<TN, TK, true>::kFloats : F32Operand<TN, TK, false>::kFloats;
    return 2 * (a + b) * (int64_t)sizeof(float);
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
  static constexpr int64_t lds(bool, bool) {
    return 2 * (X3 ? 2 : 1) * (int64_t)(TM + TN) * Bf16Rows<TK>::kRowBytes;
  }
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

static const MfmaEntry kF32Menu[] = {
    HPVM_F32_ENTRY(128, 128, 16, 64, 64),
    HPVM_F32_ENTRY(256, 128, 16, 128, 64),
    HPVM_F32_ENTRY(128, 128, 32, 64, 64),
    HPVM_F32_ENTRY(64, 64, 16, 32, 32),
    HPVM_F32_ENTRY(128, 64, 16, 64, 32),
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
