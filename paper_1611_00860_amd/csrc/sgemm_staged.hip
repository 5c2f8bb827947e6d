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
// lo = bf16(x - hi).  The GEMM then moves 16-byte units with no edge checks:
// straight from HBM into a ring of LDS stages (sgemm_bf16_dma, BF16 and
// bf16x3), or for some bf16x3 tiles through registers two K-slabs ahead of
// the LDS stage being multiplied (sgemm_bf16_staged).  The hierarchy is the
// same as in the other lowerings: one workgroup per SgemmInternal instance,
// the Allocation node as LDS stages, SgemmLeaf outputs as MFMA accumulators.
// The backward's conversions (stage_backward) and its paired products
// (sgemm_bf16_dma_pair) live here too.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.hpp"
#include "hpvm_sgemm.h"
#include "internal.hpp"
#include "lds_dma.hpp"
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

int64_t staged_rows_pad(int64_t rows) { return (rows + kPadMN - 1) / kPadMN * kPadMN; }
int64_t staged_k_pad(int64_t k) { return (k + kPadK - 1) / kPadK * kPadK; }

static StagedLayout staged_layout(int32_t prec, int64_t m, int64_t n, int64_t k) {
  StagedLayout L;
  L.m_pad = staged_rows_pad(m);
  L.n_pad = staged_rows_pad(n);
  L.k_pad = staged_k_pad(k);
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

// Packs 8 elements' bfloat16 bits (and their lo parts) into 16-byte units.
template <bool X3>
__device__ __forceinline__ void pack8(const float (&v)[8], u32x4& hv, u32x4& lv) {
  uint16_t h[8], l[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) to_bf16<X3>(v[e], h[e], l[e]);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    hv[q] = (uint32_t)h[2 * q] | ((uint32_t)h[2 * q + 1] << 16);
    if constexpr (X3) lv[q] = (uint32_t)l[2 * q] | ((uint32_t)l[2 * q + 1] << 16);
  }
}

// A conversion whose contraction index runs along the rows of src (the
// copy form) or down its columns (the transposing form).  src is rows x
// cols FP32, element (r, c) at src[r * ld + c].
struct StageJob {
  const float* src;
  int64_t ld, rows, cols, rows_pad, cols_pad;
  uint16_t* hi;
  uint16_t* lo;
  int32_t vec;
  int64_t blocks;  // workgroups given to this job
};

// Copy form: -> [rows_pad][cols_pad] bfloat16, zero outside rows x cols.
// 8-element units are dealt to the job's workgroups in turn; each thread
// loads four units before storing any.
template <bool X3>
__device__ __forceinline__ void stage_rows_part(const StageJob& j, int64_t block) {
  const int64_t per_row = j.cols_pad / 8;
  const int64_t units = j.rows_pad * per_row;
  const int64_t stride = j.blocks * blockDim.x;
  auto load = [&](int64_t u, float (&v)[8]) {
    const int64_t r = u / per_row, c = (u - r * per_row) * 8;
    const float* p = j.src + r * j.ld + c;
    if (j.vec && r < j.rows && c + 8 <= j.cols) {
      const f32x4 a = *reinterpret_cast<const f32x4*>(p);
      const f32x4 b = *reinterpret_cast<const f32x4*>(p + 4);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        v[e] = a[e];
        v[e + 4] = b[e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (r < j.rows && c + e < j.cols) ? p[e] : 0.0f;
    }
  };
  auto store = [&](int64_t u, const float (&v)[8]) {
    const int64_t r = u / per_row, c = (u - r * per_row) * 8;
    u32x4 hv, lv;
    pack8<X3>(v, hv, lv);
    *reinterpret_cast<u32x4*>(j.hi + r * j.cols_pad + c) = hv;
    if constexpr (X3) *reinterpret_cast<u32x4*>(j.lo + r * j.cols_pad + c) = lv;
  };
  int64_t u = block * blockDim.x + threadIdx.x;
  for (; u + 3 * stride < units; u += 4 * stride) {
    float v[4][8];
#pragma unroll
    for (int i = 0; i < 4; ++i) load(u + i * stride, v[i]);
#pragma unroll
    for (int i = 0; i < 4; ++i) store(u + i * stride, v[i]);
  }
  for (; u < units; u += stride) {
    float v0[8];
    load(u, v0);
    store(u, v0);
  }
}

// Transposing form: -> [cols_pad][rows_pad] bfloat16, so that the
// contraction index is contiguous.  The 64 x 64 blocks (numbered row-major,
// cols_pad / 64 per block row) go through LDS; the job's workgroups take
// blocks wg, wg + blocks, ... and load the next block's rows while they
// write out the current one.
constexpr int kTB = 64;
// A block reads its rows in 16-byte units when the whole 64 x 64 block is
// inside the matrix and the rows allow them (vec), element by element
// otherwise; LDS rows are 65 floats, so both the row-wise writes and the
// column-wise reads of a wavefront fall on distinct banks.
template <bool X3>
__device__ __forceinline__ void stage_cols_part(const StageJob& j, int64_t wg, float (*t)[kTB + 1]) {
  constexpr int kV = kTB * kTB / 4 / 256;  // 16-byte loads per thread and block
  const int64_t col_blocks = j.cols_pad / kTB;
  const int64_t total = col_blocks * (j.rows_pad / kTB);
  const int tid = threadIdx.x;
  auto corner = [&](int64_t b, int64_t& r0, int64_t& c0) {
    r0 = (b / col_blocks) * kTB;
    c0 = (b % col_blocks) * kTB;
  };
  auto whole = [&](int64_t b) {
    int64_t r0, c0;
    corner(b, r0, c0);
    return j.vec && r0 + kTB <= j.rows && c0 + kTB <= j.cols;
  };
  auto load = [&](int64_t b, f32x4 (&v)[kV]) {
    int64_t r0, c0;
    corner(b, r0, c0);
#pragma unroll
    for (int i = 0; i < kV; ++i) {
      const int r = i * (256 / (kTB / 4)) + tid / (kTB / 4), c = (tid % (kTB / 4)) * 4;
      v[i] = *reinterpret_cast<const f32x4*>(j.src + (r0 + r) * j.ld + c0 + c);
    }
  };
  f32x4 v[kV];
  int64_t b = wg;
  bool fast = b < total && whole(b);
  if (fast) load(b, v);
  for (; b < total; b += j.blocks) {
    int64_t r0, c0;
    corner(b, r0, c0);
    if (fast) {
#pragma unroll
      for (int i = 0; i < kV; ++i) {
        const int r = i * (256 / (kTB / 4)) + tid / (kTB / 4), c = (tid % (kTB / 4)) * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) t[r][c + e] = v[i][e];
      }
    } else {
#pragma unroll
      for (int i = 0; i < kTB * kTB / 256; ++i) {
        const int r = i * (256 / kTB) + tid / kTB, c = tid % kTB;
        const int64_t gr = r0 + r, gc = c0 + c;
        t[r][c] = (gr < j.rows && gc < j.cols) ? j.src[gr * j.ld + gc] : 0.0f;
      }
    }
    __syncthreads();
    // The next block's rows are requested before this block is written out.
    const int64_t nb = b + j.blocks;
    const bool nfast = nb < total && whole(nb);
    if (nfast) load(nb, v);
#pragma unroll
    for (int q = 0; q < kTB * kTB / 8 / 256; ++q) {
      const int u = tid + q * 256;
      const int cc = u / (kTB / 8), kc = (u % (kTB / 8)) * 8;
      float w[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) w[e] = t[kc + e][cc];
      u32x4 hv, lv;
      pack8<X3>(w, hv, lv);
      const int64_t off = (c0 + cc) * j.rows_pad + r0 + kc;
      *reinterpret_cast<u32x4*>(j.hi + off) = hv;
      if constexpr (X3) *reinterpret_cast<u32x4*>(j.lo + off) = lv;
    }
    __syncthreads();  // LDS is rewritten by the next block
    fast = nfast;
  }
}

// One conversion, either form.
// Both operands of a product in one launch: the first a.blocks workgroups
// copy A (copy form), the rest transpose B, so the two passes overlap.
template <bool X3>
__global__ void __launch_bounds__(256) stage_pair(StageJob a, StageJob b) {
  __shared__ float t[kTB][kTB + 1];
  if ((int64_t)blockIdx.x < a.blocks) stage_rows_part<X3>(a, blockIdx.x);
  else stage_cols_part<X3>(b, blockIdx.x - a.blocks, t);
}

// The backward's pass over G (see stage_backward in internal.hpp): one
// workgroup per 64 x 64 block of the round256(m) x round256(n) padded
// matrix, row-major over blocks (col_blocks per block row).
// The block goes through LDS as in stage_cols_part; the row plane is written
// when the block's columns lie within round64(n), the transposed plane when
// its rows lie within round64(m).  Each thread's share of <G, Cin> follows a
// fixed element order, so the partials repeat bit for bit.
struct GradJob {
  const float* G;
  int64_t ldg;
  const float* Cin;
  int64_t ldci;
  float* dCin;
  int64_t lddci, m, n;
  float beta;
  float* partial;
  uint16_t *gh, *gl;
  int64_t n_kp;
  uint16_t *th, *tl;
  int64_t m_kp;
  int32_t vec;
  int64_t col_blocks, blocks;
};

template <bool X3>
__device__ __forceinline__ void stage_gradient_block(const GradJob& j, int64_t block, float (*t)[kTB + 1],
                                                     float* red) {
  const float* __restrict__ G = j.G;
  const float* __restrict__ Cin = j.Cin;
  float* __restrict__ dCin = j.dCin;
  float* __restrict__ partial = j.partial;
  const int64_t ldg = j.ldg, ldci = j.ldci, lddci = j.lddci, m = j.m, n = j.n;
  const float beta = j.beta;
  const int32_t vec = j.vec;
  const int64_t r0 = (block / j.col_blocks) * kTB, c0 = (block % j.col_blocks) * kTB;
  const int tid = threadIdx.x;
  float part = 0.0f;
  if (vec && r0 + kTB <= m && c0 + kTB <= n) {
    // Every load is issued before the first store, so the loads overlap.
    constexpr int kU = kTB * kTB / 4 / 256;
    f32x4 g[kU], cv[kU];
#pragma unroll
    for (int i = 0; i < kU; ++i) {
      const int r = i * (256 / (kTB / 4)) + tid / (kTB / 4), c = (tid % (kTB / 4)) * 4;
      g[i] = *reinterpret_cast<const f32x4*>(G + (r0 + r) * ldg + c0 + c);
      if (partial) cv[i] = *reinterpret_cast<const f32x4*>(Cin + (r0 + r) * ldci + c0 + c);
    }
#pragma unroll
    for (int i = 0; i < kU; ++i) {
      const int r = i * (256 / (kTB / 4)) + tid / (kTB / 4), c = (tid % (kTB / 4)) * 4;
      if (dCin)
        *reinterpret_cast<f32x4*>(dCin + (r0 + r) * lddci + c0 + c) =
            beta == 0.0f ? f32x4{0.0f, 0.0f, 0.0f, 0.0f} : beta * g[i];
      if (partial) {
#pragma unroll
        for (int e = 0; e < 4; ++e) part = fmaf(g[i][e], cv[i][e], part);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) t[r][c + e] = g[i][e];
    }
  } else {
#pragma unroll 4
    for (int i = 0; i < kTB * kTB / 256; ++i) {
      const int r = i * (256 / kTB) + tid / kTB, c = tid % kTB;
      const int64_t gr = r0 + r, gc = c0 + c;
      float g = 0.0f;
      if (gr < m && gc < n) {
        g = G[gr * ldg + gc];
        if (dCin) dCin[gr * lddci + gc] = beta == 0.0f ? 0.0f : beta * g;
        if (partial) part = fmaf(g, Cin[gr * ldci + gc], part);
      }
      t[r][c] = g;
    }
  }
  __syncthreads();
  uint16_t* __restrict__ gh = j.gh;
  uint16_t* __restrict__ gl = j.gl;
  uint16_t* __restrict__ th = j.th;
  uint16_t* __restrict__ tl = j.tl;
  const int64_t n_kp = j.n_kp, m_kp = j.m_kp;
  if (gh && c0 < n_kp) {
#pragma unroll
    for (int j = 0; j < kTB * kTB / 8 / 256; ++j) {
      const int u = tid + j * 256;
      const int r = u / (kTB / 8), c = (u % (kTB / 8)) * 8;
      float v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = t[r][c + e];
      u32x4 hv, lv;
      pack8<X3>(v, hv, lv);
      const int64_t off = (r0 + r) * n_kp + c0 + c;
      *reinterpret_cast<u32x4*>(gh + off) = hv;
      if constexpr (X3) *reinterpret_cast<u32x4*>(gl + off) = lv;
    }
  }
  if (th && r0 < m_kp) {
#pragma unroll
    for (int j = 0; j < kTB * kTB / 8 / 256; ++j) {
      const int u = tid + j * 256;
      const int cc = u / (kTB / 8), kc = (u % (kTB / 8)) * 8;
      float v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = t[kc + e][cc];
      u32x4 hv, lv;
      pack8<X3>(v, hv, lv);
      const int64_t off = (c0 + cc) * m_kp + r0 + kc;
      *reinterpret_cast<u32x4*>(th + off) = hv;
      if constexpr (X3) *reinterpret_cast<u32x4*>(tl + off) = lv;
    }
  }
  if (!partial) return;
  const float sum = block_sum(part, red);
  if (tid == 0) partial[block] = sum;
}

// The staged backward's conversions in one launch: g.blocks workgroups for
// the pass over G, then b.blocks copying B, then a's blocks transposing A
// (a job with no blocks is absent).  All are bound by HBM; one launch lets
// them overlap instead of each draining before the next starts.
template <bool X3>
__global__ void __launch_bounds__(256) stage_backward_k(GradJob g, StageJob b, StageJob a) {
  __shared__ float t[kTB][kTB + 1];
  __shared__ float red[256 / kWave];
  int64_t blk = blockIdx.x;
  if (blk < g.blocks) {
    stage_gradient_block<X3>(g, blk, t, red);
    return;
  }
  blk -= g.blocks;
  if (blk < b.blocks) stage_rows_part<X3>(b, blk);
  else stage_cols_part<X3>(a, blk - b.blocks, t);
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

// Backward epilogue (EPI = 1): C (may be null) <- alpha acc, and this
// workgroup's partial of dalpha, the sum over its tile of aorig .* acc, into
// partial[tile].  The aorig elements of up to 64 accumulator values
// per lane are loaded together before any store (a store to C may alias
// aorig as far as the compiler knows, so loads issued after it would wait
// for it).  Reuses `smem`: every LDS transfer must be complete.
template <int BM, int BN>
__device__ __forceinline__ void dalpha_epilogue(const StagedArgs& p, const f32x16 (&acc)[BM][BN], int row0,
                                                int col0, int lane, int tile, char* smem) {
  constexpr int kBatch = (BM * BN * 16 <= 64) ? BM : 1;  // row blocks loaded together
  float part = 0.0f;
#pragma unroll
  for (int b0 = 0; b0 < BM; b0 += kBatch) {
    float a[kBatch][BN][16];
#pragma unroll
    for (int bi = 0; bi < kBatch; ++bi)
#pragma unroll
      for (int bj = 0; bj < BN; ++bj) {
        const int j = col0 + 32 * bj + acc_col(lane);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int i = row0 + 32 * (b0 + bi) + acc_row(r, lane);
          a[bi][bj][r] = (i < p.m && j < p.n) ? p.aorig[(int64_t)i * p.lda_orig + j] : 0.0f;
        }
      }
#pragma unroll
    for (int bi = 0; bi < kBatch; ++bi)
#pragma unroll
      for (int bj = 0; bj < BN; ++bj) {
        const int j = col0 + 32 * bj + acc_col(lane);
        if (j >= p.n) continue;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int i = row0 + 32 * (b0 + bi) + acc_row(r, lane);
          if (i < p.m) {
            const float v = acc[b0 + bi][bj][r];
            if (p.C) p.C[(int64_t)i * p.ldc + j] = p.alpha * v;
            part = fmaf(a[bi][bj][r], v, part);
          }
        }
      }
  }
  const float sum = block_sum(part, reinterpret_cast<float*>(smem));
  if (threadIdx.x == 0) p.partial[tile] = sum;
}

// The bf16x3 GEMM over staged planes: each K-slab (hi and lo planes) is
// loaded into registers while the previous one, already in LDS, feeds the
// matrix cores, and is written to the other LDS stage after those MFMAs;
// one barrier per slab.  PIPE reads the fragments of the next 16-k step
// ahead of the current MFMAs.
template <int TM, int TN, int TK, int WM, int WN, bool X3, bool PIPE, int EPI>
__global__ void __launch_bounds__((TM / WM) * (TN / WN) * kWave)
    sgemm_bf16_staged(StagedArgs p) {
  using T = Bf16TileShape<TM, TN, TK, WM, WN, X3>;
  constexpr int NT = T::NT, BM = T::BM, BN = T::BN, RB = T::RB, P = T::kPlanes;
  constexpr int kUnitsPerRow = TK / 8;
  constexpr int UA = TM * kUnitsPerRow / NT, UB = TN * kUnitsPerRow / NT;
  static_assert(UA * NT == TM * kUnitsPerRow && UB * NT == TN * kUnitsPerRow, "even split");
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

  u32x4 ra[P * UA], rb[P * UB];
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
  load(ra, rb, 0);
  store(ra, rb, 0);
  __syncthreads();
  for (int s = 0; s < S; ++s) {
    const int st = s & 1;
    const bool more = s + 1 < S;
    if (more) load(ra, rb, s + 1);
    mfma_stage(st);
    if (more) store(ra, rb, st ^ 1);
    __syncthreads();
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
    dalpha_epilogue<BM, BN>(p, acc, (int)m0 + wm0, (int)n0 + wn0, lane, (int)blockIdx.x, smem);
  }
}


// ---------------------------------------------------------------------------
// DMA-fed BF16 GEMM over the staged planes.  Each K-slab of A and B goes
// from HBM straight into one of NST LDS stages (slab s + NST - 1 is
// requested while slab s is multiplied), so no register holds a slab in
// transit; the registers this frees keep two sets of MFMA fragments, and
// the fragments of a step are read while the previous step's MFMAs run.
// Both tiles are rows (m or n) of TK bf16 k values, laid out by
// SwizzledRows; the planes are padded, so no access needs a check.  With
// X3 (bf16x3) a stage holds the hi and lo planes of both operands,
// [A hi][A lo][B hi][B lo], and each step is lo*hi + hi*lo + hi*hi in the
// order of the fused lowering, so the two give the same bits.
// ---------------------------------------------------------------------------
template <int TM, int TN, int TK, int WM, int WN, int NST, bool X3 = false>
struct Bf16DmaShape {
  static constexpr int NW = (TM / WM) * (TN / WN), BM = WM / 32, BN = WN / 32;
  static constexpr int RB = 2 * TK;  // bytes of a row
  static constexpr int kPlanes = X3 ? 2 : 1;
  static constexpr int kABytes = TM * RB, kBBytes = TN * RB;  // one plane
  static constexpr int kBOff = kPlanes * kABytes;             // B hi within a stage
  static constexpr int kStage = kPlanes * (TM + TN) * RB;
  static constexpr int64_t kLdsBytes = (int64_t)NST * kStage;
  static constexpr int kRowsPerDma = SwizzledRows<RB>::kRowsPerDma;
  static constexpr int QA = TM / kRowsPerDma / NW, QB = TN / kRowsPerDma / NW, Q = kPlanes * (QA + QB);
  static constexpr int kMaxWaves = (163840 / (NST * kStage)) * NW / 4;
  static_assert(QA * NW * kRowsPerDma == TM && QB * NW * kRowsPerDma == TN && QA % 2 == 0 && QB % 2 == 0,
                "even DMA split");
  static_assert((TK / 16) % 2 == 0, "a slab's last step uses fragment buffer 1");
  static_assert((NST - 2) * Q < 64, "vmcnt range");
};

// Scheduling hint: NM MFMAs with NR LDS reads spread evenly among them.
template <int NR, int NM>
__device__ __forceinline__ void interleave_mfma_reads() {
  constexpr int per = NM / NR;
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x008, per, 0);  // MFMA
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);    // LDS read
  }
  if constexpr (NM - per * NR > 0) __builtin_amdgcn_sched_group_barrier(0x008, NM - per * NR, 0);
}

// One output tile (number `tile` of the product p) on this workgroup.
template <int TM, int TN, int TK, int WM, int WN, int NST, int EPI, bool X3 = false>
__device__ __forceinline__ void bf16_dma_tile(const StagedArgs& p, int tile, char* smem) {
  using S = Bf16DmaShape<TM, TN, TK, WM, WN, NST, X3>;
  using Lay = SwizzledRows<S::RB>;
  constexpr int BM = S::BM, BN = S::BN, QA = S::QA, QB = S::QB, KS = TK / 16, R = S::kRowsPerDma;
  constexpr int P = S::kPlanes;

  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int wm0 = (wave / (TN / WN)) * WM, wn0 = (wave % (TN / WN)) * WN;
  int tm, tn;
  tile_coords(p.tiles_m, p.tiles_n, tile, tm, tn);
  const int64_t m0 = (int64_t)tm * TM, n0 = (int64_t)tn * TN;
  const int64_t rowb = p.kp * 2;
  const uint32_t lds0 = lds_addr(smem);

  // This wave fills row slots [wave*QA*R, (wave+1)*QA*R) of each A plane of
  // the stage and the same share of each B plane; instruction j's group
  // parity is j's.
  const char* asrc[P];
  const char* bsrc[P];
  asrc[0] = reinterpret_cast<const char*>(p.ah) + (m0 + (int64_t)wave * QA * R) * rowb;
  bsrc[0] = reinterpret_cast<const char*>(p.bh) + (n0 + (int64_t)wave * QB * R) * rowb;
  if constexpr (X3) {
    asrc[P - 1] = reinterpret_cast<const char*>(p.al) + (m0 + (int64_t)wave * QA * R) * rowb;
    bsrc[P - 1] = reinterpret_cast<const char*>(p.bl) + (n0 + (int64_t)wave * QB * R) * rowb;
  }
  const uint32_t voff[2] = {Lay::src(lane, 0, rowb), Lay::src(lane, 1, rowb)};
  auto dma_slab = [&](int slab, int st) {
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const uint32_t la = lds0 + st * S::kStage + q * S::kABytes + wave * QA * 1024;
      const uint32_t lb = lds0 + st * S::kStage + S::kBOff + q * S::kBBytes + wave * QB * 1024;
      const char* a = asrc[q] + slab * S::RB;
      const char* b = bsrc[q] + slab * S::RB;
#pragma unroll
      for (int j = 0; j < QA; ++j) dma16(la + j * 1024, a + j * R * rowb, voff[j & 1]);
#pragma unroll
      for (int j = 0; j < QB; ++j) dma16(lb + j * 1024, b + j * R * rowb, voff[j & 1]);
    }
  };

  int foff[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) foff[ks] = Lay::frag(lane, ks);
  f32x16 acc[BM][BN];
  zero_acc(acc);
  // [buffer][plane][block]; plane 1 (lo) only with X3.
  bf16x8 fa[2][P][BM], fb[2][P][BN];
  // B first: a step's first MFMAs use A block 0 with every B block.
  auto read = [&](int buf, const char* st, int ks) {
#pragma unroll
    for (int q = 0; q < P; ++q)
#pragma unroll
      for (int bj = 0; bj < BN; ++bj)
        fb[buf][q][bj] = *reinterpret_cast<const bf16x8*>(st + S::kBOff + q * S::kBBytes + (wn0 + 32 * bj) * S::RB +
                                                          foff[ks]);
#pragma unroll
    for (int q = 0; q < P; ++q)
#pragma unroll
      for (int bi = 0; bi < BM; ++bi)
        fa[buf][q][bi] = *reinterpret_cast<const bf16x8*>(st + q * S::kABytes + (wm0 + 32 * bi) * S::RB + foff[ks]);
  };
  auto mfma = [&](int buf) {
    if constexpr (X3) {
#pragma unroll
      for (int bi = 0; bi < BM; ++bi)
#pragma unroll
        for (int bj = 0; bj < BN; ++bj) {
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[buf][1][bi], fb[buf][0][bj], acc[bi][bj], 0, 0, 0);
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[buf][0][bi], fb[buf][1][bj], acc[bi][bj], 0, 0, 0);
        }
    }
#pragma unroll
    for (int bi = 0; bi < BM; ++bi)
#pragma unroll
      for (int bj = 0; bj < BN; ++bj)
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[buf][0][bi], fb[buf][0][bj], acc[bi][bj], 0, 0, 0);
  };
  constexpr int kReads = P * (BM + BN), kMfmas = (X3 ? 3 : 1) * BM * BN;

  const int slabs = p.slabs;
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
    for (int ks = 0; ks + 1 < KS; ++ks) {
      read((ks + 1) & 1, cur, ks + 1);
      interleave_mfma_reads<kReads, kMfmas>();
      mfma(ks & 1);
    }
    // Slab s + 1 has landed everywhere and slab s is no longer read:
    // request slab s + NST into its stage (the last slab again past the
    // end, keeping the wait counts exact) and read slab s + 1's first step
    // under the last step's MFMAs.
    const int nst = st + 1 == NST ? 0 : st + 1;
    dma_wait_barrier<(NST - 2) * S::Q>();
    read(0, smem + nst * S::kStage, 0);
    dma_slab(s + NST < slabs ? s + NST : slabs - 1, st);
    interleave_mfma_reads<kReads, kMfmas>();
    mfma(1);
    st = nst;
  }
  // No transfer may still be writing LDS when it is reused or released.
  dma_wait_barrier<0>();

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
    dalpha_epilogue<BM, BN>(p, acc, (int)m0 + wm0, (int)n0 + wn0, lane, tile, smem);
  }
}

template <int TM, int TN, int TK, int WM, int WN, int NST, int EPI, bool X3>
__global__ void __launch_bounds__((Bf16DmaShape<TM, TN, TK, WM, WN, NST, X3>::NW * kWave))
    __attribute__((amdgpu_waves_per_eu(1, (Bf16DmaShape<TM, TN, TK, WM, WN, NST, X3>::kMaxWaves))))
    sgemm_bf16_dma(StagedArgs p) {
  extern __shared__ __align__(16) char smem[];
  bf16_dma_tile<TM, TN, TK, WM, WN, NST, EPI, X3>(p, blockIdx.x, smem);
}

// Two independent products in one launch: the tiles of p1 (with the dalpha
// epilogue when p1.partial is set), then those of p2.  Small products that
// give one tile per CU each get two co-resident workgroups per CU this way.
template <int TM, int TN, int TK, int WM, int WN, int NST, bool X3>
__global__ void __launch_bounds__((Bf16DmaShape<TM, TN, TK, WM, WN, NST, X3>::NW * kWave))
    __attribute__((amdgpu_waves_per_eu(1, (Bf16DmaShape<TM, TN, TK, WM, WN, NST, X3>::kMaxWaves))))
    sgemm_bf16_dma_pair(StagedArgs p1, StagedArgs p2) {
  extern __shared__ __align__(16) char smem[];
  const int n1 = p1.tiles_m * p1.tiles_n;
  const int t = blockIdx.x;
  if (t < n1) {
    if (p1.partial) bf16_dma_tile<TM, TN, TK, WM, WN, NST, 1, X3>(p1, t, smem);
    else bf16_dma_tile<TM, TN, TK, WM, WN, NST, 0, X3>(p1, t, smem);
  } else {
    bf16_dma_tile<TM, TN, TK, WM, WN, NST, 0, X3>(p2, t - n1, smem);
  }
}

namespace {

template <typename Kernel>
hipError_t allow_lds_staged(Kernel* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

StageJob rows_job(const float* src, int64_t ld, int64_t rows, int64_t cols, int64_t rows_pad, int64_t cols_pad,
                  uint16_t* hi, uint16_t* lo, int32_t vec) {
  const int64_t units = rows_pad * cols_pad / 8;
  return StageJob{src, ld, rows, cols, rows_pad, cols_pad, hi, lo, vec,
                  std::max<int64_t>(1, std::min<int64_t>((units + 1023) / 1024, 8192))};
}
StageJob cols_job(const float* src, int64_t ld, int64_t rows, int64_t cols, int64_t rows_pad, int64_t cols_pad,
                  uint16_t* hi, uint16_t* lo, int32_t vec) {
  // Up to 2048 workgroups (eight per CU), each looping over its blocks.
  return StageJob{src, ld, rows, cols, rows_pad, cols_pad, hi, lo, vec,
                  std::min<int64_t>((cols_pad / kTB) * (rows_pad / kTB), 2048)};
}


// The forward product's planes: A (m x k, k contiguous) copied row by row
// into [m_pad][k_pad], B (k x n) transposed through LDS into [n_pad][k_pad].
template <bool X3>
hipError_t stage_operands(const GemmArgs& a, const StagedLayout& L, char* ws, hipStream_t s) {
  uint16_t* ah = reinterpret_cast<uint16_t*>(ws);
  uint16_t* al = X3 ? reinterpret_cast<uint16_t*>(ws + L.a_plane) : nullptr;
  uint16_t* bh = reinterpret_cast<uint16_t*>(ws + L.planes * L.a_plane);
  uint16_t* bl = X3 ? reinterpret_cast<uint16_t*>(ws + L.planes * L.a_plane + L.b_plane) : nullptr;
  StageJob ja = rows_job(a.A, a.lda, a.m, a.k, L.m_pad, L.k_pad, ah, al, a.vec_a);
  StageJob jb = cols_job(a.B, a.ldb, a.k, a.n, L.k_pad, L.n_pad, bh, bl, a.vec_b);
  void* args[] = {&ja, &jb};
  return hipLaunchKernel(reinterpret_cast<const void*>(&stage_pair<X3>), dim3((unsigned)(ja.blocks + jb.blocks)),
                         dim3(256), args, 0, s);
}

}  // namespace

int64_t stage_gradient_blocks(int64_t m, int64_t n) {
  return (staged_rows_pad(m) / kTB) * (staged_rows_pad(n) / kTB);
}

hipError_t stage_backward(int32_t prec, const BackwardStaging& st, hipStream_t s) {
  GradJob g{st.G,   st.ldg, st.Cin, st.ldci, st.dCin, st.lddci, st.m, st.n, st.beta, st.partial, st.gh, st.gl,
            staged_k_pad(st.n), st.th, st.tl, staged_k_pad(st.m), st.vec_g, staged_rows_pad(st.n) / kTB,
            stage_gradient_blocks(st.m, st.n)};
  StageJob b{}, a{};
  if (st.bh) b = rows_job(st.B, st.ldb, st.k, st.n, staged_rows_pad(st.k), staged_k_pad(st.n), st.bh, st.bl, st.vec_b);
  if (st.ah) a = cols_job(st.A, st.lda, st.m, st.k, staged_k_pad(st.m), staged_rows_pad(st.k), st.ah, st.al, st.vec_a);
  void* args[] = {&g, &b, &a};
  const void* fn = prec == HPVM_PREC_BF16X3 ? reinterpret_cast<const void*>(&stage_backward_k<true>)
                                            : reinterpret_cast<const void*>(&stage_backward_k<false>);
  return hipLaunchKernel(fn, dim3((unsigned)(g.blocks + b.blocks + a.blocks)), dim3(256), args, 0, s);
}

namespace {

// The planes of layout L in workspace ws.
template <bool X3>
StagedPlanes planes_in(const StagedLayout& L, char* ws) {
  StagedPlanes P;
  P.ah = reinterpret_cast<const uint16_t*>(ws);
  P.al = X3 ? reinterpret_cast<const uint16_t*>(ws + L.a_plane) : nullptr;
  P.bh = reinterpret_cast<const uint16_t*>(ws + L.planes * L.a_plane);
  P.bl = X3 ? reinterpret_cast<const uint16_t*>(ws + L.planes * L.a_plane + L.b_plane) : nullptr;
  return P;
}

// Kernel arguments for a product on planes P (rows of round64(a.k)).
StagedArgs staged_args(const GemmArgs& a, const StagedPlanes& P, int tm, int tn, int tk, const float* aorig,
                       int64_t lda_orig, float* partial) {
  StagedArgs p{};
  p.ah = P.ah;
  p.al = P.al;
  p.bh = P.bh;
  p.bl = P.bl;
  p.kp = staged_k_pad(a.k);
  p.C = a.C;
  p.ldc = a.ldc;
  p.m = a.m;
  p.n = a.n;
  p.slabs = (int32_t)(p.kp / tk);
  p.tiles_m = (a.m + tm - 1) / tm;
  p.tiles_n = (a.n + tn - 1) / tn;
  p.alpha = a.alpha;
  p.beta = a.beta;
  p.aorig = aorig;
  p.lda_orig = lda_orig;
  p.partial = partial;
  return p;
}

template <int TM, int TN, int TK, int WM, int WN, bool X3, bool PIPE>
struct StagedConfig {
  using T = Bf16TileShape<TM, TN, TK, WM, WN, X3>;
  static constexpr int kThreads = T::NT;
  static_assert(kPadMN % TM == 0 && kPadMN % TN == 0 && kPadK % TK == 0, "padding covers the tile");

  template <int EPI>
  static hipError_t gemm(const GemmArgs& a, const StagedPlanes& P, const float* aorig, int64_t lda_orig,
                         float* partial, hipStream_t s) {
    StagedArgs p = staged_args(a, P, TM, TN, TK, aorig, lda_orig, partial);
    auto* fn = &sgemm_bf16_staged<TM, TN, TK, WM, WN, X3, PIPE, EPI>;
    hipError_t e = allow_lds_staged(fn, (size_t)T::kLdsBytes);
    if (e != hipSuccess) return e;
    void* kargs[] = {&p};
    return hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3((unsigned)(p.tiles_m * p.tiles_n)),
                           dim3(kThreads), kargs, (size_t)T::kLdsBytes, s);
  }
  static hipError_t launch(const GemmArgs& a, void* workspace, hipStream_t s) {
    const StagedLayout L = staged_layout(X3 ? HPVM_PREC_BF16X3 : HPVM_PREC_BF16, a.m, a.n, a.k);
    char* ws = reinterpret_cast<char*>(workspace);
    hipError_t e = stage_operands<X3>(a, L, ws, s);
    if (e != hipSuccess) return e;
    return gemm<0>(a, planes_in<X3>(L, ws), nullptr, 0, nullptr, s);
  }
  static hipError_t launch_planes(const GemmArgs& a, const StagedPlanes& P, const float* aorig, int64_t lda_orig,
                                  float* partial, hipStream_t s) {
    return partial ? gemm<1>(a, P, aorig, lda_orig, partial, s) : gemm<0>(a, P, nullptr, 0, nullptr, s);
  }
};

#define HPVM_STAGED_ENTRY(PREC, X3, PIPE, TM, TN, TK, WM, WN)                                           \
  {{TM, TN, TK, WM, WN, 3}, PREC, StagedConfig<TM, TN, TK, WM, WN, X3, PIPE>::kThreads,                  \
   Bf16TileShape<TM, TN, TK, WM, WN, X3>::kLdsBytes, nullptr,                                             \
   &StagedConfig<TM, TN, TK, WM, WN, X3, PIPE>::launch,                                                  \
   &StagedConfig<TM, TN, TK, WM, WN, X3, PIPE>::launch_planes}

// BF16 and bf16x3 on the DMA-fed kernel (NST LDS stages); same planes and
// workspace as the other staged entries.
template <int TM, int TN, int TK, int WM, int WN, int NST, bool X3>
struct DmaConfig {
  using S = Bf16DmaShape<TM, TN, TK, WM, WN, NST, X3>;
  static constexpr int kThreads = S::NW * kWave;
  static_assert(kPadMN % TM == 0 && kPadMN % TN == 0 && kPadK % TK == 0, "padding covers the tile");

  template <int EPI>
  static hipError_t gemm(const GemmArgs& a, const StagedPlanes& P, const float* aorig, int64_t lda_orig,
                         float* partial, hipStream_t s) {
    StagedArgs p = staged_args(a, P, TM, TN, TK, aorig, lda_orig, partial);
    auto* fn = &sgemm_bf16_dma<TM, TN, TK, WM, WN, NST, EPI, X3>;
    hipError_t e = allow_lds_staged(fn, (size_t)S::kLdsBytes);
    if (e != hipSuccess) return e;
    void* kargs[] = {&p};
    return hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3((unsigned)(p.tiles_m * p.tiles_n)),
                           dim3(kThreads), kargs, (size_t)S::kLdsBytes, s);
  }
  static hipError_t launch(const GemmArgs& a, void* workspace, hipStream_t s) {
    const StagedLayout L = staged_layout(X3 ? HPVM_PREC_BF16X3 : HPVM_PREC_BF16, a.m, a.n, a.k);
    char* ws = reinterpret_cast<char*>(workspace);
    hipError_t e = stage_operands<X3>(a, L, ws, s);
    if (e != hipSuccess) return e;
    return gemm<0>(a, planes_in<X3>(L, ws), nullptr, 0, nullptr, s);
  }
  static hipError_t launch_planes(const GemmArgs& a, const StagedPlanes& P, const float* aorig, int64_t lda_orig,
                                  float* partial, hipStream_t s) {
    return partial ? gemm<1>(a, P, aorig, lda_orig, partial, s) : gemm<0>(a, P, nullptr, 0, nullptr, s);
  }
  static hipError_t launch_pair(const GemmArgs& a1, const StagedPlanes& P1, const float* aorig, int64_t lda_orig,
                                float* partial, const GemmArgs& a2, const StagedPlanes& P2, hipStream_t s) {
    StagedArgs p1 = staged_args(a1, P1, TM, TN, TK, aorig, lda_orig, partial);
    StagedArgs p2 = staged_args(a2, P2, TM, TN, TK, nullptr, 0, nullptr);
    auto* fn = &sgemm_bf16_dma_pair<TM, TN, TK, WM, WN, NST, X3>;
    hipError_t e = allow_lds_staged(fn, (size_t)S::kLdsBytes);
    if (e != hipSuccess) return e;
    void* kargs[] = {&p1, &p2};
    const int64_t tiles = (int64_t)p1.tiles_m * p1.tiles_n + (int64_t)p2.tiles_m * p2.tiles_n;
    return hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3((unsigned)tiles), dim3(kThreads), kargs,
                           (size_t)S::kLdsBytes, s);
  }
};

#define HPVM_DMA_ENTRY_P(PREC, X3, NST, TM, TN, TK, WM, WN)                                               \
  {{TM, TN, TK, WM, WN, 3}, PREC, DmaConfig<TM, TN, TK, WM, WN, NST, X3>::kThreads,                      \
   DmaConfig<TM, TN, TK, WM, WN, NST, X3>::S::kLdsBytes, nullptr,                                          \
   &DmaConfig<TM, TN, TK, WM, WN, NST, X3>::launch, &DmaConfig<TM, TN, TK, WM, WN, NST, X3>::launch_planes, \
   &DmaConfig<TM, TN, TK, WM, WN, NST, X3>::launch_pair}
#define HPVM_DMA_ENTRY(NST, TM, TN, TK, WM, WN) HPVM_DMA_ENTRY_P(HPVM_PREC_BF16, false, NST, TM, TN, TK, WM, WN)

const MfmaEntry kStagedMenuBf16[] = {
    HPVM_DMA_ENTRY(2, 256, 256, 64, 128, 64),
    HPVM_DMA_ENTRY(3, 256, 256, 32, 128, 64),
    HPVM_DMA_ENTRY(3, 256, 128, 64, 128, 64),
    HPVM_DMA_ENTRY(2, 128, 128, 64, 64, 64),
    HPVM_DMA_ENTRY(2, 128, 128, 64, 64, 32),
};
const MfmaEntry kStagedMenuBf16x3[] = {
    HPVM_DMA_ENTRY_P(HPVM_PREC_BF16X3, true, 2, 256, 256, 32, 128, 64),
    HPVM_STAGED_ENTRY(HPVM_PREC_BF16X3, true, true, 256, 128, 32, 128, 64),
    HPVM_STAGED_ENTRY(HPVM_PREC_BF16X3, true, true, 128, 128, 64, 64, 64),
    HPVM_DMA_ENTRY_P(HPVM_PREC_BF16X3, true, 2, 128, 128, 64, 64, 32),
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
