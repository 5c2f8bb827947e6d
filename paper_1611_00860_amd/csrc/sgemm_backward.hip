// Backward pass of the sgemm node: C_out = alpha A B + beta C_in.
//
// dA = alpha G B^T reuses the MFMA main loop with B read in transposed form
// and folds the scalar gradient dalpha = <A, G B^T> into its epilogue (A is
// read once more, tile by tile, where dA is written).  dB = alpha A^T G is a
// plain launch of the main loop with A read in transposed form.  One
// element-wise pass writes dC_in = beta G and the partial sums of
// dbeta = <G, C_in>; a single workgroup then reduces the partials.  Every
// reduction is FP32 with a fixed order, so results repeat bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.hpp"
#include "hpvm_sgemm.h"
#include "internal.hpp"
#include "mfma_bf16.hpp"
#include "mfma_f32.hpp"

namespace hpvm {

// Sum over a wavefront with a fixed butterfly.
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Sum over the workgroup; the result is valid in thread 0.  `red` holds one
// float per wavefront.  Ends with every thread past a barrier.
__device__ __forceinline__ float block_sum(float v, float* red) {
  v = wave_sum(v);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  float t = 0.0f;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += red[w];
  __syncthreads();
  return t;
}

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
  float part = 0.0f;
#pragma unroll
  for (int bi = 0; bi < BM; ++bi)
#pragma unroll
    for (int bj = 0; bj < BN; ++bj) {
      const int j = col0 + 32 * bj + acc_col(lane);
      if (j >= p.n) continue;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = row0 + 32 * bi + acc_row(r, lane);
        if (i < p.m) {
          const float v = acc[bi][bj][r];
          if (p.C) p.C[(int64_t)i * p.ldc + j] = p.alpha * v;
          part = fmaf(Aorig[(int64_t)i * lda + j], v, part);
        }
      }
    }
  const float s = block_sum(part, reinterpret_cast<float*>(smem));
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

constexpr int kElemThreads = 256;
constexpr int kElemBlocks = 1024;

// dC_in = beta G (zeros when beta == 0) and per-block partials of <G, C_in>.
__global__ void __launch_bounds__(kElemThreads)
    sgemm_grad_c(const float* __restrict__ G, int64_t ldg, const float* __restrict__ Cin, int64_t ldci,
                 float* __restrict__ dCin, int64_t lddci, int64_t m, int64_t n, float beta,
                 float* __restrict__ partial) {
  __shared__ float red[kElemThreads / kWave];
  const int64_t total = m * n;
  float part = 0.0f;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / n, j = e - i * n;
    const float g = G[i * ldg + j];
    if (dCin) dCin[i * lddci + j] = (beta == 0.0f) ? 0.0f : beta * g;
    if (partial) part = fmaf(g, Cin[i * ldci + j], part);
  }
  if (!partial) return;
  const float s = block_sum(part, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Final fixed-order reduction of both partial arrays.
__global__ void __launch_bounds__(kElemThreads)
    sgemm_grad_finish(const float* __restrict__ pa, int32_t na, const float* __restrict__ pb, int32_t nb,
                      float* dalpha, float* dbeta) {
  __shared__ float red[kElemThreads / kWave];
  float a = 0.0f, b = 0.0f;
  for (int t = threadIdx.x; t < na; t += blockDim.x) a += pa[t];
  for (int t = threadIdx.x; t < nb; t += blockDim.x) b += pb[t];
  const float sa = block_sum(a, red);
  const float sb = block_sum(b, red);
  if (threadIdx.x == 0) {
    if (dalpha) *dalpha = sa;
    if (dbeta) *dbeta = sb;
  }
}

namespace {

struct BwdConfig {
  hpvm_tile tile;  // also the dB launch's tile (must be in the menu)
  int32_t prec;
  int32_t threads;
  int64_t lds;
  void (*grad_a)(GemmArgs, const float*, int64_t, float*);
};

template <int TM, int TN, int TK, int WM, int WN, int PREC>
constexpr BwdConfig bwd_entry() {
  constexpr int64_t lds = PREC == HPVM_PREC_FP32
                              ? F32Tile<TM, TN, TK, WM, WN, false, true>::kLdsBytes
                              : Bf16TileShape<TM, TN, TK, WM, WN, PREC == HPVM_PREC_BF16X3>::kLdsBytes;
  return BwdConfig{{TM, TN, TK, WM, WN, 2}, PREC, (TM / WM) * (TN / WN) * kWave, lds,
                   &sgemm_grad_a<TM, TN, TK, WM, WN, PREC>};
}

// Preference order per precision: largest tile first.
const BwdConfig kBwd[] = {
    bwd_entry<128, 128, 16, 64, 64, HPVM_PREC_FP32>(),
    bwd_entry<128, 64, 16, 64, 32, HPVM_PREC_FP32>(),
    bwd_entry<64, 64, 16, 32, 32, HPVM_PREC_FP32>(),
    bwd_entry<128, 128, 32, 64, 64, HPVM_PREC_BF16>(),
    bwd_entry<64, 64, 32, 32, 32, HPVM_PREC_BF16>(),
    bwd_entry<128, 128, 32, 64, 64, HPVM_PREC_BF16X3>(),
    bwd_entry<64, 64, 32, 32, 32, HPVM_PREC_BF16X3>(),
};
constexpr int kNumBwd = sizeof(kBwd) / sizeof(kBwd[0]);

// Enough tiles to give every CU of a 256-CU part two workgroups, else the
// smallest tile.
constexpr int64_t kTargetTiles = 512;

int64_t tiles_for(const hpvm_tile& t, int64_t rows, int64_t cols) {
  return ((rows + t.tile_m - 1) / t.tile_m) * ((cols + t.tile_n - 1) / t.tile_n);
}

const BwdConfig* pick(int32_t prec, int64_t rows, int64_t cols) {
  const BwdConfig* last = nullptr;
  for (int i = 0; i < kNumBwd; ++i) {
    if (kBwd[i].prec != prec) continue;
    last = &kBwd[i];
    if (tiles_for(kBwd[i].tile, rows, cols) >= kTargetTiles) return last;
  }
  return last;
}

const MfmaEntry* menu_entry(int32_t prec, const hpvm_tile& t) {
  const MfmaEntry* menu;
  const int n = mfma_menu(prec, &menu);
  for (int i = 0; i < n; ++i) {
    const hpvm_tile& u = menu[i].tile;
    if (u.tile_m == t.tile_m && u.tile_n == t.tile_n && u.tile_k == t.tile_k && u.leaf_m == t.leaf_m &&
        u.leaf_n == t.leaf_n && u.stages == t.stages)
      return &menu[i];
  }
  return nullptr;
}

int64_t elem_blocks(int64_t m, int64_t n) {
  return std::max<int64_t>(1, std::min<int64_t>(kElemBlocks, (m * n + kElemThreads - 1) / kElemThreads));
}

// Partial-sum slots: dA tiles, then element-wise blocks (16-byte aligned).
int64_t ws_floats(int32_t prec, int64_t m, int64_t n, int64_t k, int64_t* na) {
  const BwdConfig* c = pick(prec, m, k);
  *na = (m > 0 && k > 0) ? tiles_for(c->tile, m, k) : 0;
  return ((*na + 3) / 4) * 4 + elem_blocks(m, n);
}

bool aligned16(const void* p, int64_t ld) { return ((uintptr_t)p % 16 == 0) && (ld % 4 == 0); }

}  // namespace
}  // namespace hpvm

using namespace hpvm;

extern "C" {

int hpvm_sgemm_backward_workspace_bytes(int64_t m, int64_t n, int64_t k, int32_t prec, int64_t* bytes) {
  if (m < 0 || n < 0 || k < 0) return set_error(HPVM_INVALID_ARG, "sizes must be >= 0");
  if (prec < HPVM_PREC_FP32 || prec > HPVM_PREC_BF16X3)
    return set_error(HPVM_INVALID_ARG, "argument 4: unknown precision %d", prec);
  if (!bytes) return set_error(HPVM_INVALID_ARG, "argument 5: bytes is NULL");
  int64_t na;
  *bytes = ws_floats(prec, m, n, k, &na) * (int64_t)sizeof(float);
  return clear_error();
}

int hpvm_sgemm_backward(int64_t m, int64_t n, int64_t k, float alpha, float beta, const float* A, int64_t lda,
                        const float* B, int64_t ldb, const float* C_in, int64_t ldci, const float* G, int64_t ldg,
                        float* dA, int64_t ldda, float* dB, int64_t lddb, float* dC_in, int64_t lddci,
                        float* dalpha, float* dbeta, int32_t prec, void* workspace, int64_t workspace_bytes,
                        void* stream) {
  if (m < 0) return set_error(HPVM_INVALID_ARG, "argument 1: m = %lld < 0", (long long)m);
  if (n < 0) return set_error(HPVM_INVALID_ARG, "argument 2: n = %lld < 0", (long long)n);
  if (k < 0) return set_error(HPVM_INVALID_ARG, "argument 3: k = %lld < 0", (long long)k);
  if (m > INT32_MAX || n > INT32_MAX || k > INT32_MAX)
    return set_error(HPVM_UNSUPPORTED, "sizes above 2^31 - 1 are not supported");
  const bool mn = m > 0 && n > 0, mk = m > 0 && k > 0, kn = k > 0 && n > 0;
  const bool want_a = dA != nullptr || dalpha != nullptr;  // dalpha rides on dA's pass
  const bool need_A = (want_a && mk && n > 0) || (dB && kn && m > 0);
  const bool need_B = want_a && mk && n > 0;
  if (need_A && !A) return set_error(HPVM_INVALID_ARG, "argument 6: A is NULL");
  if (lda < std::max<int64_t>(1, k)) return set_error(HPVM_INVALID_ARG, "argument 7: lda < max(1, k)");
  if (need_B && !B) return set_error(HPVM_INVALID_ARG, "argument 8: B is NULL");
  if (ldb < std::max<int64_t>(1, n)) return set_error(HPVM_INVALID_ARG, "argument 9: ldb < max(1, n)");
  if (dbeta && mn && !C_in) return set_error(HPVM_INVALID_ARG, "argument 10: C_in is NULL");
  if (ldci < std::max<int64_t>(1, n)) return set_error(HPVM_INVALID_ARG, "argument 11: ldci < max(1, n)");
  if (mn && !G && (want_a || dB || dC_in || dbeta)) return set_error(HPVM_INVALID_ARG, "argument 12: G is NULL");
  if (ldg < std::max<int64_t>(1, n)) return set_error(HPVM_INVALID_ARG, "argument 13: ldg < max(1, n)");
  if (ldda < std::max<int64_t>(1, k)) return set_error(HPVM_INVALID_ARG, "argument 15: ldda < max(1, k)");
  if (lddb < std::max<int64_t>(1, n)) return set_error(HPVM_INVALID_ARG, "argument 17: lddb < max(1, n)");
  if (lddci < std::max<int64_t>(1, n)) return set_error(HPVM_INVALID_ARG, "argument 19: lddci < max(1, n)");
  if (prec < HPVM_PREC_FP32 || prec > HPVM_PREC_BF16X3)
    return set_error(HPVM_INVALID_ARG, "argument 22: unknown precision %d", prec);
  int64_t na;
  const int64_t need = ws_floats(prec, m, n, k, &na) * (int64_t)sizeof(float);
  if ((dalpha || dbeta) && !workspace) return set_error(HPVM_INVALID_ARG, "argument 23: workspace is NULL");
  if ((dalpha || dbeta) && workspace_bytes < need)
    return set_error(HPVM_WORKSPACE_TOO_SMALL, "argument 24: workspace has %lld bytes, needs %lld",
                     (long long)workspace_bytes, (long long)need);
  if (workspace && (uintptr_t)workspace % 16)
    return set_error(HPVM_INVALID_ARG, "argument 23: workspace is not 16-byte aligned");
  if (fault_injected("launch")) return set_error(HPVM_HIP_ERROR, "injected launch failure (HPVM_FAULT_INJECT)");

  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  float* pa = reinterpret_cast<float*>(workspace);
  float* pb = pa ? pa + ((na + 3) / 4) * 4 : nullptr;
  const int64_t nb = elem_blocks(m, n);
  hipError_t e = hipSuccess;
  const BwdConfig* cfg = pick(prec, m, k);

  // dA (and dalpha's partials): contraction over n.
  if (want_a && mk) {
    if (n == 0) {
      if (dA) e = launch_scale(dA, ldda, m, k, 0.0f, s);
      na = 0;
    } else {
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
      a.vec_a = aligned16(G, ldg);
      a.vec_b = aligned16(B, ldb);
      a.tiles_m = (a.m + cfg->tile.tile_m - 1) / cfg->tile.tile_m;
      a.tiles_n = (a.n + cfg->tile.tile_n - 1) / cfg->tile.tile_n;
      if (dalpha) {
        // Fused pass: dA (when requested) and the per-tile partials of dalpha.
        if (cfg->lds > 65536)
          e = hipFuncSetAttribute(reinterpret_cast<const void*>(cfg->grad_a),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)cfg->lds);
        if (e == hipSuccess) {
          const float* Ao = A;
          int64_t ldao = lda;
          float* part = pa;
          void* kargs[] = {&a, &Ao, &ldao, &part};
          e = hipLaunchKernel(reinterpret_cast<const void*>(cfg->grad_a), dim3((unsigned)(a.tiles_m * a.tiles_n)),
                              dim3(cfg->threads), kargs, (size_t)cfg->lds, s);
        }
      } else {
        // No dalpha: dA is a plain launch of the main loop (B transposed).
        const MfmaEntry* me = menu_entry(prec, cfg->tile);
        e = me ? me->launch(a, false, true, s) : hipErrorInvalidValue;
      }
    }
  } else {
    na = 0;
  }
  if (e != hipSuccess) return hip_error(e, "backward dA launch");

  // dB: contraction over m.
  if (dB && kn) {
    if (m == 0) {
      e = launch_scale(dB, lddb, k, n, 0.0f, s);
    } else {
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
      b.vec_a = aligned16(A, lda);
      b.vec_b = aligned16(G, ldg);
      const BwdConfig* cb = pick(prec, k, n);
      const MfmaEntry* me = menu_entry(prec, cb->tile);
      e = me ? me->launch(b, true, false, s) : hipErrorInvalidValue;
    }
  }
  if (e != hipSuccess) return hip_error(e, "backward dB launch");

  // dC_in and dbeta's partials.
  if (mn && (dC_in || dbeta)) {
    float* part = dbeta ? pb : nullptr;
    const float* Gp = G;
    const float* Cp = C_in;
    float* dCp = dC_in;
    int64_t ldg_ = ldg, ldci_ = ldci, lddci_ = lddci, m_ = m, n_ = n;
    float beta_ = beta;
    void* kargs[] = {&Gp, &ldg_, &Cp, &ldci_, &dCp, &lddci_, &m_, &n_, &beta_, &part};
    e = hipLaunchKernel(reinterpret_cast<const void*>(&sgemm_grad_c), dim3((unsigned)nb), dim3(kElemThreads), kargs,
                        0, s);
  }
  if (e != hipSuccess) return hip_error(e, "backward dC_in launch");

  if (dalpha || dbeta) {
    const float* pa_ = pa;
    const float* pb_ = pb;
    int32_t na_ = (int32_t)(dalpha ? na : 0);
    int32_t nb_ = (int32_t)((dbeta && mn) ? nb : 0);
    void* kargs[] = {&pa_, &na_, &pb_, &nb_, &dalpha, &dbeta};
    e = hipLaunchKernel(reinterpret_cast<const void*>(&sgemm_grad_finish), dim3(1), dim3(kElemThreads), kargs, 0, s);
  }
  if (e != hipSuccess) return hip_error(e, "backward reduction launch");
  return clear_error();
}

}  // extern "C"
