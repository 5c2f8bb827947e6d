// CPU (vector) lowering of the sgemm dataflow graph.
//
// The paper compiles one HPVM graph to a GPU, to the vector units of a CPU
// (its AVX backend, Sec. 3.3 and the evaluation of Sec. 5) and to plain host
// threads, and shows that the tiled hierarchy pays off on the vector target
// too.  This is the same two-level graph lowered by hand onto host cores:
//
//   SgemmRoot          -> one call
//   SgemmInternal grid -> tile_m x tile_n tiles of C, pulled by worker
//                         threads from a shared counter (the instances are
//                         independent, Sec. 2.1)
//   Allocation         -> per-thread packed panels (tile_m x tile_k of A and
//                         tile_k x tile_n of B) sized for the core's caches,
//                         the CPU's counterpart of the scratchpad
//   SgemmLeaf grid     -> an MR x NR block of outputs held in vector
//                         registers, updated with one FMA per element and k
//
// FP32 throughout.  The micro-kernel comes in AVX-512, AVX2 and baseline
// x86-64 versions; the widest one the host's CPU features allow is used.
// This file is host C++ only.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "host_common.hpp"
#include "hpvm_sgemm.h"

namespace hpvm {
namespace {

constexpr int MR = 8;   // leaf rows per micro-tile
constexpr int NR = 32;  // leaf columns per micro-tile (two 16-float vectors)
typedef float v16 __attribute__((vector_size(64)));

// The compiled CPU tiles: internal tile_m x tile_n, k panel tile_k, leaf
// MR x NR, stages = 1 (one packed panel per operand).
const hpvm_tile kCpuMenu[] = {
    {128, 256, 256, MR, NR, 1},
    {64, 128, 256, MR, NR, 1},
    {256, 256, 128, MR, NR, 1},
};
constexpr int kNumCpu = (int)(sizeof(kCpuMenu) / sizeof(kCpuMenu[0]));

// The leaf micro-kernel: acc (MR x NR) = sum over p < kc of Ap[p][i] *
// Bp[p][j]; Cb (ld = ldcb) receives it (first panel) or adds it.  Ap: kc x
// MR, Bp: kc x NR, both packed.  One version per instruction set, chosen
// once by the host's CPU features; all three add the k terms in the same
// order.
typedef float v8 __attribute__((vector_size(32)));
using MicroKernel = void (*)(int, const float*, const float*, float*, int, int);

__attribute__((target("avx512f"))) void micro_avx512(int kc, const float* __restrict__ Ap,
                                                     const float* __restrict__ Bp, float* __restrict__ Cb,
                                                     int ldcb, int first) {
  v16 acc[MR][2];
  for (int i = 0; i < MR; ++i) acc[i][0] = acc[i][1] = v16{};
  for (int p = 0; p < kc; ++p) {
    v16 b0, b1;
    std::memcpy(&b0, Bp + (size_t)p * NR, sizeof b0);
    std::memcpy(&b1, Bp + (size_t)p * NR + 16, sizeof b1);
    const float* a = Ap + (size_t)p * MR;
    for (int i = 0; i < MR; ++i) {
      acc[i][0] += a[i] * b0;
      acc[i][1] += a[i] * b1;
    }
  }
  for (int i = 0; i < MR; ++i) {
    float* c = Cb + (size_t)i * ldcb;
    if (!first) {
      v16 c0, c1;
      std::memcpy(&c0, c, sizeof c0);
      std::memcpy(&c1, c + 16, sizeof c1);
      acc[i][0] += c0;
      acc[i][1] += c1;
    }
    std::memcpy(c, &acc[i][0], sizeof acc[i][0]);
    std::memcpy(c + 16, &acc[i][1], sizeof acc[i][1]);
  }
}

// Sixteen 8-wide registers cannot hold an 8 x 32 block: four passes over
// 8-column quarters, each with 8 accumulators.
__attribute__((target("avx2,fma"))) void micro_avx2(int kc, const float* __restrict__ Ap,
                                                    const float* __restrict__ Bp, float* __restrict__ Cb,
                                                    int ldcb, int first) {
  for (int q = 0; q < NR / 8; ++q) {
    v8 acc[MR];
    for (int i = 0; i < MR; ++i) acc[i] = v8{};
    for (int p = 0; p < kc; ++p) {
      v8 b;
      std::memcpy(&b, Bp + (size_t)p * NR + 8 * q, sizeof b);
      const float* a = Ap + (size_t)p * MR;
      for (int i = 0; i < MR; ++i) acc[i] += a[i] * b;
    }
    for (int i = 0; i < MR; ++i) {
      float* c = Cb + (size_t)i * ldcb + 8 * q;
      if (!first) {
        v8 c0;
        std::memcpy(&c0, c, sizeof c0);
        acc[i] += c0;
      }
      std::memcpy(c, &acc[i], sizeof acc[i]);
    }
  }
}

void micro_generic(int kc, const float* __restrict__ Ap, const float* __restrict__ Bp, float* __restrict__ Cb,
                   int ldcb, int first) {
  for (int i = 0; i < MR; ++i) {
    float acc[NR] = {};
    for (int p = 0; p < kc; ++p) {
      const float a = Ap[(size_t)p * MR + i];
      for (int j = 0; j < NR; ++j) acc[j] = std::fmaf(a, Bp[(size_t)p * NR + j], acc[j]);
    }
    float* c = Cb + (size_t)i * ldcb;
    for (int j = 0; j < NR; ++j) c[j] = first ? acc[j] : c[j] + acc[j];
  }
}

struct Isa {
  MicroKernel fn;
  const char* name;
};

Isa pick_isa() {
  __builtin_cpu_init();
  if (__builtin_cpu_supports("avx512f")) return {micro_avx512, "avx512f"};
  if (__builtin_cpu_supports("avx2") && __builtin_cpu_supports("fma")) return {micro_avx2, "avx2"};
  return {micro_generic, "x86-64"};
}

const Isa& isa() {
  static const Isa chosen = pick_isa();
  return chosen;
}

const char* micro_isa() { return isa().name; }

int default_threads() {
  int t = (int)std::thread::hardware_concurrency();
  if (const char* e = std::getenv("OMP_NUM_THREADS")) {
    const int o = std::atoi(e);
    if (o > 0) t = t > 0 ? std::min(t, o) : o;
  }
  return std::max(t, 1);
}

struct Problem {
  int64_t m, n, k;
  float alpha, beta;
  const float* A;
  int64_t lda;
  const float* B;
  int64_t ldb;
  float* C;
  int64_t ldc;
  int tm, tn, tk;
};

// One worker: pulls internal instances (tiles of C) until none are left.
void worker(const Problem& P, std::atomic<int64_t>* next, int64_t tiles_n, int64_t tiles) {
  const int TM = P.tm, TN = P.tn, TK = P.tk;
  const MicroKernel micro = isa().fn;
  // The Allocation node of this worker: packed A and B panels, and the
  // tile's FP32 accumulators across k panels.
  float* Ap = static_cast<float*>(std::aligned_alloc(64, sizeof(float) * (size_t)TM * TK));
  float* Bp = static_cast<float*>(std::aligned_alloc(64, sizeof(float) * (size_t)TK * TN));
  float* Cb = static_cast<float*>(std::aligned_alloc(64, sizeof(float) * (size_t)TM * TN));
  if (!Ap || !Bp || !Cb) std::abort();
  for (;;) {
    const int64_t t = next->fetch_add(1);
    if (t >= tiles) break;
    const int64_t m0 = (t / tiles_n) * TM, n0 = (t % tiles_n) * TN;
    const int mc = (int)std::min<int64_t>(TM, P.m - m0), nc = (int)std::min<int64_t>(TN, P.n - n0);
    const int ms = (mc + MR - 1) / MR, ns = (nc + NR - 1) / NR;
    for (int64_t k0 = 0; k0 < P.k; k0 += TK) {
      const int kc = (int)std::min<int64_t>(TK, P.k - k0);
      // Pack A: strip s holds rows m0 + s*MR .. as [kc][MR], zero past m.
      for (int s = 0; s < ms; ++s) {
        float* dst = Ap + (size_t)s * TK * MR;
        for (int i = 0; i < MR; ++i) {
          const int64_t row = m0 + s * MR + i;
          if (row < P.m) {
            const float* src = P.A + row * P.lda + k0;
            for (int p = 0; p < kc; ++p) dst[(size_t)p * MR + i] = src[p];
          } else {
            for (int p = 0; p < kc; ++p) dst[(size_t)p * MR + i] = 0.0f;
          }
        }
      }
      // Pack B: strip r holds columns n0 + r*NR .. as [kc][NR], zero past n.
      for (int r = 0; r < ns; ++r) {
        float* dst = Bp + (size_t)r * TK * NR;
        const int64_t c0 = n0 + r * NR;
        const int w = (int)std::min<int64_t>(NR, P.n - c0);
        for (int p = 0; p < kc; ++p) {
          const float* src = P.B + (k0 + p) * P.ldb + c0;
          float* d = dst + (size_t)p * NR;
          std::memcpy(d, src, sizeof(float) * (size_t)w);
          for (int j = w; j < NR; ++j) d[j] = 0.0f;
        }
      }
      for (int s = 0; s < ms; ++s)
        for (int r = 0; r < ns; ++r)
          micro(kc, Ap + (size_t)s * TK * MR, Bp + (size_t)r * TK * NR, Cb + (size_t)s * MR * TN + r * NR,
                       TN, k0 == 0);
    }
    // Epilogue: C <- alpha acc + beta C (beta == 0 never reads C).
    for (int i = 0; i < mc; ++i) {
      float* c = P.C + (m0 + i) * P.ldc + n0;
      const float* a = Cb + (size_t)i * TN;
      if (P.beta != 0.0f)
        for (int j = 0; j < nc; ++j) c[j] = std::fmaf(P.beta, c[j], P.alpha * a[j]);
      else
        for (int j = 0; j < nc; ++j) c[j] = P.alpha * a[j];
    }
  }
  std::free(Ap);
  std::free(Bp);
  std::free(Cb);
}

}  // namespace
}  // namespace hpvm

using namespace hpvm;

extern "C" {

int hpvm_cpu_menu(hpvm_tile* out, int32_t capacity, int32_t* count) {
  if (capacity < 0 || (capacity > 0 && !out)) return set_error(HPVM_INVALID_ARG, "argument 2: bad capacity or NULL output");
  if (!count) return set_error(HPVM_INVALID_ARG, "argument 3: count is NULL");
  for (int i = 0; i < kNumCpu && i < capacity; ++i) out[i] = kCpuMenu[i];
  *count = kNumCpu;
  return clear_error();
}

const char* hpvm_cpu_isa(void) { return micro_isa(); }

int hpvm_sgemm_cpu(int64_t m, int64_t n, int64_t k, float alpha, const float* A, int64_t lda, const float* B,
                   int64_t ldb, float beta, float* C, int64_t ldc, const hpvm_tile* tile, int32_t threads) {
  bool reads_ab = false;
  int rc = check_gemm_args("", m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, &reads_ab);
  if (rc != HPVM_OK) return rc;
  const hpvm_tile* t = &kCpuMenu[0];
  if (tile) {
    t = nullptr;
    for (int i = 0; i < kNumCpu; ++i)
      if (same_tile(kCpuMenu[i], *tile)) t = &kCpuMenu[i];
    if (!t)
      return set_error(HPVM_UNSUPPORTED, "argument 12: tile %dx%dx%d leaf %dx%d is not in the CPU menu",
                       tile->tile_m, tile->tile_n, tile->tile_k, tile->leaf_m, tile->leaf_n);
  }
  if (threads < 0) return set_error(HPVM_INVALID_ARG, "argument 13: threads = %d < 0", threads);
  if (m == 0 || n == 0) return clear_error();
  if (!reads_ab) {
    // k == 0 or alpha == 0: C <- beta C, A and B unread.
    for (int64_t i = 0; i < m; ++i)
      for (int64_t j = 0; j < n; ++j) C[i * ldc + j] = beta != 0.0f ? beta * C[i * ldc + j] : 0.0f;
    return clear_error();
  }
  Problem P{m, n, k, alpha, beta, A, lda, B, ldb, C, ldc, t->tile_m, t->tile_n, t->tile_k};
  const int64_t tiles_n = (n + P.tn - 1) / P.tn;
  const int64_t tiles = ((m + P.tm - 1) / P.tm) * tiles_n;
  const int nt = (int)std::min<int64_t>(threads > 0 ? threads : default_threads(), tiles);
  std::atomic<int64_t> next{0};
  std::vector<std::thread> pool;
  pool.reserve((size_t)std::max(nt - 1, 0));
  for (int i = 1; i < nt; ++i) pool.emplace_back(worker, std::cref(P), &next, tiles_n, tiles);
  worker(P, &next, tiles_n, tiles);
  for (auto& th : pool) th.join();
  return clear_error();
}

}  // extern "C"
