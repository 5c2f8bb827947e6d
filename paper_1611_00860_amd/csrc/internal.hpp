// Host-side interface between the C-ABI layer (api.hip) and the kernel
// translation units.  Not installed, not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "host_common.hpp"
#include "hpvm_sgemm.h"

namespace hpvm {

struct GemmArgs;

// Lowering ids (hpvm_dfg.lowering).
enum Lowering {
  kLiteral = 0,
  kMfmaF32 = 1,
  kMfmaBf16 = 2,
  kMfmaBf16x3 = 3,
  kStagedBf16 = 4,
  kStagedBf16x3 = 5,
  kFlat = 6,
};

// bfloat16 planes of one staged product, the contraction index contiguous:
// the A side [round256(m)][kp], the B side [round256(n)][kp], kp =
// round64(k), zero outside the matrices.  The lo planes (x - hi) exist for
// bf16x3 only.
struct StagedPlanes {
  const uint16_t* ah;
  const uint16_t* al;
  const uint16_t* bh;
  const uint16_t* bl;
};

// One compiled MFMA configuration.
struct MfmaEntry {
  hpvm_tile tile;
  int32_t prec;
  int32_t threads;
  int64_t lds_bytes;
  // Fused lowerings: launch with the given operand forms (a_trans / b_trans,
  // see GemmArgs).  Null for staged entries.
  hipError_t (*launch)(const GemmArgs& args, bool a_trans, bool b_trans, hipStream_t s);
  // Staged lowering (tile.stages == 3): operands converted into `workspace`
  // first, then the GEMM.  Null for fused entries.
  hipError_t (*launch_staged)(const GemmArgs& args, void* workspace, hipStream_t s) = nullptr;
  // Staged GEMM on planes already written (stage_backward);
  // args gives the sizes, C, alpha and beta.  With `partial` the epilogue is
  // the backward's dA one (C <- alpha acc when C is set; partial[tile] = sum
  // of aorig .* acc over the tile).
  hipError_t (*launch_staged_planes)(const GemmArgs& args, const StagedPlanes& planes, const float* aorig,
                                     int64_t lda_orig, float* partial, hipStream_t s) = nullptr;
  // Two staged products in one launch (the first with the optional dA
  // epilogue as above); null where the entry has no such kernel.
  hipError_t (*launch_staged_pair)(const GemmArgs& args1, const StagedPlanes& planes1, const float* aorig,
                                   int64_t lda_orig, float* partial, const GemmArgs& args2,
                                   const StagedPlanes& planes2, hipStream_t s) = nullptr;
  // Split contraction (FP32 DMA-fed entries): workspace bytes that let an
  // m x n x k product run as contraction slices whose partial sums go to the
  // workspace (0 when the entry would not split it), and that launch
  // (slices, then C <- alpha * sum + beta * C).  Null elsewhere.
  int64_t (*split_bytes)(int64_t m, int64_t n, int64_t k) = nullptr;
  hipError_t (*launch_split)(const GemmArgs& args, void* workspace, hipStream_t s) = nullptr;
};

inline int64_t entry_split_bytes(const MfmaEntry* e, int64_t m, int64_t n, int64_t k) {
  return e && e->split_bytes ? e->split_bytes(m, n, k) : 0;
}

// Contraction slices for a whole-tile problem of `tiles` tiles of depth-TK
// slabs whose tiles would not cover 256 CUs: doubled while they would not,
// each slice a whole number of slabs and at least 256 deep, at most 16; 1
// (no split) when the slices still would not cover them.
inline int dma_split_count(int64_t tiles, int64_t k, int tk) {
  int sp = 1;
  while (sp < 16 && tiles * sp < 256 && k % (2 * sp * tk) == 0 && k / (2 * sp) >= 256) sp *= 2;
  return tiles * sp >= 256 ? sp : 1;
}

// C <- alpha * (part[0] + ... + part[splits-1]) + beta * C, the slices
// summed in order, from partial sums [splits][m][n] (n, ldc multiples of 4,
// part and C 16-byte aligned); beta == 0 never reads C.
hipError_t launch_split_finish(const float* part, int32_t splits, int64_t m, int64_t n, float alpha, float beta,
                               float* C, int64_t ldc, hipStream_t s);

// The compiled fused menu for `prec` (FP32, BF16, BF16X3); returns the count.
int mfma_menu(int32_t prec, const MfmaEntry** entries);

// The staged menu for `prec` (BF16, BF16X3); returns the count.
int staged_menu(int32_t prec, const MfmaEntry** entries);

// Workspace bytes the staged lowering needs for one m x n x k product.
int64_t staged_workspace_bytes(int32_t prec, int64_t m, int64_t n, int64_t k);

// Deepest contraction a staged tile takes: its loads address a tile's
// rows of a bfloat16 plane with 32-bit byte offsets.
bool staged_k_ok(int64_t k);

// Padded plane extents: rows (m or n) to 256, the contraction to 64.
int64_t staged_rows_pad(int64_t rows);
int64_t staged_k_pad(int64_t k);

// The staged backward's conversion passes, in one launch (m x n G, A m x k,
// B k x n; each plane zero outside its matrix):
//   the pass over G, each 64 x 64 block read once, giving
//     gh/gl  <- G as [round256(m)][round64(n)] planes (the dA product's A side),
//     th/tl  <- G transposed as [round256(n)][round64(m)] (the dB product's
//               B side),
//     dCin   <- beta G (zeros when beta == 0),
//     partial[block] <- sum over the block of G .* Cin,
//   each skipped when its pointer is null (Cin is read only for partial);
//   partial holds stage_gradient_blocks(m, n) floats, in a fixed order;
//   when bh is set, B into bh/bl [round256(k)][round64(n)] (the dA
//   product's B side, n contiguous as stored);
//   when ah is set, A transposed into ah/al [round256(k)][round64(m)] (the
//   dB product's A side).
// vec_*: that matrix (and for G also dCin and Cin) allows 16-byte units.
struct BackwardStaging {
  const float* G;
  int64_t ldg;
  const float* Cin;
  int64_t ldci;
  float* dCin;
  int64_t lddci, m, n, k;
  float beta;
  float* partial;
  uint16_t *gh, *gl, *th, *tl;
  int32_t vec_g;
  const float* B;
  int64_t ldb;
  uint16_t *bh, *bl;
  int32_t vec_b;
  const float* A;
  int64_t lda;
  uint16_t *ah, *al;
  int32_t vec_a;
};
int64_t stage_gradient_blocks(int64_t m, int64_t n);
hipError_t stage_backward(int32_t prec, const BackwardStaging& st, hipStream_t s);

// Every compiled entry of a precision: fused first (entry 0 is the default),
// then staged.  Returns nullptr past the end.
const MfmaEntry* menu_entry_at(int32_t prec, int index);
int menu_size(int32_t prec);
const MfmaEntry* find_menu_entry(int32_t prec, const hpvm_tile& tile);

// Built-in tile for tile == NULL (no autotuned entry, no workspace) when the
// menu's entry 0 would give fewer than 256 tiles; false otherwise.
bool default_small_tile(int32_t prec, int64_t m, int64_t n, hpvm_tile* out);

// Workspace bytes an entry needs for m x n x k (0 for fused entries).
int64_t entry_workspace_bytes(const MfmaEntry* e, int64_t m, int64_t n, int64_t k);

// Backward tile cache (see hpvm_autotune_backward): 1 when found.
int tuned_backward_tile(int32_t prec, int64_t m, int64_t n, int64_t k, hpvm_tile* out);
void record_backward_tile(int32_t prec, int64_t m, int64_t n, int64_t k, const hpvm_tile& t);

// Literal lowering: block_x x block_y lanes, one output each.
hipError_t launch_literal(const GemmArgs& args, int block_x, int block_y, hipStream_t s);
// Untiled one-level graph: one lane per output, no Allocation node.
hipError_t launch_flat(const GemmArgs& args, int block_x, int block_y, hipStream_t s);
int64_t literal_alloc_bytes(int block_x, int block_y);

// C <- beta * C (beta == 0 writes zeros without reading C).
hipError_t launch_scale(float* C, int64_t ldc, int64_t m, int64_t n, float beta, hipStream_t s);

int hip_error(hipError_t e, const char* what);

// Autotuned tile for a problem: 2 exact entry, 1 shape-class entry, 0 none.
// With allow_workspace the overall winner is returned, otherwise the best
// tile that needs no workspace.
int tuned_tile(int32_t prec, int64_t m, int64_t n, int64_t k, bool allow_workspace, hpvm_tile* out);

}  // namespace hpvm
