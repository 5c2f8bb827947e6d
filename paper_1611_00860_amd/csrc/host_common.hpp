// Host helpers shared by every translation unit of the library, HIP or not:
// the error state behind hpvm_last_error and the argument checks of one
// sgemm.  Plain C++ (no HIP header), so the CPU lowering can use it too.
#pragma once

#include <stdint.h>

#include "hpvm_sgemm.h"

namespace hpvm {

// An operand allows 16-byte vector loads: 16-byte aligned base and a
// leading dimension that keeps every row 16-byte aligned.
inline bool vec16(const void* p, int64_t ld) { return ((uintptr_t)p % 16 == 0) && (ld % 4 == 0); }

inline bool same_tile(const hpvm_tile& a, const hpvm_tile& b) {
  return a.tile_m == b.tile_m && a.tile_n == b.tile_n && a.tile_k == b.tile_k && a.leaf_m == b.leaf_m &&
         a.leaf_n == b.leaf_n && a.stages == b.stages;
}

// Error state shared by every entry point (thread-local detail text).
int set_error(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int clear_error();
const char* last_error_text();
bool fault_injected(const char* site);

// Checks one sgemm's arguments in argument order (hpvm_sgemm's rules); `what`
// prefixes the message (e.g. "instance 7: ").  *reads_ab tells whether A and
// B are read at all (m, n, k > 0 and alpha != 0).
int check_gemm_args(const char* what, int64_t m, int64_t n, int64_t k, float alpha, const float* A,
                    int64_t lda, const float* B, int64_t ldb, float beta, const float* C,
                    int64_t ldc, bool* reads_ab);

// Byte range [lo, hi) of a row-major rows x cols float matrix.
void matrix_extent(const void* p, int64_t rows, int64_t cols, int64_t ld, uintptr_t* lo, uintptr_t* hi);

}  // namespace hpvm
