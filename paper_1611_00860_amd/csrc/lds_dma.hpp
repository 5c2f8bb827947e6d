// Direct HBM -> LDS transfers (gfx950 global_load_lds_dwordx4) and the LDS
// layouts the DMA-fed main loops use.
//
// One wave-wide DMA instruction moves 16 bytes per lane from any per-lane
// global address to LDS address (uniform base) + 16 * lane, so a
// wavefront fills 1 KB of consecutive LDS; which global chunk lands in which
// slot is chosen by the per-lane source offset.  No register holds the
// data in transit, and the transfer is counted by vmcnt like a load.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hpvm {

__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}

// base (uniform, 64-bit) + voff (per lane) -> LDS lds (uniform) + 16 * lane.
// The LDS address travels in M0, which the compiler sets right before the
// asm; the s_nop is the one wait state the hardware needs between a scalar
// write of M0 and an LDS-DMA load that reads it.  The compiler does not see
// this transfer (it counts no wait for it and keeps no LDS value across it,
// the asm clobbering memory): callers order it with dma_wait_barrier.
__device__ __forceinline__ void dma16(uint32_t lds, const void* base, uint32_t voff) {
  asm volatile(
      "s_nop 0\n\t"
      "global_load_lds_dwordx4 %0, %1"
      :
      : "v"(voff), "s"(base), "{m0}"(lds)
      : "memory");
}

// Wait until at most N DMA instructions of this wave are outstanding and
// its LDS reads are complete, then join the workgroup barrier.  Also a
// compiler barrier for memory operations.
template <int N>
__device__ __forceinline__ void dma_wait_barrier() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  asm volatile("s_waitcnt vmcnt(%0)\n\ts_waitcnt lgkmcnt(0)\n\ts_barrier" : : "n"(N) : "memory");
}

// Layout of a tile of rows of RB bytes (RB = 128 or 64), each row eight or
// four 16-byte chunks, fed by DMA and read as MFMA fragments: lane l reads
// chunk 2 ks + (l >> 5) of row r0 + (l & 31) of a 32-row block.
//   RB = 128: chunk c of row r sits at row slot r ^ ((r >> 3) & 1), chunk
//             slot c ^ (r & 7); one DMA instruction fills 8 row slots.
//   RB = 64:  two rows per 128-byte line L = r >> 1, chunk slot
//             (((r & 1) << 2) | c) ^ g(L), g(L) = (L & 3) ^ ((L >> 2) & 1);
//             one DMA instruction fills 16 rows.
// Either way every group of 8 (or 16) lanes of a fragment read covers all
// 32 (or 64) LDS banks once.
template <int RB>
struct SwizzledRows;

template <>
struct SwizzledRows<128> {
  static constexpr int kRowsPerDma = 8;
  // Source byte offset of this lane within its instruction's row group,
  // for a group of parity par (0 or 1); rowb = bytes between source rows.
  __device__ static uint32_t src(int lane, int par, int64_t rowb) {
    const int x = (lane >> 3) ^ par;
    return (uint32_t)(x * rowb + (((lane & 7) ^ x) << 4));
  }
  __device__ static int frag(int lane, int ks) {
    const int rslot = (lane & 31) ^ ((lane >> 3) & 1);
    return rslot * 128 + (((2 * ks + (lane >> 5)) ^ (lane & 7)) << 4);
  }
};

template <>
struct SwizzledRows<64> {
  static constexpr int kRowsPerDma = 16;
  __device__ static uint32_t src(int lane, int, int64_t rowb) {
    const int y = lane >> 3, p = lane & 7;
    const int g = (y & 3) ^ ((y >> 2) & 1);
    const int row = 2 * y + ((p >> 2) & 1), c = (p ^ g) & 3;
    return (uint32_t)(row * rowb + (c << 4));
  }
  __device__ static int frag(int lane, int ks) {
    const int l = lane & 31;
    const int g = ((l >> 1) & 3) ^ ((l >> 3) & 1);
    const int pos = (((l & 1) << 2) | (2 * ks + (lane >> 5))) ^ g;
    return (l >> 1) * 128 + (pos << 4);
  }
};

}  // namespace hpvm
