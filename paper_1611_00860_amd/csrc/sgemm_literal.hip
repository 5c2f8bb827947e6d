// Literal lowering of the sgemm dataflow graph (HPVM report, Sec. 6.1-6.3).
//
// One workgroup is one SgemmInternal instance, one lane is one SgemmLeaf
// instance computing one element of C, and the Allocation node's memory --
// block_x * block_y floats -- is the workgroup's LDS, holding a tile of B
// (the generated kernel of Sec. 6.2 places a tile of B in local memory).
// The leaf's linear id within its tile is block_x * id.y + id.x, as the
// listing computes from getNumNodeInstances.x and getNodeInstanceID.x/.y.
#include "device_common.hpp"
#include "internal.hpp"

namespace hpvm {

__global__ void sgemm_leaf_literal(GemmArgs p) {
  extern __shared__ float shB[];  // Allocation: block_x * block_y floats
  const int bx = blockDim.x, by = blockDim.y;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int lin = bx * ty + tx;  // leaf instance's linear id
  const int64_t i = (int64_t)blockIdx.y * by + ty;  // y <-> rows of C
  const int64_t j = (int64_t)blockIdx.x * bx + tx;  // x <-> columns of C
  float acc = 0.0f;
  for (int64_t k0 = 0; k0 < p.k; k0 += by) {
    // Stage rows k0 .. k0 + block_y of B, columns of this tile.
    const int64_t kk = k0 + ty;
    shB[lin] = (kk < p.k && j < p.n) ? p.B[kk * p.ldb + j] : 0.0f;
    __syncthreads();  // llvm.hpvm.barrier among the leaf instances
    const int kmax = (int)((p.k - k0) < by ? (p.k - k0) : by);
    if (i < p.m) {
      const float* a = p.A + i * p.lda + k0;
      for (int t = 0; t < kmax; ++t) acc = fmaf(a[t], shB[bx * t + tx], acc);
    }
    __syncthreads();
  }
  if (i < p.m && j < p.n) {
    float v = p.alpha * acc;
    if (p.beta != 0.0f) v = fmaf(p.beta, p.C[i * p.ldc + j], v);
    p.C[i * p.ldc + j] = v;
  }
}

// The untiled form of the same computation (the "non-tiled" version that
// Sec. 3.4 and 5.1 compare the tiled graph with): a one-level graph whose
// 2-D leaf grid covers C, one instance per element, reading its row of A
// and column of B straight from global memory -- no SgemmInternal level and
// no Allocation node.  The workgroup shape only groups leaf instances into
// launches; nothing is shared between them.
__global__ void sgemm_leaf_flat(GemmArgs p) {
  const int64_t i = (int64_t)blockIdx.y * blockDim.y + threadIdx.y;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.m || j >= p.n) return;
  const float* a = p.A + i * p.lda;
  const float* b = p.B + j;
  float acc = 0.0f;
  for (int64_t t = 0; t < p.k; ++t) acc = fmaf(a[t], b[t * p.ldb], acc);
  float v = p.alpha * acc;
  if (p.beta != 0.0f) v = fmaf(p.beta, p.C[i * p.ldc + j], v);
  p.C[i * p.ldc + j] = v;
}

hipError_t launch_flat(const GemmArgs& args, int block_x, int block_y, hipStream_t s) {
  dim3 block(block_x, block_y);
  dim3 grid((unsigned)((args.n + block_x - 1) / block_x), (unsigned)((args.m + block_y - 1) / block_y));
  GemmArgs a = args;
  void* kargs[] = {&a};
  return hipLaunchKernel(reinterpret_cast<const void*>(&sgemm_leaf_flat), grid, block, kargs, 0, s);
}

int64_t literal_alloc_bytes(int block_x, int block_y) {
  // The Allocation node function: (block_x * block_y) << 2 bytes.
  return ((int64_t)block_x * (int64_t)block_y) << 2;
}

hipError_t launch_literal(const GemmArgs& args, int block_x, int block_y, hipStream_t s) {
  dim3 block(block_x, block_y);
  dim3 grid((unsigned)((args.n + block_x - 1) / block_x), (unsigned)((args.m + block_y - 1) / block_y));
  GemmArgs a = args;
  void* kargs[] = {&a};
  return hipLaunchKernel(reinterpret_cast<const void*>(&sgemm_leaf_literal), grid, block, kargs,
                         (size_t)literal_alloc_bytes(block_x, block_y), s);
}

// C <- beta * C over an m x n block with leading dimension ldc.
__global__ void __launch_bounds__(256) scale_c(float* C, int64_t ldc, int64_t m, int64_t n,
                                               float beta) {
  const int64_t total = m * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / n, j = e - i * n;
    float* c = C + i * ldc + j;
    *c = (beta == 0.0f) ? 0.0f : beta * *c;
  }
}

hipError_t launch_scale(float* C, int64_t ldc, int64_t m, int64_t n, float beta, hipStream_t s) {
  const int64_t total = m * n;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  void* kargs[] = {&C, &ldc, &m, &n, &beta};
  return hipLaunchKernel(reinterpret_cast<const void*>(&scale_c), dim3((unsigned)blocks), dim3(256),
                         kargs, 0, s);
}

}  // namespace hpvm
