// Device helpers shared by the HIP kernel sources (gfx950: 64-wide wavefronts, 8 XCDs).
#pragma once
#include <hip/hip_runtime.h>

namespace dfdg {

static constexpr int kBlk = 256;   // facet kernels
static constexpr int kEBlk = 128;  // element kernels

static inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

__device__ inline double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}
__device__ inline double wave_max(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
  return x;
}

// Block index remapped so that each of the 8 XCDs (which take the launched blocks round
// robin, each with its own L2) works on one contiguous range of rows: neighbouring
// elements and facets, whose data a block gathers, then mostly sit in the same L2.
// A bijection of [0, gridDim.x) for every grid size.
__device__ inline int xcd_block() {
  const int G = gridDim.x, b = blockIdx.x, x = b & 7;
  return x * (G >> 3) + min(x, G & 7) + (b >> 3);
}

}  // namespace dfdg
