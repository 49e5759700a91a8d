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

// A read-only table (reference-element matrices) seen through the constant address
// space: reads at wave-uniform indices then compile to scalar loads into SGPRs.  Through
// a plain pointer the compiler cannot prove that the kernel's own stores leave the table
// alone, and loads it into vector registers of every lane instead.
template <typename T>
__device__ inline const __attribute__((address_space(4))) T* cst(const T* p) {
  return (const __attribute__((address_space(4))) T*)p;
}

// Reductions without atomics or fences: a kernel writes one partial per block; the next
// kernel on the stream (after the kernel boundary has made them visible) sums all partials
// redundantly in every block, in a fixed order, so every block gets the same bits.
template <int NV>
__device__ inline void block_write_partial(const double (&v)[NV], double* __restrict__ buf) {
  __shared__ double sh[NV][kBlk / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const double s = wave_sum(v[i]);
    if (lane == 0) sh[i][wid] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0;
      for (int w = 0; w < nw; ++w) s += sh[i][w];
      buf[blockIdx.x * NV + i] = s;
    }
  }
}

// Sum n partials of NV values each; every thread of the block receives the totals.
// Block-wide sums of per-thread values (fixed order: waves, then the waves' sums).
template <int NV>
__device__ inline void block_sum_values(const double (&acc)[NV], double (&out)[NV]) {
  __shared__ double sh[NV][kBlk / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const double s = wave_sum(acc[i]);
    if (lane == 0) sh[i][wid] = s;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = 0;
    for (int w = 0; w < nw; ++w) s += sh[i][w];
    out[i] = s;
  }
  __syncthreads();
}
template <int NV>
__device__ inline void block_sum_partials(const double* __restrict__ buf, int n, double (&out)[NV]) {
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0;
  for (int b = threadIdx.x; b < n; b += blockDim.x)
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] += buf[b * NV + i];
  block_sum_values<NV>(acc, out);
}
// The same sums in two steps: load this thread's partials (up to kPartsPerThread of them)
// now, add them up later, so that the loads' latency overlaps other work.
static constexpr int kMaxFacetGrid = 1024;
static constexpr int kPartsPerThread = (kMaxFacetGrid + kBlk - 1) / kBlk;
template <int NV>
struct PartLoad { double v[kPartsPerThread][NV]; };
template <int NV>
__device__ inline void partials_load(const double* __restrict__ buf, int n, bool on, PartLoad<NV>& q) {
#pragma unroll
  for (int j = 0; j < kPartsPerThread; ++j) {
    const int b = threadIdx.x + j * blockDim.x;
#pragma unroll
    for (int i = 0; i < NV; ++i) q.v[j][i] = (on && b < n) ? buf[b * NV + i] : 0.0;
  }
}
template <int NV>
__device__ inline void partials_sum(const PartLoad<NV>& q, int n, double (&out)[NV]) {
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0;
#pragma unroll
  for (int j = 0; j < kPartsPerThread; ++j)
    if ((int)threadIdx.x + j * (int)blockDim.x < n)
#pragma unroll
      for (int i = 0; i < NV; ++i) acc[i] += q.v[j][i];
  block_sum_values<NV>(acc, out);
}

}  // namespace dfdg
