// Device-side helpers shared by the kernels: wave64/block reductions with a
// fixed summation order (results are bit-reproducible run to run).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace spfas {

constexpr int kBlock = 256;        // threads per block of the streaming kernels
constexpr int kMaxParts = 1024;    // partial sums per reduction (blocks of a reducing grid)

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  return v;
}

// Sum over the block; result valid in thread 0.  `sh` needs blockDim/64 doubles.
__device__ inline double block_sum(double v, double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) r += sh[i];
  }
  __syncthreads();
  return r;
}

__device__ inline double block_max(double v, double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  v = wave_max(v);
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) r = fmax(r, sh[i]);
  }
  __syncthreads();
  return r;
}

// Sum of parts[0..n) in a fixed order by the whole block; valid in thread 0.
__device__ inline double reduce_parts(const double* parts, int n, double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v += parts[i];
  return block_sum(v, sh);
}

__device__ inline double reduce_parts_max(const double* parts, int n, double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v = fmax(v, parts[i]);
  return block_max(v, sh);
}

// Load of data a launch streams through once (SELL-64 matrix values and
// column indices): marked non-temporal so it does not displace the gathered
// vectors from the caches (4-6 % faster SELL products; slower for the CSR
// lane-group kernels and the fine residual, which keep plain loads).
template <class T>
__device__ inline T ld_stream(const T* p) { return __builtin_nontemporal_load(p); }

// Block index remapped so that each of the 8 XCDs, which receive the blocks
// of a launch round-robin, works on one contiguous range of logical blocks
// (neighbouring rows then share that XCD's L2).  A bijection on
// [0, gridDim.x) for any grid size.
__device__ inline int xcd_block() {
  const int nb = (int)gridDim.x, b = (int)blockIdx.x;
  const int q0 = nb >> 3, r = nb & 7, x = b & 7, q = b >> 3;
  return x * q0 + (x < r ? x : r) + q;
}

// Number of blocks of a reducing grid-stride kernel over n items.
inline int reduce_grid(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > kMaxParts) g = kMaxParts;
  return (int)g;
}

}  // namespace spfas
