// Deterministic block reductions (fixed order for a fixed launch shape).
#pragma once
#include <hip/hip_runtime.h>

namespace fde {

// Sum over the block; the result is valid in thread 0.  All threads must call.
template <int NT>
__device__ __forceinline__ double block_sum(double v) {
  static_assert(NT % 64 == 0 && NT <= 1024, "block must be whole wavefronts");
  __shared__ double ws[NT / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) ws[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += ws[w];
  }
  return s;
}

// Sum of p[0..n) in a fixed order (independent of the calling block), made
// available to every thread of the block.  All threads must call.  Each
// thread loads up to 8 of its strided elements at once (one L2 round trip
// per 8 NT elements) and adds them in a fixed tree order.
template <int NT>
__device__ __forceinline__ double block_ordered_sum(const double* __restrict__ p, int n) {
  __shared__ double bcast;
  constexpr int U = 8;
  double s = 0.0;
  for (int i0 = 0; i0 < n; i0 += U * NT) {
    double x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * NT + (int)threadIdx.x;
      x[u] = i < n ? p[i] : 0.0;
    }
    s += ((x[0] + x[1]) + (x[2] + x[3])) + ((x[4] + x[5]) + (x[6] + x[7]));
  }
  s = block_sum<NT>(s);
  if (threadIdx.x == 0) bcast = s;
  __syncthreads();
  const double r = bcast;
  __syncthreads();
  return r;
}

// NaN-propagating max of non-negative values
__device__ __forceinline__ double nanmax(double a, double b) {
  return (b > a || b != b) ? b : a;
}

template <int NT>
__device__ __forceinline__ double block_max(double v) {
  __shared__ double wm[NT / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = nanmax(v, __shfl_xor(v, off, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) wm[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s = nanmax(s, wm[w]);
  }
  return s;
}

}  // namespace fde
