// Device helpers: fixed-order wave64/block reductions and storage-type conversions.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

namespace ddg {

// Butterfly sum over the 64 lanes of a wave; every lane receives the same value
// and the summation order is fixed, so the result is reproducible.
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over a workgroup of NT threads (NT multiple of 64); result valid in thread 0.
template <int NT>
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += red[i];
  }
  __syncthreads();
  return s;
}

// Sum of np partials by one workgroup in a fixed order; result valid in thread 0.
template <int NT>
__device__ inline double sum_partials(const double* __restrict__ part, int np, double* red) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += NT) acc += part[i];
  return block_sum<NT>(acc, red);
}

// Storage conversions for the local factors.
template <class T> struct Store;
template <> struct Store<double> {
  __device__ static double to_acc(double x) { return x; }
  __device__ static double from(double x) { return x; }
};
template <> struct Store<float> {
  __device__ static float to_acc(float x) { return x; }
  __device__ static float from(double x) { return (float)x; }
};
template <> struct Store<__hip_bfloat16> {
  __device__ static float to_acc(__hip_bfloat16 x) { return __bfloat162float(x); }
  __device__ static __hip_bfloat16 from(double x) { return __float2bfloat16((float)x); }
};

}  // namespace ddg
