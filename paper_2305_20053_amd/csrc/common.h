// Shared device helpers for the SAA / MR-DINO kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SAA_WAVE 64

// Sum over a 64-lane wavefront with butterfly shuffles; every lane gets the sum.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, SAA_WAVE);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, SAA_WAVE));
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, SAA_WAVE));
  return v;
}

// Block-wide sum of K values per thread, fixed reduction order (deterministic).
// `red` must hold K * (blockDim.x / 64) doubles of LDS.  All threads must call;
// every thread receives the K sums in v[].
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* red) {
  const int lane = threadIdx.x & (SAA_WAVE - 1);
  const int wid = threadIdx.x / SAA_WAVE;
  const int nw = blockDim.x / SAA_WAVE;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) red[k * nw + wid] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[k * nw + w];
    v[k] = s;
  }
  __syncthreads();
}

__device__ __forceinline__ double block_sum1(double x, double* red) {
  double v[1] = {x};
  block_sum<1>(v, red);
  return v[0];
}

__device__ __forceinline__ double block_max1(double x, double* red) {
  const int lane = threadIdx.x & (SAA_WAVE - 1);
  const int wid = threadIdx.x / SAA_WAVE;
  const int nw = blockDim.x / SAA_WAVE;
  x = wave_max(x);
  if (lane == 0) red[wid] = x;
  __syncthreads();
  double s = red[0];
  for (int w = 1; w < nw; ++w) s = fmax(s, red[w]);
  __syncthreads();
  return s;
}

__device__ __forceinline__ double block_min1(double x, double* red) {
  const int lane = threadIdx.x & (SAA_WAVE - 1);
  const int wid = threadIdx.x / SAA_WAVE;
  const int nw = blockDim.x / SAA_WAVE;
  x = wave_min(x);
  if (lane == 0) red[wid] = x;
  __syncthreads();
  double s = red[0];
  for (int w = 1; w < nw; ++w) s = fmin(s, red[w]);
  __syncthreads();
  return s;
}
