// Work-group reductions for 64-lane waves (gfx950): a fixed shuffle tree per
// wave, then the wave sums in index order, so the result is bit-reproducible.
#pragma once

#include <hip/hip_runtime.h>

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum of v over the work-group, returned to every thread.  `sh` holds one
// double per wave plus one; every thread of the work-group must call it.
__device__ inline double block_sum_all(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < nw; ++w) r += sh[w];
    sh[nw] = r;
  }
  __syncthreads();
  const double r = sh[nw];
  __syncthreads();
  return r;
}

// Sum of n values in[0..n) in a fixed order, returned to every thread.
__device__ inline double block_sum_array(const double* in, int n, double* sh) {
  double acc = 0.0;
  for (int t = threadIdx.x; t < n; t += blockDim.x) acc += in[t];
  return block_sum_all(acc, sh);
}
