// Streaming copy used as the measured copy-rate reference of the operator
// kernels (pbr_copy_probe): every work-group copies consecutive 16-byte
// elements, four per lane in flight, with non-temporal loads and stores so the
// copy neither reuses nor pollutes the last-level cache.
#include "context.hpp"

namespace {

constexpr int PROBE_THREADS = 256;
constexpr int PROBE_UNROLL = 4;

__global__ void __launch_bounds__(PROBE_THREADS)
    copy_probe_kernel(const double2* __restrict__ src, double2* __restrict__ dst, long n) {
  const long stride = (long)gridDim.x * PROBE_THREADS * PROBE_UNROLL;
  for (long base = (long)blockIdx.x * PROBE_THREADS * PROBE_UNROLL + threadIdx.x; base < n;
       base += stride) {
    double2 v[PROBE_UNROLL];
#pragma unroll
    for (int u = 0; u < PROBE_UNROLL; ++u) {
      const long i = base + (long)u * PROBE_THREADS;
      if (i < n) {
        v[u].x = __builtin_nontemporal_load(&src[i].x);
        v[u].y = __builtin_nontemporal_load(&src[i].y);
      }
    }
#pragma unroll
    for (int u = 0; u < PROBE_UNROLL; ++u) {
      const long i = base + (long)u * PROBE_THREADS;
      if (i < n) {
        __builtin_nontemporal_store(v[u].x, &dst[i].x);
        __builtin_nontemporal_store(v[u].y, &dst[i].y);
      }
    }
  }
}

}  // namespace

// Loads this file's kernels onto the current device (see preload_kernels).
int preload_probe(pbr_ctx* c) {
  hipFuncAttributes a;
  PBR_HIP(c, hipFuncGetAttributes(&a, reinterpret_cast<const void*>(copy_probe_kernel)));
  return ST_OK;
}

int launch_copy_probe(pbr_ctx* c, const void* src, void* dst, long bytes) {
  const long n = bytes / 16;
  if (n <= 0) return ST_OK;
  // enough work-groups to keep every CU busy with several rounds in flight
  const long per_wg = (long)PROBE_THREADS * PROBE_UNROLL;
  const long want = (n + per_wg - 1) / per_wg;
  const unsigned grid = (unsigned)std::min<long>(want, (long)c->cus * 16);
  hipLaunchKernelGGL(copy_probe_kernel, dim3(grid), dim3(PROBE_THREADS), 0, c->stream,
                     (const double2*)src, (double2*)dst, n);
  PBR_HIP(c, hipGetLastError());
  return ST_OK;
}
