// Layout kernels: material upload into the natural and parity-block layouts,
// and the gather / scatter maps Q_b^* and Q_b between a full vector and a block
// vector (Corollary 4.2, Eq. 4.14).  Block position t = i + n1*(y2 + m2*y3) is
// the node (i, 2*y2 + (a+i)%2, 2*y3 + (a+c+i)%2).
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/pbr_host.h"
#include "context.hpp"

namespace {

__device__ inline long block_to_natural(int n1, int n2, int m2, int a, int c, long t) {
  const int i = (int)(t % n1);
  const long r = t / n1;
  const int y2 = (int)(r % m2);
  const int y3 = (int)(r / m2);
  const int j = 2 * y2 + ((a + i) & 1);
  const int k = 2 * y3 + ((a + c + i) & 1);
  return (long)i + (long)n1 * ((long)j + (long)n2 * k);
}

struct MapArgs {
  int n1, n2, n3, m2, a, c;
  long nb, n;
};

__global__ void gather_kernel(MapArgs m, const cplx* __restrict__ full, cplx* __restrict__ blk) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.nb) return;
  const long x = block_to_natural(m.n1, m.n2, m.m2, m.a, m.c, t);
  for (int a = 0; a < 3; ++a) blk[a * m.nb + t] = full[a * m.n + x];
}

__global__ void scatter_kernel(MapArgs m, const cplx* __restrict__ blk, cplx* __restrict__ full) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.nb) return;
  const long x = block_to_natural(m.n1, m.n2, m.m2, m.a, m.c, t);
  for (int a = 0; a < 3; ++a) full[a * m.n + x] = blk[a * m.nb + t];
}

// Repack one material plane set (nplanes planes of n doubles) into block order.
__global__ void repack_kernel(MapArgs m, int nplanes, const double* __restrict__ src,
                              double* __restrict__ dst) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.nb) return;
  const long x = block_to_natural(m.n1, m.n2, m.m2, m.a, m.c, t);
  for (int q = 0; q < nplanes; ++q) dst[q * m.nb + t] = src[q * m.n + x];
}

__global__ void repack_u8_kernel(MapArgs m, const unsigned char* __restrict__ src,
                                 unsigned char* __restrict__ dst) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.nb) return;
  dst[t] = src[block_to_natural(m.n1, m.n2, m.m2, m.a, m.c, t)];
}

__global__ void sqrt_kernel(long N, const double* __restrict__ rho, double* __restrict__ s,
                            double* __restrict__ is) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const double r = sqrt(rho[t]);
  s[t] = r;
  is[t] = 1.0 / r;
}

MapArgs map_args(const pbr_ctx* c, int block) {
  MapArgs m;
  m.n1 = c->n1;
  m.n2 = c->n2;
  m.n3 = c->n3;
  m.m2 = c->n2 / 2;
  m.a = block >> 1;
  m.c = block & 1;
  m.n = c->n;
  m.nb = c->n / 4;
  return m;
}

// Interleave 21 stiffness planes and rho (layout order, box L1 x L2 x L3) into
// the stencil's tiles; one thread per tile entry, padding written as zeros.
__global__ void tile_kernel(int L1, int L2, int tiles, long len, long N,
                            const double* __restrict__ C, const double* __restrict__ rho,
                            double* __restrict__ Ct) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  const int w = (int)(e % PBR_CT_W);
  long r = e / PBR_CT_W;
  const int q = (int)(r % 22);
  r /= 22;
  const int it = (int)(r % tiles);
  r /= tiles;  // r = k * L2 + j
  const int i = it * PBR_CT_W + w;
  double v = 0.0;
  if (i < L1) {
    const long t = (long)i + (long)L1 * r;
    v = q < 21 ? C[q * N + t] : rho[t];
  }
  Ct[e] = v;
}

int alloc_material(pbr_ctx* c, DevMaterial& M, long N, long ct_len) {
  if (M.N == N && M.Ct && M.idx) return ST_OK;
  M.N = N;
  M.ct_len = ct_len;
  PBR_TRY(dev_alloc(c, (void**)&M.Ct, sizeof(double) * ct_len));
  PBR_TRY(dev_alloc(c, (void**)&M.rho, sizeof(double) * N));
  PBR_TRY(dev_alloc(c, (void**)&M.srho, sizeof(double) * N));
  PBR_TRY(dev_alloc(c, (void**)&M.isrho, sizeof(double) * N));
  PBR_TRY(dev_alloc(c, (void**)&M.idx, (size_t)N));
  return ST_OK;
}


// Tiles of one layout from its stiffness planes and rho.
void launch_tile(pbr_ctx* c, int L1, int L2, int L3, const double* C, DevMaterial& M) {
  const int tiles = (L1 + PBR_CT_W - 1) / PBR_CT_W;
  const long len = (long)L3 * L2 * tiles * 22 * PBR_CT_W;
  hipLaunchKernelGGL(tile_kernel, dim3((unsigned)ceil_div(len, 256)), dim3(256), 0, c->stream, L1,
                     L2, tiles, len, M.N, C, (const double*)M.rho, M.Ct);
}

long tile_len(int L1, int L2, int L3) {
  return (long)L3 * L2 * ((L1 + PBR_CT_W - 1) / PBR_CT_W) * 22 * PBR_CT_W;
}

}  // namespace

// Loads this file's kernels onto the current device (see preload_kernels).
int preload_layout(pbr_ctx* c) {
  hipFuncAttributes a;
  PBR_HIP(c, hipFuncGetAttributes(&a, reinterpret_cast<const void*>(gather_kernel)));
  return ST_OK;
}

int dev_alloc(pbr_ctx* c, void** p, size_t bytes) {
  if (*p) return ST_OK;
  hipError_t e = hipMalloc(p, bytes > 0 ? bytes : 16);
  if (e != hipSuccess) {
    *p = nullptr;
    c->set_error(std::string("hipMalloc failed: ") + hipGetErrorString(e));
    return ST_ENOMEM;
  }
  return ST_OK;
}

void dev_free(void* p) {
  if (p) (void)hipFree(p);
}

int upload_material(pbr_ctx* c, const double* C21, const double* rho) {
  const long n = c->n;
  // host transpose to 21 planes
  std::vector<double> planes((size_t)21 * n);
  for (long x = 0; x < n; ++x)
    for (int q = 0; q < 21; ++q) planes[(size_t)q * n + x] = C21[(size_t)x * 21 + q];
  DevMaterial& F = c->mat[0];
  PBR_TRY(alloc_material(c, F, n, tile_len(c->n1, c->n2, c->n3)));
  // natural planes (and one block's planes) live only during the upload
  double* tmp = nullptr;
  double* tmpb = nullptr;
  std::vector<double> hpal((size_t)PBR_PAL_MAX * 22);
  std::vector<unsigned char> hidx((size_t)n);
  const int nrows = pbr_host_palette(n, C21, rho, hpal.data(), hidx.data());
  const bool fits = nrows > 0;
  c->npal = 0;
  int st = dev_alloc(c, (void**)&tmp, sizeof(double) * 21 * n);
  if (st == ST_OK && c->even) st = dev_alloc(c, (void**)&tmpb, sizeof(double) * 21 * (n / 4));
  if (st == ST_OK && fits) st = dev_alloc(c, (void**)&c->pal, sizeof(double) * PBR_PAL_MAX * 22);
  auto run = [&]() -> int {
    PBR_HIP(c, hipMemcpyAsync(tmp, planes.data(), sizeof(double) * 21 * n, hipMemcpyHostToDevice,
                              c->stream));
    PBR_HIP(c, hipMemcpyAsync(F.rho, rho, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(sqrt_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, c->stream, n, F.rho,
                       F.srho, F.isrho);
    launch_tile(c, c->n1, c->n2, c->n3, tmp, F);
    PBR_HIP(c, hipGetLastError());
    if (fits) {
      PBR_HIP(c, hipMemcpyAsync(c->pal, hpal.data(), sizeof(double) * 22 * nrows,
                                hipMemcpyHostToDevice, c->stream));
      PBR_HIP(c, hipMemcpyAsync(F.idx, hidx.data(), (size_t)n, hipMemcpyHostToDevice, c->stream));
    }
    if (c->even) {
      for (int b = 0; b < 4; ++b) {
        DevMaterial& B = c->mat[b + 1];
        const long nb = n / 4;
        PBR_TRY(alloc_material(c, B, nb, tile_len(c->n1, c->n2 / 2, c->n3 / 2)));
        MapArgs m = map_args(c, b);
        hipLaunchKernelGGL(repack_kernel, dim3(ceil_div(nb, 256)), dim3(256), 0, c->stream, m,
                           21, (const double*)tmp, tmpb);
        hipLaunchKernelGGL(repack_kernel, dim3(ceil_div(nb, 256)), dim3(256), 0, c->stream, m, 1,
                           (const double*)F.rho, B.rho);
        hipLaunchKernelGGL(sqrt_kernel, dim3(ceil_div(nb, 256)), dim3(256), 0, c->stream, nb,
                           B.rho, B.srho, B.isrho);
        launch_tile(c, c->n1, c->n2 / 2, c->n3 / 2, tmpb, B);
        if (fits)
          hipLaunchKernelGGL(repack_u8_kernel, dim3(ceil_div(nb, 256)), dim3(256), 0, c->stream,
                             m, (const unsigned char*)F.idx, B.idx);
        PBR_HIP(c, hipGetLastError());
      }
    }
    return ST_OK;
  };
  if (st == ST_OK) st = run();
  // the host staging vector and the temporaries die here: wait for the work
  const hipError_t e = hipStreamSynchronize(c->stream);
  dev_free(tmp);
  dev_free(tmpb);
  if (st != ST_OK) return st;
  PBR_HIP(c, e);
  c->npal = fits ? nrows : 0;
  return ST_OK;
}

int layout_gather(pbr_ctx* c, int block, const cplx* full, cplx* blk) {
  MapArgs m = map_args(c, block);
  hipLaunchKernelGGL(gather_kernel, dim3(ceil_div(m.nb, 256)), dim3(256), 0, c->stream, m, full,
                     blk);
  PBR_HIP(c, hipGetLastError());
  return ST_OK;
}

int layout_scatter(pbr_ctx* c, int block, const cplx* blk, cplx* full) {
  MapArgs m = map_args(c, block);
  hipLaunchKernelGGL(scatter_kernel, dim3(ceil_div(m.nb, 256)), dim3(256), 0, c->stream, m, blk,
                     full);
  PBR_HIP(c, hipGetLastError());
  return ST_OK;
}
