// Vector kernels for the inner PCG and the outer Krylov iteration.
//
// Reductions are deterministic: each work-group reduces a fixed slice in a
// fixed tree order (wave shuffles + LDS) and writes one partial; a single
// work-group then sums the partials in index order.  Repeated runs are
// therefore bit-identical.
#include <algorithm>
#include <cmath>

#include "blas.hpp"
#include "reduce.hpp"

namespace {

constexpr int RT = 256;  // threads per reduction work-group

// Sum over the work-group; result valid in thread 0.
__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
  __syncthreads();
  return r;
}

// partial[wg] = sum over the slice of Re(conj(a) b)  (or |a|^2 when b == a)
__global__ void __launch_bounds__(RT) dot_real_kernel(long n, const cplx* __restrict__ a,
                                                      const cplx* __restrict__ b,
                                                      double* __restrict__ part,
                                                      const PcgScalars* st) {
  __shared__ double sh[RT / 64];
  if (st && st->done) return;
  double acc = 0.0;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long)gridDim.x * blockDim.x) {
    const cplx x = a[t], y = b[t];
    acc = fma(x.x, y.x, fma(x.y, y.y, acc));
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// partial[wg] = (Re, Im) of sum conj(a) b
__global__ void __launch_bounds__(RT) dot_cplx_kernel(long n, const cplx* __restrict__ a,
                                                      const cplx* __restrict__ b,
                                                      double* __restrict__ part) {
  __shared__ double sh[RT / 64];
  double re = 0.0, im = 0.0;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long)gridDim.x * blockDim.x) {
    const cplx x = a[t], y = b[t];
    re = fma(x.x, y.x, fma(x.y, y.y, re));
    im = fma(x.x, y.y, fma(-x.y, y.x, im));
  }
  const double sr = block_sum(re, sh);
  const double si = block_sum(im, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sr;
    part[2 * blockIdx.x + 1] = si;
  }
}

// out[j] = sum_{p < np} part[p*stride + j] for j < width, fixed order.
__global__ void __launch_bounds__(RT) reduce_cols_kernel(int np, int width, int stride,
                                                         const double* __restrict__ part,
                                                         double* __restrict__ out) {
  __shared__ double sh[RT / 64];
  for (int j = blockIdx.x; j < width; j += gridDim.x) {  // one column per work-group
    double acc = 0.0;
    for (int p = threadIdx.x; p < np; p += blockDim.x) acc += part[(long)p * stride + j];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) out[j] = s;
  }
}

// ---- PCG step kernels (device-resident scalars; no-ops once converged) ----

__global__ void __launch_bounds__(RT) pcg_fin_alpha(int np, const double* __restrict__ part,
                                                    PcgScalars* st) {
  __shared__ double sh[RT / 64];
  if (st->done) return;
  double acc = 0.0;
  for (int p = threadIdx.x; p < np; p += blockDim.x) acc += part[p];
  const double pq = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    st->pq = pq;
    st->alpha = (pq > 0.0) ? st->rz / pq : 0.0;
    if (!(pq > 0.0)) st->done = 2;  // breakdown: operator not positive on p
  }
}

__global__ void __launch_bounds__(RT) pcg_update_xr(long n, cplx* __restrict__ x,
                                                    cplx* __restrict__ r,
                                                    const cplx* __restrict__ p,
                                                    const cplx* __restrict__ q,
                                                    double* __restrict__ part,
                                                    const PcgScalars* st) {
  __shared__ double sh[RT / 64];
  if (st->done) return;
  const double al = st->alpha;
  double acc = 0.0;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long)gridDim.x * blockDim.x) {
    x[t] = cfma(al, p[t], x[t]);
    const cplx rr = cfma(-al, q[t], r[t]);
    r[t] = rr;
    acc = fma(rr.x, rr.x, fma(rr.y, rr.y, acc));
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(RT) pcg_fin_rr(int np, const double* __restrict__ part,
                                                 PcgScalars* st) {
  __shared__ double sh[RT / 64];
  if (st->done) return;
  double acc = 0.0;
  for (int p = threadIdx.x; p < np; p += blockDim.x) acc += part[p];
  const double rr = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    st->rr = rr;
    st->iters += 1;
    if (rr <= st->tol2 * st->bb) st->done = 1;
  }
}

__global__ void __launch_bounds__(RT) pcg_fin_beta(int np, const double* __restrict__ part,
                                                   PcgScalars* st) {
  __shared__ double sh[RT / 64];
  if (st->done) return;
  double acc = 0.0;
  for (int p = threadIdx.x; p < np; p += blockDim.x) acc += part[p];
  const double rz = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    st->beta = (st->rz != 0.0) ? rz / st->rz : 0.0;
    st->rz = rz;
  }
}

__global__ void __launch_bounds__(RT) pcg_update_p(long n, cplx* __restrict__ p,
                                                   const cplx* __restrict__ z,
                                                   const PcgScalars* st) {
  if (st->done) return;
  const double be = st->beta;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long)gridDim.x * blockDim.x)
    p[t] = cfma(be, p[t], z[t]);
}

// init: rz = sum part (r.z), bb = |b|^2 from part2, iters = 0, done = (bb == 0)
__global__ void __launch_bounds__(RT) pcg_init(int np, const double* __restrict__ part_rz,
                                               const double* __restrict__ part_bb, double tol,
                                               PcgScalars* st) {
  __shared__ double sh[RT / 64];
  double a1 = 0.0, a2 = 0.0;
  for (int p = threadIdx.x; p < np; p += blockDim.x) {
    a1 += part_rz[p];
    a2 += part_bb[p];
  }
  const double rz = block_sum(a1, sh);
  const double bb = block_sum(a2, sh);
  if (threadIdx.x == 0) {
    st->rz = rz;
    st->bb = bb;
    st->rr = bb;
    st->tol2 = tol * tol;
    st->iters = 0;
    st->done = (bb == 0.0) ? 1 : 0;
    st->alpha = st->beta = st->pq = 0.0;
  }
}

// ---- general vector kernels ----

__global__ void copy_kernel(long n, const cplx* __restrict__ a, cplx* __restrict__ b) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long)gridDim.x * blockDim.x)
    b[t] = a[t];
}

__global__ void fill_zero_kernel(long n, cplx* __restrict__ a) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long)gridDim.x * blockDim.x)
    a[t] = mk(0, 0);
}

__global__ void scale_kernel(long n, cplx* __restrict__ a, double s) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long)gridDim.x * blockDim.x)
    a[t] = cscale(s, a[t]);
}

// y[a*N + t] = d[t] * x[a*N + t]  (3 components)
__global__ void diag_scale_kernel(long N, const double* __restrict__ d, const cplx* __restrict__ x,
                                  cplx* __restrict__ y) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < 3 * N;
       t += (long)gridDim.x * blockDim.x)
    y[t] = cscale(d[t % N], x[t]);
}

// w -= U h  (U column-major, ld, m columns; h complex on device)
__global__ void gemv_sub_kernel(long n, int m, const cplx* __restrict__ U, long ld,
                                const cplx* __restrict__ h, cplx* __restrict__ w) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long)gridDim.x * blockDim.x) {
    cplx acc = w[t];
    for (int j = 0; j < m; ++j) {
      const cplx u = U[(long)j * ld + t];
      const cplx c = h[j];
      acc = mk(acc.x - (u.x * c.x - u.y * c.y), acc.y - (u.x * c.y + u.y * c.x));
    }
    w[t] = acc;
  }
}

// part[wg*m + j] (complex, 2 doubles each) = slice sum of conj(U_j) w.  Four
// columns per sweep of the slice (w read once per sweep, four column loads in
// flight), their eight sums reduced together: one barrier per four columns.
constexpr int MD_COLS = 4;
__global__ void __launch_bounds__(RT) multi_dot_kernel(long n, int m, const cplx* __restrict__ U,
                                                       long ld, const cplx* __restrict__ w,
                                                       double* __restrict__ part) {
  __shared__ double sh[2 * MD_COLS][RT / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int j0 = 0; j0 < m; j0 += MD_COLS) {
    const int nc = min(MD_COLS, m - j0);
    double re[MD_COLS], im[MD_COLS];
#pragma unroll
    for (int c = 0; c < MD_COLS; ++c) re[c] = im[c] = 0.0;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (long)gridDim.x * blockDim.x) {
      const cplx x = w[t];
#pragma unroll
      for (int c = 0; c < MD_COLS; ++c) {
        if (c < nc) {
          const cplx u = U[(long)(j0 + c) * ld + t];
          re[c] = fma(u.x, x.x, fma(u.y, x.y, re[c]));
          im[c] = fma(u.x, x.y, fma(-u.y, x.x, im[c]));
        }
      }
    }
#pragma unroll
    for (int c = 0; c < MD_COLS; ++c) {
      const double a = wave_sum(re[c]), b = wave_sum(im[c]);
      if (lane == 0) {
        sh[2 * c][wid] = a;
        sh[2 * c + 1][wid] = b;
      }
    }
    __syncthreads();
    if (threadIdx.x < 2 * nc) {
      double r = 0.0;
      for (int v = 0; v < (int)(blockDim.x >> 6); ++v) r += sh[threadIdx.x][v];
      part[((long)blockIdx.x * m + j0) * 2 + threadIdx.x] = r;
    }
    __syncthreads();
  }
}

// V[:, 0:k] = U[:, 0:m] Y[0:m, 0:k]  (Y column-major m x k, complex, device).
// Eight output columns per sweep over j, so each U entry is loaded k/8 times
// rather than k times; every output sums over j in ascending order.
constexpr int CB_COLS = 8;
__global__ void combine_kernel(long n, int m, int k, const cplx* __restrict__ U, long ld,
                               const cplx* __restrict__ Y, cplx* __restrict__ V, long ldv) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long)gridDim.x * blockDim.x) {
    for (int c0 = 0; c0 < k; c0 += CB_COLS) {
      const int nc = min(CB_COLS, k - c0);
      cplx acc[CB_COLS];
#pragma unroll
      for (int cc = 0; cc < CB_COLS; ++cc) acc[cc] = mk(0, 0);
      for (int j = 0; j < m; ++j) {
        const cplx u = U[(long)j * ld + t];
#pragma unroll
        for (int cc = 0; cc < CB_COLS; ++cc)
          if (cc < nc) acc[cc] = cmad(u, Y[(long)(c0 + cc) * m + j], acc[cc]);
      }
#pragma unroll
      for (int cc = 0; cc < CB_COLS; ++cc)
        if (cc < nc) V[(long)(c0 + cc) * ldv + t] = acc[cc];
    }
  }
}

// The same product on the FP64 matrix cores (v_mfma_f64_16x16x4_f64).  In real
// arithmetic, with complex entries as (re, im) pairs, V_r = U_r Y_r where each
// complex y of Y becomes the 2 x 2 block [[re y, im y], [-im y, re y]]; the
// kernel computes its transpose V_r^T = Y_r^T U_r^T, so that the 16 output rows
// t of one tile sit on 16 consecutive lanes.  Operand and result lanes of the
// instruction: A[i][k] from lane i + 16 k, B[k][j] from lane j + 16 k, and lane
// l's result slot r holds D[4 r + l / 16][l % 16].  A wave owns 16 rows t and
// up to MM_TILES x 16 real output columns (MM_TILES x 8 complex ones); the
// work-group stages Y_r^T of its column chunk in LDS.
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int MM_TILES = 4;            // 16-column output tiles per wave
constexpr int MM_COLS = MM_TILES * 8;  // complex output columns per chunk
constexpr int MM_MAXM = 90;            // basis columns (K = 2 m real) at most

__global__ void __launch_bounds__(RT) combine_mfma_kernel(long n, int m, int k, int c0,
                                                         const cplx* __restrict__ U, long ld,
                                                         const cplx* __restrict__ Y,
                                                         cplx* __restrict__ V, long ldv) {
  // Y_r^T of output columns [c0, c0 + MM_COLS): yt[kr * (16 MM_TILES) + col],
  // kr < 2 m rounded up to a multiple of 4 (dynamic LDS of that size)
  extern __shared__ double yt[];
  const int kr_n = 2 * m + ((2 * m) & 2);  // K padded to a multiple of 4
  const int nc = min(MM_COLS, k - c0);
  for (int e = threadIdx.x; e < kr_n * 16 * MM_TILES; e += blockDim.x) {
    const int kr = e / (16 * MM_TILES), col = e % (16 * MM_TILES);
    const int j = kr >> 1, s_ = kr & 1, c = col >> 1, q = col & 1;
    double v = 0.0;
    if (j < m && c < nc) {
      const cplx y = Y[(long)(c0 + c) * m + j];
      v = s_ == 0 ? (q == 0 ? y.x : y.y) : (q == 0 ? -y.y : y.x);
    }
    yt[e] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long t0 = ((long)blockIdx.x * (RT / 64) + wave) * 16;
  if (t0 >= n) return;
  const long t = t0 + (lane & 15);
  const int kl = lane >> 4;
  v4d acc[MM_TILES];
#pragma unroll
  for (int a = 0; a < MM_TILES; ++a) acc[a] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int kk = 0; kk < kr_n; kk += 4) {
    const int kr = kk + kl, j = kr >> 1;
    double b = 0.0;
    if (t < n && j < m) {
      const cplx u = U[(long)j * ld + t];
      b = (kr & 1) ? u.y : u.x;
    }
#pragma unroll
    for (int a = 0; a < MM_TILES; ++a) {
      const double av = yt[kr * (16 * MM_TILES) + a * 16 + (lane & 15)];
      acc[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b, acc[a], 0, 0, 0);
    }
  }
  // lane l slot r: real output column a*16 + 4 r + l/16, row t0 + l%16
  double* Vd = reinterpret_cast<double*>(V);
#pragma unroll
  for (int a = 0; a < MM_TILES; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int col = a * 16 + 4 * r + kl, c = col >> 1, q = col & 1;
      if (c < nc && t < n) Vd[2 * ((long)(c0 + c) * ldv + t) + q] = acc[a][r];
    }
}

// Deterministic pseudo-random start vector (splitmix64 hash of seed and index).
__device__ inline unsigned long long splitmix(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void random_kernel(long n, unsigned long long seed, cplx* __restrict__ a) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long)gridDim.x * blockDim.x) {
    const unsigned long long h1 = splitmix(seed * 0x100000001B3ull + 2 * (unsigned long long)t);
    const unsigned long long h2 = splitmix(seed * 0x100000001B3ull + 2 * (unsigned long long)t + 1);
    const double u1 = (double)(h1 >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    const double u2 = (double)(h2 >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    a[t] = mk(u1, u2);
  }
}

// Gamma projection: part[wg*(nf*3) + f*3 + a] (complex) = slice sums of W_f[t] v_a[t]
__global__ void __launch_bounds__(RT) proj_dot_kernel(long N, int nf, const double* __restrict__ W,
                                                      const cplx* __restrict__ v,
                                                      double* __restrict__ part) {
  __shared__ double sh[RT / 64];
  for (int f = 0; f < nf; ++f)
    for (int a = 0; a < 3; ++a) {
      double re = 0.0, im = 0.0;
      for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < N;
           t += (long)gridDim.x * blockDim.x) {
        const double wv = W[(long)f * N + t];
        const cplx x = v[(long)a * N + t];
        re = fma(wv, x.x, re);
        im = fma(wv, x.y, im);
      }
      const double sr = block_sum(re, sh);
      const double si = block_sum(im, sh);
      if (threadIdx.x == 0) {
        const long o = ((long)blockIdx.x * nf * 3 + f * 3 + a) * 2;
        part[o] = sr;
        part[o + 1] = si;
      }
    }
}

__global__ void proj_sub_kernel(long N, int nf, const double* __restrict__ W,
                                const double* __restrict__ coef, cplx* __restrict__ v) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < N;
       t += (long)gridDim.x * blockDim.x) {
    for (int a = 0; a < 3; ++a) {
      cplx x = v[(long)a * N + t];
      for (int f = 0; f < nf; ++f) {
        const double wv = W[(long)f * N + t];
        x.x -= wv * coef[(f * 3 + a) * 2];
        x.y -= wv * coef[(f * 3 + a) * 2 + 1];
      }
      v[(long)a * N + t] = x;
    }
  }
}

// out = y - lam * d .* u  (3 components, d per node)
__global__ void resid_kernel(long N, double lam, const double* __restrict__ d,
                             const cplx* __restrict__ u, const cplx* __restrict__ y,
                             cplx* __restrict__ out) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < 3 * N;
       t += (long)gridDim.x * blockDim.x)
    out[t] = cfma(-lam * d[t % N], u[t], y[t]);
}

unsigned grid_for(long n) {
  long g = (n + RT - 1) / RT;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

// Loads this file's kernels onto the current device (see preload_kernels).
int preload_blas(pbr_ctx* c) {
  hipFuncAttributes a;
  PBR_HIP(c, hipFuncGetAttributes(&a, reinterpret_cast<const void*>(dot_real_kernel)));
  return ST_OK;
}

// ------------------------------ host wrappers ------------------------------

#define LAUNCH(kern, grid, ...)                                                 \
  do {                                                                          \
    hipLaunchKernelGGL(kern, dim3(grid), dim3(RT), 0, st_, __VA_ARGS__);   \
    PBR_HIP(c, hipGetLastError());                                              \
  } while (0)

int blas_part_capacity() { return 1024; }

int vec_copy(pbr_ctx* c, hipStream_t st_, long n, const cplx* a, cplx* b) {
  LAUNCH(copy_kernel, grid_for(n), n, a, b);
  return ST_OK;
}
int vec_zero(pbr_ctx* c, hipStream_t st_, long n, cplx* a) {
  LAUNCH(fill_zero_kernel, grid_for(n), n, a);
  return ST_OK;
}
int vec_scale(pbr_ctx* c, hipStream_t st_, long n, cplx* a, double s) {
  LAUNCH(scale_kernel, grid_for(n), n, a, s);
  return ST_OK;
}
int vec_diag_scale(pbr_ctx* c, hipStream_t st_, long N, const double* d, const cplx* x, cplx* y) {
  LAUNCH(diag_scale_kernel, grid_for(3 * N), N, d, x, y);
  return ST_OK;
}
int vec_resid(pbr_ctx* c, hipStream_t st_, long N, double lam, const double* d, const cplx* u, const cplx* y,
              cplx* out) {
  LAUNCH(resid_kernel, grid_for(3 * N), N, lam, d, u, y, out);
  return ST_OK;
}
int vec_random(pbr_ctx* c, hipStream_t st_, long n, unsigned long long seed, cplx* a) {
  LAUNCH(random_kernel, grid_for(n), n, seed, a);
  return ST_OK;
}

int dot_real_async(pbr_ctx* c, hipStream_t st_, long n, const cplx* a, const cplx* b, double* part, double* out) {
  const unsigned g = grid_for(n);
  LAUNCH(dot_real_kernel, g, n, a, b, part, (const PcgScalars*)nullptr);
  LAUNCH(reduce_cols_kernel, 1, (int)g, 1, 1, (const double*)part, out);
  return ST_OK;
}

int dot_cplx_async(pbr_ctx* c, hipStream_t st_, long n, const cplx* a, const cplx* b, double* part, double* out) {
  const unsigned g = grid_for(n);
  LAUNCH(dot_cplx_kernel, g, n, a, b, part);
  LAUNCH(reduce_cols_kernel, 1, (int)g, 2, 2, (const double*)part, out);
  return ST_OK;
}

int multi_dot_async(pbr_ctx* c, hipStream_t st_, long n, int m, const cplx* U, long ld, const cplx* w, double* part,
                    double* out) {
  // partials: g rows of 2m doubles in a buffer of 1024 x 256
  const unsigned gmax = (unsigned)std::max(1, 1024 * 128 / std::max(1, m));
  const unsigned g = std::min(grid_for(n), gmax);
  LAUNCH(multi_dot_kernel, g, n, m, U, ld, w, part);
  LAUNCH(reduce_cols_kernel, 2 * m, (int)g, 2 * m, 2 * m, (const double*)part, out);
  return ST_OK;
}

int gemv_sub(pbr_ctx* c, hipStream_t st_, long n, int m, const cplx* U, long ld, const cplx* h, cplx* w) {
  LAUNCH(gemv_sub_kernel, grid_for(n), n, m, U, ld, h, w);
  return ST_OK;
}

int combine(pbr_ctx* c, hipStream_t st_, long n, int m, int k, const cplx* U, long ld, const cplx* Y, cplx* V,
            long ldv) {
  if (m > MM_MAXM) {
    LAUNCH(combine_kernel, grid_for(n), n, m, k, U, ld, Y, V, ldv);
    return ST_OK;
  }
  // matrix cores: one launch per chunk of MM_COLS output columns
  const unsigned g = ceil_div(n, 16 * (RT / 64));
  const size_t lds = sizeof(double) * (2 * m + ((2 * m) & 2)) * 16 * MM_TILES;
  for (int c0 = 0; c0 < k; c0 += MM_COLS) {
    hipLaunchKernelGGL(combine_mfma_kernel, dim3(g), dim3(RT), lds, st_, n, m, k, c0, U, ld, Y, V,
                       ldv);
    PBR_HIP(c, hipGetLastError());
  }
  return ST_OK;
}

int proj_gamma(pbr_ctx* c, hipStream_t st_, long N, int nf, const double* W, cplx* v, double* part, double* coef) {
  const unsigned g = grid_for(N) > 256 ? 256 : grid_for(N);
  LAUNCH(proj_dot_kernel, g, N, nf, W, (const cplx*)v, part);
  LAUNCH(reduce_cols_kernel, std::max(1, nf * 6), (int)g, nf * 6, nf * 6, (const double*)part,
         coef);
  LAUNCH(proj_sub_kernel, grid_for(N), N, nf, W, (const double*)coef, v);
  return ST_OK;
}

int pcg_init_async(pbr_ctx* c, hipStream_t st_, long n, const cplx* r, const cplx* z, double tol, double* part,
                   double* part2, PcgScalars* st) {
  const unsigned g = grid_for(n);
  LAUNCH(dot_real_kernel, g, n, r, z, part, (const PcgScalars*)nullptr);
  LAUNCH(dot_real_kernel, g, n, r, r, part2, (const PcgScalars*)nullptr);
  LAUNCH(pcg_init, 1, (int)g, (const double*)part, (const double*)part2, tol, st);
  return ST_OK;
}

int pcg_alpha(pbr_ctx* c, hipStream_t st_, long n, const cplx* p, const cplx* q, double* part, PcgScalars* st) {
  const unsigned g = grid_for(n);
  LAUNCH(dot_real_kernel, g, n, p, q, part, (const PcgScalars*)st);
  LAUNCH(pcg_fin_alpha, 1, (int)g, (const double*)part, st);
  return ST_OK;
}

int pcg_xr(pbr_ctx* c, hipStream_t st_, long n, cplx* x, cplx* r, const cplx* p, const cplx* q, double* part,
           PcgScalars* st) {
  const unsigned g = grid_for(n);
  LAUNCH(pcg_update_xr, g, n, x, r, p, q, part, (const PcgScalars*)st);
  LAUNCH(pcg_fin_rr, 1, (int)g, (const double*)part, st);
  return ST_OK;
}

// The x update a fused PCG iteration defers to its last pass, for the layouts
// whose last iteration was cut short by convergence (done == 1): x += alpha p.
struct FixX {
  long n;
  const PcgScalars* st[PBR_MAX_BATCH];
  cplx* x[PBR_MAX_BATCH];
  const cplx* p[PBR_MAX_BATCH];
};
__global__ void pcg_fix_x_kernel(FixX F) {
  const PcgScalars* st = F.st[blockIdx.y];
  if (st->done != 1) return;
  const double a = st->alpha;
  cplx* x = F.x[blockIdx.y];
  const cplx* p = F.p[blockIdx.y];
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < F.n;
       i += (long)gridDim.x * blockDim.x)
    x[i] = cfma(a, p[i], x[i]);
}

int pcg_fix_x(pbr_ctx* c, hipStream_t st_, long n, int nb, PcgScalars* const* st,
              cplx* const* x, const cplx* const* p) {
  FixX F;
  F.n = n;
  for (int t = 0; t < nb; ++t) {
    F.st[t] = st[t];
    F.x[t] = x[t];
    F.p[t] = p[t];
  }
  hipLaunchKernelGGL(pcg_fix_x_kernel, dim3(grid_for(n), nb), dim3(RT), 0, st_, F);
  PBR_HIP(c, hipGetLastError());
  return ST_OK;
}

int pcg_beta_p(pbr_ctx* c, hipStream_t st_, long n, const cplx* r, const cplx* z, cplx* p, double* part,
               PcgScalars* st) {
  const unsigned g = grid_for(n);
  LAUNCH(dot_real_kernel, g, n, r, z, part, (const PcgScalars*)st);
  LAUNCH(pcg_fin_beta, 1, (int)g, (const double*)part, st);
  LAUNCH(pcg_update_p, grid_for(n), n, p, z, (const PcgScalars*)st);
  return ST_OK;
}
