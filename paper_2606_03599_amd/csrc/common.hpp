// Shared device/host helpers of libpbr: complex arithmetic on double2, error
// plumbing and launch-shape utilities.  Written for gfx950 (64-lane waves).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

typedef double2 cplx;

__host__ __device__ inline cplx mk(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline cplx cadd(cplx a, cplx b) { return mk(a.x + b.x, a.y + b.y); }
__host__ __device__ inline cplx csub(cplx a, cplx b) { return mk(a.x - b.x, a.y - b.y); }
__host__ __device__ inline cplx cmul(cplx a, cplx b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__host__ __device__ inline cplx cmulc(cplx a, cplx b) {
  return mk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline cplx cscale(double s, cplx a) { return mk(s * a.x, s * a.y); }
__host__ __device__ inline cplx cconj(cplx a) { return mk(a.x, -a.y); }
// a + s*b
__host__ __device__ inline cplx cfma(double s, cplx b, cplx a) {
  return mk(fma(s, b.x, a.x), fma(s, b.y, a.y));
}
// acc + a*b (complex)
__host__ __device__ inline cplx cmad(cplx a, cplx b, cplx acc) {
  return mk(fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y)));
}
// acc + conj(a)*b
__host__ __device__ inline cplx cmadc(cplx a, cplx b, cplx acc) {
  return mk(fma(a.x, b.x, fma(a.y, b.y, acc.x)), fma(a.x, b.y, fma(-a.y, b.x, acc.y)));
}

// Status codes mirror include/pbr.h.
enum {
  ST_OK = 0,
  ST_EINVAL = -1,
  ST_EODDGRID = -2,
  ST_ENOMEM = -3,
  ST_EDEVICE = -4,
  ST_ENOCONV = -5,
  ST_ESTATE = -6
};

// A failing HIP call inside a function returning int status: record and return.
#define PBR_HIP(ctx, call)                                                        \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      (ctx)->set_error(std::string(#call) + ": " + hipGetErrorString(e_));        \
      return ST_EDEVICE;                                                          \
    }                                                                             \
  } while (0)

#define PBR_TRY(expr)                 \
  do {                                \
    int s_ = (expr);                  \
    if (s_ != ST_OK) return s_;       \
  } while (0)

inline unsigned ceil_div(long a, long b) { return (unsigned)((a + b - 1) / b); }
