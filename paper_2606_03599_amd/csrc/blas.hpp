// Host wrappers of the vector kernels (blas.hip).  All work is queued on the
// context stream; `out` / scalar pointers are device memory.
#pragma once

#include "context.hpp"

// Device-resident scalars of one PCG solve.
struct PcgScalars {
  double rz;     // (r, z)
  double pq;     // (p, A p)
  double rr;     // ||r||^2
  double alpha, beta;
  double bb;     // ||b||^2
  double tol2;   // tol^2
  double rz_next;  // (r, z) of the current iteration until the p update consumes beta
  int done;      // 0 running, 1 converged, 2 breakdown
  int iters;
};

// Hooks of the fused PCG iteration into the preconditioner and matvec kernels
// (with the preconditioner on, one iteration is six launches: matvec with the
// (p, q) partials; first FFT pass with the alpha, x and r update and the |r|^2
// partials; second pass, whose first work-group finishes |r|^2 and the
// convergence test; the mode solve with the (r, z) partials by Parseval; third
// pass, whose first work-group finishes (r, z) and beta; last pass writing
// p = z + beta p).  A launch with st == nullptr is the plain preconditioner.
struct PcgHook {
  PcgScalars* st = nullptr;
  int init = 0;                 // first pass of a solve: r = b, x = 0
  int role = 0;                 // first work-group finishes: 1 |r|^2, 2 (r, z)
  cplx* x = nullptr;            // solution (first pass)
  cplx* r = nullptr;            // residual (first pass)
  const cplx* p = nullptr;      // search direction (first pass)
  const cplx* q = nullptr;      // (A + shift M) p (first pass)
  const cplx* b = nullptr;      // right-hand side (first pass, init)
  const double* red_in = nullptr;  // partials finished by this launch
  int red_n = 0;
  double* part_out = nullptr;   // partials written by this launch
  double tol2 = 0.0;            // init: tol_inner^2
  double inv_n = 1.0;           // 1 / nodes of the layout (Parseval scale of (r, z))
};

int blas_part_capacity();
int vec_copy(pbr_ctx* c, hipStream_t st_, long n, const cplx* a, cplx* b);
int vec_zero(pbr_ctx* c, hipStream_t st_, long n, cplx* a);
int vec_scale(pbr_ctx* c, hipStream_t st_, long n, cplx* a, double s);
int vec_diag_scale(pbr_ctx* c, hipStream_t st_, long N, const double* d, const cplx* x, cplx* y);
int vec_resid(pbr_ctx* c, hipStream_t st_, long N, double lam, const double* d, const cplx* u, const cplx* y,
              cplx* out);
int vec_random(pbr_ctx* c, hipStream_t st_, long n, unsigned long long seed, cplx* a);
int dot_real_async(pbr_ctx* c, hipStream_t st_, long n, const cplx* a, const cplx* b, double* part, double* out);
int dot_cplx_async(pbr_ctx* c, hipStream_t st_, long n, const cplx* a, const cplx* b, double* part, double* out);
int multi_dot_async(pbr_ctx* c, hipStream_t st_, long n, int m, const cplx* U, long ld, const cplx* w,
                    double* part, double* out);
int gemv_sub(pbr_ctx* c, hipStream_t st_, long n, int m, const cplx* U, long ld, const cplx* h, cplx* w);
int combine(pbr_ctx* c, hipStream_t st_, long n, int m, int k, const cplx* U, long ld, const cplx* Y, cplx* V,
            long ldv);
int proj_gamma(pbr_ctx* c, hipStream_t st_, long N, int nf, const double* W, cplx* v, double* part, double* coef);

int pcg_init_async(pbr_ctx* c, hipStream_t st_, long n, const cplx* r, const cplx* z, double tol, double* part,
                   double* part2, PcgScalars* st);
int pcg_alpha(pbr_ctx* c, hipStream_t st_, long n, const cplx* p, const cplx* q, double* part, PcgScalars* st);
int pcg_xr(pbr_ctx* c, hipStream_t st_, long n, cplx* x, cplx* r, const cplx* p, const cplx* q, double* part,
           PcgScalars* st);
// x += alpha p for the layouts of a fused PCG batch whose last iteration ended
// at the convergence test (the deferred update of the last pass)
int pcg_fix_x(pbr_ctx* c, hipStream_t st_, long n, int nb, PcgScalars* const* st,
              cplx* const* x, const cplx* const* p);
int pcg_beta_p(pbr_ctx* c, hipStream_t st_, long n, const cplx* r, const cplx* z, cplx* p, double* part,
               PcgScalars* st);
