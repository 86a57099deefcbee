// Derivatives of eigenvalues with respect to the nodewise material (first-order
// perturbation of the pencil A_h v = lambda M_h v, Eq. 3.15, with v^H M_h v = 1):
//
//   d lambda / d C21_q(x) = |e_a(x)|^2            (q = (a, a))
//                         = 2 Re(conj(e_a) e_b)    (q = (a, b), a < b: the stored
//                                                   entry is both C_ab and C_ba)
//   d lambda / d rho(x)   = -lambda sum_alpha |v_alpha(x)|^2
//
// with the strains e = B_h^H v recomputed here from the eigenvector (B_h^H as in
// the matvec: the real stencil D'_m = sum_d cf[m][d] S_d, whose factors -i drop
// out of |e|^2 and conj(e_a) e_b).  One thread per node of the layout; the
// weighted sum over a set of eigenvectors (a band, or the members of a cluster)
// is added to the natural-order gradient fields.
#include <algorithm>

#include "context.hpp"

namespace {

constexpr int GRAD_MAXV = 32;  // eigenvectors per launch

struct GradArgs {
  Geo g;
  long N;                  // nodes of the layout
  int nvec;
  const cplx* v;           // nvec vectors of 3N complex, vector-major
  double lam[GRAD_MAXV];
  double w[GRAD_MAXV];
  double* gC;              // n x 21, natural order
  double* grho;            // n
};

__global__ void __launch_bounds__(256) grad_kernel(GradArgs A) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= A.N) return;
  const Geo& g = A.g;
  const int i = (int)(t % g.L1);
  const long r = t / g.L1;
  const int j = (int)(r % g.L2), k = (int)(r / g.L2);
  // natural index of the node
  long nat;
  if (g.blocked) {
    const int jj = 2 * j + ((g.a + i) & 1), kk = 2 * k + ((g.a + g.c + i) & 1);
    nat = (long)i + (long)g.n1 * ((long)jj + (long)g.n2 * kk);
  } else {
    nat = t;
  }
  long nb[4];
  cplx fac[4];
#pragma unroll
  for (int d = 1; d <= 4; ++d) nb[d - 1] = neighbor(g, i, j, k, d, -1, fac[d - 1]);
  double gc[21];
#pragma unroll
  for (int q = 0; q < 21; ++q) gc[q] = 0.0;
  double gr = 0.0;
  for (int s = 0; s < A.nvec; ++s) {
    const cplx* v = A.v + (long)s * 3 * A.N;
    cplx G[3][3];
    double vv = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const cplx v0 = v[a * A.N + t];
      vv += v0.x * v0.x + v0.y * v0.y;
      cplx vb[4];
#pragma unroll
      for (int d = 0; d < 4; ++d) vb[d] = cmul(fac[d], v[a * A.N + nb[d]]);
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        cplx acc = cscale(g.cf[m][0], v0);
#pragma unroll
        for (int d = 1; d <= 4; ++d) acc = cfma(g.cf[m][d], vb[d - 1], acc);
        G[m][a] = acc;
      }
    }
    cplx e[6];
    e[0] = G[0][0];
    e[1] = G[1][1];
    e[2] = G[2][2];
    e[3] = cadd(G[2][1], G[1][2]);
    e[4] = cadd(G[2][0], G[0][2]);
    e[5] = cadd(G[1][0], G[0][1]);
    const double w = A.w[s];
    int q = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = a; b < 6; ++b, ++q) {
        const double re = e[a].x * e[b].x + e[a].y * e[b].y;  // Re(conj(e_a) e_b)
        gc[q] += w * (a == b ? re : 2.0 * re);
      }
    gr -= w * A.lam[s] * vv;
  }
  double* out = A.gC + nat * 21;
#pragma unroll
  for (int q = 0; q < 21; ++q) out[q] += gc[q];
  A.grho[nat] += gr;
}

}  // namespace

// Loads this file's kernels onto the current device (see preload_kernels).
int preload_grad(pbr_ctx* c) {
  hipFuncAttributes a;
  PBR_HIP(c, hipFuncGetAttributes(&a, reinterpret_cast<const void*>(grad_kernel)));
  return ST_OK;
}

int launch_eig_grad(pbr_ctx* c, const Geo& g, int block, int nvec, const double* lam,
                    const double* w, const cplx* v, double* gC, double* grho) {
  const long N = c->layout_nodes(block);
  for (int s0 = 0; s0 < nvec; s0 += GRAD_MAXV) {
    GradArgs A;
    A.g = g;
    A.N = N;
    A.nvec = std::min(GRAD_MAXV, nvec - s0);
    A.v = v + (long)s0 * 3 * N;
    for (int s = 0; s < A.nvec; ++s) {
      A.lam[s] = lam[s0 + s];
      A.w[s] = w[s0 + s];
    }
    A.gC = gC;
    A.grho = grho;
    hipLaunchKernelGGL(grad_kernel, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, c->stream, A);
    PBR_HIP(c, hipGetLastError());
  }
  return ST_OK;
}
