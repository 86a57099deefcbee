// Matrix-free application of A_h(k) + s M_h = B_h C_h B_h^H + s M_h (Sec. 6.1):
// strains from the velocity at a node and its four backward diagonal
// neighbours (B^H), the nodewise 6x6 Voigt stiffness (C), then the divergence
// from the stress at the node and its four forward neighbours (B).
//
// With D'_m = sum_s (A_lat^-1)_{sm} D~_s the factors -i of Eq. 3.12 cancel in
// B C B^H, so everything is written with the real stencil D'_m = sum_d cf[m][d] S_d:
//   G_{m,a}(z) = (D'_m^H v_a)(z) = sum_d cf[m][d] v_a(z - d)
//   eps = [G11, G22, G33, G32+G23, G31+G13, G21+G12]          (rows of B^H)
//   tau = C(z) eps,   S = stress tensor of tau (S11=t1, S22=t2, S33=t3,
//                                               S23=t4, S13=t5, S12=t6)
//   y_a(x) = sum_d sum_m cf[m][d] S_{m,a}(x + d) + s rho(x) v_a(x)   (rows of B)
#include "context.hpp"

namespace {

struct ApplyArgs {
  Geo g;
  long N;
  double s;
  const cplx* __restrict__ x;
  cplx* __restrict__ y;
  const double* __restrict__ C;
  const double* __restrict__ rho;
};

__device__ inline void coords(const Geo& g, long t, int& i, int& j, int& k) {
  i = (int)(t % g.L1);
  long r = t / g.L1;
  j = (int)(r % g.L2);
  k = (int)(r / g.L2);
}

// Voigt stress at node z (layout index tz with coordinates i,j,k).
__device__ void stress_at(const ApplyArgs& A, long tz, int i, int j, int k, cplx tau[6]) {
  const Geo& g = A.g;
  const long N = A.N;
  cplx G[3][3];
  for (int m = 0; m < 3; ++m)
    for (int a = 0; a < 3; ++a) G[m][a] = mk(0, 0);
  // d = 0: the node itself
  for (int a = 0; a < 3; ++a) {
    const cplx v = A.x[a * N + tz];
    for (int m = 0; m < 3; ++m) G[m][a] = cfma(g.cf[m][0], v, G[m][a]);
  }
  for (int d = 1; d <= 4; ++d) {
    cplx fac;
    const long tb = neighbor(g, i, j, k, d, -1, fac);
    for (int a = 0; a < 3; ++a) {
      const cplx v = cmul(fac, A.x[a * N + tb]);
      for (int m = 0; m < 3; ++m) G[m][a] = cfma(g.cf[m][d], v, G[m][a]);
    }
  }
  cplx eps[6];
  eps[0] = G[0][0];
  eps[1] = G[1][1];
  eps[2] = G[2][2];
  eps[3] = cadd(G[2][1], G[1][2]);
  eps[4] = cadd(G[2][0], G[0][2]);
  eps[5] = cadd(G[1][0], G[0][1]);
  double Cz[21];
  for (int q = 0; q < 21; ++q) Cz[q] = A.C[(long)q * N + tz];
  // symmetric 6x6 from its upper triangle, row by row
  int q = 0;
  double Cm[6][6];
  for (int r = 0; r < 6; ++r)
    for (int cc = r; cc < 6; ++cc) {
      Cm[r][cc] = Cz[q];
      Cm[cc][r] = Cz[q];
      ++q;
    }
  for (int r = 0; r < 6; ++r) {
    cplx acc = mk(0, 0);
    for (int cc = 0; cc < 6; ++cc) acc = cfma(Cm[r][cc], eps[cc], acc);
    tau[r] = acc;
  }
}

__global__ void __launch_bounds__(256) apply_gather_kernel(ApplyArgs A) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= A.N) return;
  const Geo& g = A.g;
  int i, j, k;
  coords(g, t, i, j, k);
  cplx y[3] = {mk(0, 0), mk(0, 0), mk(0, 0)};
  for (int d = 0; d <= 4; ++d) {
    long tz = t;
    cplx fac = mk(1, 0);
    int zi = i, zj = j, zk = k;
    if (d > 0) {
      tz = neighbor(g, i, j, k, d, +1, fac);
      coords(g, tz, zi, zj, zk);
    }
    cplx tau[6];
    stress_at(A, tz, zi, zj, zk, tau);
    // S_{m,a}: row m of the symmetric stress tensor
    const cplx S[3][3] = {{tau[0], tau[5], tau[4]},
                          {tau[5], tau[1], tau[3]},
                          {tau[4], tau[3], tau[2]}};
    for (int a = 0; a < 3; ++a) {
      cplx acc = mk(0, 0);
      for (int m = 0; m < 3; ++m) acc = cfma(g.cf[m][d], S[m][a], acc);
      y[a] = cmad(fac, acc, y[a]);
    }
  }
  const double sr = A.s * A.rho[t];
  for (int a = 0; a < 3; ++a) A.y[a * A.N + t] = cfma(sr, A.x[a * A.N + t], y[a]);
}

}  // namespace

int launch_apply(pbr_ctx* c, const Geo& g, int block, double s, const cplx* x, cplx* y) {
  DevMaterial& M = c->material(block);
  ApplyArgs A;
  A.g = g;
  A.N = M.N;
  A.s = s;
  A.x = x;
  A.y = y;
  A.C = M.C;
  A.rho = M.rho;
  hipLaunchKernelGGL(apply_gather_kernel, dim3(ceil_div(M.N, 256)), dim3(256), 0, c->stream, A);
  PBR_HIP(c, hipGetLastError());
  return ST_OK;
}
