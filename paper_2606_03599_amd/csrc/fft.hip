// FFT-diagonal preconditioner of the shifted system (A + shift M) x = b:
//     z = T_xi diag_m(K(m)^-1) T_xi^H r,   K(m) = Bhat(m) C_ref Bhat(m)^H + shift rho_ref I_3
// with the Bloch Fourier basis T (Sec. 5.1, Eqs. 5.1-5.2) in the full space and
// T_sigma = T F_sigma (Sec. 5.2, Eqs. 5.3-5.5) in a parity block.
//
// Full space: coefficient(m) = sum_x e^{-i x.theta_m} r(x), theta_m =
// ((phi1 + 2 pi p)/n1, ...): a twist by e^{-i x_l phi_l/n_l} followed by a
// plain 3D DFT.
//
// Block b: the nodes are (i, 2 y2 + o2(i), 2 y3 + o3(i)).  Taking the orbit
// representatives m = (p, q, r) with q < n2/2, r < n3/2 (one per orbit of
// Eq. 5.3), the block coefficient is a 3D DFT on the L1 x L2 x L3 = n1 x n2/2 x
// n3/2 box: along y2 a twist e^{-i y2 phi2/(n2/2)} and a length-n2/2 DFT, then
// the factor e^{-i o2(i) beta_q} (beta_q = (phi2 + 2 pi q)/n2) -- the half-node
// offset of the sub-lattice, which folds the orbit as F_sigma does -- likewise
// along y3, and finally a twisted length-n1 DFT along i.  Because the y2/y3
// factors depend on i, the y2 and y3 passes run before the i pass (and after it
// on the way back).  K(m) is the same on every orbit member (Sec. 5.3), so one
// 3x3 solve per representative suffices.
//
// Every 1D transform is a mixed radix-4/2/3 Stockham FFT in LDS on a batch of
// lines; lines along y2/y3 are batched over consecutive i for coalesced access.
// All transforms are unnormalised; the final pass multiplies by 1/N.
#include <cmath>
#include <vector>

#include "context.hpp"

namespace {

constexpr int FFT_THREADS = 256;
constexpr int FFT_ELEMS = 2048;  // complex elements per work-group batch (32 KB per buffer)

struct AxisArgs {
  int L1, L2, L3;
  int axis;          // 0, 1, 2
  int L;             // line length
  long nlines;       // lines per component
  long N;            // nodes per component
  int B;             // lines per work-group
  int nfac;
  int fac[12];       // radices in order
  int sign;          // -1 forward, +1 inverse
  const cplx* __restrict__ roots;  // e^{-2 pi i k/L}
  const cplx* __restrict__ pre;    // per element factor (or null)
  int pre_conj;
  const cplx* __restrict__ post;   // per output element factor (or null)
  int post_conj;
  int parity_mode;   // 0: pre/post for every line; 1: post/pre only on lines with odd o(i)
  int par_off;       // o(i) = (par_off + i) & 1
  int pre_is_parity; // pre factor is the parity factor (inverse direction)
  double scale;
  const cplx* in;
  cplx* out;
};

__device__ inline long line_base(const AxisArgs& A, long l, long& estride, int& iline) {
  if (A.axis == 0) {
    estride = 1;
    iline = 0;
    return l * A.L1;
  } else if (A.axis == 1) {
    estride = A.L1;
    iline = (int)(l % A.L1);
    return (l % A.L1) + (l / A.L1) * (long)A.L1 * A.L2;
  }
  estride = (long)A.L1 * A.L2;
  iline = (int)(l % A.L1);
  return l;
}

__device__ inline cplx cj(cplx a, int c) { return c ? cconj(a) : a; }

template <int R>
__device__ inline void small_dft(cplx* v, int sign) {
  if (R == 2) {
    const cplx a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if (R == 4) {
    const cplx t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const cplx t2 = cadd(v[1], v[3]);
    const cplx d = csub(v[1], v[3]);
    // multiply by w = sign * i
    const cplx t3 = (sign < 0) ? mk(d.y, -d.x) : mk(-d.y, d.x);
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  } else if (R == 3) {
    const double h = 0.86602540378443864676;  // sqrt(3)/2
    const cplx t = cadd(v[1], v[2]);
    const cplx u = csub(v[1], v[2]);
    const cplx m = mk(v[0].x - 0.5 * t.x, v[0].y - 0.5 * t.y);
    // s * i * h * u
    const cplx iu = (sign < 0) ? mk(h * u.y, -h * u.x) : mk(-h * u.y, h * u.x);
    v[0] = cadd(v[0], t);
    v[1] = cadd(m, iu);
    v[2] = csub(m, iu);
  }
}

template <int R>
__device__ inline void stage(const AxisArgs& A, const cplx* src, cplx* dst, int Ns, int nb) {
  const int L = A.L;
  const int LR = L / R;
  const int tw_step = L / (Ns * R);
  for (int w = threadIdx.x; w < nb * LR; w += blockDim.x) {
    const int b = w / LR;
    const int j = w - b * LR;
    const int jm = j % Ns;
    cplx v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      cplx x = src[b * L + j + r * LR];
      if (r > 0) {
        const cplx wv = cj(A.roots[(jm * r * tw_step) % L], A.sign > 0);
        x = cmul(x, wv);
      }
      v[r] = x;
    }
    small_dft<R>(v, A.sign);
    const int idx = (j / Ns) * Ns * R + jm;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[b * L + idx + r * Ns] = v[r];
  }
}

__global__ void __launch_bounds__(FFT_THREADS) fft_axis_kernel(AxisArgs A) {
  extern __shared__ cplx lds[];
  cplx* buf0 = lds;
  cplx* buf1 = lds + FFT_ELEMS;
  const int comp = blockIdx.y;
  const long l0 = (long)blockIdx.x * A.B;
  const int nb = (int)min((long)A.B, A.nlines - l0);
  const cplx* in = A.in + comp * A.N;
  cplx* out = A.out + comp * A.N;
  const int L = A.L;
  // load (elements of consecutive lines adjacent in memory for axes 1, 2)
  for (int w = threadIdx.x; w < nb * L; w += blockDim.x) {
    int b, e;
    if (A.axis == 0) {
      b = w / L;
      e = w - b * L;
    } else {
      e = w / nb;
      b = w - e * nb;
    }
    long es;
    int il;
    const long base = line_base(A, l0 + b, es, il);
    cplx x = in[base + e * es];
    if (A.pre) {
      if (A.pre_is_parity) {
        if (((A.par_off + il) & 1)) x = cmul(x, cj(A.pre[e], A.pre_conj));
      } else {
        x = cmul(x, cj(A.pre[e], A.pre_conj));
      }
    }
    buf0[b * L + e] = x;
  }
  __syncthreads();
  cplx* src = buf0;
  cplx* dst = buf1;
  int Ns = 1;
  for (int s = 0; s < A.nfac; ++s) {
    const int R = A.fac[s];
    if (R == 4)
      stage<4>(A, src, dst, Ns, nb);
    else if (R == 2)
      stage<2>(A, src, dst, Ns, nb);
    else
      stage<3>(A, src, dst, Ns, nb);
    __syncthreads();
    cplx* t = src;
    src = dst;
    dst = t;
    Ns *= R;
  }
  for (int w = threadIdx.x; w < nb * L; w += blockDim.x) {
    int b, e;
    if (A.axis == 0) {
      b = w / L;
      e = w - b * L;
    } else {
      e = w / nb;
      b = w - e * nb;
    }
    long es;
    int il;
    const long base = line_base(A, l0 + b, es, il);
    cplx x = src[b * L + e];
    if (A.post) {
      if (A.parity_mode) {
        if (((A.par_off + il) & 1)) x = cmul(x, cj(A.post[e], A.post_conj));
      } else {
        x = cmul(x, cj(A.post[e], A.post_conj));
      }
    }
    out[base + e * es] = cscale(A.scale, x);
  }
}

struct SolveArgs {
  int L1, L2, L3;
  long N;
  double th0[3];     // phi_l / n_l
  double dth[3];     // 2 pi / n_l
  double cf[3][5];
  double Cref[21];
  double shift_rho;  // shift * rho_ref
  cplx* data;
};

__global__ void __launch_bounds__(256) mode_solve_kernel(SolveArgs S) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= S.N) return;
  const int p = (int)(t % S.L1);
  const long rr = t / S.L1;
  const int q = (int)(rr % S.L2);
  const int r = (int)(rr / S.L2);
  const double al = S.th0[0] + S.dth[0] * p;
  const double be = S.th0[1] + S.dth[1] * q;
  const double ga = S.th0[2] + S.dth[2] * r;
  // shift symbols e^{i d.theta} of the four diagonal steps
  cplx sd[5];
  sd[0] = mk(1.0, 0.0);
  for (int d = 1; d <= 4; ++d) {
    const double ang = al + step_s2(d) * be + step_s3(d) * ga;
    double sn, cs;
    sincos(ang, &sn, &cs);
    sd[d] = mk(cs, sn);
  }
  // symbols of D'_m (the -i factors cancel in Bhat C Bhat^H)
  cplx e[3];
  for (int m = 0; m < 3; ++m) {
    cplx acc = mk(0, 0);
    for (int d = 0; d <= 4; ++d) acc = cfma(S.cf[m][d], sd[d], acc);
    e[m] = acc;
  }
  // P = Bhat (3x6), rows as in Eq. 5.11
  const cplx z = mk(0, 0);
  const cplx P[3][6] = {{e[0], z, z, z, e[2], e[1]},
                        {z, e[1], z, e[2], z, e[0]},
                        {z, z, e[2], e[1], e[0], z}};
  double Cm[6][6];
  {
    int qq = 0;
    for (int a = 0; a < 6; ++a)
      for (int b = a; b < 6; ++b) {
        Cm[a][b] = S.Cref[qq];
        Cm[b][a] = S.Cref[qq];
        ++qq;
      }
  }
  // W = P C (3x6), K = W P^H (3x3 Hermitian)
  cplx W[3][6];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 6; ++b) {
      cplx acc = mk(0, 0);
      for (int k = 0; k < 6; ++k) acc = cfma(Cm[k][b], P[a][k], acc);
      W[a][b] = acc;
    }
  cplx K[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      cplx acc = mk(0, 0);
      for (int k = 0; k < 6; ++k) acc = cmad(W[a][k], cconj(P[b][k]), acc);
      K[a][b] = acc;
    }
  for (int a = 0; a < 3; ++a) K[a][a].x += S.shift_rho;
  // Cholesky K = L L^H
  const double l00 = sqrt(K[0][0].x);
  const cplx l10 = cscale(1.0 / l00, K[1][0]);
  const cplx l20 = cscale(1.0 / l00, K[2][0]);
  const double l11 = sqrt(K[1][1].x - (l10.x * l10.x + l10.y * l10.y));
  const cplx l21 = cscale(1.0 / l11, csub(K[2][1], cmul(l20, cconj(l10))));
  const double l22 =
      sqrt(K[2][2].x - (l20.x * l20.x + l20.y * l20.y) - (l21.x * l21.x + l21.y * l21.y));
  cplx b0 = S.data[t], b1 = S.data[S.N + t], b2 = S.data[2 * S.N + t];
  const cplx y0 = cscale(1.0 / l00, b0);
  const cplx y1 = cscale(1.0 / l11, csub(b1, cmul(l10, y0)));
  const cplx y2 = cscale(1.0 / l22, csub(csub(b2, cmul(l20, y0)), cmul(l21, y1)));
  const cplx x2 = cscale(1.0 / l22, y2);
  const cplx x1 = cscale(1.0 / l11, csub(y1, cmulc(l21, x2)));
  const cplx x0 = cscale(1.0 / l00, csub(csub(y0, cmulc(l10, x1)), cmulc(l20, x2)));
  S.data[t] = x0;
  S.data[S.N + t] = x1;
  S.data[2 * S.N + t] = x2;
}

__global__ void table_kernel(int L, double phi, double nfull, int kind, cplx* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L) return;
  double ang;
  if (kind == 0)
    ang = -(double)t * phi / (double)L;          // twist e^{-i x phi / L}
  else if (kind == 1)
    ang = -(phi + 2.0 * M_PI * t) / nfull;       // e^{-i beta_q}
  else
    ang = -2.0 * M_PI * (double)t / (double)L;   // roots
  double s, c;
  sincos(ang, &s, &c);
  out[t] = mk(c, s);
}

int factorize(int L, int* fac) {
  int n = 0;
  while (L % 4 == 0) { fac[n++] = 4; L /= 4; }
  while (L % 2 == 0) { fac[n++] = 2; L /= 2; }
  while (L % 3 == 0) { fac[n++] = 3; L /= 3; }
  return (L == 1) ? n : -1;
}

int ensure_tables(pbr_ctx* c, int block, const double kappa[3]) {
  FftTables& T = c->fft[block + 1];
  const int L[3] = {c->n1, block < 0 ? c->n2 : c->n2 / 2, block < 0 ? c->n3 : c->n3 / 2};
  const int nf[3] = {c->n1, c->n2, c->n3};
  for (int l = 0; l < 3; ++l) {
    if (!T.roots[l]) {
      T.L[l] = L[l];
      PBR_TRY(dev_alloc(c, (void**)&T.roots[l], sizeof(cplx) * L[l]));
      PBR_TRY(dev_alloc(c, (void**)&T.twist[l], sizeof(cplx) * L[l]));
      PBR_TRY(dev_alloc(c, (void**)&T.post[l], sizeof(cplx) * L[l]));
      hipLaunchKernelGGL(table_kernel, dim3(ceil_div(L[l], 256)), dim3(256), 0, c->stream, L[l],
                         0.0, (double)nf[l], 2, T.roots[l]);
    }
  }
  if (T.kappa[0] != kappa[0] || T.kappa[1] != kappa[1] || T.kappa[2] != kappa[2]) {
    for (int l = 0; l < 3; ++l) {
      const double phi = 2.0 * M_PI * kappa[l];
      hipLaunchKernelGGL(table_kernel, dim3(ceil_div(L[l], 256)), dim3(256), 0, c->stream, L[l],
                         phi, (double)nf[l], 0, T.twist[l]);
      hipLaunchKernelGGL(table_kernel, dim3(ceil_div(L[l], 256)), dim3(256), 0, c->stream, L[l],
                         phi, (double)nf[l], 1, T.post[l]);
      T.kappa[l] = kappa[l];
    }
  }
  PBR_HIP(c, hipGetLastError());
  return ST_OK;
}

int run_axis(pbr_ctx* c, int block, int axis, int sign, const cplx* in, cplx* out, double scale) {
  FftTables& T = c->fft[block + 1];
  const long N = c->layout_nodes(block);
  AxisArgs A;
  A.L1 = T.L[0];
  A.L2 = T.L[1];
  A.L3 = T.L[2];
  A.axis = axis;
  A.L = T.L[axis];
  A.nlines = N / A.L;
  A.N = N;
  A.B = FFT_ELEMS / A.L;
  if (A.B < 1) {
    c->set_error("FFT line longer than the LDS batch");
    return ST_EINVAL;
  }
  A.nfac = factorize(A.L, A.fac);
  if (A.nfac < 0) {
    c->set_error("FFT length must be of the form 2^a 3^b");
    return ST_EINVAL;
  }
  A.sign = sign;
  A.roots = T.roots[axis];
  A.scale = scale;
  A.in = in;
  A.out = out;
  const bool blocked = block >= 0;
  const int a = block >> 1, cc = block & 1;
  A.par_off = (axis == 1) ? a : (a + cc);
  A.pre = nullptr;
  A.post = nullptr;
  A.pre_conj = 0;
  A.post_conj = 0;
  A.parity_mode = 0;
  A.pre_is_parity = 0;
  if (sign < 0) {
    A.pre = T.twist[axis];
    if (blocked && axis > 0) {
      A.post = T.post[axis];
      A.parity_mode = 1;
    }
  } else {
    A.post = T.twist[axis];
    A.post_conj = 1;
    if (blocked && axis > 0) {
      A.pre = T.post[axis];
      A.pre_conj = 1;
      A.pre_is_parity = 1;
    }
  }
  dim3 grid(ceil_div(A.nlines, A.B), 3);
  hipLaunchKernelGGL(fft_axis_kernel, grid, dim3(FFT_THREADS), 2 * FFT_ELEMS * sizeof(cplx),
                     c->stream, A);
  PBR_HIP(c, hipGetLastError());
  return ST_OK;
}

}  // namespace

int launch_precond(pbr_ctx* c, const double kappa[3], int block, double shift, const cplx* r,
                   cplx* z) {
  PBR_TRY(ensure_tables(c, block, kappa));
  const long N = c->layout_nodes(block);
  // forward: y2, y3, then i (the block factors depend on i)
  PBR_TRY(run_axis(c, block, 1, -1, r, z, 1.0));
  PBR_TRY(run_axis(c, block, 2, -1, z, z, 1.0));
  PBR_TRY(run_axis(c, block, 0, -1, z, z, 1.0));
  SolveArgs S;
  const FftTables& T = c->fft[block + 1];
  S.L1 = T.L[0];
  S.L2 = T.L[1];
  S.L3 = T.L[2];
  S.N = N;
  const int nf[3] = {c->n1, c->n2, c->n3};
  for (int l = 0; l < 3; ++l) {
    S.th0[l] = 2.0 * M_PI * kappa[l] / nf[l];
    S.dth[l] = 2.0 * M_PI / nf[l];
  }
  for (int m = 0; m < 3; ++m)
    for (int d = 0; d < 5; ++d) S.cf[m][d] = c->cf[m][d];
  for (int q = 0; q < 21; ++q) S.Cref[q] = c->Cref[q];
  S.shift_rho = shift * c->rho_ref;
  S.data = z;
  hipLaunchKernelGGL(mode_solve_kernel, dim3(ceil_div(N, 256)), dim3(256), 0, c->stream, S);
  PBR_HIP(c, hipGetLastError());
  PBR_TRY(run_axis(c, block, 0, +1, z, z, 1.0));
  PBR_TRY(run_axis(c, block, 2, +1, z, z, 1.0));
  PBR_TRY(run_axis(c, block, 1, +1, z, z, 1.0 / (double)N));
  return ST_OK;
}
