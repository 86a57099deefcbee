// FFT-diagonal preconditioner of the shifted system (A + shift M) x = b:
//     z = T_xi diag_m(K(m)^-1) T_xi^H r,   K(m) = Bhat(m) C_ref Bhat(m)^H + shift rho_ref I_3
// with the Bloch Fourier basis T (Sec. 5.1, Eqs. 5.1-5.2) in the full space and
// T_sigma = T F_sigma (Sec. 5.2, Eqs. 5.3-5.5) in a parity block.
//
// Full space: coefficient(m) = sum_x e^{-i x.theta_m} r(x) with theta_m =
// ((phi1 + 2 pi p)/n1, ...): a twist e^{-i x_l phi_l/n_l} and a 3D DFT.
//
// Block b: its nodes form two simple-cubic sub-lattices, p = i mod 2, node
// (2i'+p, 2y2+o2(p), 2y3+o3(p)) with o2 = (a+p) mod 2, o3 = (a+c+p) mod 2.  For
// the orbit representatives m = (m1, q, r), q < n2/2, r < n3/2 (one per orbit
// of Eq. 5.3) the block coefficient splits into the two sub-lattice transforms
//     V_p(m1', q, r) = sum e^{-i(2i' alpha + 2 y2 beta + 2 y3 gamma)} r_p,
// plain twisted 3D DFTs of size n1/2 x n2/2 x n3/2, combined pointwise:
//     c_b = T_0 V_0 + (-1)^b e^{-i alpha} T_1 V_1,   m1 = m1' + b n1/2,
//     T_p = e^{-i(o2(p) beta_q + o3(p) gamma_r)},
// which is the folding F_sigma of Eq. 5.4 written in sub-lattice variables.
// K(m) is the same on every member of an orbit (Sec. 5.3), so the block
// preconditioner is: sub-lattice DFTs, fold, two 3x3 solves, unfold, inverse.
//
// Passes (each reads and writes the 3-component vector once; the first
// pass reads r, every later pass works in place on z).  A parity block whose
// box has them takes three:
//   1. plane pass: one (y3, component) plane of both sub-lattices per
//      work-group, transformed along i' and y2 in place in LDS;
//   2. y3 axis forward, fold + 3x3 solves + unfold per orbit pair, y3 axis
//      inverse, in place in LDS;
//   3. plane pass inverse, times 1/N;
// the in-place transforms (plane_r1 plans) leave the modes in digit-reversed
// order along each axis, which the solve reads through permuted phase tables.
// The full space, and blocks without such a box, take five:
//   1. i axis: length-n1 lines, split into even/odd half lines for a block;
//   2. j (y2) axis;
//   3. k (y3) axis forward, fold + 3x3 solves + unfold per mode, k axis
//      inverse -- all in LDS;
//   4. j axis inverse;   5. i axis inverse, times 1/N.
// There every 1D transform is a mixed radix-4/2/3/5 Stockham FFT in LDS on a
// batch of lines; lines along j and k are batched over consecutive i for
// coalescing.
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "blas.hpp"
#include "context.hpp"
#include "reduce.hpp"

namespace {

constexpr int FFT_THREADS = 256;
// Line batch of a work-group: about 512 complex elements per LDS buffer (more
// work-groups per CU; 1024 and 2048 measured slower), but at least 8 lines
// along the second axis, whose batch runs over consecutive i (8 x 16 bytes: whole
// 128-byte segments).
constexpr int FFT_ELEMS = 512;
__host__ __device__ constexpr int line_batch(int LM, int axis) {
  return FFT_ELEMS / LM >= (axis == 1 ? 8 : 1) ? FFT_ELEMS / LM : (axis == 1 ? 8 : 1);
}

__device__ inline cplx cj(cplx a, int c) { return c ? cconj(a) : a; }

template <int R, int SIGN>
__device__ inline void small_dft(cplx* v) {
  if constexpr (R == 2) {
    const cplx a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const cplx t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const cplx t2 = cadd(v[1], v[3]);
    const cplx d = csub(v[1], v[3]);
    const cplx t3 = (SIGN < 0) ? mk(d.y, -d.x) : mk(-d.y, d.x);  // d * (SIGN i)
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  } else if constexpr (R == 5) {
    // X_k = sum_j x_j W^{jk}, W = e^{SIGN 2 pi i / 5}: with t = x1 + x4, x2 + x3
    // and u = x1 - x4, x2 - x3, X_1,4 = a1 +- SIGN i b1, X_2,3 = a2 +- SIGN i b2
    const double c1 = 0.30901699437494742410;   // cos(2 pi / 5)
    const double c2 = -0.80901699437494742410;  // cos(4 pi / 5)
    const double s1 = 0.95105651629515357212;   // sin(2 pi / 5)
    const double s2 = 0.58778525229247312917;   // sin(4 pi / 5)
    const cplx t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    const cplx u1 = csub(v[1], v[4]), u2 = csub(v[2], v[3]);
    const cplx a1 = cfma(c2, t2, cfma(c1, t1, v[0]));
    const cplx a2 = cfma(c1, t2, cfma(c2, t1, v[0]));
    const cplx b1 = cfma(s2, u2, cscale(s1, u1));
    const cplx b2 = cfma(-s1, u2, cscale(s2, u1));
    const cplx ib1 = (SIGN < 0) ? mk(b1.y, -b1.x) : mk(-b1.y, b1.x);  // SIGN i b1
    const cplx ib2 = (SIGN < 0) ? mk(b2.y, -b2.x) : mk(-b2.y, b2.x);
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = cadd(a1, ib1);
    v[4] = csub(a1, ib1);
    v[2] = cadd(a2, ib2);
    v[3] = csub(a2, ib2);
  } else {
    static_assert(R == 3, "radix");
    const double h = 0.86602540378443864676;  // sqrt(3)/2
    const cplx t = cadd(v[1], v[2]);
    const cplx u = csub(v[1], v[2]);
    const cplx m = mk(v[0].x - 0.5 * t.x, v[0].y - 0.5 * t.y);
    const cplx iu = (SIGN < 0) ? mk(h * u.y, -h * u.x) : mk(-h * u.y, h * u.x);
    v[0] = cadd(v[0], t);
    v[1] = cadd(m, iu);
    v[2] = csub(m, iu);
  }
}

// DFT of R = 1..6, 8 values held in registers (same convention as small_dft):
// R = 6 and 8 as two interleaved halves of size 3 / 4 combined with e^{SIGN 2 pi i k / R}.
template <int R, int SIGN>
__device__ inline void reg_dft(cplx* v) {
  if constexpr (R == 1) {
  } else if constexpr (R == 6) {
    cplx e[3] = {v[0], v[2], v[4]}, o[3] = {v[1], v[3], v[5]};
    small_dft<3, SIGN>(e);
    small_dft<3, SIGN>(o);
    const double h = 0.86602540378443864676;  // sin(pi / 3)
    const cplx o1 = cmul(mk(0.5, SIGN * h), o[1]), o2 = cmul(mk(-0.5, SIGN * h), o[2]);
    v[0] = cadd(e[0], o[0]);
    v[3] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[4] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[5] = csub(e[2], o2);
  } else if constexpr (R == 8) {
    cplx e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    small_dft<4, SIGN>(e);
    small_dft<4, SIGN>(o);
    const double c = 0.70710678118654752440;  // cos(pi / 4)
    const cplx o1 = cmul(mk(c, SIGN * c), o[1]);
    const cplx o2 = (SIGN < 0) ? mk(o[2].y, -o[2].x) : mk(-o[2].y, o[2].x);  // SIGN i o2
    const cplx o3 = cmul(mk(-c, SIGN * c), o[3]);
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  } else {
    small_dft<R, SIGN>(v);
  }
}

// In-place plan of a length L = R1 * R2 for the plane pass: a strided step of
// R1-point DFTs (elements R2 n1 + n2) with twiddles, then a contiguous step of
// R2-point DFTs; the result sits in digit-reversed order, position R2 k1 + k2
// holding frequency k1 + R1 k2 (plane_freq).  R1 = L, R2 = 1 for a single step;
// 0 when L has no such split.
__host__ __device__ constexpr int plane_r1(int L) {
  switch (L) {
    case 2: case 3: case 4: case 5: case 6: case 8: return L;
    case 9: case 12: case 15: case 16: case 20: case 25: return L % 5 == 0 ? 5 : (L % 4 == 0 ? 4 : 3);
    case 10: return 5;
    case 18: case 24: case 30: case 36: return 6;
    case 32: case 40: case 48: case 64: return 8;
    default: return 0;
  }
}
__host__ __device__ inline int plane_freq(int pos, int L) {
  const int r1 = plane_r1(L), r2 = L / r1;
  return pos / r2 + r1 * (pos % r2);
}

// Radix plan of a length 2^a 3^b 5^c, fixed at compile time: radix-4 stages,
// then one radix-2 stage if needed, then radix-3 and radix-5 stages.
constexpr int plan_nfac(int L) {
  int n = 0;
  while (L % 4 == 0) { ++n; L /= 4; }
  while (L % 2 == 0) { ++n; L /= 2; }
  while (L % 3 == 0) { ++n; L /= 3; }
  while (L % 5 == 0) { ++n; L /= 5; }
  return n;
}
constexpr int plan_fac(int L, int s) {
  int n = 0;
  while (L % 4 == 0) { if (n == s) return 4; ++n; L /= 4; }
  while (L % 2 == 0) { if (n == s) return 2; ++n; L /= 2; }
  while (L % 3 == 0) { if (n == s) return 3; ++n; L /= 3; }
  while (L % 5 == 0) { if (n == s) return 5; ++n; L /= 5; }
  return 1;
}

// One Stockham stage on nb lines of length L stored back to back in LDS.
// Lines sit in LDS P >= L elements apart (P = L + 1 keeps a transposing access,
// one lane per line, off a single bank group).
template <int L, int P, int R, int NS, int SIGN>
__device__ inline void stage(const cplx* __restrict__ roots, const cplx* src, cplx* dst, int nb) {
  constexpr int LR = L / R;
  constexpr int TW = L / (NS * R);
  for (int w = threadIdx.x; w < nb * LR; w += blockDim.x) {
    const int b = w / LR;
    const int j = w - b * LR;
    const int jm = j % NS;
    cplx v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      cplx x = src[b * P + j + r * LR];
      if (r > 0 && NS > 1) x = cmul(x, cj(roots[(jm * r * TW) % L], SIGN > 0));
      v[r] = x;
    }
    small_dft<R, SIGN>(v);
    const int idx = (j / NS) * NS * R + jm;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[b * P + idx + r * NS] = v[r];
  }
}

// Stages S.. of a length-L transform of nb lines; the input is in a, the
// other buffer is b; returns the buffer that holds the result.
template <int L, int P, int S, int NS, int SIGN>
__device__ inline cplx* fft_stages(const cplx* __restrict__ roots, cplx* a, cplx* b, int nb) {
  if constexpr (S >= plan_nfac(L)) {
    return a;
  } else {
    constexpr int R = plan_fac(L, S);
    stage<L, P, R, NS, SIGN>(roots, a, b, nb);
    __syncthreads();
    return fft_stages<L, P, S + 1, NS * R, SIGN>(roots, b, a, nb);
  }
}

// ---------------------------------------------------------------------------
// Passes 1, 2, 4, 5: lines along axis 0 (i) or 1 (j).
// ---------------------------------------------------------------------------
struct LineArgs {
  int L1, L2, L3;
  long nlines;       // lines per component
  long N;
  const cplx* __restrict__ roots;
  double scale;
  struct {
    const cplx* in;
    cplx* out;
    const cplx* twist;  // e^{-i y phi / L}, y in [0, L) of the transform, this layout's k
    PcgHook h;          // fused PCG work (h.st == nullptr: plain transform)
  } b[PBR_MAX_BATCH];   // layout blockIdx.z of the batch
};

// First work-group of a PCG launch: finish the partials of the previous launch.
__device__ inline void pcg_finish(const PcgHook& H, double* sh) {
  const double v = block_sum_array(H.red_in, H.red_n, sh);
  if (threadIdx.x != 0) return;
  PcgScalars* st = H.st;
  if (H.role == 1) {  // |r|^2: convergence test
    if (H.init) {
      st->bb = v;
      st->rr = v;
      st->done = (v == 0.0) ? 1 : 0;
    } else {
      st->rr = v;
      st->iters += 1;
      if (v <= st->tol2 * st->bb) st->done = 1;
    }
  } else if (H.role == 2) {  // (r, z) = (1/N) sum_m c_m^H K(m)^-1 c_m
    const double rz = v * H.inv_n;
    st->beta = H.init ? 0.0 : rz / st->rz;
    st->rz_next = rz;
  }
}

// LT: transform length; AXIS: 0 (memory-contiguous lines of length LM) or 1;
// SPLIT: axis-0 lines of a block, LM = 2 LT, even and odd elements transformed
// separately.  MODE: 0 plain; 1 first PCG pass (input r after the update
// r -= alpha q, or r = b, x = 0 at init; |r|^2 partials); 2 last PCG pass
// (output p = scale z + beta p instead of z, and the update x += alpha p with
// the old p, deferred from the first pass so that pass reads neither x nor p;
// an iteration cut short by convergence gets it from pcg_fix_x).
template <int LT, int AXIS, int SPLIT, int SIGN, int MODE>
__global__ void __launch_bounds__(FFT_THREADS) fft_lines_kernel(LineArgs A) {
  constexpr int LM = SPLIT ? 2 * LT : LT;          // line length in memory
  constexpr int B = line_batch(LM, AXIS);  // lines per work-group
  constexpr int PL = LT + 1;                      // LDS pitch of a line
  __shared__ cplx buf0[(SPLIT ? 2 * B : B) * PL], buf1[(SPLIT ? 2 * B : B) * PL];
  __shared__ cplx roots_s[LT], twist_s[LT];  // the stages' twiddles and this layout's twist
  __shared__ double red[FFT_THREADS / 64 + 1];
  const PcgHook& H = A.b[blockIdx.z].h;
  const cplx* in_ = A.b[blockIdx.z].in;
  cplx* out_ = A.b[blockIdx.z].out;
  const cplx* __restrict__ twist = twist_s;
  PcgScalars* st = H.st;
  const bool first_wg = blockIdx.x == 0 && blockIdx.y == 0;
  const int comp = blockIdx.y;
  const long l0 = (long)blockIdx.x * B;
  const int nb = (int)min((long)B, A.nlines - l0);
  const long co = comp * A.N;
  const long es = AXIS == 0 ? 1 : A.L1;
  auto base_of = [&](long l) -> long {
    if (AXIS == 0) return l * LM;
    return (l % A.L1) + (l / A.L1) * (long)A.L1 * A.L2;
  };
  // element p of this thread: w = threadIdx.x + p * FFT_THREADS
  constexpr int PER = (B * LM + FFT_THREADS - 1) / FFT_THREADS;
  auto elem = [&](int w, int& b, int& e) {
    if (AXIS == 0) {
      b = w / LM;
      e = w - b * LM;
    } else {
      e = w / B;
      b = w - e * B;
    }
  };
  // Operands are loaded first, before the CG scalars (which need the partials
  // of the previous launch) and the convergence flag, so their latency overlaps
  // those reads: MODE 1 r, q (or b at init); MODE 2 the old p and x; else the input.
  cplx va[PER], vb[PER], vc[PER], vd[PER];
  long ix[PER];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int w = threadIdx.x + p * FFT_THREADS;
    int b, e;
    elem(w, b, e);
    const bool ok = w < B * LM && b < nb;
    ix[p] = ok ? co + base_of(l0 + b) + e * es : -1;
    va[p] = vb[p] = vc[p] = vd[p] = mk(0, 0);
    if (!ok) continue;
    if (MODE == 1) {
      if (H.init) {
        va[p] = H.b[ix[p]];
      } else {
        vc[p] = H.r[ix[p]];
        vd[p] = H.q[ix[p]];
      }
    } else {
      va[p] = in_[ix[p]];
      if (MODE == 2 && !H.init) {
        vb[p] = out_[ix[p]];
        vc[p] = H.x[ix[p]];
      }
    }
  }
  if (st && !(MODE == 1 && H.init) && st->done) return;  // uniform per work-group
  double alpha = 0.0;
  if (MODE == 1) {
    if (H.init) {
      if (first_wg && threadIdx.x == 0) {
        st->tol2 = H.tol2;
        st->iters = 0;
        st->done = 0;
        st->alpha = st->beta = st->pq = 0.0;
      }
    } else {
      const double pq = block_sum_array(H.red_in, H.red_n, red);
      if (!(pq > 0.0)) {  // breakdown: the operator is not positive on p
        if (first_wg && threadIdx.x == 0) {
          st->pq = pq;
          st->done = 2;
        }
        return;
      }
      alpha = st->rz / pq;
      if (first_wg && threadIdx.x == 0) {
        st->pq = pq;
        st->alpha = alpha;
      }
    }
  } else if (st && H.role && first_wg) {
    pcg_finish(H, red);
  }
  double beta = 0.0, alpha_x = 0.0;
  if (MODE == 2) {
    beta = st->beta;
    alpha_x = st->alpha;
    if (first_wg && threadIdx.x == 0) st->rz = st->rz_next;
  }
  // (visible to the stages and the output loop after the barrier that follows
  // the input loop; the input loop itself reads the twist from global memory)
  for (int t = threadIdx.x; t < LT; t += blockDim.x) {
    roots_s[t] = A.roots[t];
    twist_s[t] = A.b[blockIdx.z].twist[t];
  }
  const cplx* __restrict__ twist_g = A.b[blockIdx.z].twist;
  double rr = 0.0;
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    if (ix[p] < 0) continue;
    const int w = threadIdx.x + p * FFT_THREADS;
    int b, e;
    elem(w, b, e);
    const long idx = ix[p];
    cplx x;
    if (MODE == 1) {
      if (H.init) {
        x = va[p];
        H.r[idx] = x;
        H.x[idx] = mk(0, 0);
      } else {
        x = cfma(-alpha, vd[p], vc[p]);
        H.r[idx] = x;
      }
      rr = fma(x.x, x.x, fma(x.y, x.y, rr));
    } else {
      x = va[p];
    }
    const int slot = SPLIT ? 2 * b + (e & 1) : b;
    const int y = SPLIT ? e >> 1 : e;
    if (SIGN < 0) x = cmul(x, twist_g[y]);
    buf0[slot * PL + y] = x;
  }
  if (MODE == 1) {
    const double s = block_sum_all(rr, red);
    if (threadIdx.x == 0) H.part_out[comp * gridDim.x + blockIdx.x] = s;
  }
  __syncthreads();
  const cplx* res = fft_stages<LT, PL, 0, 1, SIGN>(roots_s, buf0, buf1, SPLIT ? 2 * nb : nb);
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    if (ix[p] < 0) continue;
    const int w = threadIdx.x + p * FFT_THREADS;
    int b, e;
    elem(w, b, e);
    const int slot = SPLIT ? 2 * b + (e & 1) : b;
    const int y = SPLIT ? e >> 1 : e;
    cplx x = res[slot * PL + y];
    if (SIGN > 0) x = cmul(x, cconj(twist[y]));
    if (MODE == 2 && !H.init) {
      out_[ix[p]] = cfma(beta, vb[p], cscale(A.scale, x));
      H.x[ix[p]] = cfma(alpha_x, vb[p], vc[p]);
    } else {
      out_[ix[p]] = cscale(A.scale, x);
    }
  }
}

// ---------------------------------------------------------------------------
// Plane pass of a parity block: both in-plane axes in one pass.  A work-group
// holds one (y3, component) plane of the block, both sub-lattices (2 L0 x L1
// complex; 128 KB at n = 128), in LDS and transforms it in place along i' and
// y2 for each sub-lattice (plane_r1 plans; the forward transform leaves both
// axes in digit-reversed order, which the mode solve reads through permuted
// mode-phase tables, and the inverse takes that order back to natural).
// MODE 0: plain transform in -> out (scale on the inverse).  MODE 1 (forward):
// first PCG pass, r -= alpha q (or r = b, x = 0 at init) with the |r|^2
// partials, then the transform of r.  MODE 2 (inverse): last PCG pass, every
// work-group finishes (r, z) from the mode solve's partials, beta = (r, z) /
// (r, z)_old; out p = scale z + beta p and x += alpha p (the old p).
// Scalars: alpha uses rz_next (the previous last pass's (r, z)); the first
// work-group of the first pass moves it to rz, which the last pass divides by.
// ---------------------------------------------------------------------------
// Work-group size of a plane pass: one work-group holds a whole plane (133 KB
// of LDS at n = 128), so it is alone on its CU and its transform phase issues
// no memory traffic; 1024 threads (16 waves) shorten that phase.  The inverse
// pass holds z, the old p and x in registers and keeps 512 threads: at 1024
// (a 128-register bound) it spills.
constexpr int plane_threads(int mode) { return mode == 2 ? 512 : 1024; }

struct PlaneArgs {
  int L3;            // planes (y3 extent)
  long N;            // block nodes
  double scale;
  const cplx* __restrict__ roots0;  // e^{-2 pi i t / L0}
  const cplx* __restrict__ roots1;  // e^{-2 pi i t / L1}
  struct {
    const cplx* in;
    cplx* out;
    const cplx* tw0;  // twist along i' (length L0), this layout's k
    const cplx* tw1;  // twist along y2 (length L1)
    PcgHook h;
  } b[PBR_MAX_BATCH];
};

// LDS geometry of a plane: row (p, y2) of L0 elements, pitch L0 + 1; the two
// sub-lattice planes SP apart with SP = 8 mod 16 (elements) so that lanes
// alternating between sub-lattices fall in different banks.
__host__ __device__ constexpr int plane_sp(int L0, int L1) {
  return L1 * (L0 + 1) + ((8 - (L1 * (L0 + 1)) % 16) + 16) % 16;
}

// One strided step (R1-point DFTs of elements R2 n1 + n2 of each line, then the
// twiddle W_L^(n2 k1)) or one contiguous step (R2-point DFTs of elements
// R2 k1 + k2, with the twiddle W_L^(-n2 k1) applied after them on the inverse),
// in place on nl lines.  Line l starts at lbase(l); consecutive elements of a
// line are ES apart.
template <int L, int ES, int SIGN, bool STRIDED, class LB>
__device__ inline void plane_step(cplx* sm, const cplx* __restrict__ roots, int nl, LB lbase) {
  constexpr int R1 = plane_r1(L), R2 = L / R1;
  constexpr int R = STRIDED ? R1 : R2;   // DFT size of this step
  constexpr int NT = STRIDED ? R2 : R1;  // DFTs per line
  if constexpr (R == 1) return;
#pragma unroll 1
  for (int t = threadIdx.x; t < nl * NT; t += blockDim.x) {
    const int l = t % nl, j = t / nl;
    cplx* base = sm + lbase(l);
    cplx v[R];
    if constexpr (STRIDED) {
      // forward: x[R2 n1 + j] -> DFT over n1 -> times W^(j k1) -> position R2 k1 + j
      // inverse: position R2 k1 + j -> DFT over k1 -> x[R2 n1 + j]
#pragma unroll
      for (int a = 0; a < R; ++a) v[a] = base[(R2 * a + j) * ES];
      reg_dft<R, SIGN>(v);
      if (SIGN < 0 && R2 > 1) {
#pragma unroll
        for (int a = 1; a < R; ++a) v[a] = cmul(v[a], roots[(j * a) % L]);
      }
#pragma unroll
      for (int a = 0; a < R; ++a) base[(R2 * a + j) * ES] = v[a];
    } else {
      // forward: contiguous group j (= k1): DFT over n2 -> position R2 j + k2
      // inverse: DFT over k2 -> times W^(-n2 j) -> position R2 j + n2
#pragma unroll
      for (int a = 0; a < R; ++a) v[a] = base[(R2 * j + a) * ES];
      reg_dft<R, SIGN>(v);
      if (SIGN > 0 && R1 > 1) {
#pragma unroll
        for (int a = 1; a < R; ++a) v[a] = cmul(v[a], cconj(roots[(j * a) % L]));
      }
#pragma unroll
      for (int a = 0; a < R; ++a) base[(R2 * j + a) * ES] = v[a];
    }
  }
}

// Both steps of the transform of every row (axis i') or every column (axis y2).
template <int L0, int L1, int SIGN, int AXIS>
__device__ inline void plane_axis(cplx* sm, const cplx* __restrict__ roots) {
  constexpr int RP = L0 + 1, SP = plane_sp(L0, L1);
  if constexpr (AXIS == 0) {
    // lines: rows (p, y2), line-fastest lanes (rows RP apart spread the banks)
    auto lb = [](int l) { return (l / L1) * SP + (l % L1) * RP; };
    if (SIGN < 0) {
      plane_step<L0, 1, SIGN, true>(sm, roots, 2 * L1, lb);
      __syncthreads();
      plane_step<L0, 1, SIGN, false>(sm, roots, 2 * L1, lb);
    } else {
      plane_step<L0, 1, SIGN, false>(sm, roots, 2 * L1, lb);
      __syncthreads();
      plane_step<L0, 1, SIGN, true>(sm, roots, 2 * L1, lb);
    }
  } else {
    // lines: columns (p, i'), consecutive lanes on consecutive i'
    auto lb = [](int l) { return (l / L0) * SP + (l % L0); };
    if (SIGN < 0) {
      plane_step<L1, RP, SIGN, true>(sm, roots, 2 * L0, lb);
      __syncthreads();
      plane_step<L1, RP, SIGN, false>(sm, roots, 2 * L0, lb);
    } else {
      plane_step<L1, RP, SIGN, false>(sm, roots, 2 * L0, lb);
      __syncthreads();
      plane_step<L1, RP, SIGN, true>(sm, roots, 2 * L0, lb);
    }
  }
  __syncthreads();
}

template <int L0, int L1, int SIGN, int MODE>
__global__ void __launch_bounds__(plane_threads(MODE)) plane_kernel(PlaneArgs A) {
  constexpr int PLANE_THREADS = plane_threads(MODE);
  constexpr int NEL = 2 * L0 * L1;  // plane elements, both sub-lattices
  constexpr int N1 = 2 * L0;        // i extent of the block box
  constexpr int RP = L0 + 1, SP = plane_sp(L0, L1);
  constexpr int PER = (NEL + PLANE_THREADS - 1) / PLANE_THREADS;
  __shared__ cplx sm[2 * SP];
  __shared__ cplx roots0_s[L0], roots1_s[L1];
  __shared__ double red[PLANE_THREADS / 64 + 1];
  const PcgHook& H = A.b[blockIdx.z].h;
  const cplx* in_ = A.b[blockIdx.z].in;
  cplx* out_ = A.b[blockIdx.z].out;
  const cplx* __restrict__ tw0 = A.b[blockIdx.z].tw0;
  const cplx* __restrict__ tw1 = A.b[blockIdx.z].tw1;
  PcgScalars* st = H.st;
  const int comp = blockIdx.y;
  const bool first_wg = blockIdx.x == 0 && blockIdx.y == 0;
  const long base = comp * A.N + (long)blockIdx.x * NEL;
  auto lds_of = [](int e) {  // element e of the plane in memory -> LDS position
    const int i = e % N1, y2 = e / N1;
    return (i & 1) * SP + y2 * RP + (i >> 1);
  };
  // Operands first (MODE 1: r, q or b; MODE 2: the transformed z, the old p, x;
  // MODE 0: the input), then the scalars, so their latencies overlap.
  cplx va[PER], vb[PER], vc[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = threadIdx.x + k * PLANE_THREADS;
    va[k] = vb[k] = vc[k] = mk(0, 0);
    if (e >= NEL) continue;
    if (MODE == 1) {
      if (H.init) {
        va[k] = H.b[base + e];
      } else {
        va[k] = H.r[base + e];
        vb[k] = H.q[base + e];
      }
    } else {
      va[k] = in_[base + e];
      if (MODE == 2 && !H.init) vb[k] = out_[base + e];  // old p
    }
  }
  for (int t = threadIdx.x; t < L0; t += blockDim.x) roots0_s[t] = A.roots0[t];
  for (int t = threadIdx.x; t < L1; t += blockDim.x) roots1_s[t] = A.roots1[t];
  if (st && !(MODE == 1 && H.init) && st->done) return;  // uniform per work-group
  double alpha = 0.0, beta = 0.0;
  if (MODE == 1) {
    if (H.init) {
      if (first_wg && threadIdx.x == 0) {
        st->tol2 = H.tol2;
        st->iters = 0;
        st->done = 0;
        st->alpha = st->beta = st->pq = 0.0;
      }
    } else {
      const double pq = block_sum_array(H.red_in, H.red_n, red);
      if (!(pq > 0.0)) {  // breakdown: the operator is not positive on p
        if (first_wg && threadIdx.x == 0) {
          st->pq = pq;
          st->done = 2;
        }
        return;
      }
      alpha = st->rz_next / pq;
      if (first_wg && threadIdx.x == 0) {
        st->pq = pq;
        st->alpha = alpha;
        st->rz = st->rz_next;
      }
    }
  } else if (MODE == 2) {
    const double rz = block_sum_array(H.red_in, H.red_n, red) * H.inv_n;
    alpha = st->alpha;
    beta = H.init ? 0.0 : rz / st->rz;
    if (first_wg && threadIdx.x == 0) {
      st->rz_next = rz;
      st->beta = beta;
    }
  }
  // into LDS (forward: r update and twist first)
  double rr = 0.0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = threadIdx.x + k * PLANE_THREADS;
    if (e >= NEL) continue;
    cplx x = va[k];
    if (MODE == 1) {
      if (H.init) {
        H.r[base + e] = x;
        H.x[base + e] = mk(0, 0);
      } else {
        x = cfma(-alpha, vb[k], x);
        H.r[base + e] = x;
      }
      rr = fma(x.x, x.x, fma(x.y, x.y, rr));
    }
    if (SIGN < 0) {
      const int i = e % N1, y2 = e / N1;
      x = cmul(x, cmul(tw0[i >> 1], tw1[y2]));
    }
    sm[lds_of(e)] = x;
  }
  if (MODE == 1) {
    const double s2 = block_sum_all(rr, red);
    if (threadIdx.x == 0) H.part_out[comp * gridDim.x + blockIdx.x] = s2;
  }
  if (MODE == 2 && !H.init) {
    // x is requested once z sits in LDS (its registers are free), so the
    // transform hides the latency
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = threadIdx.x + k * PLANE_THREADS;
      if (e < NEL) vc[k] = H.x[base + e];
    }
  }
  __syncthreads();
  if (SIGN < 0) {
    plane_axis<L0, L1, SIGN, 0>(sm, roots0_s);
    plane_axis<L0, L1, SIGN, 1>(sm, roots1_s);
  } else {
    plane_axis<L0, L1, SIGN, 1>(sm, roots1_s);
    plane_axis<L0, L1, SIGN, 0>(sm, roots0_s);
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = threadIdx.x + k * PLANE_THREADS;
    if (e >= NEL) continue;
    cplx x = sm[lds_of(e)];
    if (SIGN > 0) {
      const int i = e % N1, y2 = e / N1;
      x = cmul(x, cconj(cmul(tw0[i >> 1], tw1[y2])));
    }
    if (MODE == 2 && !H.init) {
      out_[base + e] = cfma(beta, vb[k], cscale(A.scale, x));
      H.x[base + e] = cfma(alpha, vb[k], vc[k]);
    } else {
      out_[base + e] = SIGN > 0 ? cscale(A.scale, x) : x;
    }
  }
}

// ---------------------------------------------------------------------------
// Pass 3: k axis forward, per-mode solve (with the orbit fold for a block),
// k axis inverse.
// ---------------------------------------------------------------------------
struct SolveArgs {
  int L1, L2, L3;
  int nb;  // layouts of the launch
  long N;
  const cplx* __restrict__ roots;  // length-L3 roots
  double cf[3][5];
  double Cref[21];
  double shift_rho;
  struct {
    cplx* data;
    PcgScalars* st;   // fused PCG: skip once converged, write (r, z) partials
    double* part_out;
    const double* rr_in;  // fused PCG after a plane pass: |r|^2 partials to finish
    int rr_n;             // (every work-group sums them; the first records the test)
    int init;
    int a, c;         // block class bits
    const cplx* twist;  // e^{-i y phi3 / L3} of this layout's k
    const cplx* e1;     // e^{i alpha_m} = e^{i (phi1 + 2 pi m)/n1}, m < n1
    const cplx* e2;     // e^{i beta_q},  q < n2
    const cplx* e3;     // e^{i gamma_r}, r < n3
  } b[PBR_MAX_BATCH];   // layout blockIdx.y of the batch
};

// Symbols of D'_m for the mode whose one-step phases are Ea = e^{i alpha},
// Eb = e^{i beta}, Eg = e^{i gamma}: the diagonal shifts have symbols
// e^{i(alpha +- beta +- gamma)} (Eq. 4.1), so e_m = cf[m][0] + h_m with
// h_m = sum_{d>0} cf[m][d] sd_d linear in Ea; the mode with -Ea (m1 + n/2 in a
// block's orbit) has e_m = cf[m][0] - h_m.  (The factors -i of the symbols
// cancel in Bhat C Bhat^H.)
__device__ inline void mode_half_symbols(const SolveArgs& S, cplx Ea, cplx Eb, cplx Eg,
                                         cplx h[3]) {
  const cplx ab = cmul(Ea, Eb), abc = cmulc(Eb, Ea);  // e^{i(a+b)}, e^{i(a-b)}
  cplx sd[4];
  sd[0] = cmul(ab, Eg);
  sd[1] = cmulc(Eg, ab);
  sd[2] = cmul(abc, Eg);
  sd[3] = cmulc(Eg, abc);
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    cplx acc = mk(0, 0);
#pragma unroll
    for (int d = 1; d <= 4; ++d) acc = cfma(S.cf[m][d], sd[d - 1], acc);
    h[m] = acc;
  }
}

// K^-1 for the symbols e, K = Bhat C_ref Bhat^H + shift rho_ref I_3
// (Sec. 5.3-5.4), as 9 doubles: the real diagonal (0, 1, 2) and the upper
// entries (0,1), (0,2), (1,2) (re, im at 3..8).  K is Hermitian positive
// definite; it is inverted through its adjugate (one division, no square roots).
__device__ inline void symbol_inverse(const SolveArgs& S, const cplx e[3], double kinv[9]) {
  // K = Bhat C Bhat^H with Bhat's rows (Voigt columns, symbol) sparse:
  //   u1: (11, e1) (13, e3) (12, e2);  u2: (22, e2) (23, e3) (12, e1);
  //   u3: (33, e3) (23, e2) (13, e1)
  // so K[r][c] = sum over the 3 x 3 pairs of C[k][l] e_a conj(e_b).
  constexpr int VK[3][3] = {{0, 4, 5}, {1, 3, 5}, {2, 3, 4}};  // Voigt columns of row r
  constexpr int VE[3][3] = {{0, 2, 1}, {1, 2, 0}, {2, 1, 0}};  // symbol index of each
  cplx G[3][3];  // G[a][b] = e_a conj(e_b) = conj(G[b][a])
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    G[a][a] = mk(e[a].x * e[a].x + e[a].y * e[a].y, 0.0);
#pragma unroll
    for (int b2 = a + 1; b2 < 3; ++b2) {
      G[a][b2] = cmulc(e[b2], e[a]);
      G[b2][a] = cconj(G[a][b2]);
    }
  }
  cplx K[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int col = r; col < 3; ++col) {
      cplx acc = mk(0, 0);
#pragma unroll
      for (int u = 0; u < 3; ++u)
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          const int k = VK[r][u], l = VK[col][v];
          const int rr = k <= l ? k : l, cc = k <= l ? l : k;
          const double cv = S.Cref[rr * 6 - (rr * (rr - 1)) / 2 + (cc - rr)];
          acc = cfma(cv, G[VE[r][u]][VE[col][v]], acc);
        }
      K[r][col] = acc;
    }
  // K = [[a, d, e], [conj d, bb, f], [conj e, conj f, c]]; K^-1 = adj(K) / det K
  const double a = K[0][0].x + S.shift_rho, bb = K[1][1].x + S.shift_rho,
               c = K[2][2].x + S.shift_rho;
  const cplx d = K[0][1], ee = K[0][2], f = K[1][2];
  const double A00 = fma(bb, c, -(f.x * f.x + f.y * f.y));
  const double A11 = fma(a, c, -(ee.x * ee.x + ee.y * ee.y));
  const double A22 = fma(a, bb, -(d.x * d.x + d.y * d.y));
  const cplx A01 = csub(cmulc(f, ee), cscale(c, d));   // e conj(f) - c d
  const cplx A02 = csub(cmul(d, f), cscale(bb, ee));   // d f - bb e
  const cplx A12 = csub(cmulc(d, ee), cscale(a, f));   // conj(d) e - a f
  const double det = fma(a, A00, fma(d.x, A01.x, fma(d.y, A01.y, fma(ee.x, A02.x, ee.y * A02.y))));
  const double id = 1.0 / det;
  kinv[0] = id * A00;
  kinv[1] = id * A11;
  kinv[2] = id * A22;
  kinv[3] = id * A01.x;
  kinv[4] = id * A01.y;
  kinv[5] = id * A02.x;
  kinv[6] = id * A02.y;
  kinv[7] = id * A12.x;
  kinv[8] = id * A12.y;
}

// x = K^-1 b for K^-1 in the 9-double form of symbol_inverse.
__device__ inline void inverse_apply(const double ki[9], const cplx b[3], cplx x[3]) {
  const cplx A01 = mk(ki[3], ki[4]), A02 = mk(ki[5], ki[6]), A12 = mk(ki[7], ki[8]);
  x[0] = cadd(cscale(ki[0], b[0]), cadd(cmul(A01, b[1]), cmul(A02, b[2])));
  x[1] = cadd(cmulc(A01, b[0]), cadd(cscale(ki[1], b[1]), cmul(A12, b[2])));
  x[2] = cadd(cmulc(A02, b[0]), cadd(cmulc(A12, b[1]), cscale(ki[2], b[2])));
}

__device__ inline void symbol_solve(const SolveArgs& S, const cplx e[3], const cplx b[3],
                                    cplx x[3]) {
  double ki[9];
  symbol_inverse(S, e, ki);
  inverse_apply(ki, b, x);
}

// i-values per work-group of the solve pass: 1536 complex per LDS buffer gives
// 8 consecutive i (128-byte segments) for a 64-long third axis.
constexpr int SOLVE_ELEMS = 1536;
constexpr int solve_bi(int L3, int blocked) {
  const int b = SOLVE_ELEMS / (3 * L3);
  return blocked ? (b >= 2 ? (b & ~1) : 2) : (b >= 1 ? b : 1);
}

template <int L3T, int BLK>
__global__ void __launch_bounds__(FFT_THREADS) fft_solve_kernel(SolveArgs S) {
  constexpr int BI = solve_bi(L3T, BLK);
  constexpr int NL = 3 * BI;  // lines of one work-group: component-major
  constexpr int PT = L3T + 1;  // LDS pitch of a line
  __shared__ cplx buf0[NL * PT], buf1[NL * PT];
  __shared__ cplx roots_s[L3T], twist_s[L3T], e3_s[L3T], e1_s[BI];
  __shared__ double red[FFT_THREADS / 64 + 1];
  // One-dimensional grid of tiles x layouts.  Work-group g runs on XCD g mod 8;
  // each XCD takes a contiguous range of (tile, layout) indices, layout fastest
  // (neighbouring tiles of a layout read neighbouring 128-byte runs together).
  long lin;
  {
    const long T = (long)gridDim.x, g = blockIdx.x, x = g % 8, j = g / 8;
    lin = x * (T / 8) + min(x, T % 8) + j;
  }
  const int lay = (int)(lin % S.nb);
  const int tile = (int)(lin / S.nb);
  cplx* const data = S.b[lay].data;
  PcgScalars* const st = S.b[lay].st;
  double* const part_out = S.b[lay].part_out;
  const int ca = S.b[lay].a, cc = S.b[lay].c;
  const cplx* __restrict__ e2 = S.b[lay].e2;
  const int groups_i = (S.L1 + BI - 1) / BI;
  const int q = tile / groups_i;
  const int i0 = (tile % groups_i) * BI;
  const int bi = min(BI, S.L1 - i0);
  const long kstride = (long)S.L1 * S.L2;
  const long base = i0 + (long)S.L1 * q;
  // tables of this work-group in LDS: twiddles, twist, e^{i gamma_r}, and
  // e^{i alpha} of its i-values (block: of its BI/2 sub-lattice pairs)
  {
    const cplx* __restrict__ e1g = S.b[lay].e1;
    const int e1o = BLK ? (i0 >> 1) : i0;
    for (int t = threadIdx.x; t < L3T; t += blockDim.x) {
      roots_s[t] = S.roots[t];
      twist_s[t] = S.b[lay].twist[t];
      e3_s[t] = S.b[lay].e3[t];
    }
    for (int t = threadIdx.x; t < (BLK ? bi / 2 : bi); t += blockDim.x) e1_s[t] = e1g[e1o + t];
  }
  // (the tables are read after the barrier below; the input loop reads the
  // twist from global memory)
  const cplx* __restrict__ twist = twist_s;
  const cplx* __restrict__ e3 = e3_s;
  const cplx* __restrict__ twist_g = S.b[lay].twist;
  for (int w = threadIdx.x; w < NL * L3T; w += blockDim.x) {
    const int y = w / NL;
    const int rem = w - y * NL;
    const int comp = rem / BI, di = rem - comp * BI;
    if (di < bi)
      buf0[(comp * BI + di) * PT + y] =
          cmul(data[comp * S.N + base + di + y * kstride], twist_g[y]);
  }
  // (the operands are requested before the convergence flag is read)
  if (st && st->done) return;  // uniform per work-group
  if (const double* rr_in = S.b[lay].rr_in) {
    // |r|^2 of this iteration and the convergence test, reduced in the same
    // order by every work-group, so all of them take the same decision
    const double v = block_sum_array(rr_in, S.b[lay].rr_n, red);
    const int init = S.b[lay].init;
    const bool conv = init ? (v == 0.0) : (v <= st->tol2 * st->bb);
    if (tile == 0 && threadIdx.x == 0) {
      st->rr = v;
      if (init) {
        st->bb = v;
      } else {
        st->iters += 1;
      }
      if (conv) st->done = 1;
    }
    if (conv) return;  // uniform per work-group
  }
  __syncthreads();
  cplx* f = fft_stages<L3T, PT, 0, 1, -1>(roots_s, buf0, buf1, NL);
  cplx* g = (f == buf0) ? buf1 : buf0;
  const cplx Eb = e2[q];
  double rz = 0.0;  // sum over this work-group's modes of Re(c^H K^-1 c)
  if (!BLK) {
    for (int w = threadIdx.x; w < bi * L3T; w += blockDim.x) {
      const int di = w / L3T, r = w - di * L3T;
      cplx bv[3], xv[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) bv[a] = f[(a * BI + di) * PT + r];
      cplx h[3], e[3];
      mode_half_symbols(S, e1_s[di], Eb, e3[r], h);
#pragma unroll
      for (int m = 0; m < 3; ++m) e[m] = mk(S.cf[m][0] + h[m].x, h[m].y);
      symbol_solve(S, e, bv, xv);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        g[(a * BI + di) * PT + r] = xv[a];
        rz = fma(bv[a].x, xv[a].x, fma(bv[a].y, xv[a].y, rz));
      }
    }
  } else {
    // sub-lattice p has offsets o2(p) = (a+p)&1, o3(p) = (a+c+p)&1
    const int o20 = ca & 1, o30 = (ca + cc) & 1;
    for (int w = threadIdx.x; w < (bi / 2) * L3T; w += blockDim.x) {
      const int dp = w / L3T, r = w - dp * L3T;
      const cplx Ea = e1_s[dp], Eg = e3[r];
      // T_p = e^{-i(o2 beta + o3 gamma)}: conj(Eb)^o2 conj(Eg)^o3
      const cplx cb = cconj(Eb), cg = cconj(Eg);
      const cplx one = mk(1.0, 0.0);
      const cplx T0 = cmul(o20 ? cb : one, o30 ? cg : one);
      const cplx T1 = cmul(o20 ? one : cb, o30 ? one : cg);
      const cplx t1e = cmulc(Ea, T1);  // T1 e^{-i alpha}
      cplx c0[3], c1[3], z0[3], z1[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const cplx v0 = cmul(T0, f[(a * BI + 2 * dp) * PT + r]);
        const cplx v1 = cmul(t1e, f[(a * BI + 2 * dp + 1) * PT + r]);
        c0[a] = cadd(v0, v1);
        c1[a] = csub(v0, v1);
      }
      // m1 = m1' and m1 = m1' + n1/2 (alpha + pi: -Ea) share the half symbols
      cplx h[3], ep[3], em[3];
      mode_half_symbols(S, Ea, Eb, Eg, h);
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        ep[m] = mk(S.cf[m][0] + h[m].x, h[m].y);
        em[m] = mk(S.cf[m][0] - h[m].x, -h[m].y);
      }
      symbol_solve(S, ep, c0, z0);
      symbol_solve(S, em, c1, z1);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        rz = fma(c0[a].x, z0[a].x, fma(c0[a].y, z0[a].y, rz));
        rz = fma(c1[a].x, z1[a].x, fma(c1[a].y, z1[a].y, rz));
        g[(a * BI + 2 * dp) * PT + r] = cmulc(T0, cadd(z0[a], z1[a]));
        g[(a * BI + 2 * dp + 1) * PT + r] = cmulc(t1e, csub(z0[a], z1[a]));
      }
    }
  }
  if (part_out) {
    const double v = block_sum_all(rz, red);
    if (threadIdx.x == 0) part_out[tile] = v;
  }
  __syncthreads();
  const cplx* res = fft_stages<L3T, PT, 0, 1, +1>(roots_s, g, f, NL);
  for (int w = threadIdx.x; w < NL * L3T; w += blockDim.x) {
    const int y = w / NL;
    const int rem = w - y * NL;
    const int comp = rem / BI, di = rem - comp * BI;
    if (di < bi)
      data[comp * S.N + base + di + y * kstride] =
          cmul(res[(comp * BI + di) * PT + y], cconj(twist[y]));
  }
}

// Mode-solve pass of the three-pass block structure.  A work-group takes bi
// consecutive i (both sub-lattices, bi / 2 orbit pairs; a contiguous run of
// 16 bi bytes per line), one y2 position q and all L3 positions r of the three
// components, transforms them in place along r (plane_r1 plan; the mode order
// along r is then digit-reversed, as it already is along i' and y2 after the
// plane pass), folds each orbit pair, solves the two 3x3 systems of its
// symbols, unfolds, transforms back and writes in place.  Also finishes |r|^2 and the convergence test (rr_in) and
// writes the (r, z) partials, like fft_solve_kernel.
// Instances: BIM = 8 with 256 threads (26 KB of LDS at L3 = 64, so four
// work-groups of four waves share a CU and one's loads overlap another's
// transforms), BIM = 16 and 32 with 512 threads; a launch uses bi <= BIM
// i-values per work-group, picked per (box, batch size) by tuned_solve_width.
// The register count (124-128 VGPRs at L3 = 64, set by the 3 x 3 adjugate
// solves) allows four waves per SIMD: two 512-thread work-groups per CU (their
// LDS would allow three) or four 256-thread ones.

template <int L3T, int BIM, int NT>
__global__ void __launch_bounds__(NT) solve_plane_kernel(SolveArgs S, int bi) {
  constexpr int PT = L3T + 1;  // LDS pitch of a line along r
  __shared__ cplx sm[3 * BIM * PT];
  __shared__ cplx roots_s[L3T], e3_s[L3T], tw_s[L3T], e1_s[BIM / 2];
  __shared__ double red[NT / 64 + 1];
  long lin;  // XCD-aware numbering of (tile, layout), as in fft_solve_kernel
  {
    const long T = (long)gridDim.x, g = blockIdx.x, x = g % 8, j = g / 8;
    lin = x * (T / 8) + min(x, T % 8) + j;
  }
  const int lay = (int)(lin % S.nb);
  const int tile = (int)(lin / S.nb);
  cplx* const data = S.b[lay].data;
  PcgScalars* const st = S.b[lay].st;
  const int ca = S.b[lay].a, cc = S.b[lay].c;
  const int groups_i = S.L1 / bi;
  const int q = tile / groups_i;
  const int i0 = (tile % groups_i) * bi;
  const long kstride = (long)S.L1 * S.L2;
  const long base = i0 + (long)S.L1 * q;
  constexpr int PER = (3 * BIM * L3T + NT - 1) / NT;
  const cplx* __restrict__ twist_g = S.b[lay].twist;
  // element e = threadIdx.x + k NT of the (comp, r, di) box, di fastest: NT is
  // a multiple of bi (both powers of two), so di is the same for all k of a
  // thread and (comp, r) = e / bi advances by NT / bi (one division per thread)
  const int di = threadIdx.x % bi, rest0 = threadIdx.x / bi, rstep = NT / bi;
  cplx v[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int rest = rest0 + k * rstep;
    v[k] = mk(0, 0);
    if (rest < 3 * L3T) {
      const int r = rest % L3T, comp = rest / L3T;
      v[k] = data[comp * S.N + base + di + r * kstride];
    }
  }
  for (int t = threadIdx.x; t < L3T; t += blockDim.x) {
    roots_s[t] = S.roots[t];
    e3_s[t] = S.b[lay].e3[t];
    tw_s[t] = twist_g[t];
  }
  for (int t = threadIdx.x; t < bi / 2; t += blockDim.x) e1_s[t] = S.b[lay].e1[(i0 >> 1) + t];
  if (st && st->done) return;  // uniform per work-group
  if (const double* rr_in = S.b[lay].rr_in) {
    const double vv = block_sum_array(rr_in, S.b[lay].rr_n, red);
    const int init = S.b[lay].init;
    const bool conv = init ? (vv == 0.0) : (vv <= st->tol2 * st->bb);
    if (tile == 0 && threadIdx.x == 0) {
      st->rr = vv;
      if (init) {
        st->bb = vv;
      } else {
        st->iters += 1;
      }
      if (conv) st->done = 1;
    }
    if (conv) return;  // uniform per work-group
  }
  __syncthreads();  // the tables
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int rest = rest0 + k * rstep;
    if (rest < 3 * L3T) {
      const int r = rest % L3T, comp = rest / L3T;
      sm[(comp * bi + di) * PT + r] = cmul(v[k], tw_s[r]);
    }
  }
  __syncthreads();
  const int nl = 3 * bi;
  auto lb = [](int l) { return l * PT; };
  plane_step<L3T, 1, -1, true>(sm, roots_s, nl, lb);
  __syncthreads();
  plane_step<L3T, 1, -1, false>(sm, roots_s, nl, lb);
  __syncthreads();
  const cplx Eb = S.b[lay].e2[q];
  const int o20 = ca & 1, o30 = (ca + cc) & 1;
  double rz = 0.0;
  for (int w = threadIdx.x; w < (bi / 2) * L3T; w += blockDim.x) {
    const int dp = w / L3T, r = w - dp * L3T;
    const cplx Ea = e1_s[dp], Eg = e3_s[r];
    const cplx cb = cconj(Eb), cg = cconj(Eg);
    const cplx one = mk(1.0, 0.0);
    const cplx T0 = cmul(o20 ? cb : one, o30 ? cg : one);
    const cplx T1 = cmul(o20 ? one : cb, o30 ? one : cg);
    const cplx t1e = cmulc(Ea, T1);  // T1 e^{-i alpha}
    // m1 = m1' and m1 = m1' + n1/2 (alpha + pi: -Ea) share the half symbols.
    // The two 3x3 solves run one after the other, each from right-hand sides
    // read from LDS (the inputs stay there until the pair's outputs replace
    // them), so only the first solution is live across the second solve.
    cplx c[3], z0[3], z[3], e[3], h[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      c[a] = cadd(cmul(T0, sm[(a * bi + 2 * dp) * PT + r]),
                  cmul(t1e, sm[(a * bi + 2 * dp + 1) * PT + r]));
    mode_half_symbols(S, Ea, Eb, Eg, h);
#pragma unroll
    for (int m = 0; m < 3; ++m) e[m] = mk(S.cf[m][0] + h[m].x, h[m].y);
    symbol_solve(S, e, c, z0);
#pragma unroll
    for (int a = 0; a < 3; ++a) rz = fma(c[a].x, z0[a].x, fma(c[a].y, z0[a].y, rz));
#pragma unroll
    for (int a = 0; a < 3; ++a)
      c[a] = csub(cmul(T0, sm[(a * bi + 2 * dp) * PT + r]),
                  cmul(t1e, sm[(a * bi + 2 * dp + 1) * PT + r]));
    mode_half_symbols(S, Ea, Eb, Eg, h);
#pragma unroll
    for (int m = 0; m < 3; ++m) e[m] = mk(S.cf[m][0] - h[m].x, -h[m].y);
    symbol_solve(S, e, c, z);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      rz = fma(c[a].x, z[a].x, fma(c[a].y, z[a].y, rz));
      sm[(a * bi + 2 * dp) * PT + r] = cmulc(T0, cadd(z0[a], z[a]));
      sm[(a * bi + 2 * dp + 1) * PT + r] = cmulc(t1e, csub(z0[a], z[a]));
    }
  }
  if (double* part_out = S.b[lay].part_out) {
    const double vv = block_sum_all(rz, red);
    if (threadIdx.x == 0) part_out[tile] = vv;
  }
  __syncthreads();
  plane_step<L3T, 1, +1, false>(sm, roots_s, nl, lb);
  __syncthreads();
  plane_step<L3T, 1, +1, true>(sm, roots_s, nl, lb);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int rest = rest0 + k * rstep;
    if (rest < 3 * L3T) {
      const int r = rest % L3T, comp = rest / L3T;
      data[comp * S.N + base + di + r * kstride] =
          cmul(sm[(comp * bi + di) * PT + r], cconj(tw_s[r]));
    }
  }
}

__global__ void table_kernel(int L, double phi, int kind, cplx* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L) return;
  double ang;
  if (kind == 0)
    ang = -(double)t * phi / (double)L;              // twist e^{-i t phi / L}
  else if (kind == 1)
    ang = -2.0 * M_PI * (double)t / (double)L;       // roots e^{-2 pi i t / L}
  else
    ang = (phi + 2.0 * M_PI * (double)t) / (double)L;  // mode phase e^{i (phi + 2 pi t)/L}
  double s, c;
  sincos(ang, &s, &c);
  out[t] = mk(c, s);
}

// Mode phases e^{i (phi + 2 pi f) / n} in the digit-reversed order the plane
// pass leaves along an axis of length L (f = plane_freq(t, L), t < L).
__global__ void perm_phase_kernel(int L, int n, double phi, cplx* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L) return;
  const double ang = (phi + 2.0 * M_PI * (double)plane_freq(t, L)) / (double)n;
  double sn, cs;
  sincos(ang, &sn, &cs);
  out[t] = mk(cs, sn);
}

bool plane_pass(const pbr_ctx* c);

// Tables of a layout kind (natural: slot 0; parity blocks, which share the box
// shape: slot 1): for each transform length Lt[l] (axis 0 of a block: n1/2) the
// roots and the twist, and the mode phases e^{i(phi_l + 2 pi t)/n_l}.
int ensure_tables(pbr_ctx* c, int slot, bool blocked, const double kappa[3]) {
  FftTables& T = c->tables(slot, blocked);
  const int Lt[3] = {blocked ? c->n1 / 2 : c->n1, blocked ? c->n2 / 2 : c->n2,
                     blocked ? c->n3 / 2 : c->n3};
  const int nf[3] = {c->n1, c->n2, c->n3};
  for (int l = 0; l < 3; ++l) {
    if (!T.roots[l]) {
      T.L[l] = Lt[l];
      PBR_TRY(dev_alloc(c, (void**)&T.roots[l], sizeof(cplx) * Lt[l]));
      PBR_TRY(dev_alloc(c, (void**)&T.twist[l], sizeof(cplx) * Lt[l]));
      PBR_TRY(dev_alloc(c, (void**)&T.post[l], sizeof(cplx) * nf[l]));
      hipLaunchKernelGGL(table_kernel, dim3(ceil_div(Lt[l], 256)), dim3(256), 0, c->stream,
                         Lt[l], 0.0, 1, T.roots[l]);
    }
  }
  const bool perm = blocked && plane_pass(c);
  for (int l = 0; perm && l < 3; ++l)
    if (!T.postp[l]) {
      PBR_TRY(dev_alloc(c, (void**)&T.postp[l], sizeof(cplx) * Lt[l]));
      T.kappa[0] = 1e300;  // (re)build every table below
    }
  if (T.kappa[0] != kappa[0] || T.kappa[1] != kappa[1] || T.kappa[2] != kappa[2]) {
    for (int l = 0; l < 3; ++l) {
      const double phi = 2.0 * M_PI * kappa[l];
      hipLaunchKernelGGL(table_kernel, dim3(ceil_div(Lt[l], 256)), dim3(256), 0, c->stream,
                         Lt[l], phi, 0, T.twist[l]);
      hipLaunchKernelGGL(table_kernel, dim3(ceil_div(nf[l], 256)), dim3(256), 0, c->stream,
                         nf[l], phi, 2, T.post[l]);
      if (T.postp[l])
        hipLaunchKernelGGL(perm_phase_kernel, dim3(ceil_div(Lt[l], 256)), dim3(256), 0,
                           c->stream, Lt[l], nf[l], phi, T.postp[l]);
      T.kappa[l] = kappa[l];
    }
  }
  PBR_HIP(c, hipGetLastError());
  return ST_OK;
}

// ---- launch helpers: one kernel instance per supported transform length ----
#define PBR_FFT_LENGTHS(X)                                                                 \
  X(1) X(2) X(3) X(4) X(5) X(6) X(8) X(10) X(12) X(15) X(16) X(20) X(24) X(30) X(32) X(40) \
  X(48) X(60) X(64) X(80) X(96) X(120) X(128) X(160) X(192) X(240) X(256)

typedef void (*LineKernel)(LineArgs);
typedef void (*SolveKernel)(SolveArgs);

template <int AXIS, int SPLIT, int SIGN, int MODE>
LineKernel line_kernel(int L) {
  switch (L) {
#define PBR_CASE(n) \
  case n:           \
    return fft_lines_kernel<n, AXIS, SPLIT, SIGN, MODE>;
    PBR_FFT_LENGTHS(PBR_CASE)
#undef PBR_CASE
    default:
      return nullptr;
  }
}

template <int BLK>
SolveKernel solve_kernel(int L) {
  switch (L) {
#define PBR_CASE(n) \
  case n:           \
    return fft_solve_kernel<n, BLK>;
    PBR_FFT_LENGTHS(PBR_CASE)
#undef PBR_CASE
    default:
      return nullptr;
  }
}

// One pass of lines along `axis` for nb layouts of one kind; mode 1 / 2 are
// the first / last PCG pass.  *nparts receives the partials per layout that a
// mode-1 launch writes.  T supplies the transform length and roots (the same
// for every layout of the batch); each layout brings its own twist.
struct LineIO {
  const cplx* in;
  cplx* out;
  const cplx* twist;
  PcgHook h;
};

int run_lines(pbr_ctx* c, const FftTables& T, bool blocked, int nb, int axis, int sign, int mode,
              const LineIO* io, double scale, long part_cap, int* nparts) {
  const long N = c->layout_nodes(blocked ? 0 : -1);
  LineArgs A;
  A.L1 = c->n1;
  A.L2 = blocked ? c->n2 / 2 : c->n2;
  A.L3 = blocked ? c->n3 / 2 : c->n3;
  const int split = (axis == 0 && blocked) ? 1 : 0;
  const int LT = T.L[axis];
  const int LM = split ? 2 * LT : LT;
  A.nlines = N / LM;
  A.N = N;
  A.roots = T.roots[axis];
  A.scale = scale;
  for (int t = 0; t < nb; ++t) {
    A.b[t].in = io[t].in;
    A.b[t].out = io[t].out;
    A.b[t].twist = io[t].twist;
    A.b[t].h = io[t].h;
  }
  LineKernel k = nullptr;
  if (axis == 0 && split) {
    if (sign < 0)
      k = mode == 1 ? line_kernel<0, 1, -1, 1>(LT) : line_kernel<0, 1, -1, 0>(LT);
    else
      k = mode == 2 ? line_kernel<0, 1, 1, 2>(LT) : line_kernel<0, 1, 1, 0>(LT);
  } else if (axis == 0) {
    if (sign < 0)
      k = mode == 1 ? line_kernel<0, 0, -1, 1>(LT) : line_kernel<0, 0, -1, 0>(LT);
    else
      k = mode == 2 ? line_kernel<0, 0, 1, 2>(LT) : line_kernel<0, 0, 1, 0>(LT);
  } else {
    k = sign < 0 ? line_kernel<1, 0, -1, 0>(LT) : line_kernel<1, 0, 1, 0>(LT);
  }
  if (!k) {
    c->set_error("unsupported FFT length (2^a 3^b 5^c from the supported list, up to 256; blocks: n_l / 2)");
    return ST_EINVAL;
  }
  const int B = line_batch(LM, axis);
  dim3 grid(ceil_div(A.nlines, B), 3, nb);
  if (nparts) *nparts = (int)(grid.x * 3);
  if (mode == 1 && (long)grid.x * 3 > part_cap) {
    c->set_error("grid too large for the PCG partial buffers");
    return ST_EINVAL;
  }
  hipLaunchKernelGGL(k, grid, dim3(FFT_THREADS), 0, c->stream, A);
  PBR_HIP(c, hipGetLastError());
  return ST_OK;
}

typedef void (*PlaneKernel)(PlaneArgs);

#define PBR_PLANE_LENGTHS(X) \
  X(2) X(3) X(4) X(5) X(6) X(8) X(10) X(12) X(15) X(16) X(20) X(24) X(30) X(32) X(40) X(48) X(64)

template <int SIGN, int MODE>
PlaneKernel plane_kernel_for(int L0, int L1) {
  if (L0 != L1) return nullptr;
  switch (L0) {
#define PBR_CASE(n) \
  case n:           \
    return plane_kernel<n, n, SIGN, MODE>;
    PBR_PLANE_LENGTHS(PBR_CASE)
#undef PBR_CASE
    default:
      return nullptr;
  }
}

// Whether the block preconditioner runs as three passes (plane, mode solve,
// plane): the block box has a plane kernel and the setting allows it.
bool plane_length(int L) {
  switch (L) {
#define PBR_CASE(n) \
  case n:           \
    return true;
    PBR_PLANE_LENGTHS(PBR_CASE)
#undef PBR_CASE
    default:
      return false;
  }
}

bool plane_pass(const pbr_ctx* c) {
  if (c->precond_passes == 5 || !c->even) return false;
  return plane_kernel_for<-1, 1>(c->n1 / 2, c->n2 / 2) != nullptr && plane_length(c->n3 / 2);
}

// One plane pass over nb parity-block layouts: sign -1 forward (mode 0 or 1),
// +1 inverse (mode 0 or 2).  *nparts receives the partials per layout a mode-1
// launch writes.
struct PlaneIO {
  const cplx* in;
  cplx* out;
  const FftTables* T;
  PcgHook h;
};

int run_plane(pbr_ctx* c, int nb, int sign, int mode, const PlaneIO* io, double scale,
              long part_cap, int* nparts) {
  const int L0 = c->n1 / 2, L1 = c->n2 / 2, L3 = c->n3 / 2;
  PlaneKernel k = nullptr;
  // MODE of the instance chosen (its work-group size follows from it)
  const int kmode = sign < 0 ? (mode == 1 ? 1 : 0) : (mode == 2 ? 2 : 0);
  if (sign < 0)
    k = kmode == 1 ? plane_kernel_for<-1, 1>(L0, L1) : plane_kernel_for<-1, 0>(L0, L1);
  else
    k = kmode == 2 ? plane_kernel_for<1, 2>(L0, L1) : plane_kernel_for<1, 0>(L0, L1);
  if (!k) {
    c->set_error("no plane pass for this block box");
    return ST_EINVAL;
  }
  PlaneArgs A;
  A.L3 = L3;
  A.N = c->layout_nodes(0);
  A.scale = scale;
  A.roots0 = io[0].T->roots[0];
  A.roots1 = io[0].T->roots[1];
  for (int t = 0; t < nb; ++t) {
    A.b[t].in = io[t].in;
    A.b[t].out = io[t].out;
    A.b[t].tw0 = io[t].T->twist[0];
    A.b[t].tw1 = io[t].T->twist[1];
    A.b[t].h = io[t].h;
  }
  if (nparts) *nparts = 3 * L3;
  if (mode == 1 && 3L * L3 > part_cap) {
    c->set_error("grid too large for the PCG partial buffers");
    return ST_EINVAL;
  }
  hipLaunchKernelGGL(k, dim3(L3, 3, nb), dim3(plane_threads(kmode)), 0, c->stream, A);
  PBR_HIP(c, hipGetLastError());
  return ST_OK;
}

struct SolveIO {
  int block;
  cplx* data;
  PcgScalars* st;
  double* part_out;
  const FftTables* T;  // this layout's k-point tables
  bool perm = false;   // input left by the plane pass: digit-reversed i' and y2
  const double* rr_in = nullptr;  // |r|^2 partials to finish (fused PCG after a plane pass)
  int rr_n = 0;
  int init = 0;
};

struct PlaneSolveKernel {
  void (*fn)(SolveArgs, int) = nullptr;
  int threads = 0;
};

// Mode-solve kernel of the three-pass structure for third-axis length L3 and
// i-width bi: the smallest instance whose LDS holds bi (8, 16 or 32 i-values)
// and its work-group size.
PlaneSolveKernel solve_plane_for(int L3, int bi) {
  PlaneSolveKernel k;
  switch (L3) {
#define PBR_CASE(n)                                                           \
  case n:                                                                     \
    if (bi <= 8) {                                                            \
      k.fn = solve_plane_kernel<n, 8, 256>;                                   \
      k.threads = 256;                                                        \
    } else {                                                                  \
      k.fn = bi <= 16 ? solve_plane_kernel<n, 16, 512> : solve_plane_kernel<n, 32, 512>; \
      k.threads = 512;                                                        \
    }                                                                         \
    break;
    PBR_PLANE_LENGTHS(PBR_CASE)
#undef PBR_CASE
    default:
      break;
  }
  return k;
}

// i-width of the mode-solve pass for this box and batch size: the cost model's
// choice (16, or the largest power of two <= 16 dividing n1; at most 32 for
// third axes up to 32) unless another candidate (8, 16, 32 dividing n1) is at
// least 5 % faster when timed on a copy of the batch's data at the first call
// (the pass works in place; the copy is refreshed before each timed launch).
// Widths 8 run on 256-thread work-groups, 16 and 32 on 512-thread ones.  A
// width pinned by pbr_set_solve_width that divides n1 replaces all this.
// The choice is kept per context, so later launches, and the graphs that
// capture them, use it.  The 5 % margin keeps it stable where one width is
// clearly faster; where two time within noise of each other (four layouts at
// n = 128: 8 and 16) fresh contexts may choose differently, and with the width
// the grouping of the (r, z) partials, so the last bits of a solve.
// pbr_set_solve_width pins the width where that matters.
int tuned_solve_width(pbr_ctx* c, const SolveArgs& S, int nb, bool may_tune, int* bi_out) {
  if (c->pin_bi > 0 && S.L1 % c->pin_bi == 0) {  // pinned by pbr_set_solve_width
    *bi_out = c->pin_bi;
    return ST_OK;
  }
  for (const auto& e : c->solve_tune)
    if (e.nb == nb && e.L1 == S.L1 && e.L2 == S.L2 && e.L3 == S.L3 && e.bi > 0) {
      *bi_out = e.bi;
      return ST_OK;
    }
  auto fits = [&](int bi) { return bi >= 2 && S.L1 % bi == 0; };
  int model = S.L3 > 32 ? 16 : 32;
  while (model > 2 && !fits(model)) model >>= 1;
  int cand[3], ncand = 0;
  cand[ncand++] = model;
  for (int bi : {8, 16, 32})
    if (bi != model && fits(bi)) cand[ncand++] = bi;
  *bi_out = model;
  if (!may_tune) return ST_OK;  // no timing, no allocation, nothing recorded
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  const bool capturing =
      hipStreamIsCapturing(c->stream, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone;
  const long n3 = 3 * S.N;
  cplx* scratch = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!capturing && ncand > 1 && S.N >= 4096 &&
      dev_alloc(c, (void**)&scratch, sizeof(cplx) * n3 * nb) == ST_OK &&
      hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
    SolveArgs T = S;
    for (int t = 0; t < nb; ++t) {
      T.b[t].data = scratch + (long)t * n3;
      T.b[t].st = nullptr;
      T.b[t].part_out = nullptr;
      T.b[t].rr_in = nullptr;
    }
    float best_ms = -1.0f;
    bool ok = true;
    for (int r = 0; r < 2 && ok; ++r)  // the first round warms the caches
      for (int k = 0; k < ncand && ok; ++k) {
        float tot = 0.0f;
        for (int rep = 0; ok && rep < (r == 1 ? 3 : 1); ++rep) {
          for (int t = 0; t < nb && ok; ++t)
            ok = hipMemcpyAsync(T.b[t].data, S.b[t].data, sizeof(cplx) * n3,
                                hipMemcpyDeviceToDevice, c->stream) == hipSuccess;
          const long nwg = (long)(S.L1 / cand[k]) * S.L2;
          ok = ok && hipEventRecord(e0, c->stream) == hipSuccess;
          const PlaneSolveKernel kk = solve_plane_for(S.L3, cand[k]);
          ok = ok && kk.fn;
          if (ok)
            hipLaunchKernelGGL(kk.fn, dim3((unsigned)(nwg * nb)), dim3(kk.threads), 0,
                               c->stream, T, cand[k]);
          ok = ok && hipGetLastError() == hipSuccess &&
               hipEventRecord(e1, c->stream) == hipSuccess &&
               hipEventSynchronize(e1) == hipSuccess;
          float ms = 0.0f;
          ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
          tot += ms;
        }
        if (ok && r == 1 && (best_ms < 0.0f || tot < 0.95f * best_ms)) {
          best_ms = tot;
          *bi_out = cand[k];
        }
      }
    if (!ok) *bi_out = model;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (scratch) {
    (void)hipStreamSynchronize(c->stream);
    dev_free(scratch);
  }
  if (capturing) return ST_OK;  // not recorded: the next eager call tunes
  auto& slot = c->solve_tune[c->solve_tune_next];
  c->solve_tune_next = (c->solve_tune_next + 1) % PBR_TUNE_SLOTS;
  slot.nb = nb;
  slot.L1 = S.L1;
  slot.L2 = S.L2;
  slot.L3 = S.L3;
  slot.bi = *bi_out;
  return ST_OK;
}

void fill_symbol_args(const pbr_ctx* c, double shift, SolveArgs& S) {
  for (int m = 0; m < 3; ++m)
    for (int d = 0; d < 5; ++d) S.cf[m][d] = c->cf[m][d];
  for (int qq = 0; qq < 21; ++qq) S.Cref[qq] = c->Cref[qq];
  S.shift_rho = shift * c->rho_ref;
}

int run_solve(pbr_ctx* c, bool blocked, int nb, const SolveIO* io, double shift, long part_cap,
              int* nparts, bool may_tune = true) {
  const FftTables& T = *io[0].T;
  SolveArgs S;
  S.L1 = c->n1;
  S.L2 = blocked ? c->n2 / 2 : c->n2;
  S.L3 = blocked ? c->n3 / 2 : c->n3;
  S.N = c->layout_nodes(blocked ? 0 : -1);
  S.roots = T.roots[2];
  S.nb = nb;
  fill_symbol_args(c, shift, S);
  for (int t = 0; t < nb; ++t) {
    S.b[t].data = io[t].data;
    S.b[t].st = io[t].st;
    S.b[t].part_out = io[t].part_out;
    S.b[t].a = io[t].block >= 0 ? io[t].block >> 1 : 0;
    S.b[t].c = io[t].block >= 0 ? io[t].block & 1 : 0;
    S.b[t].twist = io[t].T->twist[2];
    S.b[t].e1 = io[t].perm ? io[t].T->postp[0] : io[t].T->post[0];
    S.b[t].e2 = io[t].perm ? io[t].T->postp[1] : io[t].T->post[1];
    S.b[t].e3 = io[t].perm ? io[t].T->postp[2] : io[t].T->post[2];
    S.b[t].rr_in = io[t].rr_in;
    S.b[t].rr_n = io[t].rr_n;
    S.b[t].init = io[t].init;
  }
  if (io[0].perm) {
    // three-pass structure: every axis in digit-reversed mode order; the
    // i-width of a work-group is tuned per (box, batch size)
    int bi = 0;
    PBR_TRY(tuned_solve_width(c, S, nb, may_tune, &bi));
    const PlaneSolveKernel k = solve_plane_for(S.L3, bi);
    if (!k.fn) {
      c->set_error("no mode-solve pass for this block box");
      return ST_EINVAL;
    }
    const long nwg = (long)(S.L1 / bi) * S.L2;
    if (nparts) *nparts = (int)nwg;
    if (io[0].part_out && nwg > part_cap) {
      c->set_error("grid too large for the PCG partial buffers");
      return ST_EINVAL;
    }
    hipLaunchKernelGGL(k.fn, dim3((unsigned)(nwg * nb)), dim3(k.threads), 0, c->stream, S, bi);
    PBR_HIP(c, hipGetLastError());
    return ST_OK;
  }
  const SolveKernel k = blocked ? solve_kernel<1>(S.L3) : solve_kernel<0>(S.L3);
  if (!k) {
    c->set_error("unsupported FFT length (2^a 3^b 5^c from the supported list, up to 256; blocks: n_l / 2)");
    return ST_EINVAL;
  }
  const int bi = solve_bi(S.L3, blocked ? 1 : 0);
  const int groups_i = (S.L1 + bi - 1) / bi;
  const long nwg = (long)groups_i * S.L2;
  if (nparts) *nparts = (int)nwg;
  if (io[0].part_out && nwg > part_cap) {
    c->set_error("grid too large for the PCG partial buffers");
    return ST_EINVAL;
  }
  hipLaunchKernelGGL(k, dim3((unsigned)(nwg * nb)), dim3(FFT_THREADS), 0, c->stream, S);
  PBR_HIP(c, hipGetLastError());
  return ST_OK;
}

}  // namespace

namespace {

// The passes of the preconditioner of one layout with the tables T: three for
// a block with a plane pass (T then holds the permuted mode phases), else five.
int precond_passes(pbr_ctx* c, const FftTables& T, int block, double shift, const cplx* r,
                   cplx* z, bool may_tune) {
  const bool blocked = block >= 0;
  const long N = c->layout_nodes(block);
  if (blocked && plane_pass(c)) {
    PlaneIO f{r, z, &T, PcgHook()}, v{z, z, &T, PcgHook()};
    SolveIO s{block, z, nullptr, nullptr, &T};
    s.perm = true;
    PBR_TRY(run_plane(c, 1, -1, 0, &f, 1.0, 0, nullptr));
    PBR_TRY(run_solve(c, true, 1, &s, shift, 0, nullptr, may_tune));
    PBR_TRY(run_plane(c, 1, +1, 0, &v, 1.0 / (double)N, 0, nullptr));
    return ST_OK;
  }
  LineIO a{r, z, nullptr, PcgHook()}, b{z, z, nullptr, PcgHook()};
  SolveIO s{block, z, nullptr, nullptr, &T};
  LineIO a0 = a, b0 = b, b1 = b;
  a0.twist = T.twist[0];
  b0.twist = T.twist[1];
  b1.twist = T.twist[0];
  PBR_TRY(run_lines(c, T, blocked, 1, 0, -1, 0, &a0, 1.0, 0, nullptr));
  PBR_TRY(run_lines(c, T, blocked, 1, 1, -1, 0, &b0, 1.0, 0, nullptr));
  PBR_TRY(run_solve(c, blocked, 1, &s, shift, 0, nullptr));
  PBR_TRY(run_lines(c, T, blocked, 1, 1, +1, 0, &b0, 1.0, 0, nullptr));
  PBR_TRY(run_lines(c, T, blocked, 1, 0, +1, 0, &b1, 1.0 / (double)N, 0, nullptr));
  return ST_OK;
}

// Tables of pbr_precond_noalloc, for callers that cannot allocate: the roots,
// twist and mode phases of the three axes (each at most SCRATCH_L entries),
// rewritten by every call.  Each device holds its own copy; its address is
// looked up once per device (scratch_init) and kernels are handed that address.
constexpr int SCRATCH_L = 256;
// [axis][roots, twist, post][SCRATCH_L], then the permuted phases of the 3 axes
constexpr int SCRATCH_CPLX = 12 * SCRATCH_L;
static __device__ __align__(256) cplx scratch[SCRATCH_CPLX];

constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
cplx* g_scratch_ptr[SCRATCH_DEVICES] = {};

}  // namespace

int scratch_init(pbr_ctx* c) {
  if (c->device < 0 || c->device >= SCRATCH_DEVICES) {
    c->set_error("device index beyond the no-allocation scratch table");
    return ST_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[c->device]) {
    void* ptr = nullptr;
    PBR_HIP(c, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) {
      c->set_error("hipGetSymbolAddress returned a null address for the scratch tables");
      return ST_EDEVICE;
    }
    g_scratch_ptr[c->device] = (cplx*)ptr;
  }
  c->scratch = g_scratch_ptr[c->device];
  return ST_OK;
}

int launch_precond(pbr_ctx* c, const double kappa[3], int block, double shift, const cplx* r,
                   cplx* z) {
  const bool blocked = block >= 0;
  PBR_TRY(ensure_tables(c, 0, blocked, kappa));
  return precond_passes(c, c->tables(0, blocked), block, shift, r, z, true);
}

int launch_precond_noalloc(pbr_ctx* c, const double kappa[3], int block, double shift,
                           const cplx* r, cplx* z) {
  const bool blocked = block >= 0;
  const int Lt[3] = {blocked ? c->n1 / 2 : c->n1, blocked ? c->n2 / 2 : c->n2,
                     blocked ? c->n3 / 2 : c->n3};
  const int nf[3] = {c->n1, c->n2, c->n3};
  for (int l = 0; l < 3; ++l)
    if (nf[l] > SCRATCH_L) {
      c->set_error("pbr_precond_noalloc: grid size " + std::to_string(nf[l]) +
                   " beyond the fixed scratch tables (n_l <= 256)");
      return ST_EINVAL;
    }
  if (!c->scratch) {
    c->set_error("pbr_precond_noalloc: scratch tables not set up for this context");
    return ST_ESTATE;
  }
  FftTables T;
  for (int l = 0; l < 3; ++l) {
    const double phi = 2.0 * M_PI * kappa[l];
    T.kappa[l] = kappa[l];
    T.L[l] = Lt[l];
    T.roots[l] = c->scratch + (3 * l + 0) * SCRATCH_L;
    T.twist[l] = c->scratch + (3 * l + 1) * SCRATCH_L;
    T.post[l] = c->scratch + (3 * l + 2) * SCRATCH_L;
    hipLaunchKernelGGL(table_kernel, dim3(ceil_div(Lt[l], 256)), dim3(256), 0, c->stream, Lt[l],
                       0.0, 1, T.roots[l]);
    hipLaunchKernelGGL(table_kernel, dim3(ceil_div(Lt[l], 256)), dim3(256), 0, c->stream, Lt[l],
                       phi, 0, T.twist[l]);
    hipLaunchKernelGGL(table_kernel, dim3(ceil_div(nf[l], 256)), dim3(256), 0, c->stream, nf[l],
                       phi, 2, T.post[l]);
    if (blocked && plane_pass(c)) {
      T.postp[l] = c->scratch + (9 + l) * SCRATCH_L;
      hipLaunchKernelGGL(perm_phase_kernel, dim3(ceil_div(Lt[l], 256)), dim3(256), 0, c->stream,
                         Lt[l], nf[l], phi, T.postp[l]);
    }
  }
  PBR_HIP(c, hipGetLastError());
  return precond_passes(c, T, block, shift, r, z, false);
}

int launch_pcg_precond_batch(pbr_ctx* c, int nb, const PcgStep* P, double shift) {
  if (nb < 1 || nb > PBR_MAX_BATCH) {
    c->set_error("batch of 1 to PBR_MAX_BATCH layouts expected");
    return ST_EINVAL;
  }
  const bool blocked = P[0].block >= 0;
  for (int t = 0; t < nb; ++t) PBR_TRY(ensure_tables(c, P[t].slot, blocked, P[t].kappa));
  const bool planar = blocked && plane_pass(c);
  const FftTables& T0 = c->tables(P[0].slot, blocked);
  const long N = c->layout_nodes(P[0].block);
  const long cap = P[0].part_cap;
  LineIO io1[PBR_MAX_BATCH], io2[PBR_MAX_BATCH], io4[PBR_MAX_BATCH], io5[PBR_MAX_BATCH];
  SolveIO sio[PBR_MAX_BATCH];
  int n_rr = 0, n_rz = 0;
  for (int t = 0; t < nb; ++t) {
    const FftTables& T = c->tables(P[t].slot, blocked);
    PcgHook h;
    h.st = P[t].st;
    h.init = P[t].init;
    h.tol2 = P[t].tol2;
    h.inv_n = 1.0 / (double)N;
    // pass 1: update (or initialise) x and r, |r|^2 partials, forward lines of r
    PcgHook h1 = h;
    h1.x = P[t].x;
    h1.r = P[t].r;
    h1.p = P[t].p;
    h1.q = P[t].q;
    h1.b = P[t].b;
    h1.red_in = P[t].part_pq;
    h1.red_n = P[t].n_pq;
    h1.part_out = P[t].part_rr;
    io1[t] = LineIO{nullptr, P[t].z, T.twist[0], h1};
    io2[t] = LineIO{P[t].z, P[t].z, T.twist[1], h};
    io2[t].h.role = 1;  // first work-group finishes |r|^2 and the convergence test
    io2[t].h.red_in = P[t].part_rr;
    io4[t] = LineIO{P[t].z, P[t].z, T.twist[1], h};
    io4[t].h.role = 2;  // first work-group finishes (r, z) and beta
    io4[t].h.red_in = P[t].part_rz;
    io5[t] = LineIO{P[t].z, P[t].pout, T.twist[0], h};  // p = z + beta p, x += alpha p
    io5[t].h.x = P[t].x;
    sio[t] = SolveIO{P[t].block, P[t].z, P[t].st, P[t].part_rz, &T};
  }
  if (planar) {
    // three passes: plane (r update, forward i' and y2), mode solve (finishes
    // |r|^2 and the test, third axis, fold, solves, (r, z) partials), plane
    // (finishes (r, z) and beta, inverse y2 and i', p and x updates)
    PlaneIO pa[PBR_MAX_BATCH], pc[PBR_MAX_BATCH];
    for (int t = 0; t < nb; ++t) {
      const FftTables& T = c->tables(P[t].slot, blocked);
      pa[t] = PlaneIO{nullptr, P[t].z, &T, io1[t].h};
      pc[t] = PlaneIO{P[t].z, P[t].pout, &T, io5[t].h};
      pc[t].h.red_in = P[t].part_rz;
      sio[t].perm = true;
      sio[t].rr_in = P[t].part_rr;
      sio[t].init = P[t].init;
    }
    PBR_TRY(run_plane(c, nb, -1, 1, pa, 1.0, cap, &n_rr));
    for (int t = 0; t < nb; ++t) sio[t].rr_n = n_rr;
    PBR_TRY(run_solve(c, blocked, nb, sio, shift, cap, &n_rz));
    for (int t = 0; t < nb; ++t) pc[t].h.red_n = n_rz;
    PBR_TRY(run_plane(c, nb, +1, 2, pc, 1.0 / (double)N, cap, nullptr));
    return ST_OK;
  }
  PBR_TRY(run_lines(c, T0, blocked, nb, 0, -1, 1, io1, 1.0, cap, &n_rr));
  for (int t = 0; t < nb; ++t) io2[t].h.red_n = n_rr;
  PBR_TRY(run_lines(c, T0, blocked, nb, 1, -1, 0, io2, 1.0, cap, nullptr));
  PBR_TRY(run_solve(c, blocked, nb, sio, shift, cap, &n_rz));
  for (int t = 0; t < nb; ++t) io4[t].h.red_n = n_rz;
  PBR_TRY(run_lines(c, T0, blocked, nb, 1, +1, 0, io4, 1.0, cap, nullptr));
  PBR_TRY(run_lines(c, T0, blocked, nb, 0, +1, 2, io5, 1.0 / (double)N, cap, nullptr));
  return ST_OK;
}

// Loads this file's kernels onto the current device (see preload_kernels).
int preload_fft(pbr_ctx* c) {
  hipFuncAttributes a;
  PBR_HIP(c, hipFuncGetAttributes(&a, reinterpret_cast<const void*>(table_kernel)));
  return ST_OK;
}
