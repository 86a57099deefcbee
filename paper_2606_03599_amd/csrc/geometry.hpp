// Grid geometry shared by the stencil, layout and FFT kernels.
//
// Two layouts are used on the device.
//   natural: the full n1 x n2 x n3 grid, index i + n1*(j + n2*k).
//   block b: the n/4 nodes of parity class b = 2a + c (a = (i+j)%2, c = (j+k)%2),
//            index t = i + n1*(y2 + m2*y3) with m2 = n2/2, m3 = n3/2; the node is
//            (i, 2*y2 + o2(i), 2*y3 + o3(i)), o2 = (a+i)%2, o3 = (a+c+i)%2.
//
// Both layouts are handled as an L1 x L2 x L3 box with coordinates (i, j, k)
// (for a block j = y2, k = y3).  The four body-diagonal steps are
// d1=(1,1,1), d2=(1,1,-1), d3=(1,-1,1), d4=(1,-1,-1) (Sec. 3.3, Eq. 3.9).  A step
// x -> x + d (forward, dir=+1) or x - d (backward, dir=-1) in the natural layout
// moves by (±1, ±s2, ±s3).  In a block layout it changes i by ±1 and (y2, y3) by
// (s + w(i))/2 forward or (w(i) - s)/2 backward with w2(i) = 2*o2(i)-1,
// w3(i) = 2*o3(i)-1 -- the class of the node is preserved because every step
// has d1+d2 and d1+d3 even (proof of Theorem 4.1).  Leaving the box on axis l
// wraps around and multiplies by e^{+i phi_l} (upward) or e^{-i phi_l}
// (downward): the Bloch extension v(x + n_l e_l) = e^{i phi_l} v(x) of Eq. 3.2
// that the shift K_l encodes (Eq. 3.4).  For a block, leaving the half-grid box
// happens exactly when the original coordinate leaves [0, n_l).
#pragma once

#include "common.hpp"

struct Geo {
  int L1, L2, L3;       // box dims of the layout
  int n1, n2, n3;       // full grid dims (symbols use them)
  int blocked;          // 0 natural, 1 parity block
  int a, c;             // class bits of the block
  cplx ph[3];           // e^{i phi_l}
  double cf[3][5];      // D'_m = sum_d cf[m][d] S_d, d = 0 identity, 1..4 diagonals
};

// s2, s3 of diagonal step d in 1..4
__host__ __device__ inline int step_s2(int d) { return (d <= 2) ? 1 : -1; }
__host__ __device__ inline int step_s3(int d) { return (d & 1) ? 1 : -1; }

__host__ __device__ inline void wrap_axis(int& x, int L, cplx ph, cplx& fac) {
  if (x >= L) {
    x -= L;
    fac = cmul(fac, ph);
  } else if (x < 0) {
    x += L;
    fac = cmul(fac, cconj(ph));
  }
}

// Neighbour of (i,j,k) along diagonal d (1..4) in direction dir (+1 / -1).
// Returns the layout index and the Bloch phase of the wrap.
__host__ __device__ inline long neighbor(const Geo& g, int i, int j, int k, int d, int dir,
                                         cplx& fac) {
  const int s2 = step_s2(d), s3 = step_s3(d);
  int ii, jj, kk;
  if (!g.blocked) {
    ii = i + dir;
    jj = j + dir * s2;
    kk = k + dir * s3;
  } else {
    const int w2 = 2 * ((g.a + i) & 1) - 1;
    const int w3 = 2 * ((g.a + g.c + i) & 1) - 1;
    if (dir > 0) {
      ii = i + 1;
      jj = j + (s2 + w2) / 2;
      kk = k + (s3 + w3) / 2;
    } else {
      ii = i - 1;
      jj = j + (w2 - s2) / 2;
      kk = k + (w3 - s3) / 2;
    }
  }
  fac = mk(1.0, 0.0);
  wrap_axis(ii, g.L1, g.ph[0], fac);
  wrap_axis(jj, g.L2, g.ph[1], fac);
  wrap_axis(kk, g.L3, g.ph[2], fac);
  return (long)ii + (long)g.L1 * ((long)jj + (long)g.L2 * kk);
}

// Host: fill the layout part of a Geo.
inline void geo_layout(Geo& g, int n1, int n2, int n3, int block) {
  g.n1 = n1;
  g.n2 = n2;
  g.n3 = n3;
  if (block < 0) {
    g.L1 = n1; g.L2 = n2; g.L3 = n3;
    g.blocked = 0; g.a = 0; g.c = 0;
  } else {
    g.L1 = n1; g.L2 = n2 / 2; g.L3 = n3 / 2;
    g.blocked = 1; g.a = block >> 1; g.c = block & 1;
  }
}
