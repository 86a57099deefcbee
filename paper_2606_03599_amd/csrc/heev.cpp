// Small dense Hermitian eigensolver for the Rayleigh-Ritz step of the outer
// Krylov iteration: cyclic complex Jacobi rotations.  Each rotation first turns
// the pivot entry real with a diagonal phase, then applies the classical real
// symmetric Jacobi rotation (tan of the angle from (a_qq - a_pp)/(2|a_pq|)).
// Sizes here are the Krylov basis size (tens), so O(m^3) per sweep is cheap and
// the method's high relative accuracy is welcome.
#include <cmath>
#include <complex>
#include <vector>

#include "../../include/pbr_host.h"

typedef std::complex<double> zc;

extern "C" int pbr_host_heev(int m, const double* A_in, double* w, double* V_out) {
  if (m < 1 || !A_in || !w) return -1;
  std::vector<zc> A((size_t)m * m), V((size_t)m * m, zc(0, 0));
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) A[(size_t)j * m + i] = zc(A_in[2 * ((size_t)j * m + i)],
                                                          A_in[2 * ((size_t)j * m + i) + 1]);
  // Hermitian part
  for (int j = 0; j < m; ++j)
    for (int i = 0; i <= j; ++i) {
      const zc a = 0.5 * (A[(size_t)j * m + i] + std::conj(A[(size_t)i * m + j]));
      A[(size_t)j * m + i] = a;
      A[(size_t)i * m + j] = std::conj(a);
    }
  for (int i = 0; i < m; ++i) {
    A[(size_t)i * m + i] = zc(A[(size_t)i * m + i].real(), 0.0);
    V[(size_t)i * m + i] = 1.0;
  }
  auto at = [&](int i, int j) -> zc& { return A[(size_t)j * m + i]; };
  auto vt = [&](int i, int j) -> zc& { return V[(size_t)j * m + i]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) {
        if (i == j)
          diag += std::norm(at(i, j));
        else
          off += std::norm(at(i, j));
      }
    if (off <= 1e-32 * diag || off == 0.0) break;
    for (int p = 0; p < m - 1; ++p)
      for (int q = p + 1; q < m; ++q) {
        const zc apq = at(p, q);
        const double mag = std::abs(apq);
        if (mag == 0.0) continue;
        const double app = at(p, p).real(), aqq = at(q, q).real();
        if (mag < 1e-300) continue;
        const zc ph = apq / mag;  // e^{i theta}
        const double tau = (aqq - app) / (2.0 * mag);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double cs = 1.0 / std::sqrt(1.0 + t * t);
        const double sn = t * cs;
        // G = diag(1, conj(ph)) * [[c, s], [-s, c]]:
        // G = [[c, s], [-s conj(ph), c conj(ph)]]
        const zc g00 = cs, g01 = sn, g10 = -sn * std::conj(ph), g11 = cs * std::conj(ph);
        // A <- A G (columns p, q)
        for (int r = 0; r < m; ++r) {
          const zc arp = at(r, p), arq = at(r, q);
          at(r, p) = arp * g00 + arq * g10;
          at(r, q) = arp * g01 + arq * g11;
        }
        // A <- G^H A (rows p, q)
        for (int cc = 0; cc < m; ++cc) {
          const zc apc = at(p, cc), aqc = at(q, cc);
          at(p, cc) = std::conj(g00) * apc + std::conj(g10) * aqc;
          at(q, cc) = std::conj(g01) * apc + std::conj(g11) * aqc;
        }
        at(p, q) = 0.0;
        at(q, p) = 0.0;
        at(p, p) = zc(at(p, p).real(), 0.0);
        at(q, q) = zc(at(q, q).real(), 0.0);
        for (int r = 0; r < m; ++r) {
          const zc vrp = vt(r, p), vrq = vt(r, q);
          vt(r, p) = vrp * g00 + vrq * g10;
          vt(r, q) = vrp * g01 + vrq * g11;
        }
      }
  }
  // sort ascending
  std::vector<int> idx(m);
  for (int i = 0; i < m; ++i) idx[i] = i;
  for (int i = 0; i < m; ++i)
    for (int j = i + 1; j < m; ++j)
      if (at(idx[j], idx[j]).real() < at(idx[i], idx[i]).real()) std::swap(idx[i], idx[j]);
  for (int c = 0; c < m; ++c) {
    w[c] = at(idx[c], idx[c]).real();
    if (V_out)
      for (int r = 0; r < m; ++r) {
        V_out[2 * ((size_t)c * m + r)] = vt(r, idx[c]).real();
        V_out[2 * ((size_t)c * m + r) + 1] = vt(r, idx[c]).imag();
      }
  }
  return 0;
}
