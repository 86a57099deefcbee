// Palette form of the nodewise material C_h, rho (Eq. 3.15): the distinct
// (C21, rho) rows and each node's row, on the host (see pbr_host_palette).
#include <cstring>

#include "../../include/pbr_host.h"

// Rows are compared bit for bit and numbered in order of first appearance.
// Runs of equal rows are checked against the previous node's row first; other
// rows go through a small open-address hash table over the row's bits.
extern "C" int pbr_host_palette(long n, const double* C21, const double* rho, double* rows,
                                unsigned char* idx) {
  constexpr int MAXR = 256;
  constexpr int HS = 4 * MAXR;  // power of two
  if (n < 1 || !C21 || !rho || !rows || !idx) return -1;
  int slot_row[HS];
  for (int& v : slot_row) v = -1;
  int nrows = 0;
  int last = -1;
  double row[22];
  for (long x = 0; x < n; ++x) {
    std::memcpy(row, C21 + (size_t)x * 21, 21 * sizeof(double));
    row[21] = rho[x];
    if (last >= 0 && std::memcmp(row, rows + (size_t)last * 22, sizeof(row)) == 0) {
      idx[x] = (unsigned char)last;
      continue;
    }
    unsigned long long h = 0x9e3779b97f4a7c15ULL;
    for (int q = 0; q < 22; ++q) {
      unsigned long long b;
      std::memcpy(&b, &row[q], 8);
      h = (h ^ b) * 0xff51afd7ed558ccdULL;
      h ^= h >> 29;
    }
    int sl = (int)(h & (HS - 1));
    int found = -1;
    while (slot_row[sl] >= 0) {
      if (std::memcmp(row, rows + (size_t)slot_row[sl] * 22, sizeof(row)) == 0) {
        found = slot_row[sl];
        break;
      }
      sl = (sl + 1) & (HS - 1);
    }
    if (found < 0) {
      if (nrows == MAXR) return 0;
      std::memcpy(rows + (size_t)nrows * 22, row, sizeof(row));
      slot_row[sl] = nrows;
      found = nrows++;
    }
    idx[x] = (unsigned char)found;
    last = found;
  }
  return nrows;
}
