/*
 * pbr_host.h -- host-side building blocks of libpbr's outer eigensolver, exported
 * so they can be used and checked without a GPU.
 */
#ifndef PBR_HOST_H
#define PBR_HOST_H

#ifdef __cplusplus
extern "C" {
#endif

/* Eigen-decomposition of a small dense Hermitian matrix, used for the
 * Rayleigh-Ritz step of the shift-invert Krylov iteration (Sec. 6.1).
 * A: m x m complex128, column-major, interleaved (re, im); only its Hermitian
 * part (A + A^H)/2 is used.  w: m eigenvalues, ascending.  V: NULL or m x m
 * complex128 column-major unit eigenvectors (column c belongs to w[c]).  All
 * pointers are host memory owned by the caller.  Returns 0, or -1 on bad
 * arguments. */
int pbr_host_heev(int m, const double *A, double *w, double *V);

/* Certification rule of the block merge (Sec. 6.1: the full spectrum is the
 * sorted union of the four block spectra).  vals[b] holds the nev_b[b] lowest
 * eigenvalues of block b, ascending (host arrays).  Writes the nev lowest values
 * of the union into merged (ascending) and returns a bit mask of the blocks that
 * must compute more eigenvalues: block b is flagged when its largest computed
 * value is strictly below the merged nev-th value, because an eigenvalue of b
 * not yet computed could then still belong to the lowest nev.  Returns -1 on bad
 * arguments or when the union holds fewer than nev values. */
int pbr_host_merge(int nev, const int nev_b[4], const double *const vals[4],
                   double *merged);

#ifdef __cplusplus
}
#endif

#endif /* PBR_HOST_H */
