/*
 * pbr_host.h -- host-side building blocks of libpbr (the outer eigensolver's
 * dense steps and the material's palette form), exported so they can be used
 * and checked without a GPU.
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

/* Palette form of the nodewise material (Eq. 3.15; the form the operator
 * kernels read when it exists, see pbr_set_material): the distinct rows
 * (C21[x][0..20], rho[x]) of the n nodes, compared bit for bit and numbered in
 * order of first appearance, written to rows (22 doubles each, capacity 256
 * rows), and each node's row number to idx[x].  C21 (n x 21), rho (n) in the
 * layout of pbr_set_material; all pointers host memory owned by the caller.
 * Returns the number of rows (1..256), 0 when the material has more than 256
 * distinct rows (rows and idx then hold partial results), -1 on bad arguments. */
int pbr_host_palette(long n, const double *C21, const double *rho, double *rows,
                     unsigned char *idx);

#ifdef __cplusplus
}
#endif

#endif /* PBR_HOST_H */
