"""Dense reference spectra of (A_h(k), M_h), full space and per parity block.

* Full space: eigenvalues of the pencil A v = lambda M v (Eq. 3.15), lambda = omega^2,
  with scipy.linalg.eigh (LAPACK zhegv*).
* Block sigma: the pencil (A_sigma, M_sigma) of Corollary 4.2; the merged and
  sorted block spectra form the full spectrum (Sec. 6.1).
* Gamma point (kappa integer): the null space N_Gamma is spanned by chi_mu e_alpha
  with the scalar modes chi_0 = 1, chi_12 = (-1)^{i+j}, chi_13 = (-1)^{i+k},
  chi_23 = (-1)^{j+k} (Sec. 6.2, Eq. 6.4, Appendix C): 12 vectors in the full space
  and 3 per block.  We report eigenvalues on the M-orthogonal complement of that
  space, i.e. the spectrum with the zero-derivative modes removed, which is what
  deflation with d0 > 0 (Eqs. 6.5-6.6) leaves unchanged.

Pins: block union == full spectrum, exactly 12 (3 per block) zero eigenvalues at
Gamma and none elsewhere (tests/test_oracle_spectrum.py).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .blocks import block_nodes, block_operator
from .discretization import as_dims, assemble_A, assemble_M


def is_gamma(kappa) -> bool:
    k = np.asarray(kappa, dtype=np.float64)
    return bool(np.all(k == np.round(k)))


def dense(A):
    return A.toarray() if hasattr(A, "toarray") else np.asarray(A)


def pencil_eigvals(A, M):
    """All eigenvalues of A v = lambda M v, ascending."""
    return sla.eigh(dense(A), dense(M), eigvals_only=True)


def pencil_eig(A, M):
    return sla.eigh(dense(A), dense(M))


def gamma_scalar_modes(dims):
    """chi_0, chi_12, chi_13, chi_23 on the grid (natural node order)."""
    n1, n2, n3 = as_dims(dims)
    k, j, i = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    return [np.ones(n1 * n2 * n3),
            ((-1.0) ** (i + j)).ravel(),
            ((-1.0) ** (i + k)).ravel(),
            ((-1.0) ** (j + k)).ravel()]


def gamma_null_basis(dims, rho):
    """M-orthonormal basis Q0 (3n x 12) of N_Gamma (Q0^H M Q0 = I)."""
    dims = as_dims(dims)
    n = dims[0] * dims[1] * dims[2]
    chis = gamma_scalar_modes(dims)
    cols = []
    for a in range(3):
        for chi in chis:
            v = np.zeros(3 * n, dtype=np.complex128)
            v[a * n:(a + 1) * n] = chi
            cols.append(v)
    Z = np.stack(cols, axis=1)
    rho3 = np.concatenate([rho, rho, rho])
    G = Z.conj().T @ (rho3[:, None] * Z)
    L = np.linalg.cholesky(G)
    return Z @ np.linalg.inv(L).conj().T


def block_gamma_null_basis(dims, rho, b):
    """M_sigma-orthonormal null basis (3n/4 x 3) of block b: 1_sigma e_alpha/sqrt(sum rho)."""
    nodes = block_nodes(dims, b)
    rb = np.asarray(rho)[nodes]
    nb = nodes.size
    Q = np.zeros((3 * nb, 3), dtype=np.complex128)
    for a in range(3):
        Q[a * nb:(a + 1) * nb, a] = 1.0 / np.sqrt(rb.sum())
    return Q


def complement_eigvals(A, M, Q0):
    """Eigenvalues of the pencil on the M-orthogonal complement of range(Q0)."""
    Ad, Md = dense(A), dense(M)
    # basis of {v : Q0^H M v = 0}
    W = sla.null_space((Q0.conj().T @ Md))
    return sla.eigh(W.conj().T @ Ad @ W, W.conj().T @ Md @ W, eigvals_only=True)


def full_spectrum(dims, kappa, C21, rho, A_lat=None, exclude_gamma_null=True):
    """Full-space eigenvalues (ascending); at Gamma the 12 null modes removed."""
    A = assemble_A(dims, kappa, C21, A_lat)
    M = assemble_M(rho)
    if exclude_gamma_null and is_gamma(kappa):
        return complement_eigvals(A, M, gamma_null_basis(dims, rho))
    return pencil_eigvals(A, M)


def block_spectrum(dims, kappa, C21, rho, b, A_lat=None, exclude_gamma_null=True):
    """Eigenvalues of block b (ascending); at Gamma its 3 null modes removed."""
    A = assemble_A(dims, kappa, C21, A_lat)
    M = assemble_M(rho)
    Ab = block_operator(A, dims, b)
    Mb = block_operator(M, dims, b)
    if exclude_gamma_null and is_gamma(kappa):
        return complement_eigvals(Ab, Mb, block_gamma_null_basis(dims, rho, b))
    return pencil_eigvals(Ab, Mb)


def merged_block_spectrum(dims, kappa, C21, rho, A_lat=None, exclude_gamma_null=True):
    """Sorted union of the four block spectra (Sec. 6.1)."""
    parts = [block_spectrum(dims, kappa, C21, rho, b, A_lat, exclude_gamma_null)
             for b in range(4)]
    return np.sort(np.concatenate(parts))


def lowest(vals, nev):
    return np.sort(np.asarray(vals))[:nev]
