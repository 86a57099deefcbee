"""Direct solution of the shift-invert system (Sec. 6.1, Eq. 6.2).

(A_h(k) + delta M_h) x = b, solved by sparse LU (scipy SuperLU).  The GPU solves
the same system with preconditioned CG; this is the plain definition of its
answer.  For a block, the system is (A_sigma + delta M_sigma) y = b_sigma.

Also: shift-invert eigenvalues with scipy's ARPACK wrapper, used as the mid-size
eigenvalue reference (n = 16..32) where dense eigh is too large.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .blocks import block_operator
from .discretization import assemble_A, assemble_M


def shifted_operator(dims, kappa, C21, rho, delta, block=-1, A_lat=None):
    A = assemble_A(dims, kappa, C21, A_lat)
    M = assemble_M(rho)
    if block >= 0:
        A = block_operator(A, dims, block)
        M = block_operator(M, dims, block)
    return (A + delta * M).tocsc(), M


def shifted_solve(dims, kappa, C21, rho, delta, b, block=-1, A_lat=None):
    K, _ = shifted_operator(dims, kappa, C21, rho, delta, block, A_lat)
    return spla.spsolve(K, np.asarray(b, dtype=np.complex128))


def shift_invert_lowest(dims, kappa, C21, rho, nev, sigma, block=-1, A_lat=None,
                        tol=1e-13):
    """nev eigenvalues of (A, M) nearest sigma (ARPACK shift-invert, SuperLU)."""
    A = assemble_A(dims, kappa, C21, A_lat)
    M = assemble_M(rho)
    if block >= 0:
        A = block_operator(A, dims, block)
        M = block_operator(M, dims, block)
    vals = spla.eigsh(A.tocsc(), k=nev, M=M.tocsc(), sigma=sigma, which="LM",
                      tol=tol, return_eigenvectors=False)
    return np.sort(vals.real)
