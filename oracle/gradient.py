"""Derivatives of the Bloch eigenvalues with respect to the nodewise material.

TEST INFRASTRUCTURE ONLY (see the package header).

For the Hermitian pencil A(p) v = lambda M(p) v with M positive definite, an
eigenvector normalised by v^H M v = 1 and a simple eigenvalue lambda, first-order
perturbation gives the Hellmann-Feynman formula

    d lambda / d p = v^H (dA/dp - lambda dM/dp) v.

Here A = B_h C_h B_h^H (Eq. 3.15) with C_h nodewise and M_h = I_3 (x) diag(rho),
so with the strain field e = B_h^H v (six components per node, rows of B_h^H,
Eq. 3.14):

* the stored upper-triangle entry C21_q(x), q = (a, b), is both C_ab(x) and
  C_ba(x): d lambda / d C21_q(x) = 2 Re(conj(e_a(x)) e_b(x)) for a != b and
  |e_a(x)|^2 for a == b;
* d lambda / d rho(x) = -lambda sum_alpha |v_alpha(x)|^2.

For a parity block the eigenvector of (A_sigma, M_sigma) is scattered into the
full space (Q_sigma v); the formula is then the full-space one, and the
derivative vanishes off the block's nodes.  Inside a cluster of equal
eigenvalues single derivatives are not defined; the sum over an orthonormal
basis of the cluster is (the trace of the projected perturbation), which is what
cluster_gradient returns.

Pins (tests/test_oracle_gradient.py): central finite differences of the dense
eigenvalues, Euler's relations for the homogeneity of lambda (degree 1 in C,
degree -1 in rho), invariance of a cluster sum under a unitary change of basis.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .blocks import block_nodes
from .discretization import UPPER21, as_dims, assemble_A, assemble_B, assemble_M
from .eigen import block_gamma_null_basis, dense, gamma_null_basis, is_gamma


def eigenpairs(dims, kappa, C21, rho, block=-1, A_lat=None):
    """All eigenpairs of the full pencil (block = -1) or of block sigma, with the
    Gamma null modes removed at Gamma.  Returns (lambda ascending, V) with V's
    columns M-normalised full-space vectors (block vectors scattered)."""
    dims = as_dims(dims)
    n = dims[0] * dims[1] * dims[2]
    A = dense(assemble_A(dims, kappa, C21, A_lat))
    M = dense(assemble_M(rho))
    if block >= 0:
        nodes = block_nodes(dims, block)
        rows = np.concatenate([a * n + nodes for a in range(3)])
        Q = np.zeros((3 * n, rows.size))
        Q[rows, np.arange(rows.size)] = 1.0
    else:
        Q = np.eye(3 * n)
    Ab, Mb = Q.T @ A @ Q, Q.T @ M @ Q
    if is_gamma(kappa):
        Z = (block_gamma_null_basis(dims, rho, block) if block >= 0
             else gamma_null_basis(dims, rho))
        W = sla.null_space(Z.conj().T @ Mb)
    else:
        W = np.eye(Ab.shape[0])
    lam, Y = sla.eigh(W.conj().T @ Ab @ W, W.conj().T @ Mb @ W)
    return lam, Q @ (W @ Y)


def hf_gradient(dims, kappa, v, lam, A_lat=None):
    """d lambda / d C21 (n x 21) and d lambda / d rho (n,) for one M-normalised
    full-space eigenvector v of eigenvalue lam."""
    dims = as_dims(dims)
    n = dims[0] * dims[1] * dims[2]
    B = assemble_B(dims, kappa, A_lat)
    e = (B.conj().T @ v).reshape(6, n)
    gC = np.zeros((n, 21))
    for q, (a, b) in enumerate(UPPER21):
        if a == b:
            gC[:, q] = np.abs(e[a]) ** 2
        else:
            gC[:, q] = 2.0 * np.real(np.conj(e[a]) * e[b])
    V = np.asarray(v).reshape(3, n)
    grho = -lam * np.sum(np.abs(V) ** 2, axis=0)
    return gC, grho


def cluster_gradient(dims, kappa, V, lams, weights=None, A_lat=None):
    """Weighted sum of hf_gradient over the columns of V (e.g. an orthonormal
    basis of a cluster with equal weights)."""
    V = np.asarray(V)
    w = np.ones(V.shape[1]) if weights is None else np.asarray(weights, float)
    gC = 0.0
    gr = 0.0
    for i in range(V.shape[1]):
        c, r = hf_gradient(dims, kappa, V[:, i], lams[i], A_lat)
        gC = gC + w[i] * c
        gr = gr + w[i] * r
    return gC, gr
