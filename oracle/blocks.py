"""Parity classes and the block node order (Sec. 4).

Parity labels (Sec. 4, Eqs. 4.2-4.5): g12(x) = (-1)^{i+j}, g13(x) = (-1)^{i+k}.
Their common eigenspaces V_sigma (Eq. 4.11) are spanned by vectors supported on
one class of nodes.  Blocks are numbered b = 2a + c with a = (i+j) mod 2 and
c = (j+k) mod 2; the paper's signs are sigma12 = (-1)^a, sigma13 = (-1)^(a+c)
(because i+k = (i+j) + (j+k) mod 2).

Block node order (a written definition shared with the C interface): block
position t = i + n1*(y2 + (n2/2)*y3) for i in [0,n1), y2 in [0,n2/2),
y3 in [0,n3/2), which is the node (i, 2*y2 + o2, 2*y3 + o3) with
o2 = (a + i) mod 2 and o3 = (a + c + i) mod 2.  A block vector is
component-major [v1 | v2 | v3], each of length n/4.

Q_sigma (Corollary 4.2, Eq. 4.14) is the 3n x 3n/4 selection matrix whose
column (alpha, t) is the unit vector of component alpha at that node, so
Q_sigma^* Q_sigma = I and A_sigma = Q^* A Q, M_sigma = Q^* M Q.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .discretization import as_dims


def node_class(dims) -> np.ndarray:
    """Block id b = 2*((i+j)%2) + (j+k)%2 of every node, natural order."""
    n1, n2, n3 = as_dims(dims)
    k, j, i = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    a = (i + j) % 2
    c = (j + k) % 2
    return (2 * a + c).ravel()


def parity_signs(dims):
    """(g12, g13) as float arrays over nodes (Eq. 4.2)."""
    n1, n2, n3 = as_dims(dims)
    k, j, i = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    return ((-1.0) ** (i + j)).ravel(), ((-1.0) ** (i + k)).ravel()


def block_sigma(b: int):
    """(sigma12, sigma13) of block b."""
    a, c = divmod(int(b), 2)
    return (-1) ** a, (-1) ** ((a + c) % 2)


def block_nodes(dims, b: int) -> np.ndarray:
    """Natural node indices of block b, in block order (i fastest, then y2, y3)."""
    n1, n2, n3 = as_dims(dims)
    if n1 % 2 or n2 % 2 or n3 % 2:
        raise ValueError("parity blocks need even n1, n2, n3 (Theorem 4.1)")
    a, c = divmod(int(b), 2)
    out = np.empty(n1 * (n2 // 2) * (n3 // 2), dtype=np.int64)
    t = 0
    for y3 in range(n3 // 2):
        for y2 in range(n2 // 2):
            for i in range(n1):
                o2 = (a + i) % 2
                o3 = (a + c + i) % 2
                j = 2 * y2 + o2
                k = 2 * y3 + o3
                out[t] = i + n1 * (j + n2 * k)
                t += 1
    return out


def selection_Q(dims, b: int) -> sp.csr_matrix:
    """Q_sigma (3n x 3n/4), component-major on both sides."""
    dims = as_dims(dims)
    n = dims[0] * dims[1] * dims[2]
    nodes = block_nodes(dims, b)
    nb = nodes.size
    rows = np.concatenate([nodes + a * n for a in range(3)])
    cols = np.arange(3 * nb)
    return sp.csr_matrix((np.ones(3 * nb, dtype=np.complex128), (rows, cols)),
                         shape=(3 * n, 3 * nb))


def gather(vfull, dims, b):
    """Q_sigma^* v: block vector (3n/4,) from a full vector (3n,)."""
    dims = as_dims(dims)
    n = dims[0] * dims[1] * dims[2]
    nodes = block_nodes(dims, b)
    V = np.asarray(vfull).reshape(3, n)
    return V[:, nodes].reshape(-1)


def scatter(vblk, dims, b, out=None):
    """Q_sigma y: writes the block vector into a (zero or given) full vector."""
    dims = as_dims(dims)
    n = dims[0] * dims[1] * dims[2]
    nodes = block_nodes(dims, b)
    full = np.zeros(3 * n, dtype=np.complex128) if out is None else out
    F = full.reshape(3, n)
    F[:, nodes] = np.asarray(vblk).reshape(3, -1)
    return full


def block_operator(A, dims, b):
    """A_sigma = Q^* A Q (Eq. 4.14) as a sparse matrix."""
    Q = selection_Q(dims, b)
    return (Q.conj().T @ A @ Q).tocsr()


def block_material(C21, rho, dims, b):
    """Per-node material of block b in block order."""
    nodes = block_nodes(dims, b)
    return np.asarray(C21)[nodes], np.asarray(rho)[nodes]
