"""Seeded material fields on the unit-cube grid.

The workload is a two-phase cell: a cubic matrix phase with a centred spherical
inclusion whose 6x6 Voigt stiffness is a random symmetric positive definite
matrix.  Fields are returned per node in the natural node order
``x = i + n1*(j + n2*k)`` (i fastest), as

* ``C21``: float64 array ``(n, 21)`` holding the upper triangle of each node's
  Voigt stiffness row by row: C11..C16, C22..C26, C33..C36, C44..C46, C55, C56,
  C66 (Voigt order [11,22,33,23,13,12], engineering shear);
* ``rho``: float64 array ``(n,)`` of densities.

Node (i, j, k) sits at the reduced position (i/n1, j/n2, k/n3); it belongs to the
inclusion iff its Euclidean distance to (1/2, 1/2, 1/2) is strictly below the
radius.  No sub-cell smoothing is applied.
"""

from __future__ import annotations

import numpy as np

# Upper-triangle index pairs of a 6x6 matrix, row by row.
_UPPER = [(a, b) for a in range(6) for b in range(a, 6)]


def cubic_stiffness(c11: float, c12: float, c44: float) -> np.ndarray:
    """Voigt matrix of a cubic crystal aligned with the axes (engineering shear)."""
    C = np.zeros((6, 6))
    C[:3, :3] = c12
    for a in range(3):
        C[a, a] = c11
        C[3 + a, 3 + a] = c44
    return C


def haar_orthogonal(rng: np.random.Generator, n: int = 6) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of a standard normal matrix with the
    columns of Q multiplied by sign(diag R)."""
    G = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    return Q * np.sign(np.diag(R))


def random_spd_stiffness(rng: np.random.Generator, lo: float = 5.0,
                         hi: float = 50.0) -> np.ndarray:
    """C = Q diag(e) Q^T with Q Haar-random and e log-uniform on [lo, hi]."""
    Q = haar_orthogonal(rng, 6)
    e = np.exp(rng.uniform(np.log(lo), np.log(hi), size=6))
    C = (Q * e) @ Q.T
    return 0.5 * (C + C.T)


def pack_c21(C: np.ndarray) -> np.ndarray:
    """Pack a symmetric 6x6 matrix (or a stack ``(..., 6, 6)``) into 21 values."""
    C = np.asarray(C, dtype=np.float64)
    return np.stack([C[..., a, b] for (a, b) in _UPPER], axis=-1)


def _node_positions(dims):
    n1, n2, n3 = dims
    k, j, i = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    return (i.ravel() / n1, j.ravel() / n2, k.ravel() / n3)


def two_phase_cell(dims, radius: float = 0.35, seed: int = 0,
                   matrix=(1.0, 0.4, 0.3), rho_matrix: float = 1.0,
                   rho_inclusion: float = 4.0, rng: np.random.Generator | None = None):
    """Two-phase unit cube: cubic matrix (C11, C12, C44) + random SPD sphere.

    Returns ``(C21, rho, C_inclusion)``.  ``rng`` overrides ``seed`` so several
    cells can be drawn from one generator.
    """
    if isinstance(dims, int):
        dims = (dims, dims, dims)
    if rng is None:
        rng = np.random.default_rng(seed)
    C_inc = random_spd_stiffness(rng)
    C_mat = cubic_stiffness(*matrix)
    x1, x2, x3 = _node_positions(dims)
    r2 = (x1 - 0.5) ** 2 + (x2 - 0.5) ** 2 + (x3 - 0.5) ** 2
    inside = r2 < radius * radius
    n = dims[0] * dims[1] * dims[2]
    C21 = np.empty((n, 21))
    C21[:] = pack_c21(C_mat)
    C21[inside] = pack_c21(C_inc)
    rho = np.full(n, float(rho_matrix))
    rho[inside] = float(rho_inclusion)
    return C21, rho, C_inc


def homogeneous_cell(dims, C: np.ndarray, rho: float):
    """Spatially constant material (used for closed-form checks)."""
    if isinstance(dims, int):
        dims = (dims, dims, dims)
    n = dims[0] * dims[1] * dims[2]
    C21 = np.empty((n, 21))
    C21[:] = pack_c21(C)
    return C21, np.full(n, float(rho))


def random_spd_field(dims, seed: int = 0, lo: float = 0.5, hi: float = 5.0):
    """Independent random SPD stiffness and density at every node (stress tests
    of nodewise-local material; no geometric structure)."""
    if isinstance(dims, int):
        dims = (dims, dims, dims)
    rng = np.random.default_rng(seed)
    n = dims[0] * dims[1] * dims[2]
    G = rng.standard_normal((n, 6, 6))
    C = G @ np.swapaxes(G, 1, 2) / 6.0 + lo * np.eye(6)
    C = 0.5 * (C + np.swapaxes(C, 1, 2))
    rho = rng.uniform(lo, hi, size=n)
    return pack_c21(C), rho


def batch_cells(count: int = 8, seed: int = 0, sizes=(64, 96, 128),
                rlo: float = 0.2, rhi: float = 0.4):
    """Uneven batch of two-phase cells: for each cell draw n from ``sizes`` and the
    radius from U[rlo, rhi], then its inclusion stiffness, all from one generator.

    Returns a list of ``(n, radius, C21, rho)``.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice(np.asarray(sizes)))
        r = float(rng.uniform(rlo, rhi))
        C21, rho, _ = two_phase_cell((n, n, n), radius=r, rng=rng)
        out.append((n, r, C21, rho))
    return out
