"""Literal Kronecker assembly of the rotated staggered operator (Sec. 3).

Every matrix is built exactly as the paper writes it, as a scipy.sparse matrix
in complex128:

* K_l: one-dimensional Bloch shift, ones on the superdiagonal and e^{i phi_l}
  in the bottom-left corner (Sec. 3.1, Eq. 3.4);
* H_1 = I (x) I (x) K_1, H_2 = I (x) K_2 (x) I, H_3 = K_3 (x) I (x) I
  (Eq. 3.5), so the node index is i + n1*(j + n2*k);
* S_d1 = H3 H2 H1, S_d2 = H3^-1 H2 H1, S_d3 = H3 H2^-1 H1,
  S_d4 = H3^-1 H2^-1 H1 (Sec. 3.3, Eq. 3.9);
* D_d = (S_d - I)/h_d with h_d = sqrt(h1^2+h2^2+h3^2) (Eq. 3.10);
* D~_1..3 from the four diagonal differences (Eq. 3.11);
* Dhat_s = -i D~_s (Eq. 3.12) and D_m = sum_s (A_lat^-1)_{sm} Dhat_s (Eq. 3.13);
* B_h (Eq. 3.14), C_h nodewise 6x6, M_h = I_3 (x) diag(rho), and
  A_h = B_h C_h B_h^H (Eq. 3.15).

Readings of points the paper leaves implicit: the grid spacing in reduced
coordinates is h_s = 1/n_s (the reconstructed derivatives approximate d/dr_s on
r in [0,1)^3); H_l^-1 is taken as H_l^H (K_l is unitary); the mass matrix is
I_3 (x) diag(rho) ("nodewise local multiplication", Theorem 4.1).

Parity pins (tests/test_oracle_*): A_h Hermitian PSD; agreement with the
independent index-formula build; homogeneous closed form; continuum
Christoffel limit; Theorem 4.1 commutation; Gamma null space of dimension 12.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# Upper-triangle pairs of the per-node 21-value Voigt stiffness, row by row.
UPPER21 = [(a, b) for a in range(6) for b in range(a, 6)]


def as_dims(dims):
    if isinstance(dims, (int, np.integer)):
        return (int(dims),) * 3
    return tuple(int(d) for d in dims)


def phases(kappa):
    """phi_l = 2*pi*kappa_l (Sec. 3.1, Eq. 3.3)."""
    return 2.0 * np.pi * np.asarray(kappa, dtype=np.float64)


def spacings(dims):
    """h_s = 1/n_s and h_d = sqrt(h1^2 + h2^2 + h3^2)."""
    h = np.array([1.0 / d for d in as_dims(dims)])
    return h, float(np.sqrt(np.sum(h * h)))


def bloch_shift_1d(n: int, phi: float) -> sp.csr_matrix:
    """K_l (Eq. 3.4): forward shift, phase e^{i phi} when the index wraps."""
    rows, cols, vals = [], [], []
    for r in range(n - 1):
        rows.append(r)
        cols.append(r + 1)
        vals.append(1.0 + 0j)
    rows.append(n - 1)
    cols.append(0)
    vals.append(np.exp(1j * phi))
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n), dtype=np.complex128)


def coordinate_shifts(dims, kappa):
    """(H_1, H_2, H_3) of Eq. 3.5."""
    n1, n2, n3 = as_dims(dims)
    p = phases(kappa)
    K1, K2, K3 = (bloch_shift_1d(n1, p[0]), bloch_shift_1d(n2, p[1]),
                  bloch_shift_1d(n3, p[2]))
    I1, I2, I3 = (sp.identity(n1, dtype=np.complex128, format="csr"),
                  sp.identity(n2, dtype=np.complex128, format="csr"),
                  sp.identity(n3, dtype=np.complex128, format="csr"))
    H1 = sp.kron(I3, sp.kron(I2, K1), format="csr")
    H2 = sp.kron(I3, sp.kron(K2, I1), format="csr")
    H3 = sp.kron(K3, sp.kron(I2, I1), format="csr")
    return H1, H2, H3


def _inv_unitary(H):
    return H.conj().T.tocsr()


def diagonal_shifts(dims, kappa):
    """(S_d1, S_d2, S_d3, S_d4) of Eq. 3.9."""
    H1, H2, H3 = coordinate_shifts(dims, kappa)
    H2i, H3i = _inv_unitary(H2), _inv_unitary(H3)
    S1 = (H3 @ H2 @ H1).tocsr()
    S2 = (H3i @ H2 @ H1).tocsr()
    S3 = (H3 @ H2i @ H1).tocsr()
    S4 = (H3i @ H2i @ H1).tocsr()
    return S1, S2, S3, S4


def diagonal_differences(dims, kappa):
    """D_d = (S_d - I)/h_d (Eq. 3.10)."""
    n = int(np.prod(as_dims(dims)))
    _, hd = spacings(dims)
    I = sp.identity(n, dtype=np.complex128, format="csr")
    return tuple(((S - I) / hd).tocsr() for S in diagonal_shifts(dims, kappa))


def reconstructed_derivatives(dims, kappa):
    """D~_1, D~_2, D~_3 of Eq. 3.11 (coefficients c_s = h_d/(4 h_s), Eq. 3.8)."""
    h, hd = spacings(dims)
    D1, D2, D3, D4 = diagonal_differences(dims, kappa)
    Dt1 = (hd / (4 * h[0])) * (D1 + D2 + D3 + D4)
    Dt2 = (hd / (4 * h[1])) * (D1 + D2 - D3 - D4)
    Dt3 = (hd / (4 * h[2])) * (D1 - D2 + D3 - D4)
    return Dt1.tocsr(), Dt2.tocsr(), Dt3.tocsr()


def cartesian_derivatives(dims, kappa, A_lat=None):
    """D_m = sum_s (A_lat^-1)_{sm} (-i D~_s) (Eqs. 3.12-3.13)."""
    Dt = reconstructed_derivatives(dims, kappa)
    Dhat = [(-1j) * D for D in Dt]
    Ainv = np.eye(3) if A_lat is None else np.linalg.inv(np.asarray(A_lat, dtype=np.float64))
    out = []
    for m in range(3):
        Dm = Ainv[0, m] * Dhat[0] + Ainv[1, m] * Dhat[1] + Ainv[2, m] * Dhat[2]
        out.append(sp.csr_matrix(Dm))
    return tuple(out)


def assemble_B(dims, kappa, A_lat=None) -> sp.csr_matrix:
    """B_h(k), 3n x 6n (Eq. 3.14)."""
    D1, D2, D3 = cartesian_derivatives(dims, kappa, A_lat)
    return sp.bmat([[D1, None, None, None, D3, D2],
                    [None, D2, None, D3, None, D1],
                    [None, None, D3, D2, D1, None]], format="csr")


def unpack_c21(C21) -> np.ndarray:
    """(n, 21) upper triangles -> (n, 6, 6) symmetric Voigt matrices."""
    C21 = np.asarray(C21, dtype=np.float64)
    C = np.zeros(C21.shape[:-1] + (6, 6))
    for t, (a, b) in enumerate(UPPER21):
        C[..., a, b] = C21[..., t]
        C[..., b, a] = C21[..., t]
    return C


def assemble_C(C21) -> sp.csr_matrix:
    """C_h, 6n x 6n: entry ((a,x),(b,x)) = C_ab(x), nodewise local."""
    C = unpack_c21(C21)
    blocks = [[sp.diags(C[:, a, b].astype(np.complex128)) for b in range(6)]
              for a in range(6)]
    return sp.bmat(blocks, format="csr")


def assemble_M(rho) -> sp.csr_matrix:
    """M_h = I_3 (x) diag(rho)."""
    d = sp.diags(np.asarray(rho, dtype=np.complex128))
    return sp.block_diag([d, d, d], format="csr")


def assemble_A(dims, kappa, C21, A_lat=None) -> sp.csr_matrix:
    """A_h(k) = B_h C_h B_h^H (Eq. 3.15)."""
    B = assemble_B(dims, kappa, A_lat)
    return (B @ assemble_C(C21) @ B.conj().T).tocsr()


def shift_max_entry(C21) -> float:
    """C_max = max |C_pq| over all nodes and entries (Eq. 7.7, read per node)."""
    return float(np.max(np.abs(np.asarray(C21))))


def default_shift(C21) -> float:
    """delta = 0.30 * C_max (Eq. 7.7)."""
    return 0.30 * shift_max_entry(C21)
