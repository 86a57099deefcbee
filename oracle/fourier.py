"""Bloch Fourier bases, derivative symbols and the FFT-diagonal preconditioner (Sec. 5).

* X_l: unitary eigenvector matrix of K_l with columns
  x_{l,p} = n_l^{-1/2} (1, lam, lam^2, ...), lam = exp(i(phi_l + 2 pi p)/n_l)
  (Appendix B.1); T = X_3 (x) X_2 (x) X_1 (Eq. 5.1); its columns are the Bloch
  DFT modes psi_pqr of Eq. 5.2.
* Orbits O(m) = {m, m+h12, m+h13, m+h23} (Eq. 5.3).  Representatives
  R = {(p, q, r): 0 <= q < n2/2, 0 <= r < n3/2} (one per orbit).
* Folding vectors f_m^(sigma) (Eq. 5.4), F_sigma, T_sigma = T F_sigma (Eq. 5.5).
* Symbols: s_d(m) = exp(i d.theta_m), theta_m = (alpha_p, beta_q, gamma_r);
  d_l = (s_dl - 1)/h_d; delta_1..3 (Eqs. 5.8-5.10); eta_j = -i delta_j and the
  3x6 block Bhat(m) (Eq. 5.11).  With a lattice matrix the Cartesian symbols are
  eta'_m = sum_s (A_lat^-1)_{sm} eta_s, mirroring Eq. 3.13.

Preconditioner (a reading: the paper states only that the Fourier/SVD variables
of Sec. 5.4 give the framework for the inner preconditioner, Sec. 6.1): for the
shifted operator A + delta*M use, mode by mode,

    K(m) = Bhat(m) C_ref Bhat(m)^H + delta * rho_ref * I_3,

with constant reference stiffness C_ref and density rho_ref, and apply
z = T_xi diag_m(K(m)^-1) T_xi^H r (per velocity component).  For homogeneous
material with C_ref = C and rho_ref = rho this is exactly (A + delta M)^-1
(Sec. 5.3: C is then diagonal by mode), which is how it is pinned.

Two implementations: ``precond_dense`` forms T and T_sigma explicitly (small n);
``precond_fft`` uses numpy.fft on the twisted field (pinned against the dense one).
"""

from __future__ import annotations

import numpy as np

from .blocks import block_nodes, block_sigma
from .discretization import as_dims, phases, spacings, unpack_c21

STEPS = np.array([(1, 1, 1), (1, 1, -1), (1, -1, 1), (1, -1, -1)], dtype=np.float64)


def bloch_dft_1d(n: int, phi: float) -> np.ndarray:
    """X_l (Appendix B.1)."""
    lam = np.exp(1j * (phi + 2 * np.pi * np.arange(n)) / n)
    powers = np.arange(n)[:, None]
    return lam[None, :] ** powers / np.sqrt(n)


def full_basis(dims, kappa) -> np.ndarray:
    """T = X_3 (x) X_2 (x) X_1 (dense n x n)."""
    n1, n2, n3 = as_dims(dims)
    p = phases(kappa)
    return np.kron(bloch_dft_1d(n3, p[2]), np.kron(bloch_dft_1d(n2, p[1]),
                                                   bloch_dft_1d(n1, p[0])))


def mode_index(m, dims):
    n1, n2, _ = as_dims(dims)
    return m[0] + n1 * (m[1] + n2 * m[2])


def orbit(m, dims):
    """O(m) of Eq. 5.3 (indices taken modulo n_l)."""
    n1, n2, n3 = as_dims(dims)
    h12 = (n1 // 2, n2 // 2, 0)
    h13 = (n1 // 2, 0, n3 // 2)
    h23 = ((h12[0] + h13[0]), h12[1] + h13[1], h12[2] + h13[2])
    out = []
    for h in ((0, 0, 0), h12, h13, h23):
        out.append(((m[0] + h[0]) % n1, (m[1] + h[1]) % n2, (m[2] + h[2]) % n3))
    return out


def representatives(dims):
    """R: one representative per orbit, ordered p fastest, then q, r."""
    n1, n2, n3 = as_dims(dims)
    return [(p, q, r) for r in range(n3 // 2) for q in range(n2 // 2) for p in range(n1)]


def folding_matrix(dims, b: int) -> np.ndarray:
    """F_sigma (n x n/4) of Eq. 5.4 for block b."""
    dims = as_dims(dims)
    n = dims[0] * dims[1] * dims[2]
    s12, s13 = block_sigma(b)
    coef = (1.0, s12, s13, s12 * s13)
    R = representatives(dims)
    F = np.zeros((n, len(R)), dtype=np.complex128)
    for col, m in enumerate(R):
        for c, mm in zip(coef, orbit(m, dims)):
            F[mode_index(mm, dims), col] += 0.5 * c
    return F


def block_basis(dims, kappa, b):
    """T_sigma = T F_sigma (Eq. 5.5)."""
    return full_basis(dims, kappa) @ folding_matrix(dims, b)


def mode_angles(m, dims, kappa):
    """theta_m = (alpha_p, beta_q, gamma_r)."""
    dims = as_dims(dims)
    ph = phases(kappa)
    return np.array([(ph[l] + 2 * np.pi * m[l]) / dims[l] for l in range(3)])


def derivative_symbols(theta, dims, A_lat=None):
    """Cartesian symbols eta'_1..3 of the derivative operators at angles theta."""
    h, hd = spacings(dims)
    s = np.exp(1j * (STEPS @ theta))          # shift symbols of S_d1..S_d4
    dl = (s - 1.0) / hd                       # symbols of D_d1..D_d4
    c = hd / (4 * h)                          # Eq. 3.8
    delta = np.array([c[0] * (dl[0] + dl[1] + dl[2] + dl[3]),
                      c[1] * (dl[0] + dl[1] - dl[2] - dl[3]),
                      c[2] * (dl[0] - dl[1] + dl[2] - dl[3])])
    eta = -1j * delta
    Ainv = np.eye(3) if A_lat is None else np.linalg.inv(np.asarray(A_lat, float))
    return Ainv.T @ eta


def symbol_block(eta) -> np.ndarray:
    """Bhat(m), 3x6 (Eq. 5.11)."""
    e1, e2, e3 = eta
    return np.array([[e1, 0, 0, 0, e3, e2],
                     [0, e2, 0, e3, 0, e1],
                     [0, 0, e3, e2, e1, 0]], dtype=np.complex128)


def mode_matrix(m, dims, kappa, C_ref, rho_ref, delta, A_lat=None):
    """K(m) = Bhat C_ref Bhat^H + delta rho_ref I_3."""
    Bh = symbol_block(derivative_symbols(mode_angles(m, dims, kappa), dims, A_lat))
    return Bh @ C_ref @ Bh.conj().T + delta * rho_ref * np.eye(3)


def reference_material(C21, rho):
    """Volume means: C_ref (6x6) and rho_ref (the default reference)."""
    return unpack_c21(np.mean(np.asarray(C21), axis=0)), float(np.mean(rho))


def homogeneous_closed_form(dims, kappa, C, rho, A_lat=None):
    """Spectrum of A v = lambda M v for constant C, rho: union over modes of
    eig(Bhat C Bhat^H)/rho (Sec. 5.3; Appendix B)."""
    n1, n2, n3 = as_dims(dims)
    vals = []
    for r in range(n3):
        for q in range(n2):
            for p in range(n1):
                Bh = symbol_block(derivative_symbols(mode_angles((p, q, r), dims, kappa),
                                                     dims, A_lat))
                vals.extend(np.linalg.eigvalsh(Bh @ C @ Bh.conj().T) / rho)
    return np.sort(np.array(vals))


def homogeneous_spectrum(dims, kappa, C, rho, A_lat=None):
    """The same union as homogeneous_closed_form, for large grids: the symbol
    matrices Bhat(m) C Bhat(m)^H of all modes at once (mode_matrices with a zero
    shift) and a batched Hermitian eigensolve (Sec. 5.3; Appendix B).  Pinned
    against the looped form on small grids."""
    K = mode_matrices(dims, kappa, C, 1.0, 0.0, A_lat)
    return np.sort(np.linalg.eigvalsh(K).ravel()) / rho


def precond_dense(r, dims, kappa, block, C_ref, rho_ref, delta, A_lat=None):
    """z = Q^H (I_3 (x) T_xi) diag K(m)^-1 (I_3 (x) T_xi)^H Q r, literally.

    block = -1: full space (r has 3n entries, T_xi = T, m over I).
    block = b:  r is a block vector (3n/4), T_xi = T_sigma, m over R.
    """
    dims = as_dims(dims)
    n = dims[0] * dims[1] * dims[2]
    if block < 0:
        Tx = full_basis(dims, kappa)
        modes = [(p, q, rr) for rr in range(dims[2]) for q in range(dims[1])
                 for p in range(dims[0])]
        rf = np.asarray(r, dtype=np.complex128).reshape(3, n)
    else:
        Tx = block_basis(dims, kappa, block)
        modes = representatives(dims)
        nodes = block_nodes(dims, block)
        rf = np.zeros((3, n), dtype=np.complex128)
        rf[:, nodes] = np.asarray(r, dtype=np.complex128).reshape(3, -1)
    coef = rf @ Tx.conj()                     # (3, modes): T_xi^H r per component
    zc = np.empty_like(coef)
    for t, m in enumerate(modes):
        K = mode_matrix(m, dims, kappa, C_ref, rho_ref, delta, A_lat)
        zc[:, t] = np.linalg.solve(K, coef[:, t])
    zf = zc @ Tx.T                            # T_xi zc per component
    if block < 0:
        return zf.reshape(-1)
    return zf[:, block_nodes(dims, block)].reshape(-1)


def _twist(dims, kappa, sign):
    n1, n2, n3 = as_dims(dims)
    ph = phases(kappa)
    k, j, i = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    return np.exp(sign * 1j * (i * ph[0] / n1 + j * ph[1] / n2 + k * ph[2] / n3))


def mode_matrices(dims, kappa, C_ref, rho_ref, delta, A_lat=None):
    """K(m) for all m in I, shaped (n3, n2, n1, 3, 3) (vectorised Eq. 5.8-5.11)."""
    n1, n2, n3 = as_dims(dims)
    h, hd = spacings(dims)
    ph = phases(kappa)
    R, Q, P = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    th = np.stack([(ph[0] + 2 * np.pi * P) / n1, (ph[1] + 2 * np.pi * Q) / n2,
                   (ph[2] + 2 * np.pi * R) / n3], axis=-1)
    s = np.exp(1j * np.einsum("...l,dl->...d", th, STEPS))
    dl = (s - 1.0) / hd
    c = hd / (4 * h)
    delta_s = np.stack([c[0] * (dl[..., 0] + dl[..., 1] + dl[..., 2] + dl[..., 3]),
                        c[1] * (dl[..., 0] + dl[..., 1] - dl[..., 2] - dl[..., 3]),
                        c[2] * (dl[..., 0] - dl[..., 1] + dl[..., 2] - dl[..., 3])], -1)
    eta = -1j * delta_s
    Ainv = np.eye(3) if A_lat is None else np.linalg.inv(np.asarray(A_lat, float))
    eta = np.einsum("sm,...s->...m", Ainv, eta)
    e1, e2, e3 = eta[..., 0], eta[..., 1], eta[..., 2]
    z = np.zeros_like(e1)
    Bh = np.stack([np.stack([e1, z, z, z, e3, e2], -1),
                   np.stack([z, e2, z, e3, z, e1], -1),
                   np.stack([z, z, e3, e2, e1, z], -1)], -2)
    K = Bh @ C_ref @ np.conj(np.swapaxes(Bh, -1, -2))
    return K + delta * rho_ref * np.eye(3)


def precond_fft(r, dims, kappa, block, C_ref, rho_ref, delta, A_lat=None):
    """Same operator as precond_dense, via numpy.fft on the twisted field.

    A block vector is zero-extended to the full grid; because K(m) is the same on
    all four members of an orbit (Sec. 5.3) the full-space operator maps V_sigma to
    itself and agrees there with the block operator (pinned against precond_dense).
    """
    dims = as_dims(dims)
    n1, n2, n3 = dims
    n = n1 * n2 * n3
    if block < 0:
        rf = np.asarray(r, dtype=np.complex128).reshape(3, n)
    else:
        nodes = block_nodes(dims, block)
        rf = np.zeros((3, n), dtype=np.complex128)
        rf[:, nodes] = np.asarray(r, dtype=np.complex128).reshape(3, -1)
    tw = _twist(dims, kappa, -1)
    coef = np.stack([np.fft.fftn(rf[a].reshape(n3, n2, n1) * tw, norm="ortho")
                     for a in range(3)], axis=-1)            # (n3, n2, n1, 3)
    K = mode_matrices(dims, kappa, C_ref, rho_ref, delta, A_lat)
    zc = np.linalg.solve(K, coef[..., None])[..., 0]
    untw = _twist(dims, kappa, +1)
    zf = np.stack([(np.fft.ifftn(zc[..., a], norm="ortho") * untw).ravel()
                   for a in range(3)])
    if block < 0:
        return zf.reshape(-1)
    return zf[:, block_nodes(dims, block)].reshape(-1)
