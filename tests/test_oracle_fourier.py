"""Pins for the Fourier bases and the preconditioner oracle (Sec. 5, Appendix B).

* X_l unitary, diagonalises K_l with eigenvalues exp(i(phi+2 pi p)/n) (App. B.1);
* T unitary and diagonalises H_1, H_2, H_3 (App. B.2);
* F_sigma^H F_sigma = I and T_sigma^H T_sigma = I (Eqs. 5.4-5.5); columns of
  T_sigma lie in V_sigma (they are eigenvectors of both parity operators with the
  block's signs) and the four T_sigma together span C^n;
* the half-period shifts of Sec. 5.2 act as the parity multipliers;
* preconditioner: numpy.fft implementation equals the literal dense T_xi one;
  for homogeneous material with C_ref = C it is exactly (A + delta M)^-1, full
  and per block (Sec. 5.3: constant C is diagonal by mode).
"""

import numpy as np
import pytest

from oracle import blocks as Bk, discretization as D, fourier as F
from synth import complex_gaussian, pack_c21, random_spd_field
from synth.materials import random_spd_stiffness

KAPPA = (0.15, 0.05, 0.10)
FCC = 0.5 * np.array([[0, 1, 1], [1, 0, 1], [1, 1, 0]], dtype=float)


@pytest.mark.parametrize("n,phi", [(1, 0.3), (4, 1.1), (6, -2.0)])
def test_X_diagonalises_K(n, phi):
    X = F.bloch_dft_1d(n, phi)
    K = D.bloch_shift_1d(n, phi).toarray()
    assert np.allclose(X.conj().T @ X, np.eye(n), atol=1e-14)
    lam = np.exp(1j * (phi + 2 * np.pi * np.arange(n)) / n)
    assert np.allclose(X.conj().T @ K @ X, np.diag(lam), atol=1e-13)


def test_T_diagonalises_H():
    dims = (4, 2, 6)
    T = F.full_basis(dims, KAPPA)
    assert np.allclose(T.conj().T @ T, np.eye(48), atol=1e-13)
    for H in D.coordinate_shifts(dims, KAPPA):
        Md = T.conj().T @ H.toarray() @ T
        assert np.abs(Md - np.diag(np.diag(Md))).max() < 1e-13


@pytest.mark.parametrize("dims", [(2, 2, 2), (4, 2, 6), (4, 4, 4)])
def test_block_basis_orthonormal_and_in_block(dims):
    n = int(np.prod(dims))
    g12, g13 = Bk.parity_signs(dims)
    Tall = []
    for b in range(4):
        Fs = F.folding_matrix(dims, b)
        assert np.allclose(Fs.conj().T @ Fs, np.eye(n // 4), atol=1e-14)
        Ts = F.block_basis(dims, KAPPA, b)
        assert np.allclose(Ts.conj().T @ Ts, np.eye(n // 4), atol=1e-13)
        s12, s13 = Bk.block_sigma(b)
        assert np.allclose(g12[:, None] * Ts, s12 * Ts, atol=1e-13)
        assert np.allclose(g13[:, None] * Ts, s13 * Ts, atol=1e-13)
        Tall.append(Ts)
    Tcat = np.concatenate(Tall, axis=1)
    assert np.allclose(Tcat.conj().T @ Tcat, np.eye(n), atol=1e-13)


def test_half_period_shift_is_parity_multiplier():
    dims = (4, 6, 2)
    T = F.full_basis(dims, KAPPA)
    g12, g13 = Bk.parity_signs(dims)
    for m in [(0, 0, 0), (1, 2, 1), (3, 5, 0)]:
        col = T[:, F.mode_index(m, dims)]
        o = F.orbit(m, dims)
        assert np.allclose(g12 * col, T[:, F.mode_index(o[1], dims)], atol=1e-13)
        assert np.allclose(g13 * col, T[:, F.mode_index(o[2], dims)], atol=1e-13)


def test_representatives_one_per_orbit():
    dims = (4, 6, 2)
    seen = {}
    for m in F.representatives(dims):
        for mm in F.orbit(m, dims):
            seen[mm] = seen.get(mm, 0) + 1
    assert len(seen) == 48 and all(v == 1 for v in seen.values())


@pytest.mark.parametrize("block", [-1, 0, 1, 2, 3])
@pytest.mark.parametrize("A_lat", [None, "fcc"])
def test_precond_fft_matches_dense(block, A_lat):
    Al = FCC if A_lat == "fcc" else None
    dims = (4, 2, 6)
    C21, rho = random_spd_field(dims, seed=3)
    Cref, rref = F.reference_material(C21, rho)
    n = 48 if block < 0 else 12
    r = complex_gaussian(3 * n, seed=17)
    z1 = F.precond_dense(r, dims, KAPPA, block, Cref, rref, 1.7, Al)
    z2 = F.precond_fft(r, dims, KAPPA, block, Cref, rref, 1.7, Al)
    assert np.linalg.norm(z1 - z2) <= 1e-13 * np.linalg.norm(z1)


@pytest.mark.parametrize("kappa", [(0.15, 0.05, 0.10), (0.0, 0.0, 0.0)])
@pytest.mark.parametrize("A_lat", [None, "fcc"])
def test_precond_exact_for_homogeneous(kappa, A_lat):
    Al = FCC if A_lat == "fcc" else None
    dims = (4, 4, 6)
    n = 96
    C = random_spd_stiffness(np.random.default_rng(1))
    C21 = np.tile(pack_c21(C), (n, 1))
    rho = np.full(n, 1.9)
    delta = 2.3
    A = D.assemble_A(dims, kappa, C21, Al)
    M = D.assemble_M(rho)
    x = complex_gaussian(3 * n, seed=4)
    b = A @ x + delta * (M @ x)
    z = F.precond_fft(b, dims, kappa, -1, C, 1.9, delta, Al)
    assert np.linalg.norm(z - x) <= 1e-12 * np.linalg.norm(x)
    for blk in range(4):
        xb = Bk.gather(x, dims, blk)
        Ab = Bk.block_operator(A, dims, blk)
        Mb = Bk.block_operator(M, dims, blk)
        zb = F.precond_fft(Ab @ xb + delta * (Mb @ xb), dims, kappa, blk, C, 1.9, delta, Al)
        assert np.linalg.norm(zb - xb) <= 1e-12 * np.linalg.norm(xb)


def test_precond_hermitian_positive():
    dims = (4, 2, 2)
    C21, rho = random_spd_field(dims, seed=5)
    Cref, rref = F.reference_material(C21, rho)
    n = 16
    P = np.stack([F.precond_fft(e, dims, KAPPA, -1, Cref, rref, 0.9)
                  for e in np.eye(3 * n)], axis=1)
    assert np.abs(P - P.conj().T).max() < 1e-13 * np.abs(P).max()
    assert np.linalg.eigvalsh(P).min() > 0
