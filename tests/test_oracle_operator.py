"""Pins for the oracle's operator (Sec. 3): properties fixed by the paper and by
mathematics, not by re-typing the formulas.

* the two constructions (Kronecker product of Eq. 3.4-3.15 and the Bloch-extension
  index formula) agree element by element, including n_l = 2 where the +1 and -1
  neighbours coincide, odd grids and a non-orthogonal lattice;
* K_l is unitary, K_l^{n} = e^{i phi} I and has eigenvalues exp(i(phi+2 pi p)/n)
  (Appendix B.1); the H_l commute (Sec. 3.1);
* A_h is Hermitian positive semidefinite (it is B C B^H with C SPD);
* kappa -> -kappa conjugates A (real C); kappa -> kappa + e_l leaves A unchanged;
* homogeneous material: spectrum = union of modewise 3x3 symbol problems
  (Sec. 5.3, Appendix B) -- an independent derivation through the Fourier basis;
* low-frequency limit equals the continuum Christoffel equation (Remark 3.1),
  which fixes h_s = 1/n_s, the reconstruction coefficients, the Voigt order,
  engineering shear and the lattice transform of Eq. 2.8/3.13.
"""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import continuum, discretization as D, fourier as F, pointwise as P
from synth import complex_gaussian, cubic_stiffness, pack_c21, random_spd_field
from synth.materials import random_spd_stiffness

KAPPA = (0.15, 0.05, 0.10)
FCC = 0.5 * np.array([[0, 1, 1], [1, 0, 1], [1, 1, 0]], dtype=float)  # columns a1,a2,a3 (Eq. 7.3, a0=1)


@pytest.mark.parametrize("n,phi", [(1, 0.7), (2, -1.3), (5, 2.2), (8, 0.0)])
def test_K_unitary_power_and_eigs(n, phi):
    K = D.bloch_shift_1d(n, phi).toarray()
    assert np.allclose(K @ K.conj().T, np.eye(n), atol=1e-15)
    assert np.allclose(np.linalg.matrix_power(K, n), np.exp(1j * phi) * np.eye(n), atol=1e-13)
    lam = np.exp(1j * (phi + 2 * np.pi * np.arange(n)) / n)
    ev = np.linalg.eigvals(K)
    for l in lam:
        assert np.min(np.abs(ev - l)) < 1e-12


def test_H_commute():
    H1, H2, H3 = D.coordinate_shifts((3, 4, 2), (0.2, -0.3, 0.45))
    for X, Y in ((H1, H2), (H1, H3), (H2, H3)):
        assert abs(X @ Y - Y @ X).max() < 1e-15


def _rand_case(dims, seed):
    C21, rho = random_spd_field(dims, seed=seed)
    n = int(np.prod(dims))
    v = complex_gaussian(3 * n, seed=seed + 100)
    return C21, rho, v


@pytest.mark.parametrize("dims", [(2, 2, 2), (4, 4, 4), (3, 3, 3), (2, 4, 6), (1, 2, 3), (5, 2, 4)])
@pytest.mark.parametrize("A_lat", [None, "fcc"])
def test_two_constructions_agree(dims, A_lat):
    Al = FCC if A_lat == "fcc" else None
    C21, rho, v = _rand_case(dims, 7)
    kap = (0.31, -0.12, 0.27)
    A = D.assemble_A(dims, kap, C21, Al)
    M = D.assemble_M(rho)
    y_kron = A @ v + 0.7 * (M @ v)
    y_pt = P.apply_A(v, dims, kap, C21, rho, s=0.7, A_lat=Al)
    assert np.linalg.norm(y_kron - y_pt) <= 1e-13 * np.linalg.norm(y_kron)


def test_single_node_evaluation_matches():
    dims = (4, 6, 2)
    C21, rho, v = _rand_case(dims, 3)
    y = P.apply_A(v, dims, KAPPA, C21, rho, s=1.5).reshape(3, -1)
    pts = [(0, 0, 0), (3, 5, 1), (1, 2, 0), (2, 0, 1)]
    ya = P.apply_A_at(pts, v, dims, KAPPA, C21, rho, s=1.5)
    for t, x in enumerate(pts):
        idx = x[0] + dims[0] * (x[1] + dims[1] * x[2])
        assert np.allclose(ya[t], y[:, idx], rtol=0, atol=1e-12 * np.abs(y).max())


@pytest.mark.parametrize("dims", [(2, 2, 2), (4, 4, 4), (3, 5, 2)])
def test_hermitian_psd(dims):
    C21, rho, _ = _rand_case(dims, 11)
    A = D.assemble_A(dims, KAPPA, C21).toarray()
    scale = np.abs(A).max()
    assert np.abs(A - A.conj().T).max() <= 1e-14 * scale
    assert np.linalg.eigvalsh(A).min() >= -1e-12 * scale


def test_kappa_symmetries():
    dims = (4, 4, 2)
    C21, _, _ = _rand_case(dims, 5)
    A = D.assemble_A(dims, KAPPA, C21)
    Am = D.assemble_A(dims, tuple(-k for k in KAPPA), C21)
    assert abs(Am - A.conj()).max() <= 1e-13 * abs(A).max()
    for l in range(3):
        k2 = list(KAPPA)
        k2[l] += 1.0
        assert abs(D.assemble_A(dims, k2, C21) - A).max() <= 1e-12 * abs(A).max()


def test_identity_cancels_in_D2_D3():
    """D~_2 and D~_3 have no diagonal term: the identity drops out (Eq. 3.11)."""
    Dt = D.reconstructed_derivatives((4, 4, 4), KAPPA)
    assert np.all(Dt[1].diagonal() == 0) and np.all(Dt[2].diagonal() == 0)
    assert np.allclose(Dt[0].diagonal(), -4.0)  # -1/h1 with h1 = 1/4


@pytest.mark.parametrize("A_lat", [None, "fcc"])
def test_homogeneous_closed_form(A_lat):
    Al = FCC if A_lat == "fcc" else None
    dims = (4, 2, 6)
    rng = np.random.default_rng(4)
    C = random_spd_stiffness(rng)
    n = int(np.prod(dims))
    C21 = np.tile(pack_c21(C), (n, 1))
    rho = np.full(n, 2.5)
    ev = np.linalg.eigvalsh(D.assemble_A(dims, KAPPA, C21, Al).toarray()) / 2.5
    cf = F.homogeneous_closed_form(dims, KAPPA, C, 2.5, Al)
    assert np.abs(np.sort(ev) - cf).max() <= 1e-13 * cf.max()


@pytest.mark.parametrize("A_lat", [None, "fcc"])
@pytest.mark.parametrize("kappa", [KAPPA, (0.0, 0.0, 0.0), (0.5, 0.25, -0.3)])
def test_homogeneous_spectrum_vectorised(A_lat, kappa):
    """The batched closed form (used at n = 128) equals the dense spectrum of the
    assembled operator, independently of the looped form it restates."""
    Al = FCC if A_lat == "fcc" else None
    dims = (4, 2, 6)
    C = random_spd_stiffness(np.random.default_rng(7))
    n = int(np.prod(dims))
    C21 = np.tile(pack_c21(C), (n, 1))
    ev = np.sort(np.linalg.eigvalsh(D.assemble_A(dims, kappa, C21, Al).toarray())) / 1.7
    hs = F.homogeneous_spectrum(dims, kappa, C, 1.7, Al)
    assert hs.shape == (3 * n,)
    assert np.abs(ev - hs).max() <= 1e-13 * hs.max()
    cf = F.homogeneous_closed_form((6, 4, 8), kappa, C, 1.7, Al)
    assert np.abs(F.homogeneous_spectrum((6, 4, 8), kappa, C, 1.7, Al) - cf).max() <= \
        1e-13 * cf.max()


def test_homogeneous_spectrum_orbit_multiplicity():
    """Every value of the homogeneous full spectrum on an even grid appears a
    multiple of four times: K(m) is the same on each orbit of Eq. 5.3."""
    C = random_spd_stiffness(np.random.default_rng(8))
    hs = F.homogeneous_spectrum((8, 8, 8), KAPPA, C, 1.0)
    assert np.abs(hs[0::4] - hs[3::4]).max() <= 1e-12 * hs.max()


@pytest.mark.parametrize("A_lat", [None, "fcc"])
def test_continuum_limit(A_lat):
    """Lowest three discrete eigenvalues -> Christoffel eigenvalues, error O(h^2)."""
    Al = np.eye(3) if A_lat is None else FCC
    rng = np.random.default_rng(9)
    C = random_spd_stiffness(rng)
    kap = np.array([0.011, -0.007, 0.004])
    q = 2 * np.pi * np.linalg.solve(Al.T, kap)     # physical wave vector, Eq. 3.1
    exact = continuum.christoffel_eigs(C, 1.3, q)
    errs = []
    for n in (32, 64, 128):
        theta = 2 * np.pi * kap / n                    # mode m = 0 of Eq. 5.2
        Bh = F.symbol_block(F.derivative_symbols(theta, (n, n, n), Al))
        disc = np.sort(np.linalg.eigvalsh(Bh @ C @ Bh.conj().T)) / 1.3
        errs.append(np.abs(disc - exact).max() / exact.max())
    assert errs[0] < 1e-3
    assert errs[1] < errs[0] / 3.0 and errs[2] < errs[1] / 3.0


def test_continuum_isotropic_speeds():
    """Isotropic: omega^2 = C44 |q|^2/rho (twice) and C11 |q|^2/rho (engineering shear)."""
    C = cubic_stiffness(1.0, 0.4, 0.3)
    n = 256
    kap = np.array([0.003, 0.002, -0.001])
    q2 = float(np.sum((2 * np.pi * kap) ** 2))
    Bh = F.symbol_block(F.derivative_symbols(2 * np.pi * kap / n, (n, n, n)))
    disc = np.sort(np.linalg.eigvalsh(Bh @ C @ Bh.conj().T))
    assert np.allclose(disc, [0.3 * q2, 0.3 * q2, 1.0 * q2], rtol=1e-5)


def test_symbols_diagonalize_operator():
    """T^H S_d T is diagonal with entries exp(i d.theta_m) (Eq. 4.1, Appendix B.2)."""
    dims = (4, 2, 4)
    T = F.full_basis(dims, KAPPA)
    S = D.diagonal_shifts(dims, KAPPA)
    modes = [(p, q, r) for r in range(dims[2]) for q in range(dims[1]) for p in range(dims[0])]
    for l, Sd in enumerate(S):
        Md = T.conj().T @ Sd.toarray() @ T
        want = np.array([np.exp(1j * F.STEPS[l] @ F.mode_angles(m, dims, KAPPA)) for m in modes])
        assert np.abs(Md - np.diag(want)).max() < 1e-13


def test_B_block_diagonal_in_fourier():
    """(I3 x T)^H B_h (I6 x T) = direct sum of Bhat(m) (Eq. 5.7, 5.11)."""
    dims = (2, 4, 2)
    n = 16
    T = F.full_basis(dims, KAPPA)
    B = D.assemble_B(dims, KAPPA, FCC).toarray()
    Bf = sp.block_diag([T] * 3).toarray().conj().T @ B @ sp.block_diag([T] * 6).toarray()
    modes = [(p, q, r) for r in range(2) for q in range(4) for p in range(2)]
    for t, m in enumerate(modes):
        Bh = F.symbol_block(F.derivative_symbols(F.mode_angles(m, dims, KAPPA), dims, FCC))
        sub = Bf[t::n, t::n]
        assert np.abs(sub - Bh).max() < 1e-12
    # everything outside the mode-diagonal positions vanishes
    mask = np.zeros_like(Bf, dtype=bool)
    for t in range(n):
        mask[t::n, t::n] = True
    assert np.abs(Bf[~mask]).max() < 1e-12
