"""Pins for parity blocking, the Gamma null space and the merged spectrum (Sec. 4, 6).

* Theorem 4.1: A and M commute with the lifted parity operators on even grids,
  cross-class entries of A are structurally zero, and the commutation fails on an
  odd grid (the theorem's hypothesis matters);
* Corollary 4.2 / Sec. 6.1: the sorted union of the four block spectra is the full
  spectrum (random per-node SPD material, several k, non-orthogonal lattice);
* Appendix C: at Gamma the four checkerboards are annihilated by every D_d,
  dim ker B^H = 12, the full pencil has exactly 12 zero eigenvalues and each block
  exactly 3; away from Gamma there are none;
* the block node order is a partition of the grid consistent with the classes.
"""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import blocks as Bk, discretization as D, eigen as E
from synth import random_spd_field, two_phase_cell

FCC = 0.5 * np.array([[0, 1, 1], [1, 0, 1], [1, 1, 0]], dtype=float)


def _lifted(dims):
    g12, g13 = Bk.parity_signs(dims)
    G12 = sp.diags(np.concatenate([g12] * 3))
    G13 = sp.diags(np.concatenate([g13] * 3))
    return G12, G13


@pytest.mark.parametrize("dims", [(2, 2, 2), (4, 2, 6), (4, 4, 4)])
def test_theorem_4_1_commutation(dims):
    C21, rho = random_spd_field(dims, seed=2)
    A = D.assemble_A(dims, (0.21, -0.4, 0.33), C21, FCC)
    M = D.assemble_M(rho)
    for G in _lifted(dims):
        assert abs(A @ G - G @ A).max() <= 1e-13 * abs(A).max()
        assert abs(M @ G - G @ M).max() == 0.0


def test_cross_class_entries_exactly_zero():
    dims = (4, 4, 4)
    C21, _ = random_spd_field(dims, seed=3)
    A = D.assemble_A(dims, (0.1, 0.2, 0.3), C21).tocoo()
    cls = np.concatenate([Bk.node_class(dims)] * 3)
    big = np.abs(A.data) > 0
    assert np.all(cls[A.row[big]] == cls[A.col[big]])


def test_odd_grid_breaks_commutation():
    dims = (3, 3, 3)
    C21, _ = random_spd_field(dims, seed=4)
    A = D.assemble_A(dims, (0.1, 0.2, 0.3), C21)
    G12, _ = _lifted(dims)
    assert abs(A @ G12 - G12 @ A).max() > 1e-3 * abs(A).max()


def test_block_order_partitions_grid():
    dims = (4, 6, 2)
    cls = Bk.node_class(dims)
    seen = np.zeros(48, dtype=int)
    for b in range(4):
        nodes = Bk.block_nodes(dims, b)
        assert nodes.size == 12
        assert np.all(cls[nodes] == b)
        seen[nodes] += 1
        # block position t = i + n1*(y2 + (n2/2) y3) with y2 = j//2, y3 = k//2
        i = nodes % 4
        j = (nodes // 4) % 6
        k = nodes // 24
        t = i + 4 * (j // 2 + 3 * (k // 2))
        assert np.array_equal(t, np.arange(12))
    assert np.all(seen == 1)


def test_block_labels_match_paper_signs():
    dims = (4, 4, 4)
    g12, g13 = Bk.parity_signs(dims)
    for b in range(4):
        s12, s13 = Bk.block_sigma(b)
        nodes = Bk.block_nodes(dims, b)
        assert np.all(g12[nodes] == s12) and np.all(g13[nodes] == s13)


@pytest.mark.parametrize("kappa", [(0.15, 0.05, 0.10), (0.5, 0.5, 0.0), (0.0, 0.0, 0.0),
                                   (0.37, -0.21, 0.5)])
@pytest.mark.parametrize("A_lat", [None, "fcc"])
def test_block_union_equals_full(kappa, A_lat):
    Al = FCC if A_lat == "fcc" else None
    dims = (4, 4, 2)
    C21, rho = random_spd_field(dims, seed=8)
    full = E.full_spectrum(dims, kappa, C21, rho, Al, exclude_gamma_null=False)
    merged = E.merged_block_spectrum(dims, kappa, C21, rho, Al, exclude_gamma_null=False)
    assert np.abs(full - merged).max() <= 1e-12 * np.abs(full).max()


def test_block_union_two_phase_n8():
    dims = (8, 8, 8)
    C21, rho, _ = two_phase_cell(dims, radius=0.35, seed=0)
    kap = (0.15, 0.05, 0.10)
    full = E.full_spectrum(dims, kap, C21, rho)
    merged = E.merged_block_spectrum(dims, kap, C21, rho)
    assert np.abs(full[:40] - merged[:40]).max() <= 1e-12 * full[39]


def test_gamma_checkerboards_annihilated():
    dims = (4, 2, 6)
    Dd = D.diagonal_differences(dims, (0, 0, 0))
    for chi in E.gamma_scalar_modes(dims):
        for Dl in Dd:
            assert np.abs(Dl @ chi).max() < 1e-12
    # a generic vector is not annihilated
    assert np.abs(Dd[0] @ np.arange(48.0)).max() > 1.0


def test_gamma_null_dimension():
    dims = (4, 4, 2)
    n = 32
    BH = D.assemble_B(dims, (0, 0, 0)).conj().T.toarray()
    sv = np.linalg.svd(BH, compute_uv=False)
    assert np.sum(sv < 1e-10 * sv.max()) == 12
    C21, rho = random_spd_field(dims, seed=1)
    A = D.assemble_A(dims, (0, 0, 0), C21)
    M = D.assemble_M(rho)
    ev = E.pencil_eigvals(A, M)
    assert np.sum(np.abs(ev) < 1e-9 * ev.max()) == 12
    for b in range(4):
        evb = E.pencil_eigvals(Bk.block_operator(A, dims, b), Bk.block_operator(M, dims, b))
        assert np.sum(np.abs(evb) < 1e-9 * evb.max()) == 3
    evk = E.pencil_eigvals(D.assemble_A(dims, (0.1, 0, 0), C21), M)
    assert evk.min() > 1e-6 * evk.max()
    # the null basis is M-orthonormal and annihilated by A
    Q0 = E.gamma_null_basis(dims, rho)
    assert np.allclose(Q0.conj().T @ (M @ Q0), np.eye(12), atol=1e-13)
    assert np.abs(A @ Q0).max() < 1e-10 * abs(A).max()
    assert Q0.shape == (3 * n, 12)


def test_complement_removes_exactly_null_modes():
    dims = (4, 4, 4)
    C21, rho = random_spd_field(dims, seed=6)
    A = D.assemble_A(dims, (0, 0, 0), C21)
    M = D.assemble_M(rho)
    allv = E.pencil_eigvals(A, M)
    comp = E.full_spectrum(dims, (0, 0, 0), C21, rho)
    assert comp.size == allv.size - 12
    assert np.abs(np.sort(allv)[12:] - comp).max() <= 1e-10 * allv.max()
    merged = E.merged_block_spectrum(dims, (0, 0, 0), C21, rho)
    assert np.abs(merged - comp).max() <= 1e-10 * allv.max()
