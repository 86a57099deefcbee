"""Input generators: shapes, seeds, structure of the synthetic workloads."""

import numpy as np

from synth import (batch_cells, haar_orthogonal, pack_c21, random_spd_stiffness, sc_path,
                   split_intervals, two_phase_cell)


def test_haar_orthogonal():
    Q = haar_orthogonal(np.random.default_rng(0))
    assert np.allclose(Q @ Q.T, np.eye(6), atol=1e-14)


def test_inclusion_spd_in_range():
    C = random_spd_stiffness(np.random.default_rng(3))
    ev = np.linalg.eigvalsh(C)
    assert ev.min() >= 5 - 1e-12 and ev.max() <= 50 + 1e-12


def test_two_phase_cell_structure():
    C21, rho, C_inc = two_phase_cell((16, 16, 16), radius=0.35, seed=0)
    assert C21.shape == (4096, 21) and rho.shape == (4096,)
    inside = rho == 4.0
    frac = inside.mean()
    assert abs(frac - 4 / 3 * np.pi * 0.35 ** 3) < 0.03
    assert np.allclose(C21[inside], pack_c21(C_inc))
    # matrix entries: C11=1, C12=0.4, C44=0.3
    m = C21[~inside][0]
    assert m[0] == 1.0 and m[1] == 0.4 and m[15] == 0.3
    # deterministic in the seed
    C21b, _, _ = two_phase_cell((16, 16, 16), radius=0.35, seed=0)
    assert np.array_equal(C21, C21b)


def test_sc_path_split():
    assert split_intervals([0.5, 0.5, np.sqrt(0.5), np.sqrt(0.75)], 15) == [3, 3, 4, 5]
    assert split_intervals([0.5, 0.5, np.sqrt(0.5), np.sqrt(0.75)], 23) == [5, 4, 6, 8]
    assert split_intervals([0.5, 0.5, np.sqrt(0.5), np.sqrt(0.75)], 59) == [12, 11, 16, 20]
    ks, labels = sc_path(16)
    assert ks.shape == (16, 3)
    assert np.allclose(ks[0], 0) and np.allclose(ks[-1], 0.5)
    assert labels == {0: "G", 3: "X", 6: "M", 10: "G", 15: "R"}


def test_batch_cells_uneven():
    cells = batch_cells(8, seed=0)
    ns = [c[0] for c in cells]
    assert set(ns) <= {64, 96, 128}
    assert all(0.2 <= c[1] <= 0.4 for c in cells)


def test_fcc_materials_and_path():
    """The FCC quartz/Si workload of Sec. 7: SPD stiffnesses, a silicon volume
    fraction equal to the sphere's share of the cell, 91 path points through the
    listed vertices."""
    from synth import fcc_path, fcc_quartz_si_cell, quartz_stiffness, silicon_stiffness
    for C in (quartz_stiffness(), silicon_stiffness()):
        assert np.allclose(C, C.T) and np.linalg.eigvalsh(C).min() > 0
    C21, rho, A, theta = fcc_quartz_si_cell((16, 16, 16), supersample=4)
    assert theta.min() == 0.0 and theta.max() == 1.0
    assert 0.0 < theta[(theta > 0) & (theta < 1)].size < theta.size
    frac = 4.0 / 3.0 * np.pi * 0.25 ** 3 / abs(np.linalg.det(A))
    assert abs(theta.mean() - frac) < 0.01 * frac
    assert np.all((rho >= 2.329 - 1e-12) & (rho <= 2.65 + 1e-12))
    for reading, X in (("reduced", (0, 0.5, 0.5)), ("cartesian", (0.5, 0.25, 0.25))):
        ks, labels = fcc_path(10, reading)
        assert ks.shape == (91, 3)
        assert [labels[i] for i in sorted(labels)] == list("GXWKGLUWLK")
        assert np.allclose(ks[10], X) and np.allclose(ks[40], (0, 0, 0))
        assert np.allclose(ks[50], (0.5, 0.5, 0.5))  # L: both readings agree
