"""Pins of the oracle's eigenvalue derivatives (oracle/gradient.py).

* central finite differences of dense eigenvalues (step 1e-6) at several nodes,
  all 21 stiffness entries and the density, full space and one block;
* Euler's relations: lambda is homogeneous of degree 1 in C and of degree -1
  in rho, so sum C21 . dlambda/dC21 = lambda and sum rho . dlambda/drho = -lambda
  (a dropped factor 2 on the off-diagonal entries, or a wrong sign, breaks them);
* the sum over a degenerate cluster does not depend on the basis of the cluster.
"""

import numpy as np

from oracle import gradient as Gr
from oracle.eigen import block_spectrum, full_spectrum
from synth import cubic_stiffness, homogeneous_cell, random_spd_field

DIMS = (4, 4, 4)
KAPPA = (0.21, -0.13, 0.07)


def _simple_index(lam, start):
    """First index >= start whose eigenvalue is well separated from its neighbours."""
    for i in range(start, lam.size - 1):
        gap = min(lam[i + 1] - lam[i], lam[i] - lam[i - 1] if i else np.inf)
        if gap > 1e-3 * abs(lam[i]):
            return i
    raise AssertionError("no simple eigenvalue")


def _fd(fun, p0, h):
    return (fun(p0 + h) - fun(p0 - h)) / (2 * h)


def test_hf_matches_finite_differences_full():
    C21, rho = random_spd_field(DIMS, seed=11)
    lam, V = Gr.eigenpairs(DIMS, KAPPA, C21, rho)
    i = _simple_index(lam, 5)
    gC, gr = Gr.hf_gradient(DIMS, KAPPA, V[:, i], lam[i])
    for x in (0, 21, 63):
        for q in range(21):
            def f(t, q=q):
                C = C21.copy()
                C[x, q] = t
                return full_spectrum(DIMS, KAPPA, C, rho)[i]
            d = _fd(f, C21[x, q], 1e-6)
            assert abs(d - gC[x, q]) <= 1e-6 * np.abs(gC).max() + 1e-8, (x, q, d, gC[x, q])
        def g(t):
            r = rho.copy()
            r[x] = t
            return full_spectrum(DIMS, KAPPA, C21, r)[i]
        d = _fd(g, rho[x], 1e-6)
        assert abs(d - gr[x]) <= 1e-6 * np.abs(gr).max() + 1e-8


def test_hf_matches_finite_differences_block():
    C21, rho = random_spd_field(DIMS, seed=12)
    b = 2
    lam, V = Gr.eigenpairs(DIMS, KAPPA, C21, rho, block=b)
    i = _simple_index(lam, 3)
    gC, gr = Gr.hf_gradient(DIMS, KAPPA, V[:, i], lam[i])
    from oracle.blocks import block_nodes
    nodes = block_nodes(DIMS, b)
    off = np.setdiff1d(np.arange(64), nodes)
    assert np.abs(gC[off]).max() == 0.0 and np.abs(gr[off]).max() == 0.0
    x = int(nodes[5])
    for q in (0, 4, 9, 20):
        def f(t, q=q):
            C = C21.copy()
            C[x, q] = t
            return block_spectrum(DIMS, KAPPA, C, rho, b)[i]
        d = _fd(f, C21[x, q], 1e-6)
        assert abs(d - gC[x, q]) <= 1e-6 * np.abs(gC).max() + 1e-8


def test_euler_homogeneity():
    C21, rho = random_spd_field(DIMS, seed=13)
    lam, V = Gr.eigenpairs(DIMS, KAPPA, C21, rho)
    for i in (0, 7, 40):
        gC, gr = Gr.hf_gradient(DIMS, KAPPA, V[:, i], lam[i])
        assert abs(np.sum(C21 * gC) - lam[i]) <= 1e-10 * abs(lam[i])
        assert abs(np.sum(rho * gr) + lam[i]) <= 1e-10 * abs(lam[i])


def test_euler_homogeneity_gamma_block():
    C21, rho = random_spd_field(DIMS, seed=14)
    lam, V = Gr.eigenpairs(DIMS, (0.0, 0.0, 0.0), C21, rho, block=1)
    gC, gr = Gr.hf_gradient(DIMS, (0.0, 0.0, 0.0), V[:, 0], lam[0])
    assert lam[0] > 1e-8
    assert abs(np.sum(C21 * gC) - lam[0]) <= 1e-10 * lam[0]
    assert abs(np.sum(rho * gr) + lam[0]) <= 1e-10 * lam[0]


def test_cluster_sum_basis_independent():
    C21, rho = homogeneous_cell(DIMS, cubic_stiffness(1.0, 0.4, 0.3), 1.0)
    kap = (0.25, 0.0, 0.0)
    lam, V = Gr.eigenpairs(DIMS, kap, C21, rho)
    # a cluster of equal eigenvalues (homogeneous material: multiplicities)
    i0 = None
    for i in range(lam.size - 1):
        if abs(lam[i + 1] - lam[i]) <= 1e-10 * abs(lam[i]) and lam[i] > 1e-8:
            i0 = i
            break
    assert i0 is not None
    i1 = i0
    while i1 + 1 < lam.size and abs(lam[i1 + 1] - lam[i0]) <= 1e-10 * abs(lam[i0]):
        i1 += 1
    idx = np.arange(i0, i1 + 1)
    g1 = Gr.cluster_gradient(DIMS, kap, V[:, idx], lam[idx])
    rng = np.random.default_rng(3)
    Z = rng.standard_normal((idx.size, idx.size)) + 1j * rng.standard_normal((idx.size, idx.size))
    U, _ = np.linalg.qr(Z)
    g2 = Gr.cluster_gradient(DIMS, kap, V[:, idx] @ U, lam[idx])
    assert np.allclose(g1[0], g2[0], rtol=0, atol=1e-10 * np.abs(g1[0]).max())
    assert np.allclose(g1[1], g2[1], rtol=0, atol=1e-10 * np.abs(g1[1]).max())
