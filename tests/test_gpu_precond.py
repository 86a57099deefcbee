"""GPU FFT-diagonal preconditioner (pbr_precond) vs the oracle.

The oracle applies z = T_xi diag K(m)^-1 T_xi^H r with numpy.fft (itself pinned
against the literal dense T and T_sigma).  Radix-2, radix-4 and radix-3 lengths
are covered (n = 6, 12, 24 give 3-factors; block axes are n/2).  For homogeneous
material the preconditioner is exactly (A + delta M)^-1, checked at n = 64.
"""

import numpy as np
import pytest

from oracle import blocks as Bk, discretization as D, fourier as F, pointwise as P
from synth import complex_gaussian, pack_c21, random_spd_field
from synth.materials import random_spd_stiffness

from gpu_util import log, make_ctx, rel, to_dev, to_host
from paper_2606_03599_amd import pbr

pytestmark = pytest.mark.gpu

KAPPA = (0.15, 0.05, 0.10)
FCC = 0.5 * np.array([[0, 1, 1], [1, 0, 1], [1, 1, 0]], dtype=float)
TOL = 1e-12


@pytest.mark.parametrize("dims", [(2, 2, 2), (4, 4, 4), (8, 8, 8), (6, 12, 6), (16, 8, 4),
                                  (24, 6, 12), (10, 10, 10), (20, 6, 30), (30, 20, 10),
                                  (60, 10, 4)])
@pytest.mark.parametrize("A_lat", [None, "fcc"])
def test_precond_matches_oracle(dims, A_lat):
    Al = FCC if A_lat == "fcc" else None
    log(f"precond dims={dims} A_lat={A_lat}")
    C21, rho = random_spd_field(dims, seed=11)
    n = int(np.prod(dims))
    ctx = make_ctx(dims, C21, rho, Al)
    Cref, rref = F.reference_material(C21, rho)
    shift = 1.7
    for kap in (KAPPA, (0.0, 0.0, 0.0)):
        r = complex_gaussian(3 * n, seed=21)
        z_or = F.precond_fft(r, dims, kap, -1, Cref, rref, shift, Al)
        z = to_host(ctx.precond(kap, -1, shift, to_dev(r), to_dev(np.zeros_like(r))))
        assert rel(z, z_or) <= TOL
        for b in range(4):
            rb = complex_gaussian(3 * n // 4, seed=22 + b)
            zb_or = F.precond_fft(rb, dims, kap, b, Cref, rref, shift, Al)
            zb = to_host(ctx.precond(kap, b, shift, to_dev(rb), to_dev(np.zeros_like(rb))))
            assert rel(zb, zb_or) <= TOL, (kap, b)
    ctx.close()


@pytest.mark.parametrize("dims", [(4, 4, 4), (8, 8, 6), (10, 10, 10), (12, 12, 8), (16, 16, 16),
                                  (20, 20, 12), (24, 24, 24), (30, 30, 6), (32, 32, 16),
                                  (40, 40, 8), (48, 48, 4), (64, 64, 8)])
@pytest.mark.parametrize("passes", [3, 5])
def test_block_precond_pass_structures(dims, passes):
    """Blocks with n1 = n2 run the three-pass structure (whole planes, in-place
    transforms in digit-reversed order) unless five passes are asked for; both
    match the oracle, at a generic wave vector, at a zone corner and at Gamma."""
    log(f"block precond dims={dims} passes={passes}")
    C21, rho = random_spd_field(dims, seed=12)
    n = int(np.prod(dims))
    ctx = make_ctx(dims, C21, rho)
    ctx.set_precond_passes(passes)
    Cref, rref = F.reference_material(C21, rho)
    for kap in (KAPPA, (0.5, 0.5, 0.5), (0.0, 0.0, 0.0)):
        for b in range(4):
            rb = complex_gaussian(3 * n // 4, seed=60 + b)
            zb_or = F.precond_fft(rb, dims, kap, b, Cref, rref, 1.3)
            zb = to_host(ctx.precond(kap, b, 1.3, to_dev(rb), to_dev(np.zeros_like(rb))))
            assert rel(zb, zb_or) <= TOL, (kap, b)
    ctx.close()


@pytest.mark.parametrize("dims", [(32, 32, 16), (64, 64, 8)])
@pytest.mark.parametrize("width", [8, 16, 32])
def test_block_precond_solve_widths(dims, width):
    """The three-pass structure with the mode-solve pass pinned to each i-width
    (8 on 256-thread work-groups, 16 and 32 on 512-thread ones) matches the
    oracle at a generic wave vector and at Gamma."""
    log(f"block precond dims={dims} solve width {width}")
    C21, rho = random_spd_field(dims, seed=13)
    n = int(np.prod(dims))
    ctx = make_ctx(dims, C21, rho)
    ctx.set_precond_passes(3)
    ctx.set_solve_width(width)
    Cref, rref = F.reference_material(C21, rho)
    for kap in (KAPPA, (0.0, 0.0, 0.0)):
        for b in range(4):
            rb = complex_gaussian(3 * n // 4, seed=70 + b)
            zb_or = F.precond_fft(rb, dims, kap, b, Cref, rref, 0.7)
            zb = to_host(ctx.precond(kap, b, 0.7, to_dev(rb), to_dev(np.zeros_like(rb))))
            assert rel(zb, zb_or) <= TOL, (kap, b)
    with pytest.raises(pbr.PbrError):
        ctx.set_solve_width(12)
    ctx.close()


def test_precond_reference_override():
    dims = (8, 4, 4)
    C21, rho = random_spd_field(dims, seed=1)
    ctx = make_ctx(dims, C21, rho)
    C = random_spd_stiffness(np.random.default_rng(3))
    ctx.set_reference(pack_c21(C), 2.5)
    r = complex_gaussian(3 * 128, seed=2)
    z_or = F.precond_fft(r, dims, KAPPA, -1, C, 2.5, 0.9)
    z = to_host(ctx.precond(KAPPA, -1, 0.9, to_dev(r), to_dev(np.zeros_like(r))))
    assert rel(z, z_or) <= TOL
    ctx.close()


@pytest.mark.parametrize("kappa", [KAPPA, (0.0, 0.0, 0.0)])
def test_precond_inverts_homogeneous_n64(kappa):
    dims = (64, 64, 64)
    log(f"precond homogeneous n=64 kappa={kappa}")
    n = 64 ** 3
    C = random_spd_stiffness(np.random.default_rng(5))
    C21 = np.tile(pack_c21(C), (n, 1))
    rho = np.full(n, 1.6)
    ctx = make_ctx(dims, C21, rho)
    delta = 3.1
    x = complex_gaussian(3 * n, seed=8)
    b = P.apply_A(x, dims, kappa, C21, rho, s=delta)
    z = to_host(ctx.precond(kappa, -1, delta, to_dev(b), to_dev(np.zeros_like(b))))
    assert rel(z, x) <= 1e-11
    for blk in (1, 2):
        bb = Bk.gather(b, dims, blk)
        zb = to_host(ctx.precond(kappa, blk, delta, to_dev(bb), to_dev(np.zeros_like(bb))))
        assert rel(zb, Bk.gather(x, dims, blk)) <= 1e-11
    ctx.close()
