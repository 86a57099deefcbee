"""Parity at n = 256, the largest grid the path is measured on (the 60-point
band path with 30 eigenpairs per k and the gap-width gradient; 16.7M nodes,
four parity blocks of 4.2M), against the oracle.

* The path's operator launch (pbr_apply_blocks: the four parity blocks of one
  wave vector in one launch, palette form of the two-phase cell) against the
  oracle's pointwise operator (Eq. 3.15, Sec. 6.1) at sampled nodes of every
  block, 1e-12 relative.
* The FFT-diagonal preconditioner of a parity block (Sec. 5.1-5.4; at n = 256 a
  block's in-plane lines are 128 long, so it runs the five-pass structure) against
  oracle.fourier.precond_fft, 1e-12 relative.
* The merged eigensolver on a homogeneous cell (one random SPD stiffness) against
  the closed form of Sec. 5.3 and Appendix B, the union over modes of
  eig(Bhat C Bhat^H) / rho (Corollary 4.2), 1e-9 relative.
"""

import numpy as np
import pytest

from oracle import blocks as Bk, discretization as D, fourier as F, pointwise as P
from synth import complex_gaussian, pack_c21, two_phase_cell
from synth.materials import random_spd_stiffness

from gpu_util import log, make_ctx, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

N = 256
DIMS = (N, N, N)
KAPPA = (0.15, 0.05, 0.10)
TOL = 1e-12


@pytest.fixture(scope="module")
def cell256():
    log("two-phase cell n=256")
    C21, rho, _ = two_phase_cell(DIMS, radius=0.35, seed=0)
    ctx = make_ctx(DIMS, C21, rho)
    yield ctx, C21, rho
    ctx.close()


def test_apply_blocks_n256_sampled(cell256):
    ctx, C21, rho = cell256
    assert ctx.palette_size() == 2
    n = N ** 3
    xf = complex_gaussian(3 * n, seed=21)
    log("apply_blocks n=256: gather the four blocks")
    x = to_dev(np.concatenate([Bk.gather(xf, DIMS, b) for b in range(4)]))
    s = D.default_shift(C21)
    y = to_host(ctx.apply_blocks(KAPPA, s, x, to_dev(np.zeros(3 * n, complex))))
    del x
    rng = np.random.default_rng(256)
    pts = [tuple(int(v) for v in rng.integers(0, N, 3)) for _ in range(48)]
    pts += [(0, 0, 0), (N - 1, N - 1, N - 1), (1, 0, N - 1), (N - 2, N - 1, 0), (128, 127, 128)]
    y_pts = P.apply_A_at(pts, xf, DIMS, KAPPA, C21, rho, s=s)
    idx = [p[0] + N * (p[1] + N * p[2]) for p in pts]
    cls = Bk.node_class(DIMS)
    nb3 = 3 * n // 4
    for b in range(4):
        Yb = y[b * nb3:(b + 1) * nb3].reshape(3, -1)
        pos = {int(v): t for t, v in enumerate(Bk.block_nodes(DIMS, b))}
        sel = [t for t in range(len(pts)) if cls[idx[t]] == b]
        assert sel, b
        got = np.array([Yb[:, pos[idx[t]]] for t in sel])
        log(f"  block {b}: {len(sel)} nodes, rel err {rel(got, y_pts[sel]):.2e}")
        assert rel(got, y_pts[sel]) <= TOL, b


def test_precond_block_n256(cell256):
    ctx, C21, rho = cell256
    Cref, rref = F.reference_material(C21, rho)
    shift = ctx.default_shift()
    rb = complex_gaussian(3 * N ** 3 // 4, seed=3)
    log("precond block 1 n=256 (oracle about a minute)")
    z_or = F.precond_fft(rb, DIMS, KAPPA, 1, Cref, rref, shift)
    z = to_host(ctx.precond(KAPPA, 1, shift, to_dev(rb), to_dev(np.zeros_like(rb))))
    log(f"  rel err {rel(z, z_or):.2e}")
    assert rel(z, z_or) <= TOL


def test_merged_eigs_homogeneous_n256():
    C = random_spd_stiffness(np.random.default_rng(7))
    rho = 1.3
    n = N ** 3
    log("homogeneous cell n=256")
    ctx = make_ctx(DIMS, np.tile(pack_c21(C), (n, 1)), np.full(n, rho))
    kappa = (0.37, -0.21, 0.08)
    nev = 12
    ref = F.homogeneous_spectrum(DIMS, kappa, C, rho)[:nev]
    ev, st = ctx.eigs_merged(kappa, nev)
    err = np.abs(ev - ref) / np.abs(ref)
    log(f"  merged eigs: max rel err {err.max():.2e}, solves {st.op_applies}, "
        f"pcg avg {st.pcg_avg:.2f}")
    assert err.max() <= 1e-9
    ctx.close()
