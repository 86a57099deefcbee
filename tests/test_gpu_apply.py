"""GPU matvec y = (A_h(k) + s M_h) x through pbr_apply vs the oracle.

Tolerance: 1e-12 relative in the 2-norm on seeded complex-Gaussian x (the
matvec parity target).  Small grids sweep every output against the Kronecker /
index-formula oracle; n = 64 is compared in full against the vectorised index
formula; n = 128 (the benchmark size, same launch configuration) is compared on
sampled output nodes computed one by one.
"""

import numpy as np
import pytest

from oracle import blocks as Bk, discretization as D, pointwise as P
from synth import complex_gaussian, random_spd_field, two_phase_cell

from gpu_util import log, make_ctx, rel, to_dev, to_host
from paper_2606_03599_amd import pbr

pytestmark = pytest.mark.gpu

KAPPA = (0.15, 0.05, 0.10)
FCC = 0.5 * np.array([[0, 1, 1], [1, 0, 1], [1, 1, 0]], dtype=float)
TOL = 1e-12


@pytest.mark.parametrize("dims", [(2, 2, 2), (4, 4, 4), (8, 8, 8), (4, 6, 2), (6, 4, 10)])
@pytest.mark.parametrize("A_lat", [None, "fcc"])
def test_apply_small_full_and_blocks(dims, A_lat):
    Al = FCC if A_lat == "fcc" else None
    log(f"apply dims={dims} A_lat={A_lat}")
    C21, rho = random_spd_field(dims, seed=3)
    n = int(np.prod(dims))
    ctx = make_ctx(dims, C21, rho, Al)
    for kap in (KAPPA, (0.0, 0.0, 0.0), (0.5, -0.25, 1.0)):
        A = D.assemble_A(dims, kap, C21, Al)
        M = D.assemble_M(rho)
        x = complex_gaussian(3 * n, seed=12345)
        s = 0.7
        y_or = A @ x + s * (M @ x)
        y = to_host(ctx.apply(kap, -1, s, to_dev(x), to_dev(np.zeros(3 * n, complex))))
        assert rel(y, y_or) <= TOL
        for b in range(4):
            xb = Bk.gather(x, dims, b)
            Ab = Bk.block_operator(A, dims, b)
            Mb = Bk.block_operator(M, dims, b)
            yb_or = Ab @ xb + s * (Mb @ xb)
            yb = to_host(ctx.apply(kap, b, s, to_dev(xb), to_dev(np.zeros(xb.size, complex))))
            assert rel(yb, yb_or) <= TOL, (kap, b)
    ctx.close()


@pytest.mark.parametrize("dims", [(2, 2, 2), (8, 8, 8), (4, 6, 2), (6, 4, 10)])
def test_apply_blocks_batched(dims):
    """All four blocks in one launch (pbr_apply_blocks) vs the oracle's block
    operators, and bit-identical to four single-block launches."""
    log(f"apply_blocks dims={dims}")
    C21, rho = random_spd_field(dims, seed=7)
    n = int(np.prod(dims))
    ctx = make_ctx(dims, C21, rho)
    kap, s = (0.35, -0.2, 0.15), 0.45
    A = D.assemble_A(dims, kap, C21)
    M = D.assemble_M(rho)
    x = complex_gaussian(3 * n, seed=12345)
    xs = [Bk.gather(x, dims, b) for b in range(4)]
    y = to_host(ctx.apply_blocks(kap, s, to_dev(np.concatenate(xs)),
                                 to_dev(np.zeros(3 * n, complex))))
    nb3 = 3 * n // 4
    for b in range(4):
        Ab = Bk.block_operator(A, dims, b)
        Mb = Bk.block_operator(M, dims, b)
        yb_or = Ab @ xs[b] + s * (Mb @ xs[b])
        assert rel(y[b * nb3:(b + 1) * nb3], yb_or) <= TOL, b
        yb = to_host(ctx.apply(kap, b, s, to_dev(xs[b]), to_dev(np.zeros(nb3, complex))))
        assert np.array_equal(yb, y[b * nb3:(b + 1) * nb3]), b
    ctx.close()


def test_autotuned_split_does_not_change_results():
    """The first four-block launch of a box is autotuned (several work splits
    timed with the caller's own launches); its output must equal every later
    launch's and a fresh context's, bit for bit (n=64: several candidate chunks)."""
    dims = (64, 64, 64)
    C21, rho = random_spd_field(dims, seed=3)
    n = int(np.prod(dims))
    x = to_dev(complex_gaussian(3 * n, seed=77))
    kap, s = (0.2, 0.1, -0.3), 0.6
    outs = []
    for rep in range(2):
        ctx = make_ctx(dims, C21, rho)
        for call in range(2):
            outs.append(to_host(ctx.apply_blocks(kap, s, x, to_dev(np.zeros(3 * n, complex)))))
        ctx.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_apply_blocks_rejects_odd_grid():
    C21, rho = random_spd_field((3, 4, 4), seed=1)
    ctx = make_ctx((3, 4, 4), C21, rho)
    from paper_2606_03599_amd import pbr
    with pytest.raises(pbr.PbrError) as e:
        ctx.apply_blocks(KAPPA, 0.0, to_dev(np.zeros(144, complex)), to_dev(np.zeros(144, complex)))
    assert e.value.status == pbr.PBR_EODDGRID
    ctx.close()


@pytest.mark.parametrize("dims", [(3, 3, 3), (1, 2, 3), (5, 4, 2)])
def test_apply_odd_full_space(dims):
    log(f"apply odd dims={dims}")
    C21, rho = random_spd_field(dims, seed=5)
    n = int(np.prod(dims))
    ctx = make_ctx(dims, C21, rho)
    x = complex_gaussian(3 * n, seed=12345)
    y_or = P.apply_A(x, dims, KAPPA, C21, rho, s=1.3)
    y = to_host(ctx.apply(KAPPA, -1, 1.3, to_dev(x), to_dev(np.zeros(3 * n, complex))))
    assert rel(y, y_or) <= TOL
    ctx.close()


def test_apply_host_pointers():
    dims = (4, 4, 4)
    C21, rho = random_spd_field(dims, seed=9)
    ctx = make_ctx(dims, C21, rho, device_material=False)
    x = complex_gaussian(192, seed=1)
    y = np.zeros(192, complex)
    ctx.apply(KAPPA, -1, 0.0, x, y)
    assert rel(y, P.apply_A(x, dims, KAPPA, C21, rho)) <= TOL
    ctx.close()


def test_gather_scatter_match_oracle():
    dims = (6, 4, 8)
    C21, rho = random_spd_field(dims, seed=2)
    ctx = make_ctx(dims, C21, rho)
    x = complex_gaussian(3 * 192, seed=4)
    full = np.zeros_like(x)
    for b in range(4):
        xb = to_host(ctx.gather(b, to_dev(x), to_dev(np.zeros(144, complex))))
        assert np.array_equal(xb, Bk.gather(x, dims, b))
        full = to_host(ctx.scatter(b, to_dev(xb), to_dev(full)))
    assert np.array_equal(full, x)
    ctx.close()


def test_apply_n64_full_sweep():
    dims = (64, 64, 64)
    log("apply n=64 two-phase, full sweep")
    C21, rho, _ = two_phase_cell(dims, radius=0.35, seed=0)
    ctx = make_ctx(dims, C21, rho)
    n = 64 ** 3
    x = complex_gaussian(3 * n, seed=12345)
    delta = D.default_shift(C21)
    y_or = P.apply_A(x, dims, KAPPA, C21, rho, s=delta)
    y = to_host(ctx.apply(KAPPA, -1, delta, to_dev(x), to_dev(np.zeros(3 * n, complex))))
    assert rel(y, y_or) <= TOL
    for b in (0, 3):
        xb = Bk.gather(x, dims, b)
        yb = to_host(ctx.apply(KAPPA, b, delta, to_dev(xb), to_dev(np.zeros_like(xb))))
        assert rel(yb, Bk.gather(y_or, dims, b)) <= TOL
    ctx.close()


def test_apply_n128_sampled():
    """Benchmark size: sampled outputs, full space and every block."""
    dims = (128, 128, 128)
    log("apply n=128 two-phase, sampled")
    C21, rho, _ = two_phase_cell(dims, radius=0.35, seed=0)
    ctx = make_ctx(dims, C21, rho)
    n = 128 ** 3
    x = complex_gaussian(3 * n, seed=12345)
    delta = D.default_shift(C21)
    rng = np.random.default_rng(7)
    pts = [tuple(int(v) for v in rng.integers(0, 128, 3)) for _ in range(40)]
    pts += [(0, 0, 0), (127, 127, 127), (0, 127, 64), (127, 0, 1), (64, 64, 64)]
    y_pts = P.apply_A_at(pts, x, dims, KAPPA, C21, rho, s=delta)
    y = to_host(ctx.apply(KAPPA, -1, delta, to_dev(x), to_dev(np.zeros(3 * n, complex))))
    Y = y.reshape(3, n)
    idx = [p[0] + 128 * (p[1] + 128 * p[2]) for p in pts]
    assert rel(Y[:, idx].T, y_pts) <= TOL
    cls = Bk.node_class(dims)
    for b in range(4):
        xb = Bk.gather(x, dims, b)
        yb = to_host(ctx.apply(KAPPA, b, delta, to_dev(xb), to_dev(np.zeros_like(xb))))
        nodes = Bk.block_nodes(dims, b)
        pos = {int(v): t for t, v in enumerate(nodes)}
        sel = [t for t, p in enumerate(pts) if cls[idx[t]] == b]
        Yb = yb.reshape(3, -1)
        got = np.array([Yb[:, pos[idx[t]]] for t in sel])
        assert rel(got, y_pts[sel]) <= TOL, b
    ctx.close()


def test_copy_probe_and_stream():
    """The copy probe (the bench's copy-rate reference) copies exactly and
    rejects bad sizes; pbr_stream names the stream the context launches on."""
    import torch
    ctx = pbr.Context((4, 4, 4))
    a = torch.randn(1 << 20, dtype=torch.float64, device="cuda")
    b = torch.zeros_like(a)
    ctx.copy_probe(a, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    with pytest.raises(pbr.PbrError) as e:
        pbr._check(ctx.h, pbr.lib().pbr_copy_probe(ctx.h, a.data_ptr(), b.data_ptr(), 24))
    assert e.value.status == pbr.PBR_EINVAL
    # under torch's default stream the context owns a stream of its own
    assert ctx.stream_handle() != 0
    ctx.close()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx2 = pbr.Context((4, 4, 4))
        assert ctx2.stream_handle() == s.cuda_stream
        ctx2.close()
