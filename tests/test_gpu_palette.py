"""Palette form of the material: the stencil reads one byte per node and the
distinct (C21, rho) rows from LDS when the material has at most 256 of them.

The dense and palette forms hold the same values, so their matvecs must agree
bit for bit; both are also held to the oracle's 1e-12 matvec tolerance.  The
graph test checks that a PCG graph captured under one material is not replayed
under another (a material change, or a change of form, recaptures).
"""

import numpy as np
import pytest

from oracle import blocks as Bk, discretization as D
from synth import complex_gaussian, random_spd_field, two_phase_cell
from synth.materials import pack_c21, random_spd_stiffness

from gpu_util import log, make_ctx, rel, to_dev, to_host
from paper_2606_03599_amd import pbr

pytestmark = pytest.mark.gpu

FCC = 0.5 * np.array([[0, 1, 1], [1, 0, 1], [1, 1, 0]], dtype=float)
TOL = 1e-12


def labelled_field(dims, K, seed):
    """K random SPD materials (each with its own rho) assigned to the nodes at
    random; every material appears when the grid has at least K nodes."""
    rng = np.random.default_rng(seed)
    rows = np.stack([pack_c21(random_spd_stiffness(rng)) for _ in range(K)])
    rhos = rng.uniform(0.5, 4.0, K)
    n = int(np.prod(dims))
    lab = rng.integers(0, K, n)
    if n >= K:
        lab[rng.permutation(n)[:K]] = np.arange(K)
    return rows[lab], rhos[lab]


def _apply_both(ctx, kap, block, s, x):
    out = []
    for enable in (True, False):
        ctx.set_palette(enable)
        out.append(to_host(ctx.apply(kap, block, s, to_dev(x), to_dev(np.zeros_like(x)))))
    ctx.set_palette(True)
    return out


@pytest.mark.parametrize("dims", [(2, 2, 2), (8, 8, 8), (4, 6, 2), (6, 4, 10)])
@pytest.mark.parametrize("K", [1, 3, 256])
@pytest.mark.parametrize("A_lat", [None, "fcc"])
def test_palette_matches_dense_and_oracle(dims, K, A_lat):
    n = int(np.prod(dims))
    if K > n:
        pytest.skip("fewer nodes than materials")
    log(f"palette dims={dims} K={K} A_lat={A_lat}")
    Al = FCC if A_lat == "fcc" else None
    C21, rho = labelled_field(dims, K, seed=K + n)
    ctx = make_ctx(dims, C21, rho, Al)
    assert ctx.palette_size() == K
    s = 0.55
    for kap in ((0.15, 0.05, 0.10), (0.0, 0.0, 0.0)):
        A = D.assemble_A(dims, kap, C21, Al)
        M = D.assemble_M(rho)
        x = complex_gaussian(3 * n, seed=99)
        y_pal, y_den = _apply_both(ctx, kap, -1, s, x)
        assert np.array_equal(y_pal, y_den)
        assert rel(y_pal, A @ x + s * (M @ x)) <= TOL
        xs = []
        for b in range(4):
            xb = Bk.gather(x, dims, b)
            xs.append(xb)
            yb_pal, yb_den = _apply_both(ctx, kap, b, s, xb)
            assert np.array_equal(yb_pal, yb_den), b
            yb_or = Bk.block_operator(A, dims, b) @ xb + s * (Bk.block_operator(M, dims, b) @ xb)
            assert rel(yb_pal, yb_or) <= TOL, b
            # the four-block launch gives the single-block results
            if b == 3:
                y4 = to_host(ctx.apply_blocks(kap, s, to_dev(np.concatenate(xs)),
                                              to_dev(np.zeros(3 * n, complex))))
                nb3 = 3 * n // 4
                for bb in range(4):
                    yb1 = to_host(ctx.apply(kap, bb, s, to_dev(xs[bb]),
                                            to_dev(np.zeros(nb3, complex))))
                    assert np.array_equal(y4[bb * nb3:(bb + 1) * nb3], yb1), bb
    ctx.close()


@pytest.mark.parametrize("dims,K", [((8, 8, 8), 5), ((8, 8, 8), 256), ((12, 10, 14), 5),
                                    ((34, 30, 6), 5)])
def test_every_stencil_shape_gives_the_same_operator(dims, K):
    """Each tile shape, pinned (16 x 13 in both forms, 16 x 11 in the palette
    form; 16 x 11 pinned on the dense form falls back to its own shape), gives the
    same output bit for bit, full space, single blocks and the four-block launch,
    and matches the oracle; grids with ragged tiles in i and j, and a 256-row
    palette (45 KB of LDS on top of the tile's)."""
    log(f"stencil shapes dims={dims} K={K}")
    n = int(np.prod(dims))
    C21, rho = labelled_field(dims, K, seed=n + K)
    ctx = make_ctx(dims, C21, rho)
    kap, s = (0.15, -0.05, 0.3), 0.8
    x = complex_gaussian(3 * n, seed=4)
    xs = [Bk.gather(x, dims, b) for b in range(4)]
    x4 = to_dev(np.concatenate(xs))
    A = D.assemble_A(dims, kap, C21) if n <= 2000 else None
    outs = []
    for enable, shape in ((True, (16, 11)), (True, (16, 13)), (False, (16, 13)),
                          (False, (16, 11)), (True, (0, 0))):
        ctx.set_palette(enable)
        ctx.set_stencil_shape(*shape)
        y = to_host(ctx.apply(kap, -1, s, to_dev(x), to_dev(np.zeros_like(x))))
        yb = [to_host(ctx.apply(kap, b, s, to_dev(xs[b]), to_dev(np.zeros_like(xs[b]))))
              for b in range(4)]
        y4 = to_host(ctx.apply_blocks(kap, s, x4, to_dev(np.zeros(3 * n, complex))))
        outs.append((y, yb, y4))
    for y, yb, y4 in outs[1:]:
        assert np.array_equal(y, outs[0][0])
        assert np.array_equal(y4, outs[0][2])
        for b in range(4):
            assert np.array_equal(yb[b], outs[0][1][b])
    if A is not None:
        M = D.assemble_M(rho)
        assert rel(outs[0][0], A @ x + s * (M @ x)) <= TOL
    nb3 = 3 * n // 4
    for b in range(4):
        assert np.array_equal(outs[0][2][b * nb3:(b + 1) * nb3], outs[0][1][b])
        assert rel(outs[0][1][b], Bk.gather(outs[0][0], dims, b)) <= TOL
    with pytest.raises(pbr.PbrError):
        ctx.set_stencil_shape(8, 22)
    ctx.close()


def test_palette_size_rules():
    dims = (8, 8, 8)
    ctx = pbr.Context(dims)
    assert ctx.palette_size() == -1  # no material yet
    for K, want in ((256, 256), (257, 0), (1, 1)):
        C21, rho = labelled_field(dims, K, seed=5)
        ctx.set_material(to_dev(C21), to_dev(rho))
        assert ctx.palette_size() == want, K
    C21, rho = random_spd_field(dims, seed=1)
    ctx.set_material(to_dev(C21), to_dev(rho))
    assert ctx.palette_size() == 0
    C21, rho, _ = two_phase_cell(dims, radius=0.35, seed=0)
    ctx.set_material(to_dev(C21), to_dev(rho))
    assert ctx.palette_size() == 2
    ctx.set_palette(False)
    assert ctx.palette_size() == 0
    ctx.set_palette(True)
    assert ctx.palette_size() == 2
    # a row differing from another in one bit is a row of its own
    C21b = C21.copy()
    C21b[17, 4] = np.nextafter(C21b[17, 4], np.inf)
    ctx.set_material(to_dev(C21b), to_dev(rho))
    assert ctx.palette_size() == 3
    ctx.close()


def test_palette_n128_four_blocks_bit_identical():
    """The benchmark launch (four blocks in one launch, n = 128, two-phase cell,
    the bench's wave vector and shift): palette and dense forms give the same
    output bit for bit, each form's chunk length autotuned on its own, and the
    output matches the oracle on sampled nodes of every block."""
    from oracle import pointwise as P
    dims = (128, 128, 128)
    log("palette n=128 four blocks")
    C21, rho, _ = two_phase_cell(dims, radius=0.35, seed=0)
    ctx = make_ctx(dims, C21, rho)
    assert ctx.palette_size() == 2
    n = 128 ** 3
    xf = complex_gaussian(3 * n, seed=21)
    xs = [Bk.gather(xf, dims, b) for b in range(4)]
    x = to_dev(np.concatenate(xs))
    kap, s = (0.15, 0.05, 0.10), D.default_shift(C21)
    outs = {}
    for enable in (True, False, True):
        ctx.set_palette(enable)
        outs.setdefault(enable, []).append(
            to_host(ctx.apply_blocks(kap, s, x, to_dev(np.zeros(3 * n, complex)))))
    assert np.array_equal(outs[True][0], outs[False][0])
    assert np.array_equal(outs[True][1], outs[False][0])
    rng = np.random.default_rng(11)
    pts = [tuple(int(v) for v in rng.integers(0, 128, 3)) for _ in range(32)]
    pts += [(0, 0, 0), (127, 127, 127), (1, 0, 127), (126, 127, 0), (64, 63, 64)]
    y_pts = P.apply_A_at(pts, xf, dims, kap, C21, rho, s=s)
    idx = [p[0] + 128 * (p[1] + 128 * p[2]) for p in pts]
    cls = Bk.node_class(dims)
    nb3 = 3 * n // 4
    for b in range(4):
        Yb = outs[True][0][b * nb3:(b + 1) * nb3].reshape(3, -1)
        pos = {int(v): t for t, v in enumerate(Bk.block_nodes(dims, b))}
        sel = [t for t in range(len(pts)) if cls[idx[t]] == b]
        got = np.array([Yb[:, pos[idx[t]]] for t in sel])
        assert rel(got, y_pts[sel]) <= TOL, b
    ctx.close()


def test_pcg_graph_recaptured_after_material_change():
    """Same buffers, wave vector and shift, new material (palette -> dense ->
    palette) or a new form: the graph-replayed PCG equals eager launches bit
    for bit each time, so no graph of an earlier material is replayed."""
    import torch
    dims = (32, 32, 32)
    mats = [two_phase_cell(dims, radius=0.3, seed=2)[:2], random_spd_field(dims, seed=4),
            two_phase_cell(dims, radius=0.25, seed=6)[:2]]
    ctx = pbr.Context(dims)
    nb3 = 3 * 32 ** 3 // 4
    bdev = to_dev(complex_gaussian(nb3, seed=31))
    xdev = torch.zeros_like(bdev)
    kap, shift = (0.15, 0.05, 0.10), 2.0
    steps = [(0, True), (1, True), (2, True), (2, False)]
    for m, enable in steps:
        log(f"graph after material {m} palette={enable}")
        ctx.set_material(to_dev(mats[m][0]), to_dev(mats[m][1]))
        ctx.set_palette(enable)
        res = {}
        for graphs in (1, 0):
            o = pbr.pbr_opts_default()
            o.graphs = graphs
            xdev.zero_()
            _, st = ctx.solve(kap, 1, shift, bdev, xdev, o)
            res[graphs] = (to_host(xdev), st.pcg_iters_total)
        assert res[0][1] == res[1][1] and res[0][1] > 20
        assert np.array_equal(res[0][0], res[1][0])
    ctx.close()
