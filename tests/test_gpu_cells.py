"""Several unit cells of their own grid sizes in one call (pbr_band_paths): the
cells' paths run concurrently, one native host thread per context, and every
cell's eigenvalues must equal, bit for bit, those of pbr_band_path on that cell
alone; the n=8 cell is also checked against the dense oracle spectra
(tests/golden/two_phase_n8.json) at 1e-9."""

import json
import os

import numpy as np
import pytest

from synth import sc_path, two_phase_cell

from gpu_util import log, make_ctx, torch_cuda
from paper_2606_03599_amd import pbr

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _cells():
    g = json.load(open(os.path.join(GOLD, "two_phase_n8.json")))
    cells = [((8, 8, 8), g["radius"], g["seed"]), ((12, 12, 12), 0.3, 5), ((16, 16, 16), 0.25, 9),
             ((10, 10, 6), 0.3, 7)]
    return g, cells


def test_band_paths_match_single_cells():
    g, cells = _cells()
    ctxs, paths = [], []
    ks_all, _ = sc_path(8)
    for q, (dims, r, seed) in enumerate(cells):
        C21, rho, _ = two_phase_cell(dims, radius=r, seed=seed)
        ctxs.append(make_ctx(dims, C21, rho))
        paths.append(ks_all[q:q + 3 + q % 2])
    nev = 6
    log(f"band_paths over {len(cells)} cells")
    evs, sts = pbr.band_paths(ctxs, paths, nev)
    for q, ctx in enumerate(ctxs):
        ev1, _ = ctx.band_path(paths[q], nev)
        assert np.array_equal(evs[q], ev1), q
        assert sts[q].op_applies > 0
    # the n=8 cell against the dense oracle at the golden wave vectors
    pts = [np.asarray(p["kappa"]) for p in g["points"].values()]
    ev8, _ = pbr.band_paths(ctxs[:2], [pts, paths[1]], 12)
    for p, e in zip(g["points"].values(), ev8[0]):
        ref = np.asarray(p["full_lowest"])[:12]
        assert np.max(np.abs(e - ref) / np.abs(ref)) < 1e-9
    for ctx in ctxs:
        ctx.close()


def test_band_paths_rejects_shared_stream():
    import torch
    torch_cuda()
    s = torch.cuda.Stream()
    C21, rho, _ = two_phase_cell((8, 8, 8), radius=0.3, seed=1)
    a = pbr.Context((8, 8, 8), stream=s.cuda_stream)
    b = pbr.Context((8, 8, 8), stream=s.cuda_stream)
    for c in (a, b):
        c.set_material(C21, rho)
    with pytest.raises(pbr.PbrError) as e:
        pbr.band_paths([a, b], [[(0.1, 0.2, 0.3)], [(0.1, 0.2, 0.3)]], 4)
    assert e.value.status == pbr.PBR_EINVAL
    a.close()
    b.close()
