"""The paper's FCC workload (quartz matrix, silicon sphere, FCC lattice, Sec. 7)
through the GPU eigensolver vs the dense oracle on small grids, including grid
lengths with a factor 5 (radix-5 transforms of the preconditioner).
Tolerance: 1e-9 relative on eigenvalues (the eigenvalue accuracy target)."""

import numpy as np
import pytest

from oracle.eigen import block_spectrum, full_spectrum
from synth import fcc_point, fcc_quartz_si_cell

from gpu_util import log, make_ctx

pytestmark = pytest.mark.gpu
TOL = 1e-9


@pytest.mark.parametrize("dims", [(8, 8, 8), (10, 10, 6)])
@pytest.mark.parametrize("point", ["X", "G", "W"])
def test_fcc_merged_and_full_vs_oracle(dims, point):
    kap = tuple(fcc_point(point))
    log(f"fcc dims={dims} point={point}")
    C21, rho, A, _ = fcc_quartz_si_cell(dims, supersample=3)
    ctx = make_ctx(dims, C21, rho, A)
    ref = full_spectrum(dims, kap, C21, rho, A)[:12]
    ev, st = ctx.eigs_merged(kap, 12)
    assert np.all(np.abs(ev - ref) <= TOL * np.abs(ref)), (ev, ref)
    evf, stf, _ = ctx.eigs(kap, -1, 12)
    assert np.all(np.abs(evf - ref) <= TOL * np.abs(ref)), (evf, ref)
    if point == "G":
        assert st.n_zero == 12 and stf.n_zero == 12
    for b in (0, 3):
        refb = block_spectrum(dims, kap, C21, rho, b, A)[:6]
        evb, _, _ = ctx.eigs(kap, b, 6)
        assert np.all(np.abs(evb - refb) <= TOL * np.abs(refb)), (b, evb, refb)
    ctx.close()


def test_fcc_n128_matches_paper_frequencies():
    """The paper's printed 128^3 results (four-band group averages, Sec. 7.3)
    at Gamma, X, W and L, 5 significant digits (relative rounding 2-4e-5).
    With the material sampled at the nodes (no smoothing) the computed groups
    agree with them to 1.5e-6 - 4.7e-5, about the printed precision, which
    pins the operator, the lattice, the wave vectors, the constants and the
    frequency scale; the reading's volume-fraction material (4^3 sub-samples
    per cut cell, Sec. 7.1) moves the groups by 1.4-2.4e-4 -- the paper's own
    cut-cell rule evidently moves them less, and it does not say how it
    computes the fraction."""
    import json
    import os
    from synth import frequency_hz
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "fcc_paper_table.json")))
    dims = (128, 128, 128)
    for supersample, tol in ((1, 6e-5), (4, 5e-4)):
        C21, rho, A, _ = fcc_quartz_si_cell(dims, supersample=supersample)
        ctx = make_ctx(dims, C21, rho, A)
        for row in g["rows"]:
            grp = row["group"] - (g["zero_groups_at_gamma"] if row["point"] == "G" else 0)
            log(f"fcc n=128 ({supersample}^3 samples) {row['point']} G{row['group']}")
            ev, st = ctx.eigs_merged(tuple(fcc_point(row["point"])), 4 * grp)
            f = frequency_hz(ev)[4 * (grp - 1):4 * grp].mean()
            ref = row["present_result_hz"]
            log(f"  ours {f:.5e} paper {ref:.4e} rel {(f - ref) / ref:+.2e}")
            assert abs(f - ref) <= tol * ref, (supersample, row["point"])
        ctx.close()
