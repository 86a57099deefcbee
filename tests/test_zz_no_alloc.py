"""pbr_precond_noalloc, the entry point for callers that cannot allocate device
memory, against pbr_precond (the same kernels; tables in the device's fixed
scratch array instead of context-allocated buffers) and the oracle.

Two calls in a row share the device's array: a 32^3 full-space application,
then a smaller input (a parity block of a 16 x 8 x 8 grid at another wave
vector), each bit-identical to pbr_precond on the same input.  Grids beyond the
array's 256 entries per axis are rejected before any work.
"""

import numpy as np
import pytest

from oracle import fourier as F
from synth import complex_gaussian, random_spd_field

from gpu_util import log, make_ctx, rel, to_dev, to_host
from paper_2606_03599_amd import pbr

pytestmark = pytest.mark.gpu


def test_precond_noalloc_matches_precond_two_calls():
    import torch
    cases = [((32, 32, 32), -1, (0.15, 0.05, 0.10), 1.7),
             ((16, 8, 8), 1, (0.5, 0.25, 0.0), 0.9)]
    for q, (dims, block, kap, shift) in enumerate(cases):
        log(f"precond_noalloc call {q}: dims={dims} block={block}")
        C21, rho = random_spd_field(dims, seed=40 + q)
        ctx = make_ctx(dims, C21, rho)
        n = int(np.prod(dims))
        dim = 3 * n if block < 0 else 3 * n // 4
        r = complex_gaussian(dim, seed=50 + q)
        rd = to_dev(r)
        z_ref = ctx.precond(kap, block, shift, rd, torch.zeros_like(rd))
        z = torch.full_like(rd, complex(np.nan, np.nan))
        ctx.precond_noalloc(kap, block, shift, rd, z)
        torch.cuda.synchronize()
        assert torch.equal(z, z_ref)
        Cref, rref = F.reference_material(C21, rho)
        z_or = F.precond_fft(r, dims, kap, block, Cref, rref, shift)
        assert rel(to_host(z), z_or) <= 1e-12
        ctx.close()


def test_precond_noalloc_rejects_beyond_scratch():
    import torch
    dims = (260, 2, 2)
    C21, rho = random_spd_field(dims, seed=3)
    ctx = make_ctx(dims, C21, rho)
    r = torch.zeros(3 * 260 * 4, dtype=torch.complex128, device="cuda")
    with pytest.raises(pbr.PbrError) as e:
        ctx.precond_noalloc((0.1, 0.2, 0.3), -1, 1.0, r, torch.zeros_like(r))
    assert e.value.status == pbr.PBR_EINVAL
    assert "256" in e.value.message
    ctx.close()
