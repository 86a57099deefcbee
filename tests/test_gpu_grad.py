"""Eigenvalue derivatives w.r.t. the nodewise stiffness and density on the GPU.

* The gradient kernel (pbr_eig_grad) fed with the oracle's dense eigenvectors
  must reproduce the oracle's Hellmann-Feynman gradient to rounding (1e-12
  relative in the max norm): full space, each block, a generic k and Gamma.
* End to end (GPU eigenvectors through band_eigenvalues + torch autograd) vs the
  oracle gradient of a simple eigenvalue: the eigenvectors carry the solver's
  error (relative residual <= ~1e-9, relative gaps ~1e-2 at n = 8), which
  enters the quadratic gradient at first order, so 1e-6 relative.
* n = 96 two-phase cell (the differentiation workload): eigenvalues 6 and 7 at X
  and R, directional derivative over 50 random nodes vs a central finite
  difference with relative step 1e-6; the eigenvalues are accurate to rounding
  (their error is quadratic in the eigenvector error), so the difference quotient
  carries ~1e-15 / (1e-6 * |derivative| / lambda) relative noise: 1e-3.
"""

import numpy as np
import pytest

from oracle import gradient as Gr
from oracle.blocks import block_nodes
from synth import random_spd_field, two_phase_cell

from gpu_util import log, make_ctx, to_dev, to_host

pytestmark = pytest.mark.gpu

DIMS = (8, 8, 8)


def _gather_block(Vfull, dims, b):
    n = int(np.prod(dims))
    nodes = block_nodes(dims, b)
    rows = np.concatenate([a * n + nodes for a in range(3)])
    return Vfull[rows]


@pytest.mark.parametrize("kappa", [(0.15, 0.05, 0.10), (0.0, 0.0, 0.0)])
@pytest.mark.parametrize("block", [-1, 0, 1, 2, 3])
def test_grad_kernel_matches_oracle(kappa, block):
    import torch
    log(f"eig_grad kernel n=8 kappa={kappa} block={block}")
    C21, rho = random_spd_field(DIMS, seed=21)
    n = int(np.prod(DIMS))
    ctx = make_ctx(DIMS, C21, rho)
    lam, V = Gr.eigenpairs(DIMS, kappa, C21, rho, block=block)
    idx = [0, 3, 7]
    w = [1.0, -0.5, 2.0]
    gC_or, gr_or = Gr.cluster_gradient(DIMS, kappa, V[:, idx], lam[idx], w)
    Vl = V if block < 0 else _gather_block(V, DIMS, block)
    ev = np.ascontiguousarray(Vl[:, idx].T)
    gC = torch.zeros((n, 21), dtype=torch.float64, device="cuda")
    gr = torch.zeros(n, dtype=torch.float64, device="cuda")
    ctx.eig_grad(kappa, block, lam[idx], w, to_dev(ev.ravel()), gC, gr)
    gC, gr = to_host(gC), to_host(gr)
    assert np.abs(gC - gC_or).max() <= 1e-12 * np.abs(gC_or).max()
    assert np.abs(gr - gr_or).max() <= 1e-12 * np.abs(gr_or).max()
    ctx.close()


def test_grad_host_pointers_accumulate():
    C21, rho = random_spd_field(DIMS, seed=22)
    n = int(np.prod(DIMS))
    ctx = make_ctx(DIMS, C21, rho)
    kap = (0.3, 0.1, -0.2)
    lam, V = Gr.eigenpairs(DIMS, kap, C21, rho)
    gC_or, gr_or = Gr.hf_gradient(DIMS, kap, V[:, 2], lam[2])
    gC = np.ones((n, 21))
    gr = np.ones(n)
    ctx.eig_grad(kap, -1, lam[2:3], [1.0], np.ascontiguousarray(V[:, 2]), gC, gr)
    assert np.abs(gC - 1.0 - gC_or).max() <= 1e-12 * np.abs(gC_or).max()
    assert np.abs(gr - 1.0 - gr_or).max() <= 1e-12 * np.abs(gr_or).max()
    ctx.close()


@pytest.mark.parametrize("blocked", [True, False])
def test_band_gradient_end_to_end_n8(blocked):
    import torch
    from paper_2606_03599_amd.autograd import band_eigenvalues
    log(f"band_eigenvalues autograd n=8 blocked={blocked}")
    C21, rho = two_phase_cell(DIMS, radius=0.35, seed=0)[:2]
    kap = (0.15, 0.05, 0.10)
    ctx = make_ctx(DIMS, C21, rho)
    Ct = torch.tensor(C21, device="cuda", requires_grad=True)
    rt = torch.tensor(rho, device="cuda", requires_grad=True)
    lam = band_eigenvalues(ctx, kap, Ct, rt, 10, blocked=blocked)
    lam_or, V = Gr.eigenpairs(DIMS, kap, C21, rho)
    assert np.allclose(lam.detach().cpu().numpy(), lam_or[:10], rtol=1e-9, atol=0)
    # a simple eigenvalue
    i = next(i for i in range(2, 9)
             if min(lam_or[i + 1] - lam_or[i], lam_or[i] - lam_or[i - 1]) > 1e-3 * lam_or[i])
    lam[i].backward()
    gC_or, gr_or = Gr.hf_gradient(DIMS, kap, V[:, i], lam_or[i])
    gC, gr = Ct.grad.cpu().numpy(), rt.grad.cpu().numpy()
    assert np.abs(gC - gC_or).max() <= 1e-6 * np.abs(gC_or).max()
    assert np.abs(gr - gr_or).max() <= 1e-6 * np.abs(gr_or).max()
    ctx.close()


@pytest.mark.parametrize("point", ["X", "R"])
def test_band_gradient_fd_n96(point):
    import torch
    from paper_2606_03599_amd.autograd import band_eigenvalues
    dims = (96, 96, 96)
    kap = {"X": (0.5, 0.0, 0.0), "R": (0.5, 0.5, 0.5)}[point]
    log(f"band gradient vs finite difference n=96 at {point}")
    C21, rho = two_phase_cell(dims, radius=0.35, seed=0)[:2]
    n = C21.shape[0]
    ctx = make_ctx(dims, C21, rho)
    Ct = torch.tensor(C21, device="cuda", requires_grad=True)
    rt = torch.tensor(rho, device="cuda", requires_grad=True)
    lam = band_eigenvalues(ctx, kap, Ct, rt, 8)
    l = lam.detach().cpu().numpy()
    # bands 6 and 7 (1-based): summed if they form a cluster
    sep = abs(l[6] - l[5]) > 1e-6 * l[5]
    targets = [(5,), (6,)] if sep else [(5, 6)]
    rng = np.random.default_rng(96)
    nodes = rng.choice(n, size=50, replace=False)
    dC = np.zeros_like(C21)
    dr = np.zeros_like(rho)
    dC[nodes] = rng.standard_normal((50, 21)) * np.abs(C21[nodes]).mean()
    dr[nodes] = rng.standard_normal(50) * rho[nodes]
    h = 1e-6
    lp = band_eigenvalues(ctx, kap, torch.tensor(C21 + h * dC, device="cuda"),
                          torch.tensor(rho + h * dr, device="cuda"), 8).cpu().numpy()
    lm = band_eigenvalues(ctx, kap, torch.tensor(C21 - h * dC, device="cuda"),
                          torch.tensor(rho - h * dr, device="cuda"), 8).cpu().numpy()
    for t in targets:
        gC, gr = torch.autograd.grad(sum(lam[j] for j in t), [Ct, rt], retain_graph=True)
        ana = float((gC.cpu().numpy() * dC).sum() + (gr.cpu().numpy() * dr).sum())
        fd = sum(lp[j] - lm[j] for j in t) / (2 * h)
        log(f"  bands {t}: analytic {ana:.6e}  finite difference {fd:.6e}")
        assert abs(ana - fd) <= 1e-3 * abs(fd)
    ctx.close()
