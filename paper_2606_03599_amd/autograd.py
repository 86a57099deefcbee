"""Band eigenvalues as a differentiable function of the nodewise material.

``band_eigenvalues(ctx, kappa, C21, rho, nev)`` returns the nev lowest
eigenvalues lambda = omega^2 of A_h(k) v = lambda M_h v (Eq. 3.15) for the
stiffness field C21 (n x 21) and density rho (n) given as float64 CUDA tensors;
with ``blocked=True`` they are merged from the four parity blocks by
pbr_eigs_merged_vecs (Corollary 4.2, certified merge), which also returns each
value's block and block-layout eigenvector.  Its backward pass is
the Hellmann-Feynman formula of pbr_eig_grad: the strains of each eigenvector
are recomputed on the device, nothing per node is stored between the passes but
the eigenvectors themselves.

Degenerate clusters: a single eigenvalue inside a cluster of equal eigenvalues
has no derivative; the sum over the cluster does.  Eigenvalues within
``cluster_rtol`` of each other (relative) are grouped, and every member gets the
mean of the cluster's incoming gradient weights, so the gradient of any function
of the cluster sum (band gap edges summed over a cluster, for instance) is exact.
A cluster cut by the nev boundary is summed over its computed members only.
"""

from __future__ import annotations

import numpy as np
import torch


def _cluster_weights(lam, w, rtol):
    w = np.asarray(w, dtype=np.float64).copy()
    order = np.argsort(lam, kind="stable")
    s = 0
    while s < len(order):
        e = s + 1
        while e < len(order) and abs(lam[order[e]] - lam[order[s]]) <= rtol * abs(lam[order[s]]):
            e += 1
        idx = order[s:e]
        w[idx] = w[idx].mean()
        s = e
    return w


class _BandEigenvalues(torch.autograd.Function):
    @staticmethod
    def forward(fctx, C21, rho, ctx, kappa, nev, blocked, shift, opts, cluster_rtol):
        ctx.set_material(C21.detach().contiguous(), rho.detach().contiguous())
        if blocked:
            V = torch.zeros((nev, ctx.block_dim(0)), dtype=torch.complex128, device="cuda")
            lam, blocks, _, V = ctx.eigs_merged_vecs(kappa, nev, V, shift=shift, opts=opts)
        else:
            V = torch.zeros((nev, ctx.block_dim(-1)), dtype=torch.complex128, device="cuda")
            lam, _, V = ctx.eigs(kappa, -1, nev, shift=shift, opts=opts, evecs=V)
            blocks = np.full(nev, -1)
        fctx.pbr = (ctx, tuple(float(k) for k in kappa), np.asarray(lam), np.asarray(blocks),
                    V, cluster_rtol, C21.shape, rho.shape)
        return torch.as_tensor(lam, dtype=torch.float64, device=C21.device)

    @staticmethod
    def backward(fctx, grad_out):
        ctx, kappa, lam, blocks, V, rtol, shC, shr = fctx.pbr
        w = _cluster_weights(lam, grad_out.detach().cpu().numpy(), rtol)
        gC = torch.zeros(shC, dtype=torch.float64, device="cuda")
        gr = torch.zeros(shr, dtype=torch.float64, device="cuda")
        for b in sorted(set(int(x) for x in blocks)):
            idx = np.nonzero(blocks == b)[0]
            ctx.eig_grad(kappa, b, lam[idx], w[idx], V[torch.as_tensor(idx, device=V.device)].contiguous(), gC, gr)
        return gC, gr, None, None, None, None, None, None, None


def band_eigenvalues(ctx, kappa, C21, rho, nev, blocked=True, shift=0.0, opts=None,
                     cluster_rtol=1e-8):
    """nev lowest eigenvalues at kappa as a differentiable function of (C21, rho)."""
    return _BandEigenvalues.apply(C21, rho, ctx, kappa, int(nev), bool(blocked), float(shift),
                                  opts, float(cluster_rtol))
