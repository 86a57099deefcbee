"""Band eigenvalues as a differentiable function of the nodewise material.

``band_eigenvalues(ctx, kappa, C21, rho, nev)`` returns the nev lowest
eigenvalues lambda = omega^2 of A_h(k) v = lambda M_h v (Eq. 3.15) for the
stiffness field C21 (n x 21) and density rho (n) given as float64 CUDA tensors;
with ``blocked=True`` they are merged from the four parity blocks (Corollary
4.2, with the same certification rule as pbr_eigs_merged).  Its backward pass is
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

from . import pbr


def _block_eigs(ctx, kappa, b, nev, shift, opts):
    N3 = ctx.block_dim(b)
    V = torch.zeros((nev, N3), dtype=torch.complex128, device="cuda")
    ev, st, V = ctx.eigs(kappa, b, nev, shift=shift, opts=opts, evecs=V)
    return np.asarray(ev), V


def _merged_eigenpairs(ctx, kappa, nev, shift, opts):
    """Per-block eigenpairs with the certification rule of the merged solve;
    returns (values, [(block, index)] in merged order, {block: V})."""
    dimb = ctx.block_dim(0)
    nz = 3 if all(float(k) == round(float(k)) for k in kappa) else 0
    cap = lambda v: int(min(v, dimb - nz - 1))
    nev_b = [cap((nev + 3) // 4 + 4)] * 4
    vals, vecs = {}, {}
    need = [0, 1, 2, 3]
    for _ in range(8):
        for b in need:
            vals[b], vecs[b] = _block_eigs(ctx, kappa, b, nev_b[b], shift, opts)
        mask, _ = pbr.pbr_host_merge(nev, [vals[b] for b in range(4)])
        need = []
        for b in range(4):
            if mask & (1 << b):
                nb = cap(nev_b[b] + max(4, nev_b[b] // 2))
                if nb > nev_b[b]:
                    nev_b[b] = nb
                    need.append(b)
        if not need:
            break
    items = sorted(((vals[b][i], b, i) for b in range(4) for i in range(len(vals[b]))))
    items = items[:nev]
    return np.array([v for v, _, _ in items]), [(b, i) for _, b, i in items], vals, vecs


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
            lam, where, vals, vecs = _merged_eigenpairs(ctx, kappa, nev, shift, opts)
        else:
            N3 = ctx.block_dim(-1)
            V = torch.zeros((nev, N3), dtype=torch.complex128, device="cuda")
            ev, st, V = ctx.eigs(kappa, -1, nev, shift=shift, opts=opts, evecs=V)
            lam = np.asarray(ev)
            where = [(-1, i) for i in range(nev)]
            vals, vecs = {-1: lam}, {-1: V}
        fctx.pbr = (ctx, tuple(float(k) for k in kappa), lam, where, vals, vecs, cluster_rtol,
                    C21.shape, rho.shape)
        return torch.as_tensor(lam, dtype=torch.float64, device=C21.device)

    @staticmethod
    def backward(fctx, grad_out):
        ctx, kappa, lam, where, vals, vecs, rtol, shC, shr = fctx.pbr
        w = _cluster_weights(lam, grad_out.detach().cpu().numpy(), rtol)
        gC = torch.zeros(shC, dtype=torch.float64, device="cuda")
        gr = torch.zeros(shr, dtype=torch.float64, device="cuda")
        per = {}
        for (b, i), wi in zip(where, w):
            per.setdefault(b, []).append((i, wi))
        for b, lst in per.items():
            idx = [i for i, _ in lst]
            V = vecs[b][idx].contiguous()
            ctx.eig_grad(kappa, b, vals[b][idx], [wi for _, wi in lst], V, gC, gr)
        return gC, gr, None, None, None, None, None, None, None


def band_eigenvalues(ctx, kappa, C21, rho, nev, blocked=True, shift=0.0, opts=None,
                     cluster_rtol=1e-8):
    """nev lowest eigenvalues at kappa as a differentiable function of (C21, rho)."""
    return _BandEigenvalues.apply(C21, rho, ctx, kappa, int(nev), bool(blocked), float(shift),
                                  opts, float(cluster_rtol))
