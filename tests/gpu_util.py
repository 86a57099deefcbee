"""Helpers shared by the GPU tests (run only on a machine with the GPU)."""

import numpy as np

from paper_2606_03599_amd import pbr


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def to_dev(a):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_host(t):
    torch = torch_cuda()
    torch.cuda.synchronize()
    return t.cpu().numpy()


def make_ctx(dims, C21, rho, A_lat=None, device_material=True):
    torch_cuda()
    ctx = pbr.Context(dims, A_lat=A_lat)
    if device_material:
        ctx.set_material(to_dev(C21), to_dev(rho))
    else:
        ctx.set_material(C21, rho)
    return ctx


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def log(msg):
    print(msg, flush=True)
