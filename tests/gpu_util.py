"""Helpers shared by the GPU tests (not collected)."""
import numpy as np
import torch

from oracle import Grid
from paper_1705_01423_amd.synth import zfaces

F64 = torch.float64


def grids(nx, ny, nz, lx=1.0, ly=1.0, alpha=3.0, precision="fp64", **kw):
    """(oracle grid, GPU plan) for one box."""
    from paper_1705_01423_amd.api import Plan
    zf = zfaces(nz, alpha)
    return Grid(nx, ny, nz, lx, ly, zf), Plan(nx, ny, nz, lx, ly, zf, precision=precision, **kw)


def rel(a, b):
    a = a.detach().to("cpu", F64) if a.dtype != torch.complex128 else a.detach().cpu()
    b = b.detach().to("cpu", F64) if b.dtype != torch.complex128 else b.detach().cpu()
    return float((a - b).norm() / b.norm())


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x)).to("cuda")


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
