"""Shared helpers of the GPU tests (device transfer, tolerances, operators)."""
import numpy as np

import workloads as W

FP32_TOL = 1e-5      # complex64 apply, max relative error (infinity-norm relative)
LOWP_TOL = 2e-2      # 16-bit links vs the unquantised operator
EMUL_TOL = 2e-5      # 16-bit kernels vs the oracle's emulation of the same rounding


def max_rel(y, ref):
    y = np.asarray(y)
    ref = np.asarray(ref)
    return float(np.max(np.abs(y - ref)) / np.max(np.abs(ref)))


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def make_op(links, offs, dims, dtype="c64"):
    from paper_2409_03904_amd import coarse
    geom = coarse.Geometry(dims, links.shape[2], offs)
    return coarse.pack(dev(links.astype(np.complex64)), geom, dtype)


def announce(*parts):
    """Print (flushed) what a GPU step is about to run, so a fault names its case."""
    print("[gpu-case]", *parts, flush=True)
