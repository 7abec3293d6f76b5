"""The allocation-free apply (coarse_apply_noalloc) against coarse_apply_ws.

Both run the same two-pass 16-bit kernels; the allocation-free entry point
takes the prepared input operands from the library's device scratch array
instead of a caller workspace, so the outputs must agree bit for bit. The
calls run back to back with sizes that shrink and grow again, so a call that
read operands a previous, larger call left in the shared array would differ.
"""
import numpy as np
import pytest
import torch

import workloads as W
from helpers import announce

pytestmark = pytest.mark.gpu


def _noalloc(op, x, y):
    from paper_2409_03904_amd import _lib as L
    from paper_2409_03904_amd import coarse
    lib = L.load()
    L.check(lib.coarse_apply_noalloc(op.geom.c, op.buf.data_ptr(), op.code, x.data_ptr(), y.data_ptr(),
                                     x.shape[2], L.C64, coarse._stream()))
    return y


def _case(dims, nbasis, nrhs, stencil, dtype, seed):
    """Random (non-Hermitian) complex64 links packed as `dtype` and a random
    complex64 input, drawn on the device from a seeded generator."""
    from paper_2409_03904_amd import coarse
    geom = coarse.Geometry(dims, nbasis, W.stencil(stencil))
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    links = 0.1 * torch.randn(geom.link_shape(), dtype=torch.complex64, device="cuda", generator=g)
    op = coarse.pack(links, geom, dtype)
    del links
    x = torch.randn(geom.vector_shape(nrhs), dtype=torch.complex64, device="cuda", generator=g)
    return op, x


CASES = [
    # 8^4, nbasis 64, nrhs 32, 81 points: 32.5 MiB of operands (the largest workload, within the 40 MiB limit)
    ((8, 8, 8, 8), 64, 32, "81pt", "fp16", 11),
    # a smaller second call: 4^4, nbasis 32, nrhs 16, 9 points, BF16
    ((4, 4, 4, 4), 32, 16, "9pt", "bf16", 12),
    # ragged: odd extents, nbasis 16, nrhs 5 (one partial column tile), FP16
    ((3, 2, 5, 1), 16, 5, "9pt", "fp16", 13),
    # larger again, BF16 at 81 points
    ((4, 4, 4, 6), 64, 24, "81pt", "bf16", 14),
    # complex64 links: no scratch involved, same kernels as coarse_apply
    ((4, 4, 4, 4), 32, 16, "9pt", "c64", 15),
]


def test_noalloc_matches_workspace_apply():
    from paper_2409_03904_amd import coarse
    for dims, nb, nr, st, dt, seed in CASES:
        announce("noalloc", dims, nb, nr, st, dt)
        op, x = _case(dims, nb, nr, st, dt, seed)
        ref = torch.empty_like(x)
        nbytes = max(coarse.apply_workspace_bytes(op, nr), 1)
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        coarse.apply(op, x, out=ref, workspace=ws)
        y1 = _noalloc(op, x, torch.full_like(x, float("nan")))
        y2 = _noalloc(op, x, torch.full_like(x, float("nan")))
        torch.cuda.synchronize()
        assert torch.isfinite(torch.view_as_real(ref)).all()
        assert torch.equal(torch.view_as_real(y1), torch.view_as_real(ref)), (dims, nb, nr, st, dt)
        assert torch.equal(torch.view_as_real(y2), torch.view_as_real(ref)), (dims, nb, nr, st, dt)
        del op, x, ref, ws, y1, y2
        torch.cuda.empty_cache()


def test_noalloc_rejects_oversize():
    from paper_2409_03904_amd import _lib as L
    from paper_2409_03904_amd import coarse
    announce("noalloc oversize rejection")
    # 10^4 sites at nbasis 64, nrhs 32: 160 MiB of operands, beyond the 72 MiB array
    geom = coarse.Geometry((10, 10, 10, 10), 64, W.stencil("9pt"))
    lib = L.load()
    x = torch.zeros(1, dtype=torch.complex64, device="cuda")
    y = torch.zeros(1, dtype=torch.complex64, device="cuda")
    p = torch.zeros(1, dtype=torch.uint8, device="cuda")
    rc = lib.coarse_apply_noalloc(geom.c, p.data_ptr(), L.FP16, x.data_ptr(), y.data_ptr(), 32, L.C64,
                                  coarse._stream())
    assert rc == L.CG_WORKSPACE_TOO_SMALL
    assert "allocation-free" in lib.cg_last_error().decode()
