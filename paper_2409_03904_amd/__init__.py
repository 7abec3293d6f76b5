"""Multi-RHS multigrid coarse operator and block-CG coarse solve for MI355X (gfx950).

The compute path is the HIP library ``libcoarse.so`` (C ABI in include/coarse.h);
``coarse`` and ``autograd`` are thin torch front ends over it.
"""
from . import _lib  # noqa: F401

__all__ = ["coarse", "autograd", "build"]
