"""torch.autograd Functions over the HIP coarse operator and block-CG solve.

Gradients follow PyTorch's convention for a real loss L of complex inputs
(grad = dL/dRe + i dL/dIm):

* y = M x:     dx = M^H gy (adjoint stencil),  dA_p(x) = gy(x) x(x + delta_p)^H
  (the sum over RHS of outer products, one nbasis x nbasis block per link);
* X = M^{-1} B (M Hermitian positive definite): Lambda = M^{-H} G solved by the
  same block CG (M^H = M), dB = Lambda, dA_p(x) = -Lambda(x) X(x + delta_p)^H;
  with chebyshev=(lo, hi, degree) both solves are Preconditioned BlockCGrQ with
  that stationary Chebyshev preconditioner.

The backward passes call the HIP library only (adjoint apply, link-gradient
kernel, block-CG solve).
"""
from __future__ import annotations

import weakref

import torch

from . import coarse

# The packed operator of the last links tensor seen by CoarseApplyFn, per
# geometry: reused while the same tensor object is passed again unmodified
# (same object, same version counter), repacked otherwise.
_PACK_CACHE: "weakref.WeakKeyDictionary" = weakref.WeakKeyDictionary()


def _packed_for(links: torch.Tensor, geom: coarse.Geometry, vec_dtype: torch.dtype) -> coarse.PackedLinks:
    """Links in the layout of the fastest apply for this shape: the 3M form
    (forward and adjoint on MFMA) for complex64 vectors when nbasis % 16 == 0,
    else complex64."""
    dtype = "c64_3m" if geom.nbasis % 16 == 0 and vec_dtype == torch.complex64 else "c64"
    hit = _PACK_CACHE.get(geom)
    if hit is not None:
        ref, version, packed = hit
        if ref() is links and version == links._version and packed.dtype == dtype:
            return packed
    packed = coarse.pack(links.detach().contiguous(), geom, dtype)
    _PACK_CACHE[geom] = (weakref.ref(links), links._version, packed)
    return packed


class CoarseApplyFn(torch.autograd.Function):
    """y = M(links) x with complex64 links [V, npoint, nb, nb] and x [V, nb, nrhs]."""

    @staticmethod
    def forward(ctx, links, x, geom):
        x_c = x.detach().contiguous()
        packed = _packed_for(links, geom, x_c.dtype)
        y = coarse.apply(packed, x_c)
        ctx.save_for_backward(x_c)
        ctx.packed = packed
        ctx.geom = geom
        return y

    @staticmethod
    def backward(ctx, gy):
        (x,) = ctx.saved_tensors
        gy = gy.contiguous()
        dlinks = dx = None
        if ctx.needs_input_grad[1]:
            dx = coarse.apply_adjoint(ctx.packed, gy)
        if ctx.needs_input_grad[0]:
            dlinks = coarse.link_grad(ctx.geom, gy, x)
        return dlinks, dx, None


class CoarseSolveFn(torch.autograd.Function):
    """X = M(links)^{-1} B for Hermitian positive definite M; B, X complex128."""

    @staticmethod
    def _solve(packed, rhs, params):
        # chebyshev=(lo, hi, degree): Preconditioned BlockCGrQ with that stationary
        # polynomial as preconditioner (the same solution, so the same gradients)
        p = dict(params)
        cheb = p.pop("chebyshev", None)
        if cheb is None:
            return coarse.bcg_solve(packed, rhs, **p)
        lo, hi, order = cheb
        return coarse.pbcg_solve(packed, rhs, lo, hi, order, **p)

    @staticmethod
    def forward(ctx, links, b, geom, params):
        links_c = links.detach().contiguous()
        packed = coarse.pack(links_c, geom, "c64")
        res = CoarseSolveFn._solve(packed, b.detach().contiguous(), params)
        ctx.save_for_backward(res.x)
        ctx.packed = packed
        ctx.geom = geom
        ctx.params = params
        ctx.result = res
        return res.x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        lam = CoarseSolveFn._solve(ctx.packed, gx.contiguous().to(torch.complex128), ctx.params).x
        dlinks = db = None
        if ctx.needs_input_grad[1]:
            db = lam
        if ctx.needs_input_grad[0]:
            dlinks = coarse.link_grad(ctx.geom, lam.to(torch.complex64).contiguous(),
                                      x.to(torch.complex64).contiguous(), alpha=-1.0)
        return dlinks, db, None, None


def coarse_apply(links: torch.Tensor, x: torch.Tensor, geom: coarse.Geometry) -> torch.Tensor:
    return CoarseApplyFn.apply(links, x, geom)


def coarse_solve(links: torch.Tensor, b: torch.Tensor, geom: coarse.Geometry, **params) -> torch.Tensor:
    params = dict(params)
    params.setdefault("tol", 1e-10)
    params.setdefault("inner_tol", 1e-4)
    return CoarseSolveFn.apply(links, b, geom, params)
