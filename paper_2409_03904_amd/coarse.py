"""Python front end of the multi-RHS coarse operator (torch tensors in, torch tensors out).

Every computation runs in the HIP library behind the C ABI; this module only
marshals pointers, shapes and the current HIP stream. PyTorch supplies device
memory and streams.

Layouts (see include/coarse.h): links ``[V, npoint, nbasis, nbasis]`` complex64,
vectors ``[V, nbasis, nrhs]`` complex64 or complex128, site index x0 fastest.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import C64, C128, BF16, FP16, LINK_DTYPES, check


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


class Geometry:
    """A periodic 4D coarse lattice with its stencil (keeps the host offsets alive)."""

    def __init__(self, dims: Sequence[int], nbasis: int, offsets):
        self.dims = tuple(int(d) for d in dims)
        self.nbasis = int(nbasis)
        self.offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int8).reshape(-1, 4))
        self.npoint = int(self.offsets.shape[0])
        self.volume = int(np.prod(self.dims))
        self._c = _lib.CoarseGeom()
        for mu in range(4):
            self._c.dims[mu] = self.dims[mu]
        self._c.nbasis = self.nbasis
        self._c.npoint = self.npoint
        self._c.offsets = self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))

    @property
    def c(self):
        return ctypes.byref(self._c)

    def vector_shape(self, nrhs: int):
        return (self.volume, self.nbasis, int(nrhs))

    def link_shape(self):
        return (self.volume, self.npoint, self.nbasis, self.nbasis)


@dataclass
class PackedLinks:
    geom: Geometry
    dtype: str          # "c64", "c64_3m" (3M-kernel layout), "bf16" or "fp16"
    buf: torch.Tensor   # uint8 device buffer

    @property
    def code(self) -> int:
        return LINK_DTYPES[self.dtype]

    @property
    def nbytes(self) -> int:
        return self.buf.numel()


def packed_bytes(geom: Geometry, dtype: str = "c64") -> int:
    lib = _lib.load()
    out = ctypes.c_size_t()
    check(lib.coarse_packed_bytes(geom.c, LINK_DTYPES[dtype], ctypes.byref(out)))
    return int(out.value)


def pack(links: torch.Tensor, geom: Geometry, dtype: str = "c64") -> PackedLinks:
    """Repack public complex64 links into the kernel layout (quantised for bf16/fp16)."""
    lib = _lib.load()
    if links.dtype != torch.complex64 or not links.is_cuda or not links.is_contiguous():
        raise ValueError("links must be a contiguous complex64 CUDA tensor")
    if tuple(links.shape) != geom.link_shape():
        raise ValueError(f"links shape {tuple(links.shape)} != {geom.link_shape()}")
    buf = torch.empty(packed_bytes(geom, dtype), dtype=torch.uint8, device=links.device)
    check(lib.coarse_pack_links(geom.c, _ptr(links), LINK_DTYPES[dtype], _ptr(buf), _stream()))
    return PackedLinks(geom, dtype, buf)


def pack_adjoint(links: torch.Tensor, geom: Geometry, dtype: str = "c64_3m") -> PackedLinks:
    """M^H as a forward operator: links A_p(x - delta_p)^H at displacements
    -delta_p, packed in `dtype` (the 3M layout by default), so that
    apply(pack_adjoint(links, geom), x) = M^H x with the forward kernels. Holds
    a second packed copy of the links."""
    lib = _lib.load()
    if links.dtype != torch.complex64 or not links.is_cuda or not links.is_contiguous():
        raise ValueError("links must be a contiguous complex64 CUDA tensor")
    if tuple(links.shape) != geom.link_shape():
        raise ValueError(f"links shape {tuple(links.shape)} != {geom.link_shape()}")
    adj = torch.empty_like(links)
    check(lib.coarse_adjoint_links(geom.c, _ptr(links), _ptr(adj), _stream()))
    gneg = Geometry(geom.dims, geom.nbasis, -geom.offsets.astype(np.int16))
    return pack(adj, gneg, dtype)


def _vec_code(x: torch.Tensor) -> int:
    if x.dtype == torch.complex64:
        return C64
    if x.dtype == torch.complex128:
        return C128
    raise ValueError("vectors must be complex64 or complex128")


def _check_vec(x: torch.Tensor, geom: Geometry):
    if not x.is_cuda or not x.is_contiguous():
        raise ValueError("vectors must be contiguous CUDA tensors")
    if x.dim() != 3 or tuple(x.shape[:2]) != (geom.volume, geom.nbasis):
        raise ValueError(f"vector shape {tuple(x.shape)} does not match [V={geom.volume}, nbasis={geom.nbasis}, nrhs]")


def apply_workspace_bytes(packed: PackedLinks, nrhs: int) -> int:
    """Workspace the two-pass 16-bit apply needs (0 for complex64 links)."""
    lib = _lib.load()
    n = ctypes.c_size_t()
    check(lib.coarse_apply_workspace_bytes(packed.geom.c, packed.code, int(nrhs), ctypes.byref(n)))
    return int(n.value)


def apply(packed: PackedLinks, x: torch.Tensor, out: Optional[torch.Tensor] = None,
          workspace: Optional[torch.Tensor] = None, two_pass: bool = True) -> torch.Tensor:
    """y = M x. With 16-bit links the two-pass kernels run (inputs converted to
    16-bit operands once, into `workspace`, allocated here when not given);
    two_pass=False selects the one-pass kernel that needs no workspace."""
    lib = _lib.load()
    _check_vec(x, packed.geom)
    y = torch.empty_like(x) if out is None else out
    nbytes = apply_workspace_bytes(packed, x.shape[2]) if two_pass else 0
    if nbytes == 0:
        check(lib.coarse_apply(packed.geom.c, _ptr(packed.buf), packed.code, _ptr(x), _ptr(y), x.shape[2],
                               _vec_code(x), _stream()))
        return y
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    check(lib.coarse_apply_ws(packed.geom.c, _ptr(packed.buf), packed.code, _ptr(x), _ptr(y), x.shape[2],
                              _vec_code(x), _ptr(workspace), workspace.numel(), _stream()))
    return y


def apply_gram_workspace_bytes(packed: PackedLinks, nrhs: int) -> int:
    """Workspace of apply_gram: split-K partials (+ 16-bit operands)."""
    lib = _lib.load()
    n = ctypes.c_size_t()
    check(lib.coarse_apply_gram_workspace_bytes(packed.geom.c, packed.code, int(nrhs), ctypes.byref(n)))
    return int(n.value)


def apply_gram(packed: PackedLinks, x: torch.Tensor, out: Optional[torch.Tensor] = None,
               workspace: Optional[torch.Tensor] = None):
    """(y, G) with y = M x and G = x^H y (complex64 x; G complex128, nrhs x nrhs),
    the operator application of a BlockCGrQ iteration and its Gram."""
    lib = _lib.load()
    _check_vec(x, packed.geom)
    if x.dtype != torch.complex64:
        raise ValueError("x must be complex64")
    y = torch.empty_like(x) if out is None else out
    nr = x.shape[2]
    g = torch.empty((nr, nr), dtype=torch.complex128, device=x.device)
    nbytes = apply_gram_workspace_bytes(packed, nr)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    check(lib.coarse_apply_gram(packed.geom.c, _ptr(packed.buf), packed.code, _ptr(x), _ptr(y), nr, _ptr(g),
                                _ptr(workspace), workspace.numel(), _stream()))
    return y, g


def chebyshev_coefficients(lo: float, hi: float, order: int) -> np.ndarray:
    """c_0 .. c_order of the Chebyshev interpolant of 1/x on [lo, hi] (computed by the library)."""
    lib = _lib.load()
    c = np.zeros(int(order) + 1, dtype=np.float64)
    check(lib.coarse_chebyshev_coefficients(float(lo), float(hi), int(order),
                                            c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return c


def chebyshev_workspace_bytes(packed: PackedLinks, nrhs: int) -> int:
    lib = _lib.load()
    out = ctypes.c_size_t()
    check(lib.coarse_chebyshev_workspace_bytes(packed.geom.c, packed.code, int(nrhs), ctypes.byref(out)))
    return int(out.value)


def chebyshev_apply(packed: PackedLinks, x: torch.Tensor, lo: float, hi: float, order: int,
                    out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """y = P(M) x, the stationary Chebyshev approximation to M^{-1} of degree
    `order` on [lo, hi] (complex64 vectors; any link type)."""
    lib = _lib.load()
    _check_vec(x, packed.geom)
    if x.dtype != torch.complex64:
        raise ValueError("x must be complex64")
    y = torch.empty_like(x) if out is None else out
    need = chebyshev_workspace_bytes(packed, x.shape[2])
    if workspace is None and int(order) > 0:
        workspace = torch.empty(need, dtype=torch.uint8, device=x.device)
    wp, wb = (_ptr(workspace), workspace.numel()) if workspace is not None else (None, 0)
    check(lib.coarse_chebyshev_apply(packed.geom.c, _ptr(packed.buf), packed.code, _ptr(x), _ptr(y), x.shape[2],
                                     float(lo), float(hi), int(order), wp, wb, _stream()))
    return y


def _check_basis(v: torch.Tensor, lam: torch.Tensor, geom: Geometry):
    if v.dtype != torch.complex64 or v.dim() != 3 or tuple(v.shape[:2]) != (geom.volume, geom.nbasis) \
            or not v.is_contiguous():
        raise ValueError("v must be a contiguous complex64 [V, nbasis, nev] tensor")
    if lam.dtype != torch.float64 or lam.numel() != v.shape[2] or not lam.is_contiguous() or lam.device != v.device:
        raise ValueError("lam must hold nev float64 values on the device of v")


def deflation_workspace_bytes(geom: Geometry, nev: int, nrhs: int) -> int:
    lib = _lib.load()
    out = ctypes.c_size_t()
    check(lib.coarse_deflation_workspace_bytes(geom.c, int(nev), int(nrhs), ctypes.byref(out)))
    return int(out.value)


def deflate(v: torch.Tensor, lam: torch.Tensor, x: torch.Tensor, geom: Geometry, want_perp: bool = False,
            workspace: Optional[torch.Tensor] = None):
    """Defl(x) = V diag(1/lam) V^H x for complex64 blocks x [V, nbasis, nrhs]
    and vectors v [V, nbasis, nev]; with want_perp also x - V V^H x."""
    lib = _lib.load()
    _check_basis(v, lam, geom)
    _check_vec(x, geom)
    if x.dtype != torch.complex64:
        raise ValueError("x must be complex64")
    nev, nrhs = v.shape[2], x.shape[2]
    y = torch.empty_like(x)
    xp = torch.empty_like(x) if want_perp else None
    need = deflation_workspace_bytes(geom, nev, nrhs)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=x.device)
    check(lib.coarse_deflate(geom.c, _ptr(v), nev, _ptr(lam), _ptr(x), _ptr(y), _ptr(xp) if xp is not None else None,
                             nrhs, _ptr(workspace), workspace.numel(), _stream()))
    return (y, xp) if want_perp else y


def block_lanczos(packed: PackedLinks, x0: torch.Tensor, steps: int, nev: int,
                  workspace: Optional[torch.Tensor] = None):
    """The nev lowest Ritz pairs of M from `steps` steps of block Lanczos with
    full reorthogonalisation started at x0 [V, nbasis, block] (complex64).
    Returns (v [V, nbasis, nev] complex64 on the device, lam (numpy, nev),
    residual norms (numpy, nev), basis size used)."""
    lib = _lib.load()
    geom = packed.geom
    _check_vec(x0, geom)
    if x0.dtype != torch.complex64:
        raise ValueError("x0 must be complex64")
    b = x0.shape[2]
    need = ctypes.c_size_t()
    check(lib.coarse_block_lanczos_workspace_bytes(geom.c, packed.code, b, int(steps), int(nev), ctypes.byref(need)))
    if workspace is None or workspace.numel() < need.value:
        workspace = torch.empty(need.value, dtype=torch.uint8, device=x0.device)
    v = torch.empty((geom.volume, geom.nbasis, int(nev)), dtype=torch.complex64, device=x0.device)
    lam = (ctypes.c_double * int(nev))()
    res = (ctypes.c_double * int(nev))()
    k = ctypes.c_int32()
    check(lib.coarse_block_lanczos(geom.c, _ptr(packed.buf), packed.code, _ptr(x0), b, int(steps), int(nev), _ptr(v),
                                   lam, res, ctypes.byref(k), _ptr(workspace), workspace.numel(), _stream()))
    return v, np.array(lam[:]), np.array(res[:]), int(k.value)


def deflated_chebyshev_apply(packed: PackedLinks, v: torch.Tensor, lam: torch.Tensor, x: torch.Tensor, lo: float,
                             hi: float, order: int, out: Optional[torch.Tensor] = None,
                             workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """y = Defl(x) + P(M) (x - V V^H x): the deflated stationary coarse solve."""
    lib = _lib.load()
    geom = packed.geom
    _check_basis(v, lam, geom)
    _check_vec(x, geom)
    if x.dtype != torch.complex64:
        raise ValueError("x must be complex64")
    nev, nrhs = v.shape[2], x.shape[2]
    y = torch.empty_like(x) if out is None else out
    need = ctypes.c_size_t()
    check(lib.coarse_deflated_chebyshev_workspace_bytes(geom.c, packed.code, nev, nrhs, ctypes.byref(need)))
    if workspace is None or workspace.numel() < need.value:
        workspace = torch.empty(need.value, dtype=torch.uint8, device=x.device)
    check(lib.coarse_deflated_chebyshev_apply(geom.c, _ptr(packed.buf), packed.code, _ptr(v), nev, _ptr(lam), _ptr(x),
                                              _ptr(y), nrhs, float(lo), float(hi), int(order), _ptr(workspace),
                                              workspace.numel(), _stream()))
    return y


def _check_block(basis: torch.Tensor, geom: Geometry):
    if basis.dtype != torch.complex64 or basis.dim() != 3 or basis.shape[0] != geom.volume \
            or basis.shape[2] != geom.nbasis or not basis.is_contiguous():
        raise ValueError("basis must be a contiguous complex64 [V, vblock, nbasis] tensor")


def block_project(basis: torch.Tensor, fine: torch.Tensor, geom: Geometry,
                  out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """C(x_c) = B(x_c)^H F(x_c) per coarse site: basis [V, vblock, nbasis],
    fine [V, vblock, nrhs] (block order) -> coarse [V, nbasis, nrhs], complex64."""
    lib = _lib.load()
    _check_block(basis, geom)
    if fine.dtype != torch.complex64 or fine.dim() != 3 or fine.shape[:2] != basis.shape[:2] \
            or not fine.is_contiguous():
        raise ValueError("fine must be a contiguous complex64 [V, vblock, nrhs] tensor")
    nrhs = fine.shape[2]
    y = torch.empty((geom.volume, geom.nbasis, nrhs), dtype=torch.complex64, device=fine.device) if out is None \
        else out
    check(lib.coarse_block_project(geom.c, basis.shape[1], _ptr(basis), _ptr(fine), _ptr(y), nrhs, _stream()))
    return y


def block_promote(basis: torch.Tensor, coarse_vec: torch.Tensor, geom: Geometry,
                  out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """F(x_c) = B(x_c) C(x_c) per coarse site: coarse [V, nbasis, nrhs] ->
    fine [V, vblock, nrhs], complex64."""
    lib = _lib.load()
    _check_block(basis, geom)
    _check_vec(coarse_vec, geom)
    if coarse_vec.dtype != torch.complex64:
        raise ValueError("coarse vector must be complex64")
    nrhs = coarse_vec.shape[2]
    y = torch.empty((geom.volume, basis.shape[1], nrhs), dtype=torch.complex64, device=coarse_vec.device) \
        if out is None else out
    check(lib.coarse_block_promote(geom.c, basis.shape[1], _ptr(basis), _ptr(coarse_vec), _ptr(y), nrhs, _stream()))
    return y


def apply_adjoint(packed: PackedLinks, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """y = M^H x."""
    lib = _lib.load()
    _check_vec(x, packed.geom)
    y = torch.empty_like(x) if out is None else out
    check(lib.coarse_apply_adjoint(packed.geom.c, _ptr(packed.buf), packed.code, _ptr(x), _ptr(y), x.shape[2],
                                   _vec_code(x), _stream()))
    return y


def apply_generic(packed: PackedLinks, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """y = M x through the VALU kernel (cross-check of the MFMA kernels)."""
    lib = _lib.load()
    _check_vec(x, packed.geom)
    y = torch.empty_like(x) if out is None else out
    check(lib.coarse_apply_generic(packed.geom.c, _ptr(packed.buf), packed.code, _ptr(x), _ptr(y), x.shape[2],
                                   _vec_code(x), _stream()))
    return y


def apply_adjoint_generic(packed: PackedLinks, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """y = M^H x through the VALU kernel (cross-check of the MFMA adjoint)."""
    lib = _lib.load()
    _check_vec(x, packed.geom)
    y = torch.empty_like(x) if out is None else out
    check(lib.coarse_apply_adjoint_generic(packed.geom.c, _ptr(packed.buf), packed.code, _ptr(x), _ptr(y),
                                           x.shape[2], _vec_code(x), _stream()))
    return y


def link_grad(geom: Geometry, gy: torch.Tensor, x: torch.Tensor, alpha: float = 1.0,
              out: Optional[torch.Tensor] = None, accumulate: Optional[bool] = None) -> torch.Tensor:
    """dlinks[x][p] (+)= alpha * gy(x) x(x+delta_p)^H (by default accumulates
    into `out` when given; accumulate=False overwrites it)."""
    lib = _lib.load()
    _check_vec(gy, geom)
    _check_vec(x, geom)
    if gy.dtype != torch.complex64 or x.dtype != torch.complex64:
        raise ValueError("link_grad takes complex64 vectors")
    acc = (out is not None) if accumulate is None else bool(accumulate)
    if acc and out is None:
        raise ValueError("accumulate=True needs `out`")
    if out is None:
        out = torch.empty(geom.link_shape(), dtype=torch.complex64, device=x.device)
    check(lib.coarse_link_grad(geom.c, _ptr(gy), _ptr(x), _ptr(out), float(alpha), int(acc), x.shape[2],
                               _stream()))
    return out


@dataclass
class SolveResult:
    x: torch.Tensor
    status: int
    cycles: int
    iterations: int
    relres: np.ndarray
    relres_max: float
    seconds_total: float
    seconds_inner: float
    seconds_outer: float


def solve_params(tol=1e-8, inner_tol=1e-3, max_outer=30, max_inner=2000, check_every=8, use_graph=True,
                 outer_dtype=C64):
    p = _lib.SolveParams()
    p.tol, p.inner_tol = float(tol), float(inner_tol)
    p.max_outer, p.max_inner = int(max_outer), int(max_inner)
    p.check_every, p.use_graph = int(check_every), int(bool(use_graph))
    p.outer_dtype = int(outer_dtype)
    return p


def _outer_code(op: "PackedLinks") -> int:
    """Link type of an outer operator: complex64 links in the 4M (c64) or the
    3M (c64_3m) layout; the double residual runs in that form."""
    if op.dtype not in ("c64", "c64_3m"):
        raise ValueError("the outer operator must be packed as c64 or c64_3m")
    return op.code


def workspace_bytes(geom: Geometry, nrhs: int, params=None) -> int:
    lib = _lib.load()
    params = params or solve_params()
    out = ctypes.c_size_t()
    check(lib.coarse_bcg_workspace_bytes(geom.c, int(nrhs), ctypes.byref(params), ctypes.byref(out)))
    return int(out.value)


def bcg_solve(outer: PackedLinks, b: torch.Tensor, x0: Optional[torch.Tensor] = None,
              inner: Optional[PackedLinks] = None, workspace: Optional[torch.Tensor] = None,
              raise_on_failure: bool = True, **kw) -> SolveResult:
    """Solve M X = B (M Hermitian positive definite) by double precision defect
    correction around BlockCGrQ in single / 16-bit-link precision."""
    lib = _lib.load()
    geom = outer.geom
    code = _outer_code(outer)
    _check_vec(b, geom)
    if b.dtype != torch.complex128:
        raise ValueError("b must be complex128")
    nrhs = b.shape[2]
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    params = solve_params(outer_dtype=code, **kw)
    need = workspace_bytes(geom, nrhs, params)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=b.device)
    stats = _lib.SolveStats()
    inner_ptr = _ptr(inner.buf) if inner is not None else None
    inner_code = inner.code if inner is not None else code
    rc = lib.coarse_bcg_solve(geom.c, _ptr(outer.buf), inner_ptr, inner_code, _ptr(b), _ptr(x), nrhs,
                              ctypes.byref(params), ctypes.byref(stats), _ptr(workspace), workspace.numel(),
                              _stream())
    if raise_on_failure:
        check(rc)
    res = SolveResult(x=x, status=rc, cycles=stats.cycles, iterations=stats.iterations,
                      relres=np.array(stats.relres[:nrhs]), relres_max=stats.relres_max,
                      seconds_total=stats.seconds_total, seconds_inner=stats.seconds_inner,
                      seconds_outer=stats.seconds_outer)
    return res


def pbcg_workspace_bytes(geom: Geometry, nrhs: int, lo: float, hi: float, order: int, params=None) -> int:
    lib = _lib.load()
    params = params or solve_params()
    prec = _lib.ChebPrec(float(lo), float(hi), int(order))
    out = ctypes.c_size_t()
    check(lib.coarse_pbcg_workspace_bytes(geom.c, int(nrhs), ctypes.byref(params), ctypes.byref(prec),
                                          ctypes.byref(out)))
    return int(out.value)


def pbcg_solve(outer: PackedLinks, b: torch.Tensor, lo: float, hi: float, order: int,
               x0: Optional[torch.Tensor] = None, inner: Optional[PackedLinks] = None,
               workspace: Optional[torch.Tensor] = None, raise_on_failure: bool = True, **kw) -> SolveResult:
    """Solve M X = B as `bcg_solve` does, with Preconditioned BlockCGrQ as the
    inner iteration and the degree-`order` Chebyshev approximation to 1/x on
    [lo, hi] of the inner operator as the stationary preconditioner. The inner
    tolerance is relative to the start of each cycle, in the preconditioner's
    norm."""
    lib = _lib.load()
    geom = outer.geom
    code = _outer_code(outer)
    _check_vec(b, geom)
    if b.dtype != torch.complex128:
        raise ValueError("b must be complex128")
    nrhs = b.shape[2]
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    params = solve_params(outer_dtype=code, **kw)
    prec = _lib.ChebPrec(float(lo), float(hi), int(order))
    need = pbcg_workspace_bytes(geom, nrhs, lo, hi, order, params)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=b.device)
    stats = _lib.SolveStats()
    inner_ptr = _ptr(inner.buf) if inner is not None else None
    inner_code = inner.code if inner is not None else code
    rc = lib.coarse_pbcg_solve(geom.c, _ptr(outer.buf), inner_ptr, inner_code, _ptr(b), _ptr(x), nrhs,
                               ctypes.byref(params), ctypes.byref(prec), ctypes.byref(stats), _ptr(workspace),
                               workspace.numel(), _stream())
    if raise_on_failure:
        check(rc)
    return SolveResult(x=x, status=rc, cycles=stats.cycles, iterations=stats.iterations,
                       relres=np.array(stats.relres[:nrhs]), relres_max=stats.relres_max,
                       seconds_total=stats.seconds_total, seconds_inner=stats.seconds_inner,
                       seconds_outer=stats.seconds_outer)


def bcg_solve_batched(outers, bs, x0s=None, inners=None, workspace: Optional[torch.Tensor] = None,
                      raise_on_failure: bool = True, **kw):
    """Solve M_k X_k = B_k for several independent systems at once (one graph
    with one branch per system for the inner iterations); returns a list of
    SolveResult. `outers`, `bs` (and optional `x0s`, `inners`) are lists."""
    lib = _lib.load()
    n = len(outers)
    if n == 0 or len(bs) != n:
        raise ValueError("need matching, non-empty lists of operators and right-hand sides")
    x0s = [None] * n if x0s is None else list(x0s)
    inners = [None] * n if inners is None else list(inners)
    arr = (_lib.CoarseSolveSystem * n)()
    xs = []
    codes = {_outer_code(op) for op in outers}
    if len(codes) != 1:
        raise ValueError("the outer operators of one batch must share their link type")
    code = codes.pop()
    for k in range(n):
        op, b = outers[k], bs[k]
        _check_vec(b, op.geom)
        if b.dtype != torch.complex128:
            raise ValueError("b must be complex128")
        xs.append(torch.zeros_like(b) if x0s[k] is None else x0s[k].clone())
        arr[k].geom = op.geom._c
        arr[k].nrhs = b.shape[2]
        arr[k].packed_outer = _ptr(op.buf)
        arr[k].packed_inner = _ptr(inners[k].buf) if inners[k] is not None else None
        arr[k].inner_dtype = inners[k].code if inners[k] is not None else code
        arr[k].b = _ptr(b)
        arr[k].x = _ptr(xs[k])
    params = solve_params(outer_dtype=code, **kw)
    need = ctypes.c_size_t()
    check(lib.coarse_bcg_batched_workspace_bytes(arr, n, ctypes.byref(params), ctypes.byref(need)))
    if workspace is None or workspace.numel() < need.value:
        workspace = torch.empty(max(need.value, 1), dtype=torch.uint8, device=bs[0].device)
    stats = (_lib.SolveStats * n)()
    rc = lib.coarse_bcg_solve_batched(arr, n, ctypes.byref(params), stats, _ptr(workspace), workspace.numel(),
                                      _stream())
    if raise_on_failure:
        check(rc)
    out = []
    for k in range(n):
        st = stats[k]
        nr = bs[k].shape[2]
        out.append(SolveResult(x=xs[k], status=st.status, cycles=st.cycles, iterations=st.iterations,
                               relres=np.array(st.relres[:nr]), relres_max=st.relres_max,
                               seconds_total=st.seconds_total, seconds_inner=st.seconds_inner,
                               seconds_outer=st.seconds_outer))
    return out


# ---------------------------------------------------------------------------
# Tuning and batches of systems
# ---------------------------------------------------------------------------

def tune_apply(packed: PackedLinks, x: torch.Tensor, reps: int = 20):
    """Time every apply variant for this shape (y scratch allocated here), keep the
    fastest for later calls; returns (variant, microseconds)."""
    lib = _lib.load()
    _check_vec(x, packed.geom)
    y = torch.empty_like(x)
    v = ctypes.c_int32()
    us = ctypes.c_float()
    check(lib.coarse_tune_apply(packed.geom.c, _ptr(packed.buf), packed.code, _ptr(x), _ptr(y), x.shape[2],
                                _vec_code(x), int(reps), _stream(), ctypes.byref(v), ctypes.byref(us)))
    return int(v.value), float(us.value)


def max_apply_variant(nbasis: int) -> int:
    """Largest apply variant index for this nbasis (variants are 0 .. this)."""
    n = _lib.load().coarse_apply_variant_count(int(nbasis))
    if n < 1:
        check(n)
    return n - 1


def set_apply_variant(geom: Geometry, nrhs: int, variant: int, link_dtype: str = "c64", vec_dtype=C64):
    """Pin (variant >= 0) or clear (variant < 0) the apply variant of a shape."""
    lib = _lib.load()
    check(lib.coarse_set_apply_variant(geom.nbasis, int(nrhs), geom.npoint, LINK_DTYPES[link_dtype], vec_dtype,
                                       int(variant)))


class BatchedApply:
    """y_i = M_i x_i for several systems: one persistent launch over all of
    them, or (when tune() finds it faster, e.g. for a batch dominated by a few
    large systems whose own tuned kernels run at a higher occupancy) the tuned
    single-system launches one after another."""

    def __init__(self, ops, xs, ys):
        lib = _lib.load()
        if not (len(ops) == len(xs) == len(ys)) or not ops:
            raise ValueError("need matching, non-empty lists of operators and vectors")
        self._keep = (list(ops), list(xs), list(ys))
        self.arr = (_lib.CoarseSystem * len(ops))()
        for k, (op, x, y) in enumerate(zip(ops, xs, ys)):
            if op.dtype != "c64" or x.dtype != torch.complex64 or y.dtype != torch.complex64:
                raise ValueError("batched apply takes complex64 links and vectors")
            _check_vec(x, op.geom)
            _check_vec(y, op.geom)
            self.arr[k].geom = op.geom._c
            self.arr[k].nrhs = x.shape[2]
            self.arr[k].packed = _ptr(op.buf)
            self.arr[k].x = _ptr(x)
            self.arr[k].y = _ptr(y)
        need = ctypes.c_size_t()
        check(lib.coarse_batched_workspace_bytes(self.arr, len(ops), ctypes.byref(need)))
        self.ws = torch.empty(need.value, dtype=torch.uint8, device=xs[0].device)
        self.mode = "persistent"

    def persistent(self):
        lib = _lib.load()
        check(lib.coarse_apply_batched(self.arr, len(self.arr), _ptr(self.ws), self.ws.numel(), _stream()))

    def separate(self):
        for op, x, y in zip(*self._keep):
            apply(op, x, out=y)

    def __call__(self):
        if self.mode == "persistent":
            self.persistent()
        else:
            self.separate()

    @staticmethod
    def set_occupancy(wg_per_cu: int) -> int:
        """Workgroups per CU of the persistent grid (0 = query)."""
        return int(_lib.load().coarse_batched_set_occupancy(int(wg_per_cu)))

    def _time(self, fn, reps):
        fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / reps

    def tune(self, reps: int = 20, candidates=(1, 2, 3, 4, 6, 8), compare_separate: bool = True):
        """Pick the persistent-grid occupancy by timing each candidate and, with
        compare_separate, the launch mode (persistent vs the tuned single-system
        launches); returns {occupancy or "separate": us}."""
        times = {}
        for occ in candidates:
            self.set_occupancy(occ)
            times[occ] = self._time(self.persistent, reps)
        best = min(times, key=times.get)
        self.set_occupancy(best)
        self.mode = "persistent"
        if compare_separate:
            for op, x, y in zip(*self._keep):
                tune_apply(op, x, reps=max(3, reps // 4))
            times["separate"] = self._time(self.separate, reps)
            if times["separate"] < times[best]:
                self.mode = "separate"
        return times
