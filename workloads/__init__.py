"""Seeded synthetic inputs for the multi-RHS coarse operator and its block solve.

This module is shared by the oracle, the tests and the benchmark. It holds
shapes, stencil offset lists and random draws only; it never applies the
operator, so neither side of a parity test can inherit the other's arithmetic.

Conventions (the paper's multi-RHS coarse operator, Sec. 2.6):

* a coarse lattice with extents ``dims = (L0, L1, L2, L3)``; the site index is
  ``s = x0 + L0*(x1 + L1*(x2 + L2*x3))`` (x0 fastest), periodic boundaries;
* ``links[s, p]`` is the ``nbasis x nbasis`` complex matrix ``A_p(x)``
  (row-major), for the stencil point ``p`` with displacement ``offsets[p]``;
* a multi-RHS vector is ``[V, nbasis, nrhs]``: an ``nbasis x nrhs`` block per
  site, the right-hand-side index being the extra "fifth dimension" of
  Sec. 2 (the RHS treated as a fictitious lattice direction).

The synthetic operator follows the construction the workloads ask for:
i.i.d. complex Gaussian off-diagonal links with the Hermitian pairing
``A_{-p}(x+delta_p) = A_p(x)^H`` and a self term ``(G + G^H)/2 + s*I``, which
makes the operator Hermitian positive definite once ``s`` exceeds
``-lambda_min`` of the unshifted operator. The shifts that target a condition
number are not computed here (that needs the operator); they are stored in
``shifts.json`` next to this file, written by the oracle's script.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

SEED_BASE = 240903904
SIGMA = 0.1
SELF_CANONICAL = 40  # canonical index of the zero displacement


def canonical_index(delta: Sequence[int]) -> int:
    """Index of a displacement in the 3^4 hypercube {-1,0,1}^4, x0 fastest."""
    return int(sum((3 ** mu) * (int(d) + 1) for mu, d in enumerate(delta)))


def _from_canonical(c: int) -> Tuple[int, int, int, int]:
    out = []
    for _ in range(4):
        out.append(c % 3 - 1)
        c //= 3
    return tuple(out)  # type: ignore[return-value]


def stencil(kind: str) -> np.ndarray:
    """Offset list ``[Np, 4]`` (int8).

    ``"9pt"``: self, +e0..+e3, -e0..-e3 (a one-hop coarse operator).
    ``"81pt"``: the full {-1,0,1}^4 hypercube in canonical order (the general
    coarse stencil of Sec. 2.6 for coarsened 2- and 4-hop operators).
    ``"self"``: the zero displacement only.
    """
    if kind == "9pt":
        offs = [(0, 0, 0, 0)]
        for mu in range(4):
            e = [0, 0, 0, 0]
            e[mu] = 1
            offs.append(tuple(e))
        for mu in range(4):
            e = [0, 0, 0, 0]
            e[mu] = -1
            offs.append(tuple(e))
    elif kind == "81pt":
        offs = [_from_canonical(c) for c in range(81)]
    elif kind == "self":
        offs = [(0, 0, 0, 0)]
    else:
        raise ValueError(f"unknown stencil kind {kind!r}")
    return np.asarray(offs, dtype=np.int8)


def volume(dims: Sequence[int]) -> int:
    return int(np.prod([int(d) for d in dims]))


def _displaced_sites(dims: Sequence[int], delta: Sequence[int]) -> np.ndarray:
    """Site index of (x + delta) mod L for every site x (x0 fastest)."""
    L = [int(d) for d in dims]
    # grid indexed [x3, x2, x1, x0] so that ravel() walks x0 fastest
    g = np.arange(volume(L)).reshape(L[3], L[2], L[1], L[0])
    # value at x must be the index of x + delta: roll by -delta
    for mu in range(4):
        axis = 3 - mu
        g = np.roll(g, -int(delta[mu]), axis=axis)
    return g.reshape(-1)


def _cgauss(rng: np.random.Generator, shape, sigma: float) -> np.ndarray:
    """Complex Gaussian with E|z|^2 = sigma^2: all real parts, then all imaginary parts."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) * (sigma / math.sqrt(2.0))


def hermitian_links(rng: np.random.Generator, dims: Sequence[int], nbasis: int,
                    offsets: np.ndarray, shift: float, sigma: float = SIGMA) -> np.ndarray:
    """Links ``[V, Np, nb, nb]`` complex64 of a Hermitian coarse operator.

    Draw order: for every displacement of the positive half (canonical index
    above the self index), in canonical order, one CN(0, sigma^2) block per
    site; then the self-term Gaussian G. Each drawn block is rounded to
    complex64 first, and its mirror ``A_{-p}(x+delta_p)`` is the conjugate
    transpose of the rounded block, so the complex64 operator itself is
    exactly Hermitian. ``A_0 = (G + G^H)/2 + shift*I``.
    """
    offsets = np.asarray(offsets, dtype=np.int64)
    V = volume(dims)
    Np = offsets.shape[0]
    canon = {canonical_index(o): p for p, o in enumerate(offsets)}
    if len(canon) != Np:
        raise ValueError("offsets must be unique")
    for c in canon:
        if (80 - c) not in canon:
            raise ValueError("a Hermitian operator needs a stencil closed under negation")
    if SELF_CANONICAL not in canon:
        raise ValueError("a Hermitian positive definite operator needs the self point")
    links = np.zeros((V, Np, nbasis, nbasis), dtype=np.complex64)
    for c in sorted(canon):
        if c <= SELF_CANONICAL:
            continue
        p = canon[c]
        q = canon[80 - c]
        a = _cgauss(rng, (V, nbasis, nbasis), sigma).astype(np.complex64)
        links[:, p] = a
        dst = _displaced_sites(dims, offsets[p])
        links[dst, q] = np.conj(np.transpose(a, (0, 2, 1)))
        del a
    g = _cgauss(rng, (V, nbasis, nbasis), sigma)
    a0 = 0.5 * (g + np.conj(np.transpose(g, (0, 2, 1))))
    a0 = a0 + shift * np.eye(nbasis)[None, :, :]
    links[:, canon[SELF_CANONICAL]] = a0.astype(np.complex64)
    return links


def gaussian_links(rng: np.random.Generator, dims: Sequence[int], nbasis: int,
                   npoint: int, sigma: float = SIGMA) -> np.ndarray:
    """I.i.d. (non-Hermitian) CN(0, sigma^2) links, complex64."""
    V = volume(dims)
    return _cgauss(rng, (V, npoint, nbasis, nbasis), sigma).astype(np.complex64)


def gaussian_vectors(rng: np.random.Generator, dims: Sequence[int], nbasis: int,
                     nrhs: int, dtype=np.complex64) -> np.ndarray:
    """I.i.d. CN(0, 1) multi-RHS vector ``[V, nb, nrhs]``."""
    V = volume(dims)
    return _cgauss(rng, (V, nbasis, nrhs), 1.0).astype(dtype)


def integer_links(rng: np.random.Generator, dims: Sequence[int], nbasis: int,
                  npoint: int, lo: int = -2, hi: int = 2) -> np.ndarray:
    """Links with entries in {lo..hi} + i{lo..hi}: every low-precision product is exact."""
    V = volume(dims)
    re = rng.integers(lo, hi + 1, size=(V, npoint, nbasis, nbasis))
    im = rng.integers(lo, hi + 1, size=(V, npoint, nbasis, nbasis))
    return (re + 1j * im).astype(np.complex64)


def integer_vectors(rng: np.random.Generator, dims: Sequence[int], nbasis: int,
                    nrhs: int, lo: int = -2, hi: int = 2) -> np.ndarray:
    V = volume(dims)
    re = rng.integers(lo, hi + 1, size=(V, nbasis, nrhs))
    im = rng.integers(lo, hi + 1, size=(V, nbasis, nrhs))
    return (re + 1j * im).astype(np.complex64)


# --------------------------------------------------------------------------
# Workload registry
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class System:
    """One coarse system: lattice, basis size, number of RHS, stencil, spectrum target."""
    name: str
    dims: Tuple[int, int, int, int]
    nbasis: int
    nrhs: int
    stencil: str
    kappa: Optional[float]        # target condition number (None: explicit shift)
    shift: Optional[float] = None  # explicit shift (used when kappa is None)
    tol: float = 1e-8
    seed_index: int = 0

    @property
    def volume(self) -> int:
        return volume(self.dims)

    @property
    def npoint(self) -> int:
        return int(stencil(self.stencil).shape[0])

    @property
    def seed(self) -> int:
        return SEED_BASE + self.seed_index

    def offsets(self) -> np.ndarray:
        return stencil(self.stencil)

    def link_bytes_c64(self) -> int:
        return self.volume * self.npoint * self.nbasis * self.nbasis * 8

    def link_bytes_lowp(self) -> int:
        """16-bit link storage: two 16-bit components per entry for every
        non-self point, the self block in complex64, one float32 scale per
        (site, point)."""
        return self.volume * ((self.npoint - 1) * self.nbasis * self.nbasis * 4
                              + self.nbasis * self.nbasis * 8 + self.npoint * 4)

    def vector_bytes_c64(self) -> int:
        return self.volume * self.nbasis * self.nrhs * 8

    def apply_flops(self) -> int:
        """Useful flops of one apply, 8 real flops per complex multiply-add."""
        return 8 * self.volume * self.npoint * self.nbasis * self.nbasis * self.nrhs


# The five workloads: a small parity case, the FP32 production shape, the
# precision case with the 81-point stencil, six uneven systems for batching,
# and the differentiation case (production shape plus a tiny FD instance).
C1 = System("c1", (4, 4, 4, 4), 8, 4, "9pt", kappa=None, shift=4.0, tol=1e-10, seed_index=1)
C2 = System("c2", (8, 8, 8, 8), 32, 16, "9pt", kappa=1e3, tol=1e-8, seed_index=2)
C3 = System("c3", (8, 8, 8, 8), 64, 32, "81pt", kappa=1e4, tol=1e-8, seed_index=3)
_C4_SHAPES = [(4, 4, 4, 4), (6, 6, 6, 6), (8, 8, 8, 8), (4, 4, 4, 8), (6, 6, 6, 12), (8, 8, 8, 16)]
C4 = tuple(
    System(f"c4.{i}", _C4_SHAPES[i], [24, 32, 48][i % 3], [4, 8, 16, 32][i % 4], "9pt",
           kappa=1e3, tol=1e-8, seed_index=40 + i)
    for i in range(6)
)
C5 = System("c5", (8, 8, 8, 8), 32, 16, "9pt", kappa=1e3, tol=1e-8, seed_index=5)
C5_FD = System("c5.fd", (2, 2, 2, 2), 4, 2, "9pt", kappa=None, shift=2.0, tol=1e-10, seed_index=50)

REGISTRY: Dict[str, System] = {s.name: s for s in (C1, C2, C3, C5, C5_FD) + C4}

_SHIFTS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "shifts.json")


def stored_shifts() -> Dict[str, dict]:
    if not os.path.exists(_SHIFTS_PATH):
        return {}
    with open(_SHIFTS_PATH) as f:
        return json.load(f)


def shift_for(system: System) -> float:
    """Diagonal shift of the self term: explicit, or the stored kappa-targeting value."""
    if system.kappa is None:
        return float(system.shift)
    table = stored_shifts()
    if system.name not in table:
        raise KeyError(f"no stored shift for {system.name}; run oracle/make_shifts.py")
    return float(table[system.name]["shift"])


def make_operator(system: System, shift: Optional[float] = None) -> Tuple[np.ndarray, np.ndarray, np.random.Generator]:
    """(links c64, offsets, rng positioned after the link draws) for a registered system."""
    rng = np.random.default_rng(system.seed)
    s = shift_for(system) if shift is None else shift
    offs = system.offsets()
    links = hermitian_links(rng, system.dims, system.nbasis, offs, s)
    return links, offs, rng


def make_system(system: System, shift: Optional[float] = None):
    """(links c64, offsets, B c128) with the draw order links, self term, RHS."""
    links, offs, rng = make_operator(system, shift)
    b = gaussian_vectors(rng, system.dims, system.nbasis, system.nrhs, dtype=np.complex128)
    return links, offs, b
