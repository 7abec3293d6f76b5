"""Stationary Chebyshev approximation to 1/x applied to the coarse operator
(Sec. 2.3) on the GPU, against the complex128 oracle.

Tolerance for float32 vectors: every degree adds the rounding of one apply and
one elementwise pass. In the worst case the three-term recurrence carries a
perturbation from degree j to degree k amplified by k - j + 1 (the bound of
the second-kind polynomial U_{k-j} on [-1, 1]), which would allow errors
growing like (n + 1)^2 times the per-degree error; with the spectrum inside
[lo, hi] the measured error stays at the level of one apply for every degree
tested (1e-6 .. 7e-6 up to degree 40 and at full size), so the bound is twice
the single-apply tolerance (4u for degree 0, a single scaling).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import FP32_TOL, LOWP_TOL, announce, dev, host, make_op, max_rel

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def cheb_tol(order):
    return 4.0 * U32 if order == 0 else 2.0 * FP32_TOL


def _system(dims, nb, nr, kind, seed, shift):
    rng = np.random.default_rng(seed)
    offs = W.stencil(kind)
    links = W.hermitian_links(rng, dims, nb, offs, shift=shift).astype(np.complex64)
    b = W.gaussian_vectors(rng, dims, nb, nr)
    return links, offs, b


def _range(links, offs, dims):
    """[lo, hi] holding the whole spectrum: Lanczos extremes (Ritz values lie
    inside the spectrum) widened by 10 %."""
    nb = links.shape[2]
    n = int(np.prod(dims)) * nb
    op = lambda v: O.apply(links, offs, dims, v.reshape(-1, nb, 1)).ravel()
    tmin, tmax, bmin, bmax = O.lanczos_extremes(op, n, steps=min(n, 120), seed=5)
    lo, hi = 0.9 * (tmin - bmin), 1.1 * (tmax + bmax)
    assert lo > 0, (tmin, bmin)
    return lo, hi


CASES = [((2, 4, 2, 4), 16, 5, "9pt", 4.0), ((4, 4, 4, 4), 32, 16, "9pt", 6.0), ((3, 2, 2, 4), 8, 3, "81pt", 14.0),
         ((2, 2, 2, 2), 16, 32, "81pt", 14.0)]


@pytest.mark.parametrize("dims,nb,nr,kind,shift", CASES)
@pytest.mark.parametrize("order", [0, 1, 2, 7, 40])
def test_chebyshev_matches_oracle(dims, nb, nr, kind, shift, order):
    from paper_2409_03904_amd import coarse
    links, offs, b = _system(dims, nb, nr, kind, 300 + nb + nr, shift)
    lo, hi = _range(links, offs, dims)
    ref = O.chebyshev_apply(lambda v: O.apply(links, offs, dims, v), b, lo, hi, order)
    forms = ["c64"] + (["c64_3m"] if nb % 16 == 0 else [])
    for form in forms:
        announce("chebyshev", dims, nb, nr, kind, order, form)
        op = make_op(links, offs, dims, form)
        y = host(coarse.chebyshev_apply(op, dev(b), lo, hi, order))
        assert max_rel(y, ref) <= cheb_tol(order), (form, max_rel(y, ref))


@pytest.mark.parametrize("kind", ["bf16", "fp16"])
def test_chebyshev_16bit_links(kind):
    """16-bit links: P(M~) against the unquantised P(M) at a low degree, within
    the 16-bit operator bound times the degree."""
    from paper_2409_03904_amd import coarse
    dims, nb, nr = (2, 4, 2, 4), 16, 8
    links, offs, b = _system(dims, nb, nr, "9pt", 77, 4.0)
    lo, hi = _range(links, offs, dims)
    order = 3
    ref = O.chebyshev_apply(lambda v: O.apply(links, offs, dims, v), b, lo, hi, order)
    announce("chebyshev 16-bit", kind)
    op = make_op(links, offs, dims, kind)
    y = host(coarse.chebyshev_apply(op, dev(b), lo, hi, order))
    assert max_rel(y, ref) <= order * LOWP_TOL, max_rel(y, ref)


@pytest.mark.parametrize("form", ["c64", "c64_3m"])
def test_chebyshev_full_size(form):
    """The 8^4 / nbasis 32 / nrhs 16 workload at degree 8 against the oracle, all
    outputs."""
    from paper_2409_03904_amd import coarse
    s = W.C2
    links, offs, b = W.make_system(s)
    sh = W.stored_shifts()["c2"]
    hi = 1.1 * sh["lambda_max"]
    lo = hi / 2000.0
    order = 8
    x = b.astype(np.complex64)
    ref = O.chebyshev_apply(lambda v: O.apply(links, offs, s.dims, v), x, lo, hi, order)
    announce("chebyshev full size", form)
    op = make_op(links, offs, s.dims, form)
    y = host(coarse.chebyshev_apply(op, dev(x), lo, hi, order))
    assert max_rel(y, ref) <= cheb_tol(order), max_rel(y, ref)


def test_chebyshev_approximates_the_inverse():
    """The bench configuration (8^4 / 32 / 16, degree 120 on [hi/2000, 1.1
    lambda_max]): with the spectrum inside [lo, hi], ||b - M P(M) b|| / ||b|| is
    at most max over [lo, hi] of |1 - x P(x)| (evaluated with numpy), plus the
    float32 error of the recurrence."""
    from numpy.polynomial import chebyshev as C

    from paper_2409_03904_amd import coarse
    s = W.C2
    links, offs, b = W.make_system(s)
    sh = W.stored_shifts()["c2"]
    hi = 1.1 * sh["lambda_max"]
    lo = hi / 2000.0
    order = 120
    xs = np.linspace(lo, hi, 200001)
    c = O.chebyshev_coefficients(lo, hi, order)
    bound = np.max(np.abs(1.0 - xs * C.chebval((2 * xs - (hi + lo)) / (hi - lo), c)))
    x = b.astype(np.complex64)
    announce("chebyshev inverse bound", order)
    op = make_op(links, offs, s.dims, "c64_3m")
    y = host(coarse.chebyshev_apply(op, dev(x), lo, hi, order)).astype(np.complex128)
    r = x.astype(np.complex128) - O.apply(links, offs, s.dims, y)
    rel = np.linalg.norm(O.flatten(r), axis=0) / np.linalg.norm(O.flatten(x.astype(np.complex128)), axis=0)
    assert np.max(rel) <= bound + 1e-4, (np.max(rel), bound)
