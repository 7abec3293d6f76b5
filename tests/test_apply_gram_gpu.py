"""GPU parity of the apply with the Gram x^H y (coarse_apply_gram) against the oracle.

The BlockCGrQ iteration (Fig. 2) applies the operator to the search block
and inverts the Gram D^H Z; with 3M links the library accumulates that Gram
in the apply's epilogue (one partial per workgroup of several sites, then a
fixed-order sum; one column tile, nrhs <= 16). Cases cover one and several
sites per workgroup, two to four waves (nbasis 16..64), partial column tiles
(nrhs 2, 8), both stencils, the unfused fallbacks (two column tiles,
complex64 links, 16-bit links through the two-pass apply at nrhs 16 and 32,
BF16 and FP16, both stencils, nrhs outside the MFMA set, volumes that do not
split into 64 workgroups) and the full 8^4/32/16 shape.

Expected values: y = oracle.apply in complex128 and G = x^H y of that y; for
16-bit links y = oracle.apply_lowp (the oracle's emulation of the same link
and input rounding) and G = x^H y of that y, with y also held to the
unquantised operator at LOWP_TOL. The Gram's error bound follows from the
apply's: |dG_ab| <= ||x_a|| ||dy_b||, so |G - G_ref| is held to the apply's
tolerance times the largest ||x_a|| ||y_b||.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import EMUL_TOL, FP32_TOL, LOWP_TOL, announce, dev, host, make_op, max_rel

pytestmark = pytest.mark.gpu

GRAM_TOL = 1e-5

CASES = [
    # dims, nbasis, nrhs, stencil, link type
    ((4, 4, 2, 2), 16, 16, "9pt", "c64_3m"),    # fused, one site per workgroup
    ((8, 4, 4, 8), 48, 16, "9pt", "c64_3m"),    # fused, two sites per workgroup (512 three-wave workgroups)
    ((4, 4, 4, 4), 32, 16, "81pt", "c64_3m"),   # fused, 81 points
    ((4, 4, 2, 2), 64, 8, "9pt", "c64_3m"),     # fused, half a column tile, four waves
    ((4, 4, 2, 2), 16, 2, "9pt", "c64_3m"),     # fused, nrhs 2
    ((8, 4, 4, 4), 48, 32, "9pt", "c64_3m"),    # unfused: two column tiles
    ((3, 2, 2, 2), 32, 16, "9pt", "c64_3m"),    # unfused: 24 sites
    ((4, 4, 2, 2), 16, 5, "9pt", "c64_3m"),     # unfused: nrhs 5 (VALU Gram)
    ((4, 4, 2, 2), 32, 16, "9pt", "c64"),       # unfused: complex64 links
    ((3, 2, 4, 2), 24, 8, "81pt", "c64"),       # unfused: nbasis 24 (partial row tile), 81 points
    ((4, 4, 2, 2), 32, 16, "9pt", "fp16"),      # unfused: 16-bit links, two-pass apply
    ((4, 4, 4, 8), 64, 32, "9pt", "fp16"),      # unfused: 16-bit links, nrhs 32, four row tiles
    ((8, 8, 4, 8), 48, 32, "9pt", "bf16"),      # unfused: 16-bit links, three row tiles
    ((4, 4, 4, 4), 32, 32, "81pt", "fp16"),     # unfused: 16-bit links, 81 points
    ((3, 2, 2, 2), 32, 32, "9pt", "bf16"),      # unfused: 16-bit links, 24 sites
]


def _check(dims, nb, nr, kind, dtype, seed, hermitian=False):
    from paper_2409_03904_amd import coarse
    rng = np.random.default_rng(4000 + seed)
    offs = W.stencil(kind)
    if hermitian:
        links = W.hermitian_links(rng, dims, nb, offs, shift=2.0)
    else:
        links = W.gaussian_links(rng, dims, nb, offs.shape[0])
    x = W.gaussian_vectors(rng, dims, nb, nr)
    announce("apply gram", dims, nb, nr, kind, dtype)
    op = make_op(links, offs, dims, dtype)
    xd = dev(x)
    y, g = coarse.apply_gram(op, xd)
    y, g = host(y), host(g)
    yref = O.apply(links, offs, dims, x.astype(np.complex128))
    if dtype in ("bf16", "fp16"):
        assert max_rel(y, yref) <= LOWP_TOL
        yref = O.apply_lowp(links, offs, dims, x.astype(np.complex64), dtype)
        tol = EMUL_TOL
    else:
        tol = FP32_TOL
    assert max_rel(y, yref) <= tol
    xr = x.reshape(-1, nr).astype(np.complex128)
    yr = yref.reshape(-1, nr).astype(np.complex128)
    gref = xr.conj().T @ yr
    scale = np.max(np.linalg.norm(xr, axis=0)) * np.max(np.linalg.norm(yr, axis=0))
    assert np.max(np.abs(g - gref)) <= (GRAM_TOL if tol == FP32_TOL else tol) * scale
    return op, xd, y, g


@pytest.mark.parametrize("dims,nb,nr,kind,dtype", CASES)
def test_apply_gram_matches_oracle(dims, nb, nr, kind, dtype):
    from paper_2409_03904_amd import coarse
    op, xd, y, g = _check(dims, nb, nr, kind, dtype, seed=nb + nr)
    # the apply half equals the plain apply bit for bit; the Gram repeats bit for bit
    y2 = host(coarse.apply(op, xd))
    assert np.array_equal(y, y2)
    _, g3 = coarse.apply_gram(op, xd)
    assert np.array_equal(g, host(g3))


def test_apply_gram_hermitian_operator():
    """A Hermitian operator gives a Hermitian x^H M x (up to rounding)."""
    _, _, _, g = _check((8, 4, 4, 8), 48, 16, "9pt", "c64_3m", seed=7, hermitian=True)
    assert np.max(np.abs(g - g.conj().T)) <= 1e-5 * np.max(np.abs(g))


def test_apply_gram_full_size():
    """The 8^4 / nbasis 32 / nrhs 16 / 9-point workload (two sites per workgroup)."""
    s = W.C2
    _check(s.dims, s.nbasis, s.nrhs, "9pt", "c64_3m", seed=11)
