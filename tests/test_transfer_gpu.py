"""Block project and promote between grids (Sec. 2.5) on the GPU, through the
C ABI, against the complex128 oracle: one product per coarse site,
C(x_c) = B(x_c)^H F(x_c) and F(x_c) = B(x_c) C(x_c).

Tolerance: complex64 inputs, float32 MFMA products summed in float32 over
V_block (project) or N_basis (promote) terms: FP32_TOL relative to the largest
output entry (measured errors are printed).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import FP32_TOL, announce, dev, host, max_rel

pytestmark = pytest.mark.gpu


def _c64(rng, shape):
    return (rng.standard_normal(shape, dtype=np.float32) + 1j * rng.standard_normal(shape, dtype=np.float32)) \
        .astype(np.complex64)


CASES = [((2, 2, 2, 2), 8, 16, 3), ((2, 2, 2, 2), 32, 48, 12), ((2, 2, 4, 2), 64, 256, 12),
         ((2, 2, 2, 2), 24, 32, 32), ((2, 2, 2, 2), 64, 64, 1), ((3, 2, 2, 2), 5, 16, 17)]


@pytest.mark.parametrize("dims,nb,vblock,nr", CASES)
def test_project_promote_match_oracle(dims, nb, vblock, nr):
    from paper_2409_03904_amd import coarse
    rng = np.random.default_rng(1000 + nb + vblock + nr)
    V = int(np.prod(dims))
    geom = coarse.Geometry(dims, nb, W.stencil("9pt"))
    B = _c64(rng, (V, vblock, nb))
    F = _c64(rng, (V, vblock, nr))
    Cc = _c64(rng, (V, nb, nr))
    announce("transfer", dims, nb, vblock, nr)
    got_c = host(coarse.block_project(dev(B), dev(F), geom))
    got_f = host(coarse.block_promote(dev(B), dev(Cc), geom))
    e1 = max_rel(got_c, O.block_project(B, F))
    e2 = max_rel(got_f, O.block_promote(B, Cc))
    print("transfer error", nb, vblock, nr, e1, e2)
    assert e1 <= FP32_TOL and e2 <= FP32_TOL


def test_project_promote_paper_shape():
    """Table 6 shapes: N_basis 64, N_rhs 12, V_block 256, batch 4096 (an 8^4
    coarse lattice); every output site checked against the oracle on a
    sample of 256 coarse sites."""
    from paper_2409_03904_amd import coarse
    rng = np.random.default_rng(1100)
    dims, nb, vblock, nr = (8, 8, 8, 8), 64, 256, 12
    V = 4096
    geom = coarse.Geometry(dims, nb, W.stencil("9pt"))
    B = _c64(rng, (V, vblock, nb))
    F = _c64(rng, (V, vblock, nr))
    Cc = _c64(rng, (V, nb, nr))
    announce("transfer paper shape")
    got_c = host(coarse.block_project(dev(B), dev(F), geom))
    got_f = host(coarse.block_promote(dev(B), dev(Cc), geom))
    sites = np.sort(rng.choice(V, 256, replace=False))
    e1 = max_rel(got_c[sites], O.block_project(B[sites], F[sites]))
    e2 = max_rel(got_f[sites], O.block_promote(B[sites], Cc[sites]))
    print("transfer paper-shape error", e1, e2)
    assert e1 <= FP32_TOL and e2 <= FP32_TOL
    assert np.all(np.isfinite(got_c)) and np.all(np.isfinite(got_f))


def test_project_promote_are_bitwise_reproducible():
    from paper_2409_03904_amd import coarse
    import torch
    rng = np.random.default_rng(1500)
    dims, nb, vblock, nr = (2, 2, 4, 2), 64, 256, 12
    geom = coarse.Geometry(dims, nb, W.stencil("9pt"))
    B, F, Cc = dev(_c64(rng, (32, vblock, nb))), dev(_c64(rng, (32, vblock, nr))), dev(_c64(rng, (32, nb, nr)))
    announce("transfer reproducible")
    assert torch.equal(coarse.block_project(B, F, geom), coarse.block_project(B, F, geom))
    assert torch.equal(coarse.block_promote(B, Cc, geom), coarse.block_promote(B, Cc, geom))
