"""GPU parity of the coarse apply kernels (through the C ABI) against the oracle.

Shapes span several row/column tiles with ragged tails (nbasis 24/40, nrhs
1/5/12), extent-2 and extent-3 directions (aliased +-e neighbours), both
stencils, and the full-size workloads (every output entry).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import EMUL_TOL, FP32_TOL, LOWP_TOL, announce, dev, host, make_op, max_rel

pytestmark = pytest.mark.gpu

CASES = [
    # dims, nbasis, nrhs, stencil
    ((4, 4, 4, 4), 8, 4, "9pt"),       # the small parity workload
    ((2, 3, 4, 2), 24, 12, "9pt"),     # partial row tile, partial column tile, extent 2
    ((3, 2, 2, 3), 16, 1, "81pt"),
    ((4, 2, 3, 2), 40, 5, "9pt"),
    ((2, 2, 2, 2), 64, 32, "81pt"),    # precision-workload tile shape on a tiny lattice
    ((3, 3, 2, 2), 32, 16, "81pt"),
    ((2, 2, 3, 2), 48, 8, "9pt"),
]


def _case(dims, nb, nr, kind, seed=0, hermitian=False):
    rng = np.random.default_rng(1000 + seed)
    offs = W.stencil(kind)
    if hermitian:
        links = W.hermitian_links(rng, dims, nb, offs, shift=2.0)
    else:
        links = W.gaussian_links(rng, dims, nb, offs.shape[0])
    x = W.gaussian_vectors(rng, dims, nb, nr)
    return links, offs, x


@pytest.mark.parametrize("dims,nb,nr,kind", CASES)
def test_apply_fp32_matches_oracle(dims, nb, nr, kind):
    from paper_2409_03904_amd import coarse
    links, offs, x = _case(dims, nb, nr, kind)
    announce("apply c64", dims, nb, nr, kind)
    op = make_op(links, offs, dims)
    y = host(coarse.apply(op, dev(x)))
    ref = O.apply(links, offs, dims, x)
    assert max_rel(y, ref) <= FP32_TOL
    yg = host(coarse.apply_generic(op, dev(x)))
    assert max_rel(yg, ref) <= FP32_TOL


@pytest.mark.parametrize("dims,nb,nr,kind", CASES[:4])
def test_apply_fp64_vectors_matches_oracle(dims, nb, nr, kind):
    from paper_2409_03904_amd import coarse
    links, offs, x = _case(dims, nb, nr, kind, seed=1)
    x = x.astype(np.complex128) + 1e-3j * x.astype(np.complex128) ** 2
    announce("apply c128", dims, nb, nr, kind)
    op = make_op(links, offs, dims)
    y = host(coarse.apply(op, dev(x)))
    ref = O.apply(links, offs, dims, x)
    assert max_rel(y, ref) <= 1e-13


@pytest.mark.parametrize("dims,nb,nr,kind", [((2, 2, 2, 2), 4, 2, "9pt"), ((3, 2, 2, 2), 12, 3, "81pt"),
                                             ((2, 3, 2, 2), 5, 7, "9pt")])
def test_apply_generic_shapes(dims, nb, nr, kind):
    """nbasis outside the MFMA tiling runs the VALU kernel."""
    from paper_2409_03904_amd import coarse
    links, offs, x = _case(dims, nb, nr, kind, seed=2)
    announce("apply generic", dims, nb, nr, kind)
    op = make_op(links, offs, dims)
    ref = O.apply(links, offs, dims, x)
    assert max_rel(host(coarse.apply(op, dev(x))), ref) <= FP32_TOL
    x128 = x.astype(np.complex128)
    assert max_rel(host(coarse.apply(op, dev(x128))), O.apply(links, offs, dims, x128)) <= 1e-13


@pytest.mark.parametrize("dims,nb,nr,kind", CASES + [((2, 2, 2, 2), 4, 2, "9pt")])
def test_adjoint_matches_oracle(dims, nb, nr, kind):
    from paper_2409_03904_amd import coarse
    links, offs, x = _case(dims, nb, nr, kind, seed=3)
    announce("adjoint", dims, nb, nr, kind)
    op = make_op(links, offs, dims)
    ref = O.apply_adjoint(links, offs, dims, x)
    assert max_rel(host(coarse.apply_adjoint(op, dev(x))), ref) <= FP32_TOL
    assert max_rel(host(coarse.apply_adjoint_generic(op, dev(x))), ref) <= FP32_TOL
    x128 = x.astype(np.complex128)
    assert max_rel(host(coarse.apply_adjoint(op, dev(x128))), O.apply_adjoint(links, offs, dims, x128)) <= 1e-13


def test_apply_deterministic():
    from paper_2409_03904_amd import coarse
    links, offs, x = _case((3, 3, 2, 2), 32, 16, "81pt", seed=4)
    announce("determinism")
    op = make_op(links, offs, dims=(3, 3, 2, 2))
    xd = dev(x)
    a = host(coarse.apply(op, xd))
    b = host(coarse.apply(op, xd))
    assert np.array_equal(a, b)


# ---- 16-bit links ----
LOWP_CASES = [((2, 2, 3, 2), 16, 8, "9pt"), ((2, 2, 2, 2), 32, 16, "81pt"), ((2, 2, 2, 2), 64, 32, "81pt"),
              ((3, 2, 2, 2), 48, 5, "9pt"), ((2, 2, 2, 3), 32, 3, "9pt")]


@pytest.mark.parametrize("two_pass", [True, False])
@pytest.mark.parametrize("kind", ["bf16", "fp16"])
@pytest.mark.parametrize("dims,nb,nr,st", LOWP_CASES)
def test_lowp_exact_on_integer_grid(kind, dims, nb, nr, st, two_pass):
    """Integer links and inputs: every 16-bit product and float32 sum is exact,
    so the kernel must reproduce the exact result bit for bit."""
    from paper_2409_03904_amd import coarse
    rng = np.random.default_rng(77)
    offs = W.stencil(st)
    links = W.integer_links(rng, dims, nb, offs.shape[0])
    x = W.integer_vectors(rng, dims, nb, nr)
    announce("lowp integer", kind, dims, nb, nr, st, two_pass)
    op = make_op(links, offs, dims, kind)
    y = host(coarse.apply(op, dev(x), two_pass=two_pass))
    ref = O.apply(links, offs, dims, x)
    assert np.array_equal(y.astype(np.complex128), ref)
    yg = host(coarse.apply_generic(op, dev(x)))
    assert np.array_equal(yg.astype(np.complex128), ref)


@pytest.mark.parametrize("two_pass", [True, False])
@pytest.mark.parametrize("kind", ["bf16", "fp16"])
@pytest.mark.parametrize("dims,nb,nr,st", LOWP_CASES[:3] + [((4, 2, 2, 2), 64, 7, "81pt")])
def test_lowp_matches_emulation(kind, dims, nb, nr, st, two_pass):
    from paper_2409_03904_amd import coarse
    links, offs, x = _case(dims, nb, nr, st, seed=5, hermitian=True)
    x = x * np.exp(np.random.default_rng(6).uniform(-3, 3, size=(1, 1, nr)))  # columns of different scale
    x = x.astype(np.complex64)
    announce("lowp gaussian", kind, dims, nb, nr, st, two_pass)
    op = make_op(links, offs, dims, kind)
    y = host(coarse.apply(op, dev(x), two_pass=two_pass))
    assert max_rel(y, O.apply_lowp(links, offs, dims, x, kind)) <= EMUL_TOL
    assert max_rel(y, O.apply(links, offs, dims, x)) <= LOWP_TOL
    assert max_rel(host(coarse.apply_generic(op, dev(x))), O.apply_lowp(links, offs, dims, x, kind)) <= EMUL_TOL


@pytest.mark.parametrize("kind", ["bf16", "fp16"])
def test_lowp_two_pass_equals_one_pass(kind):
    """Same operands, same MFMA order, same scaling: the two forms agree bitwise."""
    import torch
    from paper_2409_03904_amd import coarse
    links, offs, x = _case((4, 2, 2, 2), 64, 32, "81pt", seed=8, hermitian=False)
    x = (x * np.exp(np.random.default_rng(9).uniform(-4, 4, size=(1, 1, 32)))).astype(np.complex64)
    announce("lowp one vs two pass", kind)
    op = make_op(links, offs, (4, 2, 2, 2), kind)
    xd = dev(x)
    ws = torch.empty(coarse.apply_workspace_bytes(op, 32), dtype=torch.uint8, device="cuda")
    a = host(coarse.apply(op, xd, workspace=ws))
    b = host(coarse.apply(op, xd, two_pass=False))
    assert np.array_equal(a, b)


# ---- 3M form ----
CASES_3M = [((2, 2, 3, 2), 16, 16, "9pt"), ((3, 2, 2, 2), 32, 5, "9pt"), ((2, 2, 2, 2), 64, 32, "81pt"),
            ((2, 2, 2, 3), 48, 17, "9pt"), ((4, 2, 2, 2), 64, 1, "81pt"), ((2, 3, 2, 2), 32, 31, "81pt")]


@pytest.mark.parametrize("dims,nb,nr,st", CASES_3M)
def test_apply_3m_matches_oracle(dims, nb, nr, st):
    """Three real products per complex multiply-add, the 3M link layout; odd
    and small nrhs (padded column tiles), one and two column tiles."""
    from paper_2409_03904_amd import coarse
    links, offs, x = _case(dims, nb, nr, st, seed=11)
    x = x.astype(np.complex64)
    announce("3m", dims, nb, nr, st)
    op = make_op(links, offs, dims, "c64_3m")
    y = host(coarse.apply(op, dev(x)))
    assert max_rel(y, O.apply(links, offs, dims, x)) <= FP32_TOL


@pytest.mark.parametrize("dims,nb,nr,st", CASES_3M + [((2, 2, 1, 2), 16, 32, "81pt")])
def test_apply_3m_fp64_vectors_matches_oracle(dims, nb, nr, st):
    """complex128 vectors on the 3M links (the double residual of defect
    correction): T1, T2, T3 on f64 MFMA from the exact link values, against
    the complex128 oracle, with inputs that complex64 cannot hold."""
    from paper_2409_03904_amd import coarse
    links, offs, x = _case(dims, nb, nr, st, seed=13)
    x = x.astype(np.complex128) + 1e-3j * x.astype(np.complex128) ** 2
    announce("3m c128", dims, nb, nr, st)
    op = make_op(links, offs, dims, "c64_3m")
    y = host(coarse.apply(op, dev(x)))
    assert max_rel(y, O.apply(links, offs, dims, x)) <= 1e-13


@pytest.mark.parametrize("dims,nb,nr,st", CASES_3M + [((2, 4, 2, 4), 16, 5, "9pt"), ((2, 2, 1, 2), 16, 32, "81pt")])
def test_adjoint_3m_matches_oracle(dims, nb, nr, st):
    """M^H in the 3M form on the 3M link layout (contraction over the link row,
    links and input gathered from x - delta_p) against the oracle's adjoint on
    non-Hermitian links: one and two column tiles, odd and small nrhs, every
    row-tile count, an extent-1 direction."""
    from paper_2409_03904_amd import coarse
    links, offs, x = _case(dims, nb, nr, st, seed=12)
    x = x.astype(np.complex64)
    announce("adjoint 3m", dims, nb, nr, st)
    op = make_op(links, offs, dims, "c64_3m")
    y = host(coarse.apply_adjoint(op, dev(x)))
    assert max_rel(y, O.apply_adjoint(links, offs, dims, x)) <= FP32_TOL


def test_full_size_adjoint_3m():
    """8^4, nbasis 32, nrhs 16, 9-point: the whole 3M adjoint output against
    the oracle's adjoint, on non-Hermitian links."""
    from paper_2409_03904_amd import coarse
    s = W.C2
    rng = np.random.default_rng(77)
    offs = W.stencil("9pt")
    links = W.gaussian_links(rng, s.dims, s.nbasis, offs.shape[0])
    x = W.gaussian_vectors(rng, s.dims, s.nbasis, s.nrhs).astype(np.complex64)
    announce("full c2 adjoint 3m")
    op = make_op(links, offs, s.dims, "c64_3m")
    y = host(coarse.apply_adjoint(op, dev(x)))
    assert max_rel(y, O.apply_adjoint(links, offs, s.dims, x)) <= FP32_TOL


# ---- full-size workloads ----
def test_full_size_fp32_workload():
    """8^4, nbasis 32, nrhs 16, 9-point: the whole output against the oracle."""
    from paper_2409_03904_amd import coarse
    s = W.C2
    links, offs, b = W.make_system(s)
    x = b.astype(np.complex64)
    announce("full c2 apply")
    op = make_op(links, offs, s.dims)
    y = host(coarse.apply(op, dev(x)))
    assert max_rel(y, O.apply(links, offs, s.dims, x)) <= FP32_TOL


@pytest.mark.timeout(900)
def test_full_size_precision_workload():
    """8^4, nbasis 64, nrhs 32, 81-point, in complex64 (4M and 3M) and 16-bit
    links, every output entry: against the complex128 oracle, and for 16-bit
    links also against the oracle's emulation of their rounding."""
    import torch
    from paper_2409_03904_amd import coarse
    s = W.C3
    links, offs, b = W.make_system(s)
    x = b.astype(np.complex64)
    del b
    announce("full c3 apply: oracle")
    ref = O.apply(links, offs, s.dims, x)
    geom = coarse.Geometry(s.dims, s.nbasis, offs)
    lt = dev(links)
    xd = dev(x)
    ys = {}
    for kind in ("c64", "c64_3m", "bf16", "fp16"):
        announce("full c3 apply", kind)
        op = coarse.pack(lt, geom, kind)
        ys[kind] = host(coarse.apply(op, xd))
        del op
        torch.cuda.synchronize()
    del lt, xd
    assert max_rel(ys["c64"], ref) <= FP32_TOL
    assert max_rel(ys["c64_3m"], ref) <= FP32_TOL
    for kind in ("bf16", "fp16"):
        assert max_rel(ys[kind], ref) <= LOWP_TOL, kind
        announce("full c3 apply: oracle emulation", kind)
        assert max_rel(ys[kind], O.apply_lowp(links, offs, s.dims, x, kind)) <= EMUL_TOL, kind


# ---- edge cases: aliasing neighbours, self-only and self-free stencils ----
EDGE_STENCILS = {
    "self": W.stencil("self"),
    "noself": W.stencil("9pt")[1:],                      # 8 hops, no self point
    "one": np.array([[0, 1, 0, 0]], dtype=np.int8),      # a single non-self point
}


@pytest.mark.parametrize("sname", sorted(EDGE_STENCILS))
@pytest.mark.parametrize("dims", [(1, 2, 3, 2), (2, 1, 1, 1), (3, 3, 3, 3)])
@pytest.mark.parametrize("kind", ["c64", "c64_3m", "bf16", "fp16"])
def test_apply_edge_stencils_and_extents(sname, dims, kind):
    """Extent-1 directions (every displacement along them is the site itself,
    so contributions add up), a self-only stencil, a stencil without the self
    point (16-bit kernels' separate self path unused) and a single hop, in every
    link storage and, for 16-bit links, both kernel forms."""
    from paper_2409_03904_amd import coarse
    offs = EDGE_STENCILS[sname]
    nb, nr = 16, 5
    rng = np.random.default_rng(90 + len(sname))
    links = W.gaussian_links(rng, dims, nb, offs.shape[0])
    x = W.gaussian_vectors(rng, dims, nb, nr)
    announce("edge", sname, dims, kind)
    op = make_op(links, offs, dims, kind)
    xd = dev(x)
    if kind in ("bf16", "fp16"):
        ref = O.apply_lowp(links, offs, dims, x, kind)
        for two_pass in (True, False):
            assert max_rel(host(coarse.apply(op, xd, two_pass=two_pass)), ref) <= EMUL_TOL, two_pass
    else:
        ref = O.apply(links, offs, dims, x)
        assert max_rel(host(coarse.apply(op, xd)), ref) <= FP32_TOL
        assert max_rel(host(coarse.apply_adjoint(op, xd)), O.apply_adjoint(links, offs, dims, x)) <= FP32_TOL


@pytest.mark.parametrize("dims,nb,nr,kind", [((2, 4, 2, 4), 16, 5, "9pt"), ((4, 4, 4, 4), 32, 16, "9pt"),
                                             ((3, 2, 2, 4), 16, 3, "81pt"), ((2, 2, 1, 2), 16, 32, "81pt")])
def test_adjoint_as_forward_operator(dims, nb, nr, kind):
    """M^H applied as the forward operator of the adjoint links
    (A_p(x - delta_p)^H at -delta_p), packed complex64 and 3M, against the
    oracle's adjoint on non-Hermitian links; extent-1 and extent-2 directions
    included."""
    import torch
    from paper_2409_03904_amd import coarse
    rng = np.random.default_rng(1300 + nb + nr)
    offs = W.stencil(kind)
    links = W.gaussian_links(rng, dims, nb, offs.shape[0]).astype(np.complex64)
    x = W.gaussian_vectors(rng, dims, nb, nr)
    ref = O.apply_adjoint(links, offs, dims, x)
    geom = coarse.Geometry(dims, nb, offs)
    lt = dev(links)
    for dtype in ("c64", "c64_3m"):
        announce("adjoint as forward", dims, nb, nr, kind, dtype)
        op = coarse.pack_adjoint(lt, geom, dtype)
        y = host(coarse.apply(op, dev(x)))
        assert max_rel(y, ref) <= FP32_TOL
