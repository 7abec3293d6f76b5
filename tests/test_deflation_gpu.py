"""Multi-RHS deflation and the deflated Chebyshev coarse solve (Sec. 2.3) on the
GPU, through the C ABI, against the complex128 oracle.

Tolerance: complex64 inputs, float32 MFMA products; the coefficients c = V^H x
are summed in float32 within a row range and in double across ranges, the
promotion V c sums n_ev float32 products. Both stay at the level of the
complex64 apply (FP32_TOL relative to the largest output entry; measured
errors are printed); the deflated Chebyshev solve adds the polynomial's
bound (twice that).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import FP32_TOL, announce, dev, host, make_op, max_rel

pytestmark = pytest.mark.gpu


def _basis(rng, n, nev):
    a = rng.standard_normal((n, nev)) + 1j * rng.standard_normal((n, nev))
    q, _ = np.linalg.qr(a)
    return q.astype(np.complex64)


def _geom(dims, nb, kind="9pt"):
    from paper_2409_03904_amd import coarse
    return coarse.Geometry(dims, nb, W.stencil(kind))


CASES = [((2, 4, 2, 4), 16, 5), ((4, 4, 4, 4), 32, 16), ((3, 2, 2, 4), 8, 3), ((2, 2, 2, 2), 16, 32),
         ((2, 2, 4, 2), 16, 1)]


@pytest.mark.parametrize("dims,nb,nr", CASES)
@pytest.mark.parametrize("nev", [1, 7, 16, 64, 100])
def test_deflate_matches_oracle(dims, nb, nr, nev):
    import torch
    from paper_2409_03904_amd import coarse
    n = int(np.prod(dims)) * nb
    if nev > n:
        pytest.skip("more vectors than unknowns")
    rng = np.random.default_rng(700 + nev + nb + nr)
    v = _basis(rng, n, nev)
    lam = rng.uniform(0.5, 2.0, nev)
    x = W.gaussian_vectors(rng, dims, nb, nr)
    rd, rp = O.deflate(v.astype(np.complex128), lam, O.flatten(x))
    g = _geom(dims, nb)
    vd = dev(v.reshape(int(np.prod(dims)), nb, nev))
    ld = torch.from_numpy(lam).cuda()
    announce("deflate", dims, nb, nr, nev)
    y, xp = coarse.deflate(vd, ld, dev(x), g, want_perp=True)
    e1 = max_rel(O.flatten(host(y)), rd)
    e2 = max_rel(O.flatten(host(xp)), rp)
    print("deflate error", nev, e1, e2)
    assert e1 <= FP32_TOL and e2 <= FP32_TOL
    # x_perp in place of x, and the same y
    xd = dev(x)
    lib = __import__("paper_2409_03904_amd._lib", fromlist=["load"]).load()
    ws = torch.empty(coarse.deflation_workspace_bytes(g, nev, nr), dtype=torch.uint8, device="cuda")
    y2 = torch.empty_like(xd)
    rc = lib.coarse_deflate(g.c, vd.data_ptr(), nev, ld.data_ptr(), xd.data_ptr(), y2.data_ptr(), xd.data_ptr(),
                            nr, ws.data_ptr(), ws.numel(), None)
    assert rc == 0
    torch.cuda.synchronize()
    assert np.array_equal(host(y2), host(y))
    assert np.array_equal(host(xd), host(xp))


@pytest.mark.parametrize("nev,order", [(1, 6), (20, 10), (60, 3)])
def test_deflated_chebyshev_matches_oracle(nev, order):
    """Exact eigenpairs of a Hermitian 9-point operator on 2^4 sites, nbasis 16:
    the oracle's two-part solve (diagonal in the eigenbasis) against the GPU,
    with complex64 and 3M links."""
    import torch
    from paper_2409_03904_amd import coarse
    dims, nb, nr = (2, 2, 2, 2), 16, 6
    rng = np.random.default_rng(800 + nev)
    offs = W.stencil("9pt")
    links = W.hermitian_links(rng, dims, nb, offs, shift=4.0).astype(np.complex64)
    m = O.dense(links, offs, dims)
    lam, U = np.linalg.eigh(m)
    lo, hi = 0.9 * lam[nev], 1.1 * lam[-1]
    x = W.gaussian_vectors(rng, dims, nb, nr)
    ref = O.deflated_chebyshev(lambda z: m @ z, U[:, :nev], lam[:nev], O.flatten(x), lo, hi, order)
    vd = dev(U[:, :nev].astype(np.complex64).reshape(16, nb, nev))
    ld = torch.from_numpy(lam[:nev].copy()).cuda()
    for form in ("c64", "c64_3m"):
        announce("deflated chebyshev", nev, order, form)
        op = make_op(links, offs, dims, form)
        y = coarse.deflated_chebyshev_apply(op, vd, ld, dev(x), lo, hi, order)
        err = max_rel(O.flatten(host(y)), ref)
        print("deflated chebyshev error", nev, order, form, err)
        assert err <= 2 * FP32_TOL


def test_deflation_full_size():
    """8^4, nbasis 32, nrhs 16 with 192 orthonormal vectors (the paper's smallest
    deflation space): deflation against the oracle, and the deflated degree-12
    polynomial against the oracle on sampled sites of the whole result."""
    import torch
    from paper_2409_03904_amd import coarse
    s = W.C2
    links, offs, _ = W.make_system(s)
    rng = np.random.default_rng(901)
    n, nev = s.volume * s.nbasis, 192
    v = _basis(rng, n, nev)
    lam = rng.uniform(0.007, 0.06, nev)
    x = W.gaussian_vectors(rng, s.dims, s.nbasis, s.nrhs)
    rd, rp = O.deflate(v.astype(np.complex128), lam, O.flatten(x))
    g = _geom(s.dims, s.nbasis)
    vd = dev(v.reshape(s.volume, s.nbasis, nev))
    ld = torch.from_numpy(lam).cuda()
    announce("deflate full size")
    y, xp = coarse.deflate(vd, ld, dev(x), g, want_perp=True)
    e1, e2 = max_rel(O.flatten(host(y)), rd), max_rel(O.flatten(host(xp)), rp)
    print("deflate full-size error", e1, e2)
    assert e1 <= FP32_TOL and e2 <= FP32_TOL
    sh = W.stored_shifts()["c2"]
    hi = 1.1 * sh["lambda_max"]
    lo = hi / 200.0
    order = 12
    announce("deflated chebyshev full size")
    op = make_op(links, offs, s.dims, "c64_3m")
    yc = host(coarse.deflated_chebyshev_apply(op, vd, ld, dev(x), lo, hi, order))
    ref = rd + O.flatten(O.chebyshev_apply(lambda z: O.apply(links, offs, s.dims, z), rp.reshape(x.shape), lo, hi,
                                           order))
    err = max_rel(O.flatten(yc), ref)
    print("deflated chebyshev full-size error", err)
    assert err <= 2 * FP32_TOL


@pytest.mark.parametrize("form,b,steps,min_conv", [("c64", 8, 20, 4), ("c64_3m", 8, 20, 4), ("c64", 3, 33, 4),
                                                   ("c64_3m", 32, 6, 0)])
def test_block_lanczos_matches_oracle(form, b, steps, min_conv):
    """2^4 sites, nbasis 16 (n = 256), 16 Ritz pairs; blocks of 8 (20 steps), 3
    (33 steps: an odd basis width, unaligned rows) and 32 (6 steps, the largest
    block, not converged): the converged Ritz values agree with the oracle's
    (same start block); every GPU Ritz pair's residual ||M v - theta v||
    (oracle apply, double) matches its reported estimate, and the vectors are
    orthonormal."""
    import torch
    from paper_2409_03904_amd import coarse
    dims, nb, nev = (2, 2, 2, 2), 16, 16
    rng = np.random.default_rng(1200)
    offs = W.stencil("9pt")
    links = W.hermitian_links(rng, dims, nb, offs, shift=4.0).astype(np.complex64)
    x0 = W.gaussian_vectors(rng, dims, nb, 8)
    if b != 8:
        x0 = W.gaussian_vectors(np.random.default_rng(7), dims, nb, b)
    op = lambda z: O.flatten(O.apply(links, offs, dims, z.reshape(16, nb, -1)))
    th_o, V_o, res_o = O.block_lanczos(op, O.flatten(x0).astype(np.complex128), steps, nev)
    hn = float(np.max(np.abs(np.linalg.eigvalsh(O.dense(links, offs, dims)))))
    announce("block lanczos", form)
    v, lam, res, k = coarse.block_lanczos(make_op(links, offs, dims, form), dev(x0), steps, nev)
    assert k == steps * b
    V = O.flatten(host(v)).astype(np.complex128)
    direct = np.linalg.norm(op(V) - V * lam[None, :], axis=0)
    conv = res_o < 1e-4 * hn
    assert np.sum(conv) >= min_conv
    if np.any(conv):
        print("lanczos theta error", np.max(np.abs(lam[conv] - th_o[conv])) / hn)
        assert np.max(np.abs(lam[conv] - th_o[conv])) <= 1e-5 * hn
    print("lanczos residuals", b, steps, res[:4], direct[:4])
    assert np.max(np.abs(direct - res)) <= 1e-4 * hn
    np.testing.assert_allclose(V.conj().T @ V, np.eye(nev), rtol=0, atol=1e-5)


def test_block_lanczos_full_size_deflates():
    """8^4, nbasis 32 (n = 131072), block 16, 16 steps, 32 Ritz pairs: the
    Ritz values lie at or above the stored lowest eigenvalue (interlacing), the
    estimates match the direct residuals, the vectors are orthonormal, and
    deflating with the Ritz pairs leaves x_perp orthogonal to them."""
    import torch
    from paper_2409_03904_amd import coarse
    s = W.C2
    links, offs, _ = W.make_system(s)
    rng = np.random.default_rng(1201)
    x0 = W.gaussian_vectors(rng, s.dims, s.nbasis, 16)
    announce("block lanczos full size")
    op = make_op(links, offs, s.dims, "c64_3m")
    v, lam, res, k = coarse.block_lanczos(op, dev(x0), 16, 32)
    V = O.flatten(host(v)).astype(np.complex128)
    direct = np.linalg.norm(O.flatten(O.apply(links, offs, s.dims, V.reshape(s.volume, s.nbasis, 32)))
                            - V * lam[None, :], axis=0)
    lmax = W.stored_shifts()["c2"]["lambda_max"]
    print("lanczos full size", lam[:4], res[:4], direct[:4])
    assert np.max(np.abs(direct - res)) <= 1e-4 * lmax
    assert np.all(np.diff(lam) >= 0)
    assert lam[0] >= W.stored_shifts()["c2"]["lambda_min"] - 1e-4 * lmax
    np.testing.assert_allclose(V.conj().T @ V, np.eye(32), rtol=0, atol=1e-4)
    g = coarse.Geometry(s.dims, s.nbasis, offs)
    _, xp = coarse.deflate(v, torch.from_numpy(lam).cuda(), dev(x0), g, want_perp=True)
    assert np.max(np.abs(V.conj().T @ O.flatten(host(xp)))) <= 1e-4 * np.max(np.abs(x0))


def test_deflation_and_lanczos_are_bitwise_reproducible():
    """Fixed-order split-K sums and host steps: two runs give identical bits for
    the deflation outputs, the deflated Chebyshev solve and block Lanczos."""
    import torch
    from paper_2409_03904_amd import coarse
    dims, nb, nr, nev = (4, 4, 4, 4), 32, 16, 50
    rng = np.random.default_rng(1400)
    offs = W.stencil("9pt")
    links = W.hermitian_links(rng, dims, nb, offs, shift=6.0).astype(np.complex64)
    x = dev(W.gaussian_vectors(rng, dims, nb, nr))
    v = dev(_basis(rng, 256 * nb, nev).reshape(256, nb, nev))
    lam = torch.from_numpy(rng.uniform(0.5, 2.0, nev)).cuda()
    g = coarse.Geometry(dims, nb, offs)
    op = make_op(links, offs, dims, "c64_3m")
    announce("deflation reproducible")
    runs = [coarse.deflate(v, lam, x, g, want_perp=True) for _ in range(2)]
    assert all(torch.equal(a, b) for a, b in zip(runs[0], runs[1]))
    c = [coarse.deflated_chebyshev_apply(op, v, lam, x, 0.5, 14.0, 9) for _ in range(2)]
    assert torch.equal(c[0], c[1])
    lz = [coarse.block_lanczos(op, x, 6, 20) for _ in range(2)]
    assert torch.equal(lz[0][0], lz[1][0]) and np.array_equal(lz[0][1], lz[1][1])


def test_block_lanczos_exhausted_krylov_space():
    """A start block inside an invariant subspace: constant Hermitian links make
    every plane wave e^{ik.x} u an eigenvector family, M (e^{ik.x} u) =
    e^{ik.x} A(k) u with A(k) = sum_p A_p e^{ik.delta_p} (nbasis x nbasis), so
    the Krylov space of a plane-wave block has dimension nbasis. Block Lanczos
    must stop there (k < K), return the eigenvalues of A(k) with their
    residuals, zero pairs beyond, and deflation with those outputs must stay
    finite and equal the oracle's deflation on the valid pairs."""
    import torch
    from paper_2409_03904_amd import coarse
    dims, nb, b, steps, nev = (2, 2, 2, 4), 8, 4, 4, 12
    offs = W.stencil("9pt")
    V = int(np.prod(dims))
    rng = np.random.default_rng(4242)
    blocks = {}
    for p, o in enumerate(offs):
        c = W.canonical_index(o)
        if c > W.SELF_CANONICAL:
            blocks[p] = (rng.standard_normal((nb, nb)) + 1j * rng.standard_normal((nb, nb))) * 0.07
    links = np.zeros((V, len(offs), nb, nb), dtype=np.complex128)
    for p, a in blocks.items():
        q = [W.canonical_index(o) for o in offs].index(80 - W.canonical_index(offs[p]))
        links[:, p] = a
        links[:, q] = a.conj().T
    g = rng.standard_normal((nb, nb)) + 1j * rng.standard_normal((nb, nb))
    links[:, 0] = 0.05 * (g + g.conj().T) + 4.0 * np.eye(nb)
    links = links.astype(np.complex64)
    # momentum k_mu = 2 pi n_mu / L_mu
    n = np.array([1, 0, 1, 3])
    kvec = 2 * np.pi * n / np.array(dims)
    xs = O.site_coordinates(dims)
    phase = np.exp(1j * xs @ kvec)
    ak = sum(links[0, p].astype(np.complex128) * np.exp(1j * float(np.dot(kvec, offs[p]))) for p in range(len(offs)))
    ev = np.linalg.eigvalsh(0.5 * (ak + ak.conj().T))
    u = rng.standard_normal((nb, b)) + 1j * rng.standard_normal((nb, b))
    x0 = (phase[:, None, None] * u[None, :, :]).astype(np.complex64)
    op = make_op(links, offs, dims, "c64")
    announce("block lanczos exhausted", dims, nb, b, steps, nev)
    v, lam, res, k = coarse.block_lanczos(op, dev(x0), steps, nev)
    print("exhausted lanczos: k", k, "lam", lam, "res", res)
    assert k == nb < steps * b
    scale = float(np.max(np.abs(ev)))
    np.testing.assert_allclose(lam[:nb], ev, rtol=0, atol=1e-5 * scale)
    assert np.all(lam[nb:] == 0.0)
    vh = host(v).reshape(V * nb, nev)
    assert np.all(vh[:, nb:] == 0)
    # residual estimates against direct residuals of the returned pairs (oracle apply)
    mv = O.flatten(O.apply(links, offs, dims, host(v)))
    direct = np.linalg.norm(mv[:, :nb] - vh[:, :nb] * lam[None, :nb], axis=0)
    assert np.all(np.isfinite(res)) and np.all(res[:nb] <= 1e-4 * scale) and np.all(res[nb:] == 0.0)
    assert np.all(direct <= 1e-4 * scale)
    # deflation with the zero pairs included: finite, equal to the oracle on the valid pairs
    x = W.gaussian_vectors(rng, dims, nb, 4)
    ld = torch.from_numpy(np.ascontiguousarray(lam)).cuda()
    y, xp = coarse.deflate(v, ld, dev(x), coarse.Geometry(dims, nb, offs), want_perp=True)
    yh, xph = O.flatten(host(y)), O.flatten(host(xp))
    assert np.all(np.isfinite(yh)) and np.all(np.isfinite(xph))
    rd, rp = O.deflate(vh[:, :nb].astype(np.complex128), lam[:nb], O.flatten(x))
    assert max_rel(yh, rd) <= FP32_TOL and max_rel(xph, rp) <= FP32_TOL
