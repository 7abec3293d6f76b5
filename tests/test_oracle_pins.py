"""Pins of the complex128 oracle against facts fixed by the paper and by mathematics.

Each test would fail under a plausible oracle mistake: a wrong neighbour sign
or index (dense assembly, Fourier symbol, Laplacian), a missing conjugation
(adjoint identity, hermiticity), a dropped term in BlockCGrQ (dense LU,
residual invariant, N_rhs = 1 reduction, finite termination), a rounding-mode
slip (bit patterns of bf16/fp16 rounding), a wrong gradient convention (finite
differences).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed=0):
    return np.random.default_rng(seed)


def _rand_vec(rng, dims, nb, nr):
    return W.gaussian_vectors(rng, dims, nb, nr, dtype=np.complex128)


SMALL_GEOMS = [
    ((2, 2, 2, 2), 3, "9pt"),
    ((3, 3, 3, 3), 2, "9pt"),
    ((4, 3, 2, 1), 4, "9pt"),
    ((2, 3, 2, 3), 2, "81pt"),
    ((3, 2, 3, 2), 3, "81pt"),
]


# ---- P1: apply equals the dense matrix built by direct block placement ----
@pytest.mark.parametrize("dims,nb,kind", SMALL_GEOMS)
def test_apply_matches_dense_assembly(dims, nb, kind):
    rng = _rng(1)
    offs = W.stencil(kind)
    links = W.gaussian_links(rng, dims, nb, offs.shape[0])
    x = _rand_vec(rng, dims, nb, 3)
    m = O.dense(links, offs, dims)
    y = O.apply(links, offs, dims, x)
    np.testing.assert_allclose(O.flatten(y), m @ O.flatten(x), rtol=0, atol=1e-12)


def test_apply_brute_force_loops():
    """Y[x,i,r] = sum_p sum_j A[x,p,i,j] X[x+delta_p, j, r], written as scalar loops."""
    rng = _rng(2)
    dims, nb, nr = (2, 3, 1, 2), 2, 2
    offs = W.stencil("9pt")
    links = W.gaussian_links(rng, dims, nb, offs.shape[0])
    x = _rand_vec(rng, dims, nb, nr)
    V = W.volume(dims)
    L = dims
    ref = np.zeros((V, nb, nr), dtype=complex)
    for s in range(V):
        c = [s % L[0], (s // L[0]) % L[1], (s // (L[0] * L[1])) % L[2], s // (L[0] * L[1] * L[2])]
        for p in range(offs.shape[0]):
            d = [(c[m] + int(offs[p][m])) % L[m] for m in range(4)]
            t = d[0] + L[0] * (d[1] + L[1] * (d[2] + L[2] * d[3]))
            for i in range(nb):
                for r in range(nr):
                    acc = 0j
                    for j in range(nb):
                        acc += complex(links[s, p, i, j]) * x[t, j, r]
                    ref[s, i, r] += acc
    np.testing.assert_allclose(O.apply(links, offs, dims, x), ref, rtol=0, atol=1e-13)


def test_neighbour_convention_x0_fastest():
    """Site 0's +e0 neighbour is site 1; its -e3 neighbour is the last time slice."""
    dims = (3, 4, 5, 6)
    assert O.neighbour(dims, (1, 0, 0, 0))[0] == 1
    assert O.neighbour(dims, (0, 1, 0, 0))[0] == 3
    assert O.neighbour(dims, (0, 0, 1, 0))[0] == 12
    assert O.neighbour(dims, (0, 0, 0, -1))[0] == 3 * 4 * 5 * 5
    assert O.neighbour(dims, (-1, 0, 0, 0))[0] == 2


# ---- P2: adjoint identity for arbitrary (non-Hermitian) links ----
@pytest.mark.parametrize("dims,nb,kind", SMALL_GEOMS)
def test_adjoint_identity(dims, nb, kind):
    rng = _rng(3)
    offs = W.stencil(kind)
    links = W.gaussian_links(rng, dims, nb, offs.shape[0])
    u = _rand_vec(rng, dims, nb, 2)
    v = _rand_vec(rng, dims, nb, 2)
    lhs = np.vdot(u, O.apply(links, offs, dims, v))
    rhs = np.vdot(O.apply_adjoint(links, offs, dims, u), v)
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
    m = O.dense(links, offs, dims)
    np.testing.assert_allclose(O.flatten(O.apply_adjoint(links, offs, dims, u)),
                               m.conj().T @ O.flatten(u), rtol=0, atol=1e-12)


# ---- P3: the Hermitian pairing makes M Hermitian ----
@pytest.mark.parametrize("dims,nb,kind", [((2, 2, 2, 2), 3, "9pt"), ((3, 3, 2, 2), 2, "81pt"),
                                          ((4, 4, 4, 4), 2, "9pt"), ((3, 2, 1, 2), 2, "81pt")])
def test_hermitian_construction(dims, nb, kind):
    rng = _rng(4)
    offs = W.stencil(kind)
    links = W.hermitian_links(rng, dims, nb, offs, shift=0.3)
    m = O.dense(links, offs, dims)
    assert np.max(np.abs(m - m.conj().T)) == 0.0
    u = _rand_vec(rng, dims, nb, 1)
    v = _rand_vec(rng, dims, nb, 1)
    a = np.vdot(u, O.apply(links, offs, dims, v))
    b = np.vdot(O.apply(links, offs, dims, u), v)
    assert abs(a - b) <= 1e-13 * abs(a)


def test_non_hermitian_links_are_not_hermitian():
    rng = _rng(5)
    offs = W.stencil("9pt")
    links = W.gaussian_links(rng, (2, 2, 2, 2), 2, offs.shape[0])
    m = O.dense(links, offs, (2, 2, 2, 2))
    assert np.max(np.abs(m - m.conj().T)) > 0.1


# ---- P4 / P5: constant links: translation invariance and the Fourier symbol ----
def _constant_links(rng, dims, nb, offs):
    a = (rng.standard_normal((offs.shape[0], nb, nb)) + 1j * rng.standard_normal((offs.shape[0], nb, nb))) * 0.3
    V = W.volume(dims)
    return np.broadcast_to(a[None], (V,) + a.shape).astype(np.complex64).copy(), a.astype(np.complex64)


def _translate(x, dims, a):
    return x[O.neighbour(dims, a)]


@pytest.mark.parametrize("kind", ["9pt", "81pt"])
def test_translation_invariance(kind):
    rng = _rng(6)
    dims, nb = (3, 4, 2, 3), 2
    offs = W.stencil(kind)
    links, _ = _constant_links(rng, dims, nb, offs)
    x = _rand_vec(rng, dims, nb, 2)
    for a in [(1, 0, 0, 0), (0, 2, 1, 0), (2, 3, 1, 2)]:
        lhs = O.apply(links, offs, dims, _translate(x, dims, a))
        rhs = _translate(O.apply(links, offs, dims, x), dims, a)
        np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-12)


@pytest.mark.parametrize("kind", ["9pt", "81pt"])
def test_fourier_symbol_and_spectrum(kind):
    rng = _rng(7)
    dims, nb = (3, 2, 4, 2), 2
    offs = W.stencil(kind)
    links, a = _constant_links(rng, dims, nb, offs)
    xs = O.site_coordinates(dims)
    V = W.volume(dims)
    spectrum = []
    for n in np.ndindex(*dims):
        k = 2 * np.pi * np.asarray(n) / np.asarray(dims)
        ahat = sum(a[p].astype(complex) * np.exp(1j * (k @ offs[p].astype(float))) for p in range(offs.shape[0]))
        v = rng.standard_normal((nb, 1)) + 1j * rng.standard_normal((nb, 1))
        phase = np.exp(1j * (xs @ k))[:, None, None]
        x = phase * v[None]
        y = O.apply(links, offs, dims, x)
        np.testing.assert_allclose(y, phase * (ahat @ v)[None], rtol=0, atol=1e-12)
        spectrum.extend(np.linalg.eigvals(ahat))
    ev = np.linalg.eigvals(O.dense(links, offs, dims))
    assert len(spectrum) == V * nb
    # same multiset of eigenvalues
    s1 = np.sort_complex(np.round(np.asarray(spectrum), 9))
    s2 = np.sort_complex(np.round(ev, 9))
    np.testing.assert_allclose(s1, s2, atol=1e-7)


# ---- P6: the 4D lattice Laplacian ----
def test_lattice_laplacian_eigenvalues():
    dims = (4, 3, 2, 5)
    m2 = 0.25
    offs = W.stencil("9pt")
    V = W.volume(dims)
    links = np.zeros((V, offs.shape[0], 1, 1), dtype=np.complex64)
    links[:, 0] = 8.0 + m2
    links[:, 1:] = -1.0
    ev = np.sort(np.linalg.eigvalsh(O.dense(links, offs, dims)))
    expect = []
    for n in np.ndindex(*dims):
        k = 2 * np.pi * np.asarray(n) / np.asarray(dims)
        expect.append(m2 + np.sum(4 * np.sin(k / 2) ** 2))
    np.testing.assert_allclose(ev, np.sort(expect), atol=1e-10)


# ---- P7 / P8: self-only stencil, column independence, linearity ----
def test_self_only_is_per_site_matmul():
    rng = _rng(8)
    dims, nb, nr = (2, 2, 3, 1), 3, 2
    offs = W.stencil("self")
    links = W.gaussian_links(rng, dims, nb, 1)
    x = _rand_vec(rng, dims, nb, nr)
    y = O.apply(links, offs, dims, x)
    for s in range(W.volume(dims)):
        np.testing.assert_allclose(y[s], links[s, 0].astype(complex) @ x[s], atol=1e-13)


def test_columns_independent_and_linear():
    rng = _rng(9)
    dims, nb, nr = (3, 2, 2, 2), 3, 4
    offs = W.stencil("81pt")
    links = W.gaussian_links(rng, dims, nb, offs.shape[0])
    x = _rand_vec(rng, dims, nb, nr)
    z = _rand_vec(rng, dims, nb, nr)
    y = O.apply(links, offs, dims, x)
    for r in range(nr):
        np.testing.assert_allclose(O.apply(links, offs, dims, x[:, :, r:r + 1])[:, :, 0], y[:, :, r], atol=1e-13)
    perm = [2, 0, 3, 1]
    np.testing.assert_allclose(O.apply(links, offs, dims, x[:, :, perm]), y[:, :, perm], atol=1e-13)
    a, b = 0.3 - 1.1j, 2.0 + 0.5j
    np.testing.assert_allclose(O.apply(links, offs, dims, a * x + b * z),
                               a * y + b * O.apply(links, offs, dims, z), atol=1e-12)


# ---- P9 / P10 (oracle side): round-to-nearest-even emulation ----
def test_bf16_rounding_bit_patterns():
    one = 1.0
    vals = np.array([one, one + 2 ** -8, one + 3 * 2 ** -8, one + 2 ** -8 + 2 ** -20,
                     -(one + 3 * 2 ** -8), 3.0e38, 1e-40], dtype=np.float32)
    out = O.round_bf16(vals)
    assert out[0] == 1.0
    assert out[1] == 1.0                      # tie -> even
    assert out[2] == 1.0 + 2 ** -6            # tie -> even (upwards)
    assert out[3] == 1.0 + 2 ** -7            # above the tie
    assert out[4] == -(1.0 + 2 ** -6)
    assert np.isfinite(out[5]) or np.isinf(out[5])
    # every output is a bf16 value: low 16 bits zero
    assert np.all((out.view(np.uint32) & 0xFFFF) == 0)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = _rng(10)
    v = (rng.standard_normal(200000) * np.exp(rng.uniform(-20, 20, 200000))).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(O.round_bf16(v), ref)


def test_fp16_rounding_bit_patterns():
    vals = np.array([1.0 + 2 ** -11, 1.0 + 3 * 2 ** -11, 2049.0, 2051.0, 65520.0, 2 ** -25, 3 * 2 ** -26],
                    dtype=np.float32)
    out = O.round_fp16(vals)
    assert out[0] == 1.0
    assert out[1] == 1.0 + 2 ** -9
    assert out[2] == 2048.0
    assert out[3] == 2052.0
    assert np.isinf(out[4])                   # above the largest half
    assert out[5] == 0.0                      # half of the smallest subnormal: tie -> even (zero)
    assert out[6] == 2 ** -24


def test_pow2_ceil():
    got = O.pow2_ceil(np.array([0.5, 0.51, 1.0, 3.0, 0.0, 2 ** -30 * 1.5]))
    np.testing.assert_array_equal(got, [0.5, 1.0, 1.0, 4.0, 1.0, 2 ** -29])


@pytest.mark.parametrize("kind,bound", [("bf16", 2 ** -9), ("fp16", 2 ** -12)])
def test_quantised_links_error_bound_and_hermiticity(kind, bound):
    rng = _rng(11)
    dims, nb = (2, 2, 2, 2), 4
    offs = W.stencil("9pt")
    links = W.hermitian_links(rng, dims, nb, offs, shift=1.0)
    q = O.quantize_links(links, offs, kind)
    s = O.link_scales(links)
    err = np.abs(q - links.astype(complex))
    for p in range(offs.shape[0]):
        if not np.any(offs[p]):
            assert np.max(err[:, p]) == 0.0       # self block stays complex64
            continue
        lim = bound * s[:, p][:, None, None]
        assert np.all(np.abs(q[:, p].real - links[:, p].real) <= lim)
        assert np.all(np.abs(q[:, p].imag - links[:, p].imag) <= lim)
    m = O.dense(q, offs, dims)
    assert np.max(np.abs(m - m.conj().T)) == 0.0


@pytest.mark.parametrize("kind", ["bf16", "fp16"])
def test_lowp_exact_on_integer_grid(kind):
    rng = _rng(12)
    dims, nb, nr = (2, 3, 2, 2), 4, 3
    offs = W.stencil("9pt")
    links = W.integer_links(rng, dims, nb, offs.shape[0])
    x = W.integer_vectors(rng, dims, nb, nr)
    np.testing.assert_array_equal(O.apply_lowp(links, offs, dims, x, kind), O.apply(links, offs, dims, x))


def test_lowp_apply_error_small():
    rng = _rng(13)
    dims, nb, nr = (3, 2, 2, 2), 8, 4
    offs = W.stencil("9pt")
    links = W.hermitian_links(rng, dims, nb, offs, shift=3.0)
    x = _rand_vec(rng, dims, nb, nr)
    y = O.apply(links, offs, dims, x)
    for kind, lim in (("bf16", 2e-2), ("fp16", 2e-3)):
        e = np.max(np.abs(O.apply_lowp(links, offs, dims, x, kind) - y)) / np.max(np.abs(y))
        assert 0 < e < lim


# ---- P11 / P12 / P13: block CG ----
def _hpd_system(seed, dims=(2, 2, 2, 2), nb=4, nr=2, shift=2.0, kind="9pt"):
    rng = _rng(seed)
    offs = W.stencil(kind)
    links = W.hermitian_links(rng, dims, nb, offs, shift=shift)
    b = _rand_vec(rng, dims, nb, nr)
    return links, offs, dims, b


def test_bcgrq_matches_lu_c1():
    s = W.C1
    links, offs, b = W.make_system(s)
    m = O.dense(links, offs, s.dims)
    assert np.min(np.linalg.eigvalsh(m)) > 0
    op = lambda v: O.flatten(O.apply(links, offs, s.dims, v.reshape(s.volume, s.nbasis, -1)))
    x, info = O.bcgrq(op, O.flatten(b), tol=1e-12, maxiter=500)
    assert info.converged and not info.breakdown
    ref = O.solve_dense(links, offs, s.dims, b)
    np.testing.assert_allclose(x, O.flatten(ref), rtol=0, atol=1e-10 * np.max(np.abs(ref)))
    assert np.max(O.true_relres(op, O.flatten(b), x)) <= 1e-11


def test_bcgrq_without_c_in_update_fails():
    """The update printed without C_k does not solve the system (the correction is needed)."""
    links, offs, dims, b = _hpd_system(14)
    m = O.dense(links, offs, dims)
    bb = O.flatten(b) * 5.0          # C_0 far from the identity
    r = bb.copy()
    c = O.chol_upper(r.conj().T @ r)
    q = np.linalg.solve(c.T, r.T).T
    d = q.copy()
    x = np.zeros_like(bb)
    for _ in range(60):
        z = m @ d
        mk = np.linalg.inv(d.conj().T @ z)
        x = x + d @ mk                  # as printed
        t = q - z @ mk
        try:
            s = O.chol_upper(t.conj().T @ t, 1e-28)
        except O.Breakdown:
            break
        q = np.linalg.solve(s.T, t.T).T
        d = q + d @ s.conj().T
        c = s @ c
    assert np.max(np.linalg.norm(bb - m @ x, axis=0) / np.linalg.norm(bb, axis=0)) > 1e-2
    xs, info = O.bcgrq(lambda v: m @ v, bb, tol=1e-12, maxiter=200)
    assert np.max(np.linalg.norm(bb - m @ xs, axis=0) / np.linalg.norm(bb, axis=0)) < 1e-10


def test_bcgrq_invariants():
    links, offs, dims, b = _hpd_system(15, nr=3)
    m = O.dense(links, offs, dims)
    bb = O.flatten(b)
    x, info = O.bcgrq(lambda v: m @ v, bb, tol=1e-13, maxiter=200, record=True)
    assert info.converged
    for k in range(min(6, len(info.history_c))):
        xk, qk, ck, dk = info.history_x[k], info.history_q[k], info.history_c[k], info.history_d[k]
        r = bb - m @ xk
        # R_k = Q_k C_k, column norms of R equal those of C
        np.testing.assert_allclose(np.linalg.norm(r, axis=0), np.linalg.norm(ck, axis=0), rtol=1e-9)
        np.testing.assert_allclose(qk @ ck, r, atol=1e-9 * np.max(np.abs(r)))
        # Q_k orthonormal
        np.testing.assert_allclose(qk.conj().T @ qk, np.eye(qk.shape[1]), atol=1e-10)
    # block M-conjugacy of successive search directions
    ds = info.history_d[:6]
    for i in range(len(ds)):
        for j in range(i):
            g = ds[i].conj().T @ m @ ds[j]
            assert np.max(np.abs(g)) < 1e-8 * np.linalg.norm(ds[i]) * np.linalg.norm(ds[j]) * np.linalg.norm(m, 2)


def test_bcgrq_finite_termination():
    """n = 64 unknowns, 2 RHS: the block Krylov space is exhausted after n/2 = 32 steps."""
    links, offs, dims, b = _hpd_system(16, nb=4, nr=2, shift=1.5)
    m = O.dense(links, offs, dims)
    kappa = np.linalg.cond(m)
    assert kappa < 50
    x, info = O.bcgrq(lambda v: m @ v, O.flatten(b), tol=1e-11, maxiter=200)
    assert info.converged and info.iterations <= 32


def test_bcgrq_single_rhs_equals_textbook_cg():
    links, offs, dims, b = _hpd_system(17, nr=1)
    m = O.dense(links, offs, dims)
    bb = O.flatten(b)
    x, info = O.bcgrq(lambda v: m @ v, bb, tol=1e-12, maxiter=40, record=True)
    xc, res, xs = O.cg(lambda v: m @ v, bb[:, 0], tol=1e-12, maxiter=40, record=True)
    n = min(len(info.history_x), len(xs))
    assert n > 5
    for k in range(n):
        np.testing.assert_allclose(info.history_x[k][:, 0], xs[k], atol=1e-10 * np.max(np.abs(xc)))


def test_bcgrq_rank_deficient_breaks_down():
    links, offs, dims, b = _hpd_system(18, nr=2)
    m = O.dense(links, offs, dims)
    bb = O.flatten(b)
    bb[:, 1] = 2.0 * bb[:, 0]
    x, info = O.bcgrq(lambda v: m @ v, bb, tol=1e-10, maxiter=100)
    assert info.breakdown


# ---- P14: convergence rate bound and the paper's printed rates ----
def test_paper_rate_numbers():
    g = json.load(open(os.path.join(GOLDEN, "paper_rates.json")))
    kappa = g["fine_lambda_max"]["value"] / g["fine_lambda_min"]["value"]
    assert abs(O.chebyshev_rate(kappa) - g["sigma_bound"]["value"]) < 5e-7
    # the fitted CG rate sits just above the bound (bound saturated)
    assert g["sigma_cg_fit"]["value"] >= g["sigma_bound"]["value"]
    kp = O.kappa_from_rate(g["sigma_hdcg"]["value"])
    assert abs(kp - g["kappa_precon"]["value"]) < 0.1
    assert abs(g["smoother_lambda"]["value"] / kp - g["lambda_effective"]["value"]) < 5e-6


def test_cg_rate_within_chebyshev_bound():
    """Constant-link operator with an exactly known spectrum (Fourier symbol)."""
    dims = (6, 6, 6, 6)
    offs = W.stencil("9pt")
    V = W.volume(dims)
    m2 = 0.02
    links = np.zeros((V, 9, 1, 1), dtype=np.complex64)
    links[:, 0] = 8 + m2
    links[:, 1:] = -1.0
    lam = []
    for n in np.ndindex(*dims):
        k = 2 * np.pi * np.asarray(n) / 6
        lam.append(m2 + np.sum(4 * np.sin(k / 2) ** 2))
    kappa = max(lam) / min(lam)
    sigma = O.chebyshev_rate(kappa)
    rng = _rng(19)
    b = rng.standard_normal(V) + 1j * rng.standard_normal(V)
    op = lambda v: O.apply(links, offs, dims, v.reshape(V, 1, 1)).reshape(-1)
    x, res, _ = O.cg(op, b, tol=1e-10, maxiter=2000)
    # energy-norm error contracts at least as 2*sigma^k; the residual follows up to sqrt(kappa)
    k = len(res)
    assert res[-1] <= 1e-10
    assert k <= math.ceil(math.log(2e10 * math.sqrt(kappa)) / -math.log(sigma))


# ---- defect correction around a low-precision inner solve ----
@pytest.mark.parametrize("kind", ["bf16", "fp16"])
def test_defect_correction_reaches_tolerance(kind):
    s = W.C1
    links, offs, b = W.make_system(s)
    op = lambda v: O.flatten(O.apply(links, offs, s.dims, v.reshape(s.volume, s.nbasis, -1)))
    ql = O.quantize_links(links, offs, kind)
    opq = lambda v: O.flatten(O.apply(ql, offs, s.dims, v.reshape(s.volume, s.nbasis, -1)))

    def inner(r):
        e, info = O.bcgrq(opq, r, tol=1e-3, maxiter=200)
        return e, info.iterations

    x, info = O.defect_correction(op, inner, O.flatten(b), tol=1e-12, max_outer=30)
    assert info.converged
    assert np.max(O.true_relres(op, O.flatten(b), x)) <= 1e-12
    assert info.cycles <= 10


# ---- P15: gradients against central finite differences (complex128) ----
def _fd_system(seed=20):
    s = W.C5_FD
    links, offs, b = W.make_system(s)
    rng = _rng(seed)
    w = _rand_vec(rng, s.dims, s.nbasis, s.nrhs)
    return s, links.astype(np.complex128), offs, b, w


def test_apply_gradients_vs_fd():
    s, links, offs, x, w = _fd_system()
    loss_x = lambda z: float(np.real(np.vdot(w, O.apply(links, offs, s.dims, z))))
    loss_a = lambda a: float(np.real(np.vdot(w, O.apply(a, offs, s.dims, x))))
    dx, da = O.apply_vjp(links, offs, s.dims, x, w)
    np.testing.assert_allclose(dx, O.fd_gradient(loss_x, x), atol=1e-7)
    np.testing.assert_allclose(da, O.fd_gradient(loss_a, links), atol=1e-7)


def test_solve_gradients_vs_fd():
    s, links, offs, b, w = _fd_system(21)
    m = O.dense(links, offs, s.dims)
    assert np.min(np.linalg.eigvalsh(m)) > 0.1
    loss_b = lambda z: float(np.real(np.vdot(w, O.solve_dense(links, offs, s.dims, z))))
    loss_a = lambda a: float(np.real(np.vdot(w, O.solve_dense(a, offs, s.dims, b))))
    x, lam, da = O.solve_vjp_dense(links, offs, s.dims, b, w)
    np.testing.assert_allclose(lam, O.fd_gradient(loss_b, b), atol=1e-6)
    np.testing.assert_allclose(da, O.fd_gradient(loss_a, links), atol=1e-6)


def test_gradient_directional_identity():
    """dL = Re sum tr(dA^H E_A) + Re <dX, E_X> for a random direction (E_A, E_X)."""
    s, links, offs, x, w = _fd_system(22)
    rng = _rng(23)
    ea = (rng.standard_normal(links.shape) + 1j * rng.standard_normal(links.shape))
    ex = (rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape))
    dx, da = O.apply_vjp(links, offs, s.dims, x, w)
    f = lambda t: float(np.real(np.vdot(w, O.apply(links + t * ea, offs, s.dims, x + t * ex))))
    h = 1e-5
    fd = (f(h) - f(-h)) / (2 * h)
    an = float(np.real(np.vdot(da, ea)) + np.real(np.vdot(dx, ex)))
    assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


def test_apply_at_sites_matches_full_apply():
    rng = _rng(24)
    dims, nb = (3, 2, 3, 2), 3
    offs = W.stencil("81pt")
    links = W.gaussian_links(rng, dims, nb, offs.shape[0])
    x = _rand_vec(rng, dims, nb, 2)
    sites = np.array([0, 5, 17, 35])
    np.testing.assert_allclose(O.apply_at(links, offs, dims, x, sites), O.apply(links, offs, dims, x)[sites],
                               atol=1e-13)


# ---------------------------------------------------------------------------
# Stationary Chebyshev approximation to 1/x (Sec. 2.3)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("lo,hi,order", [(0.02, 40.0, 120), (2.0, 92.0, 8), (0.5, 3.0, 0), (0.1, 7.0, 33)])
def test_chebyshev_coefficients_match_numpy_interpolant(lo, hi, order):
    """The coefficients equal numpy's Chebyshev interpolant (points of the first
    kind) of 1/x mapped to [-1, 1]; the paper's two parameter sets included
    (coarse solve [0.02, 40, 120], smoother [2, 92, 8])."""
    from numpy.polynomial import chebyshev as C
    ref = C.chebinterpolate(lambda y: 1.0 / (0.5 * (hi - lo) * y + 0.5 * (hi + lo)), order)
    got = O.chebyshev_coefficients(lo, hi, order)
    assert got.shape == (order + 1,)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("lo,hi,order", [(0.02, 40.0, 120), (2.0, 92.0, 8), (0.1, 7.0, 33)])
def test_chebyshev_interpolates_at_nodes(lo, hi, order):
    """P(x_j) = 1/x_j at the n + 1 Chebyshev points (numpy's evaluation of the
    series), and away from the points P stays close to 1/x on [lo, hi] for a
    well-resolved order."""
    from numpy.polynomial import chebyshev as C
    c = O.chebyshev_coefficients(lo, hi, order)
    yj = np.cos(np.pi * (np.arange(order + 1) + 0.5) / (order + 1))
    xj = 0.5 * (hi - lo) * yj + 0.5 * (hi + lo)
    assert np.max(np.abs(C.chebval(yj, c) * xj - 1.0)) <= 1e-10
    if (hi / lo) ** 0.5 * 4 < order:  # resolved: error bound decays like ((sqrt k - 1)/(sqrt k + 1))^n
        x = np.linspace(lo, hi, 2001)
        y = (2 * x - (hi + lo)) / (hi - lo)
        assert np.max(np.abs(C.chebval(y, c) * x - 1.0)) <= 1e-3


def test_chebyshev_apply_diagonal_operator():
    """Self-only stencil with the same diagonal block at every site: P(M) acts on
    row i of every block as the scalar P(lambda_i), evaluated with numpy."""
    from numpy.polynomial import chebyshev as C
    dims, nb, nr = (2, 2, 2, 2), 6, 3
    lo, hi, order = 0.3, 5.0, 17
    lam = np.linspace(0.35, 4.9, nb).astype(np.float32).astype(np.float64)  # the stored link values
    links = np.zeros((16, 1, nb, nb), dtype=np.complex64)
    links[:, 0] = np.diag(lam).astype(np.complex64)
    offs = W.stencil("self")
    b = _rand_vec(np.random.default_rng(3), dims, nb, nr)
    got = O.chebyshev_apply(lambda v: O.apply(links, offs, dims, v), b, lo, hi, order)
    scal = C.chebval((2 * lam - (hi + lo)) / (hi - lo), O.chebyshev_coefficients(lo, hi, order))
    assert np.max(np.abs(got - scal[None, :, None] * b)) <= 1e-12 * np.max(np.abs(got))


@pytest.mark.parametrize("order", [1, 2, 30])
def test_chebyshev_apply_matches_eigendecomposition(order):
    """A Hermitian 9-point operator on 2^4 sites: P(M) b = U P(Lambda) U^H b from
    the dense eigendecomposition, P evaluated with numpy on the eigenvalues."""
    from numpy.polynomial import chebyshev as C
    dims, nb, nr = (2, 2, 2, 2), 3, 2
    rng = np.random.default_rng(11)
    offs = W.stencil("9pt")
    links = W.hermitian_links(rng, dims, nb, offs, shift=3.0)
    M = O.dense(links, offs, dims)
    lam, U = np.linalg.eigh(M)
    lo, hi = 0.9 * lam.min(), 1.1 * lam.max()
    assert lo > 0
    b = _rand_vec(rng, dims, nb, nr)
    got = O.chebyshev_apply(lambda v: O.apply(links, offs, dims, v), b, lo, hi, order)
    p = C.chebval((2 * lam - (hi + lo)) / (hi - lo), O.chebyshev_coefficients(lo, hi, order))
    ref = (U @ (p[:, None] * (U.conj().T @ O.flatten(b)))).reshape(b.shape)
    assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(ref))


# ---------------------------------------------------------------------------
# Preconditioned BlockCGrQ (Fig. 2 right, Sec. 2.2) with the Chebyshev
# polynomial as the stationary preconditioner (Sec. 2.3)
# ---------------------------------------------------------------------------

def _cheb_dense(m, lo, hi, order):
    """P(M) as a dense matrix from the eigendecomposition, P evaluated with numpy."""
    from numpy.polynomial import chebyshev as C
    lam, U = np.linalg.eigh(m)
    p = C.chebval((2 * lam - (hi + lo)) / (hi - lo), O.chebyshev_coefficients(lo, hi, order))
    return (U * p[None, :]) @ U.conj().T


@pytest.mark.parametrize("lo_frac,hi_frac,order", [(0.5, 1.1, 8), (3.0, 1.0, 5), (0.02, 1.2, 30)])
def test_chebyshev_residual_polynomial_closed_form(lo_frac, hi_frac, order):
    """x P(x) - 1 is a degree n + 1 polynomial vanishing at the n + 1 interpolation
    points and equal to -1 at x = 0, so 1 - x P(x) = T_{n+1}(y(x)) / T_{n+1}(y(0)).
    Hence 0 < x P(x) < 2 on [lo, hi] and 0 < x P(x) < 1 on (0, lo): P is positive
    on (0, hi] and P(M) is Hermitian positive definite whenever the spectrum of
    the HPD operator M lies below hi, wherever lo sits."""
    from numpy.polynomial import chebyshev as C
    lo, hi = lo_frac, 10.0 * hi_frac
    c = O.chebyshev_coefficients(lo, hi, order)
    x = np.concatenate([np.linspace(1e-3, lo, 400), np.linspace(lo, hi, 2001)])
    y = (2 * x - (hi + lo)) / (hi - lo)
    y0 = -(hi + lo) / (hi - lo)
    tn = np.zeros(order + 2)
    tn[-1] = 1.0
    ref = C.chebval(y, tn) / C.chebval(y0, tn)
    got = 1.0 - x * C.chebval(y, c)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-10)
    xp = x * C.chebval(y, c)
    assert np.all(xp > 0) and np.all(xp[x <= lo] < 1 + 1e-12) and np.all(xp < 2)


def _pcg_system(seed=21, nr=3, shift=1.2):
    links, offs, dims, b = _hpd_system(seed, nr=nr, shift=shift)
    m = O.dense(links, offs, dims)
    lam = np.linalg.eigvalsh(m)
    assert lam.min() > 0
    return m, lam, O.flatten(b)


def test_pbcgrq_matches_dense_solve():
    m, lam, bb = _pcg_system()
    P = _cheb_dense(m, 0.5 * lam.min(), 1.1 * lam.max(), 6)
    x, info = O.pbcgrq(lambda v: m @ v, lambda v: P @ v, bb, tol=1e-12, maxiter=200)
    assert info.converged and not info.breakdown
    ref = np.linalg.solve(m, bb)
    np.testing.assert_allclose(x, ref, rtol=0, atol=1e-10 * np.max(np.abs(ref)))


def test_pbcgrq_identity_preconditioner_is_bcgrq():
    """With M^{-1} = I the M inner product is the Euclidean one, q = Q and the
    iteration is BlockCGrQ step for step (the stop tests coincide too:
    ||C_0 e_j|| = ||b_j|| from X_0 = 0)."""
    m, lam, bb = _pcg_system(22)
    x1, i1 = O.bcgrq(lambda v: m @ v, bb, tol=1e-11, maxiter=200, record=True)
    x2, i2 = O.pbcgrq(lambda v: m @ v, lambda v: v, bb, tol=1e-11, maxiter=200, record=True)
    assert i1.iterations == i2.iterations
    for a, b in zip(i1.history_x, i2.history_x):
        np.testing.assert_allclose(b, a, rtol=0, atol=1e-12 * np.max(np.abs(x1)))


def test_pbcgrq_single_rhs_equals_textbook_pcg():
    """N_rhs = 1 reduces to the textbook preconditioned CG (Saad, Alg. 9.1):
    alpha = (r, z) / (A p, p), x += alpha p, r -= alpha A p, z = M^{-1} r,
    beta = (r_new, z_new) / (r, z), p = z + beta p; the iterates agree."""
    m, lam, bb = _pcg_system(23, nr=1)
    P = _cheb_dense(m, 0.3 * lam.min(), 1.05 * lam.max(), 4)
    x, info = O.pbcgrq(lambda v: m @ v, lambda v: P @ v, bb, tol=1e-12, maxiter=60, record=True)
    b1 = bb[:, 0]
    xs = [np.zeros_like(b1)]
    r = b1.copy()
    z = P @ r
    p = z.copy()
    rz = np.vdot(r, z)
    for _ in range(len(info.history_x) - 1):
        w = m @ p
        alpha = rz / np.vdot(p, w)
        xs.append(xs[-1] + alpha * p)
        r = r - alpha * w
        z = P @ r
        rz_new = np.vdot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    assert len(xs) > 5
    for k in range(len(xs)):
        np.testing.assert_allclose(info.history_x[k][:, 0], xs[k], rtol=0, atol=1e-10 * np.max(np.abs(x)))


def test_pbcgrq_exact_inverse_converges_in_one_step():
    """M^{-1} = H^{-1} makes M^{-1} H the identity: one block step solves."""
    m, lam, bb = _pcg_system(24)
    minv = np.linalg.inv(m)
    x, info = O.pbcgrq(lambda v: m @ v, lambda v: minv @ v, bb, tol=1e-10, maxiter=10)
    assert info.converged and info.iterations == 1
    np.testing.assert_allclose(m @ x, bb, rtol=0, atol=1e-10 * np.max(np.abs(bb)))


def test_pbcgrq_invariants():
    """q_k C_k = B - H X_k; Q_k = M^{-1} q_k; Q_k^H q_k = I (M-orthonormal);
    ||C_k e_j||^2 = r_j^H M^{-1} r_j; successive search directions H-conjugate."""
    m, lam, bb = _pcg_system(25)
    P = _cheb_dense(m, 0.5 * lam.min(), 1.1 * lam.max(), 5)
    x, info = O.pbcgrq(lambda v: m @ v, lambda v: P @ v, bb, tol=1e-13, maxiter=100, record=True)
    assert info.converged
    nr = bb.shape[1]
    for k in range(min(6, len(info.history_c))):
        xk, qk, ck, dk = info.history_x[k], info.history_q[k], info.history_c[k], info.history_d[k]
        r = bb - m @ xk
        np.testing.assert_allclose(qk @ ck, r, rtol=0, atol=1e-9 * np.max(np.abs(bb)))
        Qk = P @ qk
        np.testing.assert_allclose(Qk.conj().T @ qk, np.eye(nr), rtol=0, atol=1e-10)
        mn = np.sqrt(np.real(np.einsum("ij,ij->j", r.conj(), P @ r)))
        np.testing.assert_allclose(np.linalg.norm(ck, axis=0), mn, rtol=1e-9)
    ds = info.history_d[:6]
    for i in range(len(ds)):
        for j in range(i):
            g = ds[i].conj().T @ m @ ds[j]
            assert np.max(np.abs(g)) < 1e-8 * np.linalg.norm(ds[i]) * np.linalg.norm(ds[j]) * np.linalg.norm(m, 2)


def test_pbcgrq_iterations_within_preconditioned_bound():
    """The spectrum of P(H) H lies in [1 - eps, 1 + eps] with
    eps = 1 / |T_{n+1}(y(0))| when [lo, hi] covers the spectrum, so the
    preconditioned condition number is (1 + eps) / (1 - eps) and the CG bound
    2 sigma^k (sigma from that number) caps the iteration count; the
    unpreconditioned solve needs several times more."""
    m, lam, bb = _pcg_system(26, shift=1.2)
    lo, hi, order = 0.95 * lam.min(), 1.05 * lam.max(), 12
    y0 = -(hi + lo) / (hi - lo)
    eps = 1.0 / abs(np.cosh((order + 1) * np.arccosh(abs(y0))))
    kap = (1 + eps) / (1 - eps)
    ev = np.linalg.eigvals(_cheb_dense(m, lo, hi, order) @ m).real
    assert ev.min() >= 1 - eps - 1e-10 and ev.max() <= 1 + eps + 1e-10
    tol = 1e-10
    sig = O.chebyshev_rate(kap)
    # error in the H norm <= 2 sig^k; the relative M^{-1} residual norm is
    # within sqrt(kappa') of it
    bound = math.ceil(math.log(tol / (2 * math.sqrt(kap))) / math.log(sig)) + 1
    P = _cheb_dense(m, lo, hi, order)
    _, ip = O.pbcgrq(lambda v: m @ v, lambda v: P @ v, bb, tol=tol, maxiter=200)
    _, iu = O.bcgrq(lambda v: m @ v, bb, tol=tol, maxiter=400)
    assert ip.converged and iu.converged
    assert ip.iterations <= bound
    assert 2 * ip.iterations < iu.iterations


def test_pbcgrq_rank_deficient_breaks_down():
    m, lam, bb = _pcg_system(27)
    bb[:, 2] = bb[:, 0] - 3.0 * bb[:, 1]
    P = _cheb_dense(m, 0.5 * lam.min(), 1.1 * lam.max(), 4)
    x, info = O.pbcgrq(lambda v: m @ v, lambda v: P @ v, bb, tol=1e-10, maxiter=50)
    assert info.breakdown


# ---------------------------------------------------------------------------
# Multi-RHS deflation and the deflated Chebyshev coarse solve (Sec. 2.3)
# ---------------------------------------------------------------------------

def _eig_system(seed=31, nr=3):
    dims, nb = (2, 2, 2, 2), 3
    rng = np.random.default_rng(seed)
    offs = W.stencil("9pt")
    links = W.hermitian_links(rng, dims, nb, offs, shift=3.0)
    m = O.dense(links, offs, dims)
    lam, U = np.linalg.eigh(m)
    b = O.flatten(_rand_vec(rng, dims, nb, nr))
    return links, offs, dims, m, lam, U, b


def test_deflation_full_basis_is_the_inverse():
    """With every eigenpair, Defl = M^{-1} and nothing is left orthogonal."""
    links, offs, dims, m, lam, U, b = _eig_system()
    d, xp = O.deflate(U, lam, b)
    np.testing.assert_allclose(d, np.linalg.solve(m, b), rtol=0, atol=1e-12 * np.max(np.abs(d)))
    assert np.max(np.abs(xp)) <= 1e-12 * np.max(np.abs(b))


def test_deflation_projector_properties():
    """x_perp is orthogonal to the deflation space and x - x_perp lies in it;
    Defl(x) = V diag(1/lambda) V^H x entry by entry (scalar loops)."""
    links, offs, dims, m, lam, U, b = _eig_system(32)
    rng = np.random.default_rng(4)
    nev = 7
    v, _ = np.linalg.qr(rng.standard_normal((b.shape[0], nev)) + 1j * rng.standard_normal((b.shape[0], nev)))
    lv = rng.uniform(0.5, 2.0, nev)
    d, xp = O.deflate(v, lv, b)
    assert np.max(np.abs(v.conj().T @ xp)) <= 1e-12 * np.max(np.abs(b))
    par = b - xp
    np.testing.assert_allclose(v @ (v.conj().T @ par), par, rtol=0, atol=1e-12 * np.max(np.abs(b)))
    ref = np.zeros_like(d)
    for r in range(b.shape[1]):
        for i in range(nev):
            ci = sum(np.conj(v[k, i]) * b[k, r] for k in range(b.shape[0]))
            ref[:, r] += v[:, i] * ci / lv[i]
    np.testing.assert_allclose(d, ref, rtol=0, atol=1e-12 * np.max(np.abs(ref)))


@pytest.mark.parametrize("nev,order", [(0, 9), (5, 9), (20, 4)])
def test_deflated_chebyshev_is_diagonal_in_the_eigenbasis(nev, order):
    """Sec. 2.3: in the eigenbasis the stationary coarse solve is
    diag(1/lambda_1 .. 1/lambda_nev, P(lambda_nev+1) .. P(lambda_max)); with no
    deflation vectors it is the plain polynomial."""
    from numpy.polynomial import chebyshev as C
    links, offs, dims, m, lam, U, b = _eig_system(33)
    lo, hi = lam[min(nev, len(lam) - 1)] * 0.9, 1.1 * lam[-1]
    v, lv = U[:, :nev], lam[:nev]
    op = lambda z: m @ z
    got = O.deflated_chebyshev(op, v, lv, b, lo, hi, order)
    p = C.chebval((2 * lam - (hi + lo)) / (hi - lo), O.chebyshev_coefficients(lo, hi, order))
    diag = np.where(np.arange(len(lam)) < nev, 1.0 / lam, p)
    ref = U @ (diag[:, None] * (U.conj().T @ b))
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-11 * np.max(np.abs(ref)))
    if nev == 0:
        np.testing.assert_allclose(got, O.chebyshev_apply(op, b, lo, hi, order), rtol=0, atol=1e-13)


# ---------------------------------------------------------------------------
# Block project / promote (Sec. 2.5)
# ---------------------------------------------------------------------------

def _block_basis(rng, nsite, vblock, nb, orthonormal=True):
    a = rng.standard_normal((nsite, vblock, nb)) + 1j * rng.standard_normal((nsite, vblock, nb))
    if orthonormal:
        a = np.stack([np.linalg.qr(a[s])[0] for s in range(nsite)])
    return a


def test_block_project_promote_scalar_loops():
    rng = np.random.default_rng(41)
    nsite, vblock, nb, nr = 3, 5, 4, 2
    B = _block_basis(rng, nsite, vblock, nb, orthonormal=False)
    F = rng.standard_normal((nsite, vblock, nr)) + 1j * rng.standard_normal((nsite, vblock, nr))
    Cc = rng.standard_normal((nsite, nb, nr)) + 1j * rng.standard_normal((nsite, nb, nr))
    P, Q = O.block_project(B, F), O.block_promote(B, Cc)
    for s in range(nsite):
        for i in range(nb):
            for r in range(nr):
                assert abs(P[s, i, r] - sum(np.conj(B[s, k, i]) * F[s, k, r] for k in range(vblock))) < 1e-12
        for k in range(vblock):
            for r in range(nr):
                assert abs(Q[s, k, r] - sum(B[s, k, i] * Cc[s, i, r] for i in range(nb))) < 1e-12


def test_block_project_promote_adjoint_and_projector():
    """<project F, C> = <F, promote C>; with an orthonormal basis per block,
    project after promote is the identity and promote after project is the
    orthogonal projector onto the basis span (idempotent, leaves F - PF
    orthogonal to every basis vector)."""
    rng = np.random.default_rng(42)
    nsite, vblock, nb, nr = 4, 24, 8, 3
    B = _block_basis(rng, nsite, vblock, nb)
    F = rng.standard_normal((nsite, vblock, nr)) + 1j * rng.standard_normal((nsite, vblock, nr))
    Cc = rng.standard_normal((nsite, nb, nr)) + 1j * rng.standard_normal((nsite, nb, nr))
    lhs = np.vdot(O.block_project(B, F), Cc)
    rhs = np.vdot(F, O.block_promote(B, Cc))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    np.testing.assert_allclose(O.block_project(B, O.block_promote(B, Cc)), Cc, rtol=0, atol=1e-12)
    PF = O.block_promote(B, O.block_project(B, F))
    np.testing.assert_allclose(O.block_promote(B, O.block_project(B, PF)), PF, rtol=0, atol=1e-12)
    assert np.max(np.abs(O.block_project(B, F - PF))) <= 1e-12


# ---- block Lanczos for the deflation vectors ----
def test_block_lanczos_full_space_gives_every_eigenpair():
    """n = 48 unknowns, block 4, 12 steps: the Krylov space is the whole space,
    so the Ritz values are the eigenvalues (dense eigh) and every Ritz pair is
    exact."""
    dims, nb = (2, 2, 2, 2), 3
    rng = np.random.default_rng(51)
    offs = W.stencil("9pt")
    links = W.hermitian_links(rng, dims, nb, offs, shift=3.0)
    m = O.dense(links, offs, dims)
    lam = np.linalg.eigvalsh(m)
    x0 = rng.standard_normal((48, 4)) + 1j * rng.standard_normal((48, 4))
    theta, V, res = O.block_lanczos(lambda z: m @ z, x0, 12, 48)
    np.testing.assert_allclose(theta, lam, rtol=0, atol=1e-10 * np.max(np.abs(lam)))
    np.testing.assert_allclose(V.conj().T @ V, np.eye(48), rtol=0, atol=1e-10)
    np.testing.assert_allclose(m @ V, V * theta[None, :], rtol=0, atol=1e-9 * np.max(np.abs(lam)))


def test_block_lanczos_lowest_pairs_and_residual_estimate():
    """A 9-point operator on 3^4 sites (n = 324), block 8, 20 steps: the lowest
    Ritz values lie above the true eigenvalues and converge to them; each Ritz
    residual ||H v - theta v|| equals the block estimate ||B Y_last||, and every
    eigenvalue lies within its residual of its Ritz value (Kahan's bound)."""
    dims, nb = (3, 3, 3, 3), 4
    rng = np.random.default_rng(52)
    offs = W.stencil("9pt")
    links = W.hermitian_links(rng, dims, nb, offs, shift=3.0)
    m = O.dense(links, offs, dims)
    lam = np.linalg.eigvalsh(m)
    x0 = rng.standard_normal((324, 8)) + 1j * rng.standard_normal((324, 8))
    theta, V, res = O.block_lanczos(lambda z: m @ z, x0, 20, 12)
    direct = np.linalg.norm(m @ V - V * theta[None, :], axis=0)
    np.testing.assert_allclose(direct, res, rtol=1e-6, atol=1e-10)
    assert np.all(theta >= lam[:12] - 1e-10)
    for t, r in zip(theta, res):
        assert np.min(np.abs(lam - t)) <= r + 1e-10
    assert np.max(np.abs(theta[:4] - lam[:4])) <= 1e-6 * np.max(np.abs(lam))


# ---- Spectral helpers behind the kappa-targeting shifts (Sec. 3, Eq. bound) ----
def _hermitian_dense(dims, nb, shift, seed):
    offs = W.stencil("9pt")
    links = W.hermitian_links(_rng(seed), dims, nb, offs, shift)
    return O.dense(links, offs, dims)


def test_lanczos_extremes_converge_to_dense_spectrum():
    """Enough steps on a 3^4 x 4 Hermitian 9-point operator (324 unknowns): the
    extreme Ritz values equal numpy's extreme eigenvalues, their bounds are
    tiny, and the Ritz values lie inside the spectrum (interlacing)."""
    m = _hermitian_dense((3, 3, 3, 3), 4, 0.0, 11)
    ev = np.linalg.eigvalsh(m)
    tmin, tmax, bmin, bmax = O.lanczos_extremes(lambda v: m @ v, m.shape[0], 200, seed=5)
    scale = float(np.max(np.abs(ev)))
    assert abs(tmin - ev[0]) <= 1e-10 * scale and abs(tmax - ev[-1]) <= 1e-10 * scale
    assert bmin <= 1e-6 * scale and bmax <= 1e-6 * scale
    assert tmin >= ev[0] - 1e-12 * scale and tmax <= ev[-1] + 1e-12 * scale


def _krylov_ritz(m, v0, k):
    """Rayleigh-Ritz on the k-dimensional Krylov space of m from v0, by an
    orthonormal basis built with full (twice repeated) Gram-Schmidt, and the
    direct residual norms ||m y - theta y|| of the extreme Ritz pairs."""
    n = m.shape[0]
    q = np.zeros((n, k), dtype=np.complex128)
    q[:, 0] = v0 / np.linalg.norm(v0)
    for j in range(1, k):
        w = m @ q[:, j - 1]
        for _ in range(2):
            w = w - q[:, :j] @ (q[:, :j].conj().T @ w)
        q[:, j] = w / np.linalg.norm(w)
    h = q.conj().T @ m @ q
    th, s = np.linalg.eigh(0.5 * (h + h.conj().T))
    res = [float(np.linalg.norm(m @ (q @ s[:, i]) - th[i] * (q @ s[:, i]))) for i in (0, -1)]
    return float(th[0]), float(th[-1]), res[0], res[1]


@pytest.mark.parametrize("steps", [6, 12, 20])
def test_lanczos_extremes_bounds_are_the_ritz_residuals(steps):
    """Before convergence, on a 2^4 x 4 operator (64 unknowns): the returned
    Ritz values are those of the Krylov space (Rayleigh-Ritz on a basis built
    by full Gram-Schmidt, not the three-term recurrence) and each returned
    bound equals the direct residual norm of its Ritz pair; an eigenvalue of
    the dense matrix lies within that bound of each Ritz value. A wrong index
    in the bound (another component of the Ritz vector) or a sign slip in the
    recurrence fails here."""
    m = _hermitian_dense((2, 2, 2, 2), 4, 0.3, 12)
    n = m.shape[0]
    seed = 9
    rng = np.random.default_rng(seed)
    v0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)  # the oracle's documented start vector
    tmin, tmax, bmin, bmax = O.lanczos_extremes(lambda v: m @ v, n, steps, seed=seed)
    rmin_t, rmax_t, rmin_b, rmax_b = _krylov_ritz(m, v0, steps)
    scale = float(np.max(np.abs(np.linalg.eigvalsh(m))))
    assert abs(tmin - rmin_t) <= 1e-9 * scale and abs(tmax - rmax_t) <= 1e-9 * scale
    assert abs(bmin - rmin_b) <= 1e-7 * scale and abs(bmax - rmax_b) <= 1e-7 * scale
    ev = np.linalg.eigvalsh(m)
    assert np.min(np.abs(ev - tmin)) <= bmin * (1 + 1e-9) + 1e-12
    assert np.min(np.abs(ev - tmax)) <= bmax * (1 + 1e-9) + 1e-12
    # not converged yet at these step counts: the bounds carry information
    if steps <= 12:
        assert bmin > 1e-6 and bmax > 1e-6


@pytest.mark.parametrize("kappa", [10.0, 1e3, 1e4])
def test_kappa_shift_gives_the_target_condition_number(kappa):
    """The shift from the exact extremes of the unshifted operator H0 translates
    the spectrum to one whose eigenvalue ratio is kappa (dense H0 + s I in
    complex128); the workload construction, which adds s to the self term
    before rounding to complex64, gives the same spectrum up to that rounding."""
    dims, nb, seed = (2, 2, 2, 2), 4, 13
    m0 = _hermitian_dense(dims, nb, 0.0, seed)
    ev0 = np.linalg.eigvalsh(m0)
    s = O.kappa_shift(float(ev0[0]), float(ev0[-1]), kappa)
    ev = np.linalg.eigvalsh(m0 + s * np.eye(m0.shape[0]))
    assert ev[0] > 0
    assert abs(ev[-1] / ev[0] - kappa) <= 1e-9 * kappa
    ev_w = np.linalg.eigvalsh(_hermitian_dense(dims, nb, s, seed))
    np.testing.assert_allclose(ev_w, ev0 + s, rtol=0, atol=1e-6)
