"""Preconditioned BlockCGrQ (Fig. 2 right, Sec. 2.2) with the stationary
Chebyshev preconditioner (Sec. 2.3) on the GPU, through the C ABI, against the
complex128 oracle.

Iterate parity: one defect-correction cycle of k inner iterations from X = 0
gives X_1 = E diag(||b_j||) with E the k-th iterate of the inner iteration on
the normalised right-hand side; the oracle runs the same k steps of
``pbcgrq`` in complex128 with the same polynomial. The inner iteration runs in
float32 (Gram matrices and small steps in double), so each step carries the
rounding of one polynomial application (measured at the level of one apply,
about 2e-6 relative) and of the block updates; over k <= 4 steps of a system
whose preconditioned condition number is small these stay below 1e-4 of the
iterate's largest entry, the bound used here (measured: 7e-7 .. 3e-6). The
step counts stay below the point where the float32 residual reaches its
rounding floor (there the next Gram matrix is rank deficient in float32 and
the inner iteration ends by breakdown, which the double precision oracle
does not see).

Solves: the solution to the outer tolerance in the oracle's true residual,
against a dense solve on the small workload and a manufactured solution on the
8^4, nbasis 32, nrhs 16 workload.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import announce, dev, host, make_op, max_rel

pytestmark = pytest.mark.gpu

ITER_TOL = 1e-4


def _system(dims, nb, nr, kind, seed, shift):
    rng = np.random.default_rng(seed)
    offs = W.stencil(kind)
    links = W.hermitian_links(rng, dims, nb, offs, shift=shift).astype(np.complex64)
    b = W.gaussian_vectors(rng, dims, nb, nr, dtype=np.complex128)
    return links, offs, b


def _range(links, offs, dims):
    """[lo, hi] around the spectrum: Lanczos extremes widened by 10 %."""
    nb = links.shape[2]
    n = int(np.prod(dims)) * nb
    op = lambda v: O.apply(links, offs, dims, v.reshape(-1, nb, 1)).ravel()
    tmin, tmax, bmin, bmax = O.lanczos_extremes(op, n, steps=min(n, 120), seed=5)
    lo, hi = 0.9 * (tmin - bmin), 1.1 * (tmax + bmax)
    assert lo > 0
    return lo, hi


def _true_relres(links, offs, dims, b, x):
    r = b - O.apply(links, offs, dims, x)
    return np.linalg.norm(O.flatten(r), axis=0) / np.linalg.norm(O.flatten(b), axis=0)


def _oracle_one_cycle(links, offs, dims, b, lo, hi, order, k):
    op = lambda v: O.flatten(O.apply(links, offs, dims, v.reshape(b.shape)))
    prec = lambda v: O.flatten(O.chebyshev_apply(lambda u: O.apply(links, offs, dims, u), v.reshape(b.shape),
                                                 lo, hi, order))
    bb = O.flatten(b)
    rn = np.linalg.norm(bb, axis=0)
    e, info = O.pbcgrq(op, prec, bb / rn[None, :], tol=0.0, maxiter=k)
    assert info.iterations == k and not info.breakdown
    return (e * rn[None, :]).reshape(b.shape)


CASES = [((2, 4, 2, 4), 16, 5, "9pt", 4.0), ((4, 4, 4, 4), 32, 16, "9pt", 6.0), ((3, 2, 2, 4), 8, 3, "81pt", 14.0),
         ((2, 2, 2, 2), 16, 32, "81pt", 14.0), ((2, 2, 4, 2), 16, 1, "9pt", 4.0)]


@pytest.mark.parametrize("dims,nb,nr,kind,shift", CASES)
@pytest.mark.parametrize("order,k", [(0, 3), (3, 1), (2, 3), (6, 2)])
def test_pbcg_iterates_match_oracle(dims, nb, nr, kind, shift, order, k):
    from paper_2409_03904_amd import coarse
    links, offs, b = _system(dims, nb, nr, kind, 500 + nb + nr, shift)
    lo, hi = _range(links, offs, dims)
    ref = _oracle_one_cycle(links, offs, dims, b, lo, hi, order, k)
    op = make_op(links, offs, dims)
    forms = [None] + ([make_op(links, offs, dims, "c64_3m")] if nb % 16 == 0 else [])
    for inner in forms:
        announce("pbcg iterates", dims, nb, nr, kind, order, k, "3m" if inner is not None else "c64")
        res = coarse.pbcg_solve(op, dev(b), lo, hi, order, inner=inner, tol=1e-300, inner_tol=1e-300,
                                max_outer=1, max_inner=k, check_every=2, raise_on_failure=False)
        assert res.status == 1  # not converged: one cycle of k iterations
        assert res.cycles == 1 and res.iterations == k
        err = max_rel(host(res.x), ref)
        print("pbcg iterate error", order, k, err)
        assert err <= ITER_TOL


def test_pbcg_small_workload_matches_dense_solve():
    from paper_2409_03904_amd import coarse
    s = W.C1
    links, offs, b = W.make_system(s)
    lo, hi = _range(links.astype(np.complex64), offs, s.dims)
    op = make_op(links, offs, s.dims)
    announce("pbcg c1")
    for use_graph in (True, False):
        res = coarse.pbcg_solve(op, dev(b), lo, hi, 6, tol=s.tol, inner_tol=1e-4, use_graph=use_graph,
                                check_every=4)
        x = host(res.x)
        assert res.status == 0
        ref = O.solve_dense(links, offs, s.dims, b)
        assert np.max(np.abs(x - ref)) / np.max(np.abs(ref)) <= 1e-9
        assert np.max(_true_relres(links, offs, s.dims, b, x)) <= s.tol
        assert res.relres_max <= s.tol


@pytest.mark.parametrize("kind", ["c64_3m", "bf16", "fp16"])
def test_pbcg_lowp_inner(kind):
    from paper_2409_03904_amd import coarse
    s = W.System("c1.16", (4, 4, 4, 4), 16, 4, "9pt", kappa=None, shift=4.0, tol=1e-10, seed_index=61)
    links, offs, b = W.make_system(s)
    lo, hi = _range(links.astype(np.complex64), offs, s.dims)
    announce("pbcg lowp", kind)
    op = make_op(links, offs, s.dims)
    inner = make_op(links, offs, s.dims, kind)
    res = coarse.pbcg_solve(op, dev(b), lo, 1.1 * hi, 8, inner=inner, tol=s.tol, inner_tol=1e-2)
    assert res.status == 0
    assert np.max(_true_relres(links, offs, s.dims, b, host(res.x))) <= s.tol


def test_pbcg_fp32_workload_to_tolerance():
    """8^4, nbasis 32, nrhs 16, kappa 1e3, tolerance 1e-8, manufactured solution;
    degree 16 on [lambda_max / 200, 1.1 lambda_max]: fewer inner iterations
    than the unpreconditioned solve, the same true residual."""
    from paper_2409_03904_amd import coarse
    s = W.C2
    links, offs, _ = W.make_system(s)
    sh = W.stored_shifts()["c2"]
    hi = 1.1 * sh["lambda_max"]
    lo = hi / 200.0
    rng = np.random.default_rng(5)
    xt = W.gaussian_vectors(rng, s.dims, s.nbasis, s.nrhs, dtype=np.complex128)
    b = O.apply(links, offs, s.dims, xt)
    announce("pbcg c2")
    op = make_op(links, offs, s.dims)
    res = coarse.pbcg_solve(op, dev(b), lo, hi, 16, tol=s.tol, inner_tol=1e-4)
    plain = coarse.bcg_solve(op, dev(b), tol=s.tol, inner_tol=1e-4)
    x = host(res.x)
    assert res.status == 0
    rr = _true_relres(links, offs, s.dims, b, x)
    assert np.max(rr) <= s.tol * 1.01
    np.testing.assert_allclose(rr, res.relres, rtol=1e-3, atol=1e-12)
    err = np.linalg.norm(O.flatten(x - xt), axis=0) / np.linalg.norm(O.flatten(xt), axis=0)
    assert np.max(err) <= 1e3 * 1.5 * s.tol
    print("pbcg c2 iterations", res.iterations, "plain", plain.iterations)
    assert 3 * res.iterations < plain.iterations


def test_pbcg_is_bitwise_reproducible():
    from paper_2409_03904_amd import coarse
    links, offs, b = _system((4, 4, 4, 4), 16, 16, "9pt", 77, 4.0)
    lo, hi = _range(links, offs, (4, 4, 4, 4))
    op = make_op(links, offs, (4, 4, 4, 4))
    announce("pbcg reproducible")
    kw = dict(tol=1e-10, inner_tol=1e-4, check_every=3)
    runs = [coarse.pbcg_solve(op, dev(b), lo, hi, 5, **kw), coarse.pbcg_solve(op, dev(b), lo, hi, 5, **kw),
            coarse.pbcg_solve(op, dev(b), lo, hi, 5, use_graph=False, **kw)]
    assert runs[0].status == 0
    for r in runs[1:]:
        assert r.status == 0 and r.iterations == runs[0].iterations
        assert np.array_equal(host(r.x), host(runs[0].x))


def test_pbcg_graph_cache_keeps_preconditioners_apart():
    """Two solves differing only in the polynomial (degree, then interval) must
    not share a cached graph: each matches its own uncaptured run."""
    from paper_2409_03904_amd import coarse
    links, offs, b = _system((4, 4, 4, 4), 16, 4, "9pt", 78, 4.0)
    lo, hi = _range(links, offs, (4, 4, 4, 4))
    op = make_op(links, offs, (4, 4, 4, 4))
    announce("pbcg graph cache")
    kw = dict(tol=1e-10, inner_tol=1e-4, check_every=3)
    for lo_, hi_, order in [(lo, hi, 3), (lo, hi, 7), (0.5 * lo, hi, 7)]:
        g = coarse.pbcg_solve(op, dev(b), lo_, hi_, order, **kw)
        u = coarse.pbcg_solve(op, dev(b), lo_, hi_, order, use_graph=False, **kw)
        assert g.status == 0 and g.iterations == u.iterations
        assert np.array_equal(host(g.x), host(u.x))


def test_pbcg_rank_deficient_rhs_reports_breakdown():
    from paper_2409_03904_amd import coarse
    s = W.C1
    links, offs, b = W.make_system(s)
    b[:, :, 1] = b[:, :, 0]
    lo, hi = _range(links.astype(np.complex64), offs, s.dims)
    op = make_op(links, offs, s.dims)
    announce("pbcg breakdown")
    res = coarse.pbcg_solve(op, dev(b), lo, hi, 4, tol=1e-8, raise_on_failure=False)
    assert res.status == -4
