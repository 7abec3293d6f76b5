"""GPU block-CG solves (through the C ABI) against the oracle: dense LU on the
small workload, manufactured solutions and the oracle's true residual at full
size, defect correction with 16-bit inner links, failure statuses."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import announce, dev, host, make_op

pytestmark = pytest.mark.gpu


def _true_relres(links, offs, dims, b, x):
    r = b - O.apply(links, offs, dims, x)
    return np.linalg.norm(O.flatten(r), axis=0) / np.linalg.norm(O.flatten(b), axis=0)


@pytest.mark.parametrize("use_graph", [True, False])
def test_small_workload_matches_dense_lu(use_graph):
    from paper_2409_03904_amd import coarse
    s = W.C1
    links, offs, b = W.make_system(s)
    announce("solve c1", use_graph)
    op = make_op(links, offs, s.dims)
    res = coarse.bcg_solve(op, dev(b), tol=s.tol, inner_tol=1e-4, use_graph=use_graph, check_every=4)
    x = host(res.x)
    assert res.status == 0
    ref = O.solve_dense(links, offs, s.dims, b)
    assert np.max(np.abs(x - ref)) / np.max(np.abs(ref)) <= 1e-9
    assert np.max(_true_relres(links, offs, s.dims, b, x)) <= s.tol
    assert res.relres_max <= s.tol
    assert res.cycles >= 2  # float32 inner iteration alone cannot reach 1e-10


@pytest.mark.parametrize("kind", ["bf16", "fp16", "c64_3m"])
def test_small_workload_lowp_inner(kind):
    from paper_2409_03904_amd import coarse
    s = W.System("c1.16", (4, 4, 4, 4), 16, 4, "9pt", kappa=None, shift=4.0, tol=1e-10, seed_index=61)
    links, offs, b = W.make_system(s)
    announce("solve lowp", kind)
    op = make_op(links, offs, s.dims)
    inner = make_op(links, offs, s.dims, kind)
    res = coarse.bcg_solve(op, dev(b), inner=inner, tol=s.tol, inner_tol=1e-2)
    assert res.status == 0
    assert np.max(_true_relres(links, offs, s.dims, b, host(res.x))) <= s.tol


@pytest.mark.parametrize("inner", [None, "fp16", "c64"])
@pytest.mark.parametrize("dims,nb,nr", [((4, 4, 4, 4), 16, 4), ((2, 4, 2, 4), 32, 32)])
def test_outer_3m_residual_matches_dense_lu(inner, dims, nb, nr):
    """Outer links in the 3M layout: the double residual in the 3M form (f64
    MFMA), the inner iterations on the same links (None) or on others; one and
    two column tiles. Against dense LU and the oracle's true residual."""
    from paper_2409_03904_amd import coarse
    s = W.System("c1.3m", dims, nb, nr, "9pt", kappa=None, shift=4.0, tol=1e-10, seed_index=62 + nb)
    links, offs, b = W.make_system(s)
    announce("solve outer 3m", inner, dims, nb, nr)
    op = make_op(links, offs, s.dims, "c64_3m")
    inner_op = None if inner is None else make_op(links, offs, s.dims, inner)
    res = coarse.bcg_solve(op, dev(b), inner=inner_op, tol=s.tol, inner_tol=1e-3 if inner == "fp16" else 1e-4)
    x = host(res.x)
    assert res.status == 0
    ref = O.solve_dense(links, offs, s.dims, b)
    assert np.max(np.abs(x - ref)) / np.max(np.abs(ref)) <= 1e-9
    rr = _true_relres(links, offs, s.dims, b, x)
    assert np.max(rr) <= s.tol
    np.testing.assert_allclose(rr, res.relres, rtol=1e-3, atol=1e-14)


def test_fp32_workload_to_tolerance():
    """8^4, nbasis 32, nrhs 16, kappa ~ 1e3, tolerance 1e-8; manufactured solution."""
    from paper_2409_03904_amd import coarse
    s = W.C2
    links, offs, _ = W.make_system(s)
    rng = np.random.default_rng(5)
    xt = W.gaussian_vectors(rng, s.dims, s.nbasis, s.nrhs, dtype=np.complex128)
    b = O.apply(links, offs, s.dims, xt)
    announce("solve c2")
    op = make_op(links, offs, s.dims)
    res = coarse.bcg_solve(op, dev(b), tol=s.tol, inner_tol=1e-4)
    x = host(res.x)
    assert res.status == 0
    rr = _true_relres(links, offs, s.dims, b, x)
    assert np.max(rr) <= s.tol * 1.01
    np.testing.assert_allclose(rr, res.relres, rtol=1e-3, atol=1e-12)
    # error bounded by kappa * residual
    err = np.linalg.norm(O.flatten(x - xt), axis=0) / np.linalg.norm(O.flatten(xt), axis=0)
    assert np.max(err) <= 1e3 * 1.5 * s.tol


@pytest.mark.timeout(1100)
def test_precision_workload_solves():
    """8^4, nbasis 64, nrhs 32, 81-point, kappa ~ 1e4, tolerance 1e-8: complex64,
    BF16 and FP16 inner links, each to the oracle's true residual; manufactured
    solution, so the error is known exactly."""
    import torch
    from paper_2409_03904_amd import coarse
    s = W.C3
    links, offs, _ = W.make_system(s)
    rng = np.random.default_rng(7)
    xt = W.gaussian_vectors(rng, s.dims, s.nbasis, s.nrhs, dtype=np.complex128)
    b = O.apply(links, offs, s.dims, xt)
    announce("solve c3")
    geom = coarse.Geometry(s.dims, s.nbasis, offs)
    lt = dev(links)
    op = coarse.pack(lt, geom, "c64")
    bd = dev(b)
    op3m = coarse.pack(lt, geom, "c64_3m")
    # the last case: outer links in the 3M layout (the double residual in the 3M form)
    for kind, itol, outer in (("c64", 1e-4, op), ("bf16", 1e-2, op), ("fp16", 1e-3, op), ("fp16", 1e-3, op3m)):
        announce("solve c3 inner", kind, outer.dtype)
        inner = None if kind == "c64" else coarse.pack(lt, geom, kind)
        res = coarse.bcg_solve(outer, bd, inner=inner, tol=s.tol, inner_tol=itol, max_inner=5000)
        x = host(res.x)
        del inner
        torch.cuda.synchronize()
        assert res.status == 0, (kind, res.status)
        rr = _true_relres(links, offs, s.dims, b, x)
        assert np.max(rr) <= s.tol * 1.01, kind
        np.testing.assert_allclose(rr, res.relres, rtol=1e-3, atol=1e-12)
        err = np.linalg.norm(O.flatten(x - xt), axis=0) / np.linalg.norm(O.flatten(xt), axis=0)
        assert np.max(err) <= 1e4 * 1.5 * s.tol, kind
        print(f"[c3] {kind} (outer {outer.dtype}): cycles {res.cycles} inner {res.iterations} "
              f"relres {np.max(rr):.3e} err {np.max(err):.3e}", flush=True)


def test_warm_start_resumes():
    from paper_2409_03904_amd import coarse
    s = W.C1
    links, offs, b = W.make_system(s)
    op = make_op(links, offs, s.dims)
    announce("warm start")
    first = coarse.bcg_solve(op, dev(b), tol=1e-4, inner_tol=1e-2)
    second = coarse.bcg_solve(op, dev(b), x0=first.x, tol=s.tol, inner_tol=1e-4)
    assert second.status == 0
    assert np.max(_true_relres(links, offs, s.dims, b, host(second.x))) <= s.tol


def test_rank_deficient_rhs_reports_breakdown():
    from paper_2409_03904_amd import coarse
    s = W.C1
    links, offs, b = W.make_system(s)
    b[:, :, 1] = b[:, :, 0]
    op = make_op(links, offs, s.dims)
    announce("breakdown")
    res = coarse.bcg_solve(op, dev(b), tol=1e-8, raise_on_failure=False)
    assert res.status == -4


def test_iteration_limit_reports_not_converged():
    from paper_2409_03904_amd import coarse
    s = W.C2
    links, offs, b = W.make_system(s)
    op = make_op(links, offs, s.dims)
    announce("not converged")
    res = coarse.bcg_solve(op, dev(b), tol=1e-8, max_outer=1, max_inner=5, raise_on_failure=False)
    assert res.status == 1
    assert res.iterations == 5
    # the returned iterate is the one whose residual was reported
    rr = _true_relres(links, offs, s.dims, b, host(res.x))
    np.testing.assert_allclose(rr, res.relres, rtol=1e-6)


def test_nonfinite_rhs():
    from paper_2409_03904_amd import coarse
    s = W.C1
    links, offs, b = W.make_system(s)
    b[3, 2, 1] = np.nan
    op = make_op(links, offs, s.dims)
    announce("nonfinite")
    res = coarse.bcg_solve(op, dev(b), tol=1e-8, raise_on_failure=False)
    assert res.status == -5


def _batch_systems():
    """Uneven small systems: lattices, nbasis, nrhs (one not on the MFMA BLAS
    path), one with BF16 inner links."""
    specs = [((4, 4, 4, 4), 8, 4, None), ((2, 2, 4, 4), 16, 8, "bf16"), ((4, 4, 2, 2), 16, 3, None),
             ((2, 4, 2, 4), 8, 16, None)]
    out = []
    for k, (dims, nb, nr, kind) in enumerate(specs):
        s = W.System(f"b{k}", dims, nb, nr, "9pt", kappa=None, shift=4.0, tol=1e-10, seed_index=70 + k)
        links, offs, b = W.make_system(s)
        out.append((s, links, offs, b, kind))
    return out


@pytest.mark.parametrize("use_graph", [True, False])
def test_batched_solve_matches_dense_lu(use_graph):
    from paper_2409_03904_amd import coarse
    systems = _batch_systems()
    announce("batched solve", use_graph)
    outers = [make_op(links, offs, s.dims) for s, links, offs, b, kind in systems]
    inners = [None if kind is None else make_op(links, offs, s.dims, kind) for s, links, offs, b, kind in systems]
    res = coarse.bcg_solve_batched(outers, [dev(b) for s, links, offs, b, kind in systems], inners=inners,
                                   tol=1e-10, inner_tol=1e-3, use_graph=use_graph, check_every=4)
    for (s, links, offs, b, kind), r in zip(systems, res):
        assert r.status == 0, s.name
        x = host(r.x)
        ref = O.solve_dense(links, offs, s.dims, b)
        assert np.max(np.abs(x - ref)) / np.max(np.abs(ref)) <= 1e-9, s.name
        assert np.max(_true_relres(links, offs, s.dims, b, x)) <= 1e-10, s.name


def test_batched_solve_outer_3m():
    """Batched solves with 3M-layout outer links (nbasis % 16 == 0 systems)."""
    from paper_2409_03904_amd import coarse
    systems = [t for t in _batch_systems() if t[0].nbasis % 16 == 0]
    announce("batched solve outer 3m")
    outers = [make_op(links, offs, s.dims, "c64_3m") for s, links, offs, b, kind in systems]
    inners = [None if kind is None else make_op(links, offs, s.dims, kind) for s, links, offs, b, kind in systems]
    res = coarse.bcg_solve_batched(outers, [dev(b) for s, links, offs, b, kind in systems], inners=inners,
                                   tol=1e-10, inner_tol=1e-3, check_every=4)
    for (s, links, offs, b, kind), r in zip(systems, res):
        assert r.status == 0, s.name
        x = host(r.x)
        ref = O.solve_dense(links, offs, s.dims, b)
        assert np.max(np.abs(x - ref)) / np.max(np.abs(ref)) <= 1e-9, s.name


def test_batched_solve_reports_per_system_status():
    """A rank-deficient right-hand side block breaks down; the other systems still converge."""
    from paper_2409_03904_amd import coarse
    systems = _batch_systems()[:3]
    bs = [b.copy() for s, links, offs, b, kind in systems]
    bs[1][:, :, 1] = bs[1][:, :, 0]  # two equal columns
    announce("batched solve statuses")
    outers = [make_op(links, offs, s.dims) for s, links, offs, b, kind in systems]
    res = coarse.bcg_solve_batched(outers, [dev(b) for b in bs], tol=1e-10, inner_tol=1e-3,
                                   raise_on_failure=False)
    assert [r.status for r in res] == [0, -4, 0]
    for k in (0, 2):
        s, links, offs, b, kind = systems[k]
        assert np.max(_true_relres(links, offs, s.dims, b, host(res[k].x))) <= 1e-10


@pytest.mark.parametrize("shape", [((4, 4, 4, 4), 8, 4), ((4, 4, 4, 4), 16, 16), ((2, 4, 2, 4), 16, 32)])
def test_solve_is_bitwise_reproducible(shape):
    """Split-K Grams summed in a fixed order and small steps computed identically
    in every workgroup: the same solve run twice, without graph capture, and as
    one system of a batched call gives bit-identical iterates and counts (nrhs 4
    and 16 take the fused small steps, 32 the separate ones)."""
    from paper_2409_03904_amd import coarse
    dims, nb, nr = shape
    s = W.System("repro", dims, nb, nr, "9pt", kappa=None, shift=4.0, tol=1e-10, seed_index=80 + nr)
    links, offs, b = W.make_system(s)
    op = make_op(links, offs, dims)
    other = W.System("repro2", (2, 2, 2, 4), 8, 3, "9pt", kappa=None, shift=4.0, tol=1e-10, seed_index=90)
    l2, o2, b2 = W.make_system(other)
    op2 = make_op(l2, o2, other.dims)
    announce("reproducible", shape)
    kw = dict(tol=1e-10, inner_tol=1e-4, check_every=4)
    runs = [coarse.bcg_solve(op, dev(b), **kw), coarse.bcg_solve(op, dev(b), **kw),
            coarse.bcg_solve(op, dev(b), use_graph=False, **kw),
            coarse.bcg_solve_batched([op2, op], [dev(b2), dev(b)], **kw)[1]]
    ref = host(runs[0].x)
    assert runs[0].status == 0
    for r in runs[1:]:
        assert r.status == 0 and r.iterations == runs[0].iterations and r.cycles == runs[0].cycles
        assert np.array_equal(host(r.x), ref)


@pytest.mark.parametrize("nr", [1, 2, 5, 8, 12, 16, 24, 32])
def test_solve_every_small_step_path(nr):
    """Every nrhs branch of the small dense steps and block updates against the
    dense solution: fused into the updates (2, 8, 16), separate MFMA steps (32),
    VALU updates (1, 5, 12, 24; pivot-block padding at 1, 5)."""
    from paper_2409_03904_amd import coarse
    s = W.System(f"paths{nr}", (2, 2, 4, 4), 8, nr, "9pt", kappa=None, shift=4.0, tol=1e-10, seed_index=100 + nr)
    links, offs, b = W.make_system(s)
    op = make_op(links, offs, s.dims)
    announce("small-step path", nr)
    res = coarse.bcg_solve(op, dev(b), tol=1e-10, inner_tol=1e-4, check_every=4)
    assert res.status == 0
    x = host(res.x)
    ref = O.solve_dense(links, offs, s.dims, b)
    assert np.max(np.abs(x - ref)) / np.max(np.abs(ref)) <= 1e-9
    assert np.max(_true_relres(links, offs, s.dims, b, x)) <= 1e-10


def test_graph_cache_keeps_operators_apart():
    """One workspace shared by two operators of the same shape, solved in
    turn and with another iteration count per graph: every solve must use a
    graph captured for its own operator (the cache key holds the link pointer
    and the iteration count), so each result matches its dense solution."""
    import torch

    from paper_2409_03904_amd import coarse
    dims, nb, nr = (2, 2, 4, 4), 16, 8
    systems = []
    for k in range(2):
        s = W.System(f"cache{k}", dims, nb, nr, "9pt", kappa=None, shift=4.0, tol=1e-10, seed_index=120 + k)
        links, offs, b = W.make_system(s)
        systems.append((links, offs, b, make_op(links, offs, dims)))
    geom = systems[0][3].geom
    ws = torch.empty(coarse.workspace_bytes(geom, nr), dtype=torch.uint8, device="cuda")
    announce("graph cache")
    for k, ce in ((0, 4), (1, 4), (0, 4), (1, 8), (0, 8)):
        links, offs, b, op = systems[k]
        res = coarse.bcg_solve(op, dev(b), workspace=ws, tol=1e-10, inner_tol=1e-4, check_every=ce)
        assert res.status == 0, (k, ce)
        x = host(res.x)
        ref = O.solve_dense(links, offs, dims, b)
        assert np.max(np.abs(x - ref)) / np.max(np.abs(ref)) <= 1e-9, (k, ce)
