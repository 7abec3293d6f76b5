"""One persistent launch over six uneven coarse systems (lattices 4^4 .. 8^3x16,
nbasis 24/32/48, nrhs 4..32): every output against the oracle and against the
one-system kernel."""
import ctypes

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import FP32_TOL, announce, dev, host, max_rel

pytestmark = pytest.mark.gpu


def _systems():
    out = []
    for s in W.C4:
        links, offs, b = W.make_system(s)
        out.append((s, links, offs, b.astype(np.complex64)))
    return out


@pytest.mark.timeout(600)
def test_batched_matches_oracle_and_single_launches():
    import torch
    from paper_2409_03904_amd import _lib, coarse
    lib = _lib.load()
    systems = _systems()
    announce("batched six systems")
    ops, xs, ys, geoms = [], [], [], []
    arr = (_lib.CoarseSystem * len(systems))()
    for k, (s, links, offs, x) in enumerate(systems):
        geom = coarse.Geometry(s.dims, s.nbasis, offs)
        op = coarse.pack(dev(links), geom, "c64")
        xd = dev(x)
        yd = torch.zeros_like(xd)
        ops.append(op)
        xs.append(xd)
        ys.append(yd)
        geoms.append(geom)
        arr[k].geom = geom._c
        arr[k].nrhs = s.nrhs
        arr[k].packed = op.buf.data_ptr()
        arr[k].x = xd.data_ptr()
        arr[k].y = yd.data_ptr()
    need = ctypes.c_size_t()
    _lib.check(lib.coarse_batched_workspace_bytes(arr, len(systems), ctypes.byref(need)))
    ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    for rep in range(2):  # the queue counter is reset by every launch
        for yd in ys:
            yd.zero_()
        _lib.check(lib.coarse_apply_batched(arr, len(systems), ws.data_ptr(), ws.numel(), stream))
        torch.cuda.synchronize()
        for k, (s, links, offs, x) in enumerate(systems):
            y = host(ys[k])
            assert max_rel(y, O.apply(links, offs, s.dims, x)) <= FP32_TOL, (rep, s.name)
            single = host(coarse.apply(ops[k], xs[k]))
            assert max_rel(y, single) <= 5e-6, s.name  # same products, different summation split


def test_tuner_picks_a_variant_and_keeps_results():
    """Every apply variant gives the same operator; the tuner records the fastest."""
    from paper_2409_03904_amd import coarse
    for dims, nb, nr in [((4, 4, 4, 4), 16, 8), ((4, 4, 4, 4), 32, 16), ((4, 4, 2, 2), 8, 4)]:
        rng = np.random.default_rng(nb)
        offs = W.stencil("9pt")
        links = W.gaussian_links(rng, dims, nb, offs.shape[0])
        x = W.gaussian_vectors(rng, dims, nb, nr)
        announce("tune", dims, nb, nr)
        geom = coarse.Geometry(dims, nb, offs)
        op = coarse.pack(dev(links), geom, "c64")
        ref = O.apply(links, offs, dims, x)
        xd = dev(x)
        nv = coarse.max_apply_variant(nb) + 1
        assert nv == {8: 4, 16: 4, 32: 3}[nb]
        for v in range(nv):
            coarse.set_apply_variant(geom, nr, v)
            assert max_rel(host(coarse.apply(op, xd)), ref) <= FP32_TOL, (nb, nr, v)
        coarse.set_apply_variant(geom, nr, -1)
        v, us = coarse.tune_apply(op, xd, reps=5)
        assert 0 <= v < nv and us > 0
        assert max_rel(host(coarse.apply(op, xd)), ref) <= FP32_TOL
        coarse.set_apply_variant(geom, nr, -1)


def test_batched_tuner():
    import torch
    from paper_2409_03904_amd import coarse
    systems = _systems()[:3]
    announce("batched tune")
    ops, xs, ys = [], [], []
    for s, links, offs, x in systems:
        geom = coarse.Geometry(s.dims, s.nbasis, offs)
        ops.append(coarse.pack(dev(links), geom, "c64"))
        xs.append(dev(x))
        ys.append(torch.zeros_like(xs[-1]))
    b = coarse.BatchedApply(ops, xs, ys)
    times = b.tune(reps=3, candidates=(2, 4))
    assert set(times) == {2, 4, "separate"} and all(t > 0 for t in times.values())
    assert b.mode in ("persistent", "separate")
    for mode in ("persistent", "separate"):
        for y in ys:
            y.zero_()
        b.mode = mode
        b()
        torch.cuda.synchronize()
        for k, (s, links, offs, x) in enumerate(systems):
            assert max_rel(host(ys[k]), O.apply(links, offs, s.dims, x)) <= FP32_TOL, mode
    coarse.BatchedApply.set_occupancy(4)


@pytest.mark.timeout(900)
def test_batched_solve_on_the_six_systems():
    """coarse_bcg_solve_batched on the batching workload's own six systems
    (lattices 4^4 .. 8^3x16, nbasis 24/32/48, nrhs 4..32, kappa 1e3 each):
    manufactured solutions X_true with B = M X_true from the oracle; every
    system's true residual (oracle apply of the returned X) within the 1e-8
    tolerance, and its error within the bound kappa * residual."""
    import torch
    from paper_2409_03904_amd import coarse
    announce("batched solve six systems")
    # condition numbers from the stored Lanczos extremes widened by their residual bounds
    kappas = {k: (v["lambda_max"] + v["bound_max"]) / (v["lambda_min"] - v["bound_min"])
              for k, v in W.stored_shifts().items()}
    ops, bs, refs = [], [], []
    for s in W.C4:
        links, offs, rng = W.make_operator(s)
        x_true = W.gaussian_vectors(rng, s.dims, s.nbasis, s.nrhs, dtype=np.complex128)
        b = O.apply(links, offs, s.dims, x_true)
        geom = coarse.Geometry(s.dims, s.nbasis, offs)
        ops.append(coarse.pack(dev(links), geom, "c64"))
        bs.append(dev(b))
        refs.append((s, links, offs, b, x_true))
    res = coarse.bcg_solve_batched(ops, bs, tol=1e-8, inner_tol=1e-4, max_outer=30, max_inner=5000,
                                   check_every=16)
    torch.cuda.synchronize()
    for r, (s, links, offs, b, x_true) in zip(res, refs):
        x = host(r.x)
        rr = np.linalg.norm(O.flatten(b - O.apply(links, offs, s.dims, x)), axis=0) / \
            np.linalg.norm(O.flatten(b), axis=0)
        err = np.linalg.norm(O.flatten(x - x_true), axis=0) / np.linalg.norm(O.flatten(x_true), axis=0)
        print(s.name, "status", r.status, "cycles", r.cycles, "iterations", r.iterations, "true relres",
              float(rr.max()), "error", float(err.max()))
        assert r.status == 0, s.name
        assert float(rr.max()) <= 1e-8, s.name
        assert np.all(err <= 1.01 * kappas[s.name] * rr + 1e-12), s.name
