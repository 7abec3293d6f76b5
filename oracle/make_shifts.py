"""Write ``workloads/shifts.json``: the self-term shift that gives each
registered workload its target condition number.

Runs only the oracle: the unshifted operator H0 (the same draws with shift 0)
is fed to plain Lanczos for its extreme eigenvalues, then
s = (lam_max - kappa*lam_min)/(kappa - 1) puts (lam_max+s)/(lam_min+s) at kappa.
Lanczos Ritz values lie inside the spectrum, so each record keeps the
residual bounds; a second Lanczos run on the shifted operator re-measures kappa.

Usage: python -m oracle.make_shifts [name ...]   (default: every kappa-targeted workload)
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

import workloads as W
from oracle.coarse_oracle import kappa_shift, lanczos_extremes, neighbour

STEPS = 500


def _operator(system, shift):
    links, offs, _ = W.make_operator(system, shift=shift)
    blocks = [np.ascontiguousarray(links[:, p]).astype(np.complex128) for p in range(offs.shape[0])]
    del links
    nbrs = [neighbour(system.dims, offs[p]) for p in range(offs.shape[0])]
    V, nb = system.volume, system.nbasis

    def op(v):
        x = v.reshape(V, nb, 1)
        y = np.zeros_like(x)
        for a, n in zip(blocks, nbrs):
            y += np.matmul(a, x[n])
        return y.reshape(-1)

    return op


def main(names):
    path = os.path.join(os.path.dirname(os.path.abspath(W.__file__)), "shifts.json")
    table = W.stored_shifts()
    for name in names:
        system = W.REGISTRY[name]
        n = system.volume * system.nbasis
        t0 = time.time()
        op0 = _operator(system, 0.0)
        lo, hi, blo, bhi = lanczos_extremes(op0, n, STEPS, seed=1)
        del op0
        s = kappa_shift(lo, hi, system.kappa)
        op1 = _operator(system, s)
        lo1, hi1, blo1, bhi1 = lanczos_extremes(op1, n, STEPS, seed=2)
        del op1
        table[name] = {
            "shift": s,
            "kappa_target": system.kappa,
            "h0_lambda_min": lo, "h0_lambda_max": hi,
            "h0_bound_min": blo, "h0_bound_max": bhi,
            "lambda_min": lo1, "lambda_max": hi1,
            "bound_min": blo1, "bound_max": bhi1,
            "kappa_measured": hi1 / lo1,
            "lanczos_steps": STEPS,
            "seconds": round(time.time() - t0, 1),
        }
        print(name, json.dumps(table[name]), flush=True)
        with open(path, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    if not args:
        args = [k for k, v in W.REGISTRY.items() if v.kappa is not None]
    main(args)
