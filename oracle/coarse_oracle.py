"""Complex128 CPU oracle: coarse stencil apply, adjoint, dense assembly,
BlockCGrQ, defect correction, low-precision emulation and gradients.

TEST INFRASTRUCTURE ONLY: the tests, the entry module's smoke check and the
CPU-baseline leg of the benchmark call it; the product path never does.

Everything here is written from the paper's definitions (arXiv 2409.03904):

* coarse operator, Sec. 2.6 ("Applying the coarse operator"): for every
  stencil point p with displacement delta_p and every coarse site x,
  ``C(x) += A^p(x) B(x + delta_p)``, an N_basis x N_rhs block per site, the
  RHS index acting as an extra lattice direction (Sec. 2, multiple RHS);
* the stencil is a subset of the displacements {-1,0,1}^4 (Sec. 2.6);
* BlockCGrQ, Fig. 2 (left), with the iterate update ``X += D_k M_k C_k``
  (the figure prints ``D_k M_k``; see ``bcgrq`` for why C_k is required);
* the Chebyshev worst-case bound sigma = (sqrt(k)-1)/(sqrt(k)+1) of
  Sec. 3 (Eq. "bound") as a convergence-rate check;
* the stationary Chebyshev approximation to 1/x on [lo, hi] of Sec. 2.3
  (the polynomial that replaces the CG polynomial of the coarse solve), with
  coefficients from 1/x at the Chebyshev interpolation points;
* multi-RHS deflation and the deflated Chebyshev coarse solve of Sec. 2.3,
  with block Lanczos (full reorthogonalisation) for the deflation vectors;
* block project and promote between the grids, Sec. 2.5 (one product per
  coarse site);
* Preconditioned BlockCGrQ, Fig. 2 (right) and Sec. 2.2, with the same
  iterate-update reading as the unpreconditioned one (``pbcgrq``).

Precision: complex128 throughout. Link values are the complex64 values
upcast, so the oracle and the GPU path define the same operator.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

C128 = np.complex128


# ---------------------------------------------------------------------------
# Geometry (own implementation; periodic lattice, x0 fastest)
# ---------------------------------------------------------------------------

def site_coordinates(dims: Sequence[int]) -> np.ndarray:
    """[V, 4] coordinates (x0, x1, x2, x3) of site s = x0 + L0*(x1 + L1*(x2 + L2*x3))."""
    L = [int(d) for d in dims]
    s = np.arange(int(np.prod(L)))
    out = np.empty((s.size, 4), dtype=np.int64)
    rem = s.copy()
    for mu in range(4):
        out[:, mu] = rem % L[mu]
        rem //= L[mu]
    return out


def site_of(coords: np.ndarray, dims: Sequence[int]) -> np.ndarray:
    L = [int(d) for d in dims]
    c = np.mod(coords, L)
    return c[..., 0] + L[0] * (c[..., 1] + L[1] * (c[..., 2] + L[2] * c[..., 3]))


def neighbour(dims: Sequence[int], delta: Sequence[int]) -> np.ndarray:
    """For every site x, the index of the site x + delta (periodic wrap)."""
    xs = site_coordinates(dims)
    return site_of(xs + np.asarray(delta, dtype=np.int64)[None, :], dims)


# ---------------------------------------------------------------------------
# Coarse operator (Sec. 2.6)
# ---------------------------------------------------------------------------

def apply(links: np.ndarray, offsets: np.ndarray, dims: Sequence[int], x: np.ndarray) -> np.ndarray:
    """Y(x) = sum_p A_p(x) X(x + delta_p), complex128.

    The per-point statement of Sec. 2.6 summed over the stencil; points whose
    displacements land on the same neighbour (extent 1 or 2) add up.
    links: [V, Np, nb, nb]; x: [V, nb, nrhs]. One batched matmul per point,
    the batch being the coarse volume, as in the paper's formulation.
    """
    x = np.asarray(x, dtype=C128)
    y = np.zeros(x.shape, dtype=C128)
    for p in range(offsets.shape[0]):
        nb = neighbour(dims, offsets[p])
        y += np.matmul(links[:, p].astype(C128), x[nb])
    return y


def apply_at(links: np.ndarray, offsets: np.ndarray, dims: Sequence[int], x: np.ndarray,
             sites: np.ndarray) -> np.ndarray:
    """Y(x) = sum_p A_p(x) X(x + delta_p) for the listed sites only (same definition,
    for sampled checks of a large lattice)."""
    sites = np.asarray(sites, dtype=np.int64)
    y = np.zeros((sites.size,) + tuple(x.shape[1:]), dtype=C128)
    for p in range(offsets.shape[0]):
        nb = neighbour(dims, offsets[p])[sites]
        y += np.matmul(links[sites, p].astype(C128), np.asarray(x[nb], dtype=C128))
    return y


def apply_adjoint(links: np.ndarray, offsets: np.ndarray, dims: Sequence[int], x: np.ndarray) -> np.ndarray:
    """(M^H X)(x) = sum_p A_p(x - delta_p)^H X(x - delta_p), complex128.

    Transpose of the gather above: the (x, x+delta_p) block A_p(x) of M
    becomes the (x+delta_p, x) block A_p(x)^H of M^H.
    """
    x = np.asarray(x, dtype=C128)
    y = np.zeros(x.shape, dtype=C128)
    for p in range(offsets.shape[0]):
        src = neighbour(dims, -np.asarray(offsets[p], dtype=np.int64))
        a = links[src, p].astype(C128)
        y += np.matmul(np.conj(np.transpose(a, (0, 2, 1))), x[src])
    return y


def dense(links: np.ndarray, offsets: np.ndarray, dims: Sequence[int]) -> np.ndarray:
    """Dense (V*nb) x (V*nb) matrix by direct block placement M[x, x+delta_p] += A_p(x).

    Independent of ``apply``: the neighbour of each site is found by explicit
    per-site coordinate arithmetic in pure Python.
    """
    L = [int(d) for d in dims]
    V, Np, nb, _ = links.shape
    m = np.zeros((V * nb, V * nb), dtype=C128)
    for s in range(V):
        x = [s % L[0], (s // L[0]) % L[1], (s // (L[0] * L[1])) % L[2], s // (L[0] * L[1] * L[2])]
        for p in range(Np):
            y = [(x[mu] + int(offsets[p][mu])) % L[mu] for mu in range(4)]
            t = y[0] + L[0] * (y[1] + L[1] * (y[2] + L[2] * y[3]))
            m[s * nb:(s + 1) * nb, t * nb:(t + 1) * nb] += links[s, p].astype(C128)
    return m


def flatten(x: np.ndarray) -> np.ndarray:
    """[V, nb, nrhs] -> [(V*nb), nrhs], row index x*nb + i."""
    return x.reshape(-1, x.shape[-1])


# ---------------------------------------------------------------------------
# Spectral utilities
# ---------------------------------------------------------------------------

def chebyshev_rate(kappa: float) -> float:
    """Worst-case CG error reduction per iteration, (sqrt(k)-1)/(sqrt(k)+1) (Sec. 3, Eq. bound)."""
    r = math.sqrt(kappa)
    return (r - 1.0) / (r + 1.0)


def kappa_from_rate(sigma: float) -> float:
    """Inverse of ``chebyshev_rate``: the condition number a measured rate implies (Sec. 3.1)."""
    return ((1.0 + sigma) / (1.0 - sigma)) ** 2


def lanczos_extremes(op: Callable[[np.ndarray], np.ndarray], n: int, steps: int,
                     seed: int = 0) -> Tuple[float, float, float, float]:
    """Plain Lanczos (no reorthogonalisation) on a Hermitian operator of order n.

    Returns (theta_min, theta_max, bound_min, bound_max): the extreme Ritz
    values and their residual bounds |beta_k * s_k|, each Ritz value being
    within its bound of an eigenvalue.
    """
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    v /= np.linalg.norm(v)
    v_prev = np.zeros(n, dtype=C128)
    alphas: List[float] = []
    betas: List[float] = []
    beta = 0.0
    for _ in range(min(steps, n)):
        w = op(v)
        a = float(np.real(np.vdot(v, w)))
        w = w - a * v - beta * v_prev
        alphas.append(a)
        beta = float(np.linalg.norm(w))
        betas.append(beta)
        if beta == 0.0:
            break
        v_prev, v = v, w / beta
    k = len(alphas)
    t = np.diag(alphas) + np.diag(betas[:k - 1], 1) + np.diag(betas[:k - 1], -1)
    evals, evecs = np.linalg.eigh(t)
    bmin = abs(betas[k - 1] * evecs[k - 1, 0])
    bmax = abs(betas[k - 1] * evecs[k - 1, -1])
    return float(evals[0]), float(evals[-1]), float(bmin), float(bmax)


def kappa_shift(lam_min: float, lam_max: float, kappa: float) -> float:
    """Shift s with (lam_max + s)/(lam_min + s) = kappa."""
    return (lam_max - kappa * lam_min) / (kappa - 1.0)


# ---------------------------------------------------------------------------
# Stationary Chebyshev approximation to 1/x (Sec. 2.3)
# ---------------------------------------------------------------------------

def chebyshev_coefficients(lo: float, hi: float, order: int) -> np.ndarray:
    """c_0 .. c_n (n = order) of the degree-n Chebyshev interpolant of 1/x on
    [lo, hi] (Sec. 2.3: coefficients from the target function 1/x at the
    Chebyshev interpolation points). With y(x) = (2x - (hi + lo)) / (hi - lo),
    the n + 1 points y_j = cos(theta_j), theta_j = pi (j + 1/2) / (n + 1), and
    T_k(y_j) = cos(k theta_j):

        c_k = (2 / (n + 1)) sum_j f(x_j) cos(k theta_j),  c_0 halved,

    so that P(x) = sum_k c_k T_k(y(x)) equals 1/x at every x_j."""
    n = int(order)
    if n < 0 or not (0 < lo < hi):
        raise ValueError("need order >= 0 and 0 < lo < hi")
    theta = np.pi * (np.arange(n + 1) + 0.5) / (n + 1)
    x = 0.5 * (hi - lo) * np.cos(theta) + 0.5 * (hi + lo)
    f = 1.0 / x
    c = np.array([np.sum(f * np.cos(k * theta)) for k in range(n + 1)]) * (2.0 / (n + 1))
    c[0] *= 0.5
    return c


def chebyshev_apply(op: Callable[[np.ndarray], np.ndarray], b: np.ndarray, lo: float, hi: float,
                    order: int) -> np.ndarray:
    """P(M) b = sum_k c_k T_k(Y) b with Y = (2M - (hi + lo)) / (hi - lo), by the
    three-term recurrence T_0 = b, T_1 = Y b, T_{k+1} = 2 Y T_k - T_{k-1}
    (one application of M per degree), in complex128."""
    c = chebyshev_coefficients(lo, hi, order)
    a, d = 2.0 / (hi - lo), (hi + lo) / (hi - lo)

    def Y(v):
        return a * op(v) - d * v

    t_prev = np.asarray(b, dtype=C128)
    out = c[0] * t_prev
    if order >= 1:
        t = Y(t_prev)
        out = out + c[1] * t
        for k in range(2, int(order) + 1):
            t_next = 2.0 * Y(t) - t_prev
            out = out + c[k] * t_next
            t_prev, t = t, t_next
    return out


# ---------------------------------------------------------------------------
# Multi-RHS deflation and the deflated Chebyshev coarse solve (Sec. 2.3)
# ---------------------------------------------------------------------------

def deflate(v: np.ndarray, lam: np.ndarray, x: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Deflation of a block of right-hand sides on the n_ev vectors |i> (the
    columns of v, [n, n_ev]) with values lambda_i (Sec. 2.3):

        Defl(x) = sum_i |i> <i|x> / lambda_i,   x_perp = x - sum_i |i> <i|x>,

    for every column of x ([n, nrhs]) at once, as the two products
    c = V^H x and V c (the multi-RHS form of Sec. 2.5). Returns (Defl(x), x_perp)."""
    v = np.asarray(v, dtype=C128)
    x = np.asarray(x, dtype=C128)
    c = v.conj().T @ x
    return v @ (c / np.asarray(lam, dtype=np.float64)[:, None]), x - v @ c


def block_lanczos(op: Callable[[np.ndarray], np.ndarray], x0: np.ndarray, steps: int, nev: int):
    """Block Lanczos with full reorthogonalisation for the lowest eigenpairs of a
    Hermitian operator (the source of the deflation vectors, Sec. 2.3 and 3):
      Q_0 R_0 = X_0 (thin QR);  for j = 0 .. steps-1:  W = H Q_j;
      W <- W - Q_{0..j} (Q_{0..j}^H W) twice (the coefficients summed into
      column block j of T = Q^H H Q);  Q_{j+1} B_{j+1} = W (thin QR by the
      Cholesky factor of W^H W), B_{j+1} the block below the diagonal of T;
    then Rayleigh-Ritz: T = Y Theta Y^H, Ritz vectors Q Y for the nev lowest
    Ritz values, with residual norms ||B_steps Y_last|| (the last block row of
    Y). Stops early when a new block is rank deficient. Returns
    (theta[:nev], V [n, nev], residual estimates [nev])."""
    x0 = np.asarray(x0, dtype=C128)
    n, b = x0.shape
    r = chol_upper(x0.conj().T @ x0)
    qs = [np.linalg.solve(r.T, x0.T).T]
    K = steps * b
    T = np.zeros((K + b, K), dtype=C128)
    last = None
    for j in range(steps):
        Q = np.concatenate(qs, axis=1)
        w = op(qs[j])
        c = Q.conj().T @ w
        w = w - Q @ c
        c2 = Q.conj().T @ w
        w = w - Q @ c2
        T[:(j + 1) * b, j * b:(j + 1) * b] = c + c2
        try:
            bj = chol_upper(w.conj().T @ w, 1e-24)
        except Breakdown:
            T = T[:(j + 1) * b, :(j + 1) * b]
            last = None
            break
        T[(j + 1) * b:(j + 2) * b, j * b:(j + 1) * b] = bj
        last = bj
        if j + 1 < steps:
            qs.append(np.linalg.solve(bj.T, w.T).T)
    m = min(T.shape[1], len(qs) * b)
    Tm = T[:m, :m]
    Tm = 0.5 * (Tm + Tm.conj().T)
    theta, Y = np.linalg.eigh(Tm)
    Q = np.concatenate(qs, axis=1)[:, :m]
    k = min(nev, m)
    V = Q @ Y[:, :k]
    res = np.linalg.norm(last @ Y[m - b:m, :k], axis=0) if last is not None else np.zeros(k)
    return theta[:k], V, res


def deflated_chebyshev(op: Callable[[np.ndarray], np.ndarray], v: np.ndarray, lam: np.ndarray,
                       x: np.ndarray, lo: float, hi: float, order: int) -> np.ndarray:
    """The two-part stationary coarse solve of Sec. 2.3:
    Q x = Defl(x_par) + P(M) x_perp, with x split into its parts parallel and
    orthogonal to span{|i>}, Defl the deflation inverse and P the degree-`order`
    Chebyshev approximation to 1/x on [lo, hi]. ``op`` and the vectors use the
    flat [n, nrhs] layout."""
    d, xp = deflate(v, lam, x)
    return d + chebyshev_apply(op, xp, lo, hi, order)


# ---------------------------------------------------------------------------
# Transfer between grids: block project and promote (Sec. 2.5)
# ---------------------------------------------------------------------------

def block_project(basis: np.ndarray, fine: np.ndarray) -> np.ndarray:
    """C(x_c) = B(x_c)^H F(x_c) for every coarse site x_c (Sec. 2.5, the
    coarse-volume batched product): basis [V, V_block, N_basis], fine
    [V, V_block, N_rhs] (the fine degrees of freedom of each block side by
    side), result [V, N_basis, N_rhs]."""
    b = np.asarray(basis, dtype=C128)
    return np.matmul(np.conj(np.transpose(b, (0, 2, 1))), np.asarray(fine, dtype=C128))


def block_promote(basis: np.ndarray, coarse: np.ndarray) -> np.ndarray:
    """F(x_c) = B(x_c) C(x_c) for every coarse site (Sec. 2.5): basis
    [V, V_block, N_basis], coarse [V, N_basis, N_rhs], result [V, V_block, N_rhs]."""
    return np.matmul(np.asarray(basis, dtype=C128), np.asarray(coarse, dtype=C128))


# ---------------------------------------------------------------------------
# Block CG: BlockCGrQ (Fig. 2, left)
# ---------------------------------------------------------------------------

class Breakdown(RuntimeError):
    """A Gram matrix of the block iteration is not Hermitian positive definite."""


def chol_upper(g: np.ndarray, rel_eps: float = 0.0) -> np.ndarray:
    """Upper-triangular C with C^H C = g (the thin-QR normalisation of Fig. 2).

    Raises ``Breakdown`` when g is not positive definite, or when a pivot
    falls at or below ``rel_eps`` times the trace (a rank-deficient block).
    """
    g = 0.5 * (g + g.conj().T)
    n = g.shape[0]
    tr = float(np.real(np.trace(g)))
    if not np.all(np.isfinite(g)):
        raise Breakdown("non-finite Gram matrix")
    c = np.zeros_like(g)
    a = g.copy()
    for k in range(n):
        piv = float(np.real(a[k, k]))
        if not (piv > rel_eps * tr) or piv <= 0.0:
            raise Breakdown(f"pivot {k} = {piv:.3e} (trace {tr:.3e})")
        d = math.sqrt(piv)
        c[k, k] = d
        c[k, k + 1:] = a[k, k + 1:] / d
        a[k + 1:, k + 1:] -= np.outer(c[k, k + 1:].conj(), c[k, k + 1:])
    return c


@dataclass
class SolveInfo:
    iterations: int = 0
    converged: bool = False
    breakdown: bool = False
    relres_recursive: List[np.ndarray] = field(default_factory=list)
    history_x: List[np.ndarray] = field(default_factory=list)
    history_d: List[np.ndarray] = field(default_factory=list)
    history_q: List[np.ndarray] = field(default_factory=list)
    history_c: List[np.ndarray] = field(default_factory=list)


def bcgrq(op: Callable[[np.ndarray], np.ndarray], b: np.ndarray, x0: Optional[np.ndarray] = None,
          tol: float = 1e-10, maxiter: int = 1000, record: bool = False,
          breakdown_eps: float = 1e-28) -> Tuple[np.ndarray, SolveInfo]:
    """BlockCGrQ for a Hermitian positive definite operator, Fig. 2 (left).

    b, x0: [n, nrhs] complex. Steps, in the figure's order and notation:
      R_0 = B - H X_0;  Q_0 C_0 = R_0 (thin QR via the Cholesky factor of
      R_0^H R_0, kept explicit as in Sec. 2.2);  D_0 = Q_0;  then per k
      Z_k = H D_k;  M_k = (D_k^H Z_k)^{-1};  X_{k+1} = X_k + D_k M_k C_k;
      Q_{k+1} S_{k+1} = Q_k - Z_k M_k;  D_{k+1} = Q_{k+1} + D_k S_{k+1}^H;
      C_{k+1} = S_{k+1} C_k.
    The figure writes the iterate update as X_k + D_k M_k. With R_k = Q_k C_k
    and D_k^H Q_k = I, the block step length that zeroes D_k^H R_{k+1} is
    M_k D_k^H R_k = M_k C_k, so C_k must multiply the update; without it the
    recursion still drives C_k to zero but X does not solve the system.
    The recursive residual norm of column j is ||C_k e_j|| (Q_k orthonormal);
    the stop test is max_j ||C_k e_j|| / ||B e_j|| <= tol.
    """
    b = np.asarray(b, dtype=C128)
    n, nr = b.shape
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=C128).copy()
    info = SolveInfo()
    bnorm = np.linalg.norm(b, axis=0)
    bnorm = np.where(bnorm == 0.0, 1.0, bnorm)
    r = b - op(x)
    try:
        c = chol_upper(r.conj().T @ r, breakdown_eps)
    except Breakdown:
        info.breakdown = True
        return x, info
    q = np.linalg.solve(c.T, r.T).T  # q = r c^{-1}
    d = q.copy()
    for k in range(maxiter):
        if record:
            info.history_x.append(x.copy())
            info.history_d.append(d.copy())
            info.history_q.append(q.copy())
            info.history_c.append(c.copy())
        z = op(d)
        try:
            m = np.linalg.inv(d.conj().T @ z)
        except np.linalg.LinAlgError:
            info.breakdown = True
            break
        x = x + d @ (m @ c)
        t = q - z @ m
        try:
            s = chol_upper(t.conj().T @ t, breakdown_eps)
        except Breakdown:
            info.iterations = k + 1
            info.breakdown = True
            break
        q = np.linalg.solve(s.T, t.T).T  # q = t s^{-1}
        d = q + d @ s.conj().T
        c = s @ c
        info.iterations = k + 1
        rel = np.linalg.norm(c, axis=0) / bnorm
        info.relres_recursive.append(rel)
        if np.max(rel) <= tol:
            info.converged = True
            break
    if record:
        info.history_x.append(x.copy())
    return x, info


def pbcgrq(op: Callable[[np.ndarray], np.ndarray], prec: Callable[[np.ndarray], np.ndarray],
           b: np.ndarray, x0: Optional[np.ndarray] = None, tol: float = 1e-10, maxiter: int = 1000,
           record: bool = False, breakdown_eps: float = 1e-28) -> Tuple[np.ndarray, SolveInfo]:
    """Preconditioned BlockCGrQ, Fig. 2 (right), for a Hermitian positive
    definite operator H and a Hermitian positive definite preconditioner
    ``prec`` = M^{-1} (Sec. 2.2: BlockCGrQ on M^{-1} H in the M inner product,
    where <u|v>_M = u^H M v, so that <Z|Z>_M = Z^H z for Z = M^{-1} z).

    Lower-case blocks live in the space of H's range (residual-like), capitals
    are their images under M^{-1}; both are rotated, as the paper keeps them:
      z_0 = B - H X_0;  Z_0 = M^{-1} z_0;  C_0^H C_0 = Z_0^H z_0;
      q_0 = z_0 C_0^{-1};  Q_0 = Z_0 C_0^{-1};  D_0 = Q_0;  then per k
      z_k = H D_k;  Z_k = M^{-1} z_k;  N_k = (D_k^H z_k)^{-1};
      X_{k+1} = X_k + D_k N_k C_k;
      t_k = q_k - z_k N_k;  T_k = Q_k - Z_k N_k;  S^H S = T_k^H t_k;
      q_{k+1} = t_k S^{-1};  Q_{k+1} = T_k S^{-1};
      D_{k+1} = Q_{k+1} + D_k S^H;  C_{k+1} = S C_k.
    Readings: the iterate update carries C_k as in ``bcgrq`` (the residual is
    R_k = q_k C_k, and D_k N_k C_k is the step that zeroes D_k^H R_{k+1});
    the figure's factorisation line names S_k on one side and S_{k+1} on the
    other, read as one matrix S (the one used by the next three lines).
    Q_k^H q_k = I, so ||C_k e_j|| is the M^{-1} norm sqrt(r_j^H M^{-1} r_j)
    of residual column j; the stop test is that norm relative to its start,
    max_j ||C_k e_j|| / ||C_0 e_j|| <= tol.
    """
    b = np.asarray(b, dtype=C128)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=C128).copy()
    info = SolveInfo()
    zr = b - op(x)
    zp = prec(zr)
    try:
        c = chol_upper(zp.conj().T @ zr, breakdown_eps)
    except Breakdown:
        info.breakdown = True
        return x, info
    c0n = np.linalg.norm(c, axis=0)
    q = np.linalg.solve(c.T, zr.T).T   # q = z c^{-1}
    qp = np.linalg.solve(c.T, zp.T).T  # Q = Z c^{-1}
    d = qp.copy()
    for k in range(maxiter):
        if record:
            info.history_x.append(x.copy())
            info.history_d.append(d.copy())
            info.history_q.append(q.copy())
            info.history_c.append(c.copy())
        zr = op(d)
        zp = prec(zr)
        try:
            nk = np.linalg.inv(d.conj().T @ zr)
        except np.linalg.LinAlgError:
            info.breakdown = True
            break
        x = x + d @ (nk @ c)
        t = q - zr @ nk
        tp = qp - zp @ nk
        try:
            s = chol_upper(tp.conj().T @ t, breakdown_eps)
        except Breakdown:
            info.iterations = k + 1
            info.breakdown = True
            break
        q = np.linalg.solve(s.T, t.T).T
        qp = np.linalg.solve(s.T, tp.T).T
        d = qp + d @ s.conj().T
        c = s @ c
        info.iterations = k + 1
        rel = np.linalg.norm(c, axis=0) / c0n
        info.relres_recursive.append(rel)
        if np.max(rel) <= tol:
            info.converged = True
            break
    if record:
        info.history_x.append(x.copy())
    return x, info


def cg(op: Callable[[np.ndarray], np.ndarray], b: np.ndarray, x0: Optional[np.ndarray] = None,
       tol: float = 1e-10, maxiter: int = 1000, record: bool = False):
    """Textbook Hestenes-Stiefel conjugate gradients for one RHS (the N_rhs = 1 case)."""
    b = np.asarray(b, dtype=C128).reshape(-1)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=C128).reshape(-1).copy()
    r = b - op(x)
    p = r.copy()
    rr = float(np.real(np.vdot(r, r)))
    bn = float(np.linalg.norm(b)) or 1.0
    xs = [x.copy()] if record else []
    res = []
    for k in range(maxiter):
        w = op(p)
        alpha = rr / float(np.real(np.vdot(p, w)))
        x = x + alpha * p
        r = r - alpha * w
        rr_new = float(np.real(np.vdot(r, r)))
        res.append(math.sqrt(rr_new) / bn)
        if record:
            xs.append(x.copy())
        if math.sqrt(rr_new) / bn <= tol:
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, res, xs


def true_relres(op: Callable[[np.ndarray], np.ndarray], b: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Per-column ||b_j - M x_j|| / ||b_j|| in complex128."""
    b = np.asarray(b, dtype=C128)
    r = b - op(np.asarray(x, dtype=C128))
    return np.linalg.norm(r, axis=0) / np.linalg.norm(b, axis=0)


@dataclass
class DefectInfo:
    cycles: int = 0
    inner_iterations: int = 0
    converged: bool = False
    relres: List[np.ndarray] = field(default_factory=list)


def defect_correction(op_outer: Callable[[np.ndarray], np.ndarray],
                      inner_solve: Callable[[np.ndarray], Tuple[np.ndarray, int]],
                      b: np.ndarray, x0: Optional[np.ndarray] = None, tol: float = 1e-8,
                      max_outer: int = 50) -> Tuple[np.ndarray, DefectInfo]:
    """Iterative refinement around an approximate inner solve.

    Per cycle: R = B - M X (outer precision); stop when max_j ||r_j||/||b_j||
    <= tol; normalise each residual column, R^ = R diag(1/||r_j||); solve the
    inner system approximately, E ~ M~^{-1} R^; X += E diag(||r_j||).
    The paper keeps full accuracy only in the outer solver and notes that
    the coarse solves tolerate lower precision (Sec. 4); this loop is that
    outer solver around a lower-precision inner block CG.
    """
    b = np.asarray(b, dtype=C128)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=C128).copy()
    bn = np.linalg.norm(b, axis=0)
    info = DefectInfo()
    for cyc in range(max_outer + 1):
        r = b - op_outer(x)
        rn = np.linalg.norm(r, axis=0)
        rel = rn / bn
        info.relres.append(rel)
        if np.max(rel) <= tol:
            info.converged = True
            break
        if cyc == max_outer:
            break
        scale = np.where(rn == 0.0, 1.0, rn)
        e, its = inner_solve(r / scale[None, :])
        info.inner_iterations += its
        x = x + e * scale[None, :]
        info.cycles = cyc + 1
    return x, info


# ---------------------------------------------------------------------------
# Low-precision link storage, emulated (round to nearest even)
# ---------------------------------------------------------------------------

def round_bf16(v: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even); returned as float32."""
    f = np.ascontiguousarray(v, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    out = u.astype(np.uint32).view(np.float32)
    # NaN stays NaN (not expected in inputs); infinities stay infinite
    return np.where(np.isfinite(f), out, f)


def round_fp16(v: np.ndarray) -> np.ndarray:
    """Round float32 values to IEEE half (nearest, ties to even); returned as float32."""
    return np.asarray(v, dtype=np.float32).astype(np.float16).astype(np.float32)


def pow2_ceil(m: np.ndarray) -> np.ndarray:
    """Smallest power of two >= m (1 where m == 0), as float64."""
    m = np.asarray(m, dtype=np.float64)
    mant, expo = np.frexp(m)  # m = mant * 2^expo, mant in [0.5, 1)
    e = np.where(mant == 0.5, expo - 1, expo)
    return np.where(m > 0, np.ldexp(1.0, e), 1.0)


def _round(kind: str, v: np.ndarray) -> np.ndarray:
    if kind == "bf16":
        return round_bf16(v)
    if kind == "fp16":
        return round_fp16(v)
    raise ValueError(kind)


def link_scales(links: np.ndarray) -> np.ndarray:
    """One power-of-two scale per (site, point) block: 2^ceil(log2 max(|Re|,|Im|))."""
    a = links.astype(np.complex64)
    m = np.maximum(np.abs(a.real), np.abs(a.imag)).max(axis=(2, 3))
    return pow2_ceil(m)


def quantize_links(links: np.ndarray, offsets: np.ndarray, kind: str) -> np.ndarray:
    """Links as the low-precision store represents them (complex128 values).

    Every block except the self point's is divided by its power-of-two scale
    (exact), rounded component-wise to ``kind`` and multiplied back. A pair
    A_p(x), A_{-p}(x+delta_p) = A_p(x)^H has the same entries up to conjugation,
    hence the same scale and the same rounding, so the stored operator stays
    exactly Hermitian. The self block stays complex64.
    """
    a = links.astype(np.complex64)
    s = link_scales(a)
    out = np.empty(a.shape, dtype=C128)
    for p in range(offsets.shape[0]):
        blk = a[:, p]
        if not np.any(offsets[p]):
            out[:, p] = blk
            continue
        sc = s[:, p].astype(np.float32)[:, None, None]
        re = _round(kind, blk.real / sc).astype(np.float64)
        im = _round(kind, blk.imag / sc).astype(np.float64)
        out[:, p] = (re + 1j * im) * s[:, p][:, None, None]
    return out


def quantize_vector(x: np.ndarray, kind: str) -> np.ndarray:
    """The apply's low-precision view of an input vector (complex128 values).

    bf16: component-wise rounding, no scale (bf16 has the float32 exponent range).
    fp16: one power-of-two scale per (site, RHS column), 2^ceil(log2 max
    |component|) over the nbasis entries of that column at that site, then
    rounding; half's narrow exponent range needs the scale, and a per-site
    scale keeps the relative precision of every site's block.
    """
    x32 = np.asarray(x).astype(np.complex64)
    if kind == "bf16":
        return round_bf16(x32.real).astype(np.float64) + 1j * round_bf16(x32.imag).astype(np.float64)
    m = np.maximum(np.abs(x32.real), np.abs(x32.imag)).max(axis=1)  # [V, nrhs]
    s = pow2_ceil(m)
    sc = s.astype(np.float32)[:, None, :]
    re = round_fp16(x32.real / sc).astype(np.float64)
    im = round_fp16(x32.imag / sc).astype(np.float64)
    return (re + 1j * im) * s[:, None, :]


def apply_lowp(links: np.ndarray, offsets: np.ndarray, dims: Sequence[int], x: np.ndarray,
               kind: str) -> np.ndarray:
    """Emulation of the low-precision apply: rounded links and rounded input for
    every point except the self point, which uses complex64 links and the
    unrounded input; products summed in complex128."""
    ql = quantize_links(links, offsets, kind)
    xq = quantize_vector(x, kind)
    x64 = np.asarray(x).astype(np.complex64).astype(C128)
    y = np.zeros(x.shape, dtype=C128)
    for p in range(offsets.shape[0]):
        nb = neighbour(dims, offsets[p])
        src = x64 if not np.any(offsets[p]) else xq
        y += np.matmul(ql[:, p], src[nb])
    return y


# ---------------------------------------------------------------------------
# Gradients (PyTorch convention: grad = dL/dRe + i dL/dIm for a real loss L)
# ---------------------------------------------------------------------------

def link_grad(g: np.ndarray, x: np.ndarray, offsets: np.ndarray, dims: Sequence[int]) -> np.ndarray:
    """dA_p(x) = G(x) X(x + delta_p)^H: the sum over RHS of outer products."""
    g = np.asarray(g, dtype=C128)
    x = np.asarray(x, dtype=C128)
    V, nb, nr = g.shape
    out = np.empty((V, offsets.shape[0], nb, nb), dtype=C128)
    for p in range(offsets.shape[0]):
        n = neighbour(dims, offsets[p])
        out[:, p] = np.matmul(g, np.conj(np.transpose(x[n], (0, 2, 1))))
    return out


def apply_vjp(links, offsets, dims, x, gy):
    """Gradients of a real loss through Y = M X: (dX, dA) = (M^H G, G X^H per link)."""
    return apply_adjoint(links, offsets, dims, gy), link_grad(gy, x, offsets, dims)


def solve_dense(links, offsets, dims, b):
    """X = M^{-1} B by a dense LU solve (any invertible M)."""
    import scipy.linalg
    m = dense(links, offsets, dims)
    sol = scipy.linalg.lu_solve(scipy.linalg.lu_factor(m), flatten(np.asarray(b, dtype=C128)))
    return sol.reshape(np.shape(b))


def solve_vjp_dense(links, offsets, dims, b, gx):
    """Gradients through X = M^{-1} B: Lambda = M^{-H} G, dB = Lambda, dA = -Lambda X^H per link."""
    import scipy.linalg
    m = dense(links, offsets, dims)
    lu = scipy.linalg.lu_factor(m)
    x = scipy.linalg.lu_solve(lu, flatten(np.asarray(b, dtype=C128))).reshape(np.shape(b))
    lam = scipy.linalg.lu_solve(lu, flatten(np.asarray(gx, dtype=C128)), trans=2).reshape(np.shape(b))
    return x, lam, -link_grad(lam, x, offsets, dims)


def fd_gradient(loss: Callable[[np.ndarray], float], z: np.ndarray, h: float = 1e-6) -> np.ndarray:
    """Central finite differences of a real loss w.r.t. every Re and Im part of z."""
    z = np.asarray(z, dtype=C128)
    flat = z.reshape(-1)
    g = np.empty(flat.shape, dtype=C128)
    for i in range(flat.size):
        zp = flat.copy()
        zp[i] += h
        zm = flat.copy()
        zm[i] -= h
        dre = (loss(zp.reshape(z.shape)) - loss(zm.reshape(z.shape))) / (2 * h)
        zp = flat.copy()
        zp[i] += 1j * h
        zm = flat.copy()
        zm[i] -= 1j * h
        dim = (loss(zp.reshape(z.shape)) - loss(zm.reshape(z.shape))) / (2 * h)
        g[i] = dre + 1j * dim
    return g.reshape(z.shape)
