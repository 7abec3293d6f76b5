// Dense nrhs x nrhs double-precision steps of BlockCGrQ (Fig. 2, left) on one
// workgroup: the Cholesky factor of the thin QR kept explicit (Sec. 2.2), its
// inverse, the small products, the residual column norms ||C e_j|| and the
// convergence and breakdown flags. Device code only: included by the stand-alone
// step kernels and by the block-update kernels that run the steps in every
// workgroup's prologue.
#pragma once
#include "blas.hpp"

namespace coarse {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ double2 to_d2(double2 v) { return v; }

// ---------------------------------------------------------------------------
// Small dense double-precision steps: one workgroup; thread (i, j) owns entry
// (i, j) of every np x np matrix in LDS, np = n rounded up to the pivot block
// size P (the padding rows and columns hold the identity: they factor to the
// identity and never mix with the live entries).
//
// A Hermitian positive definite A is factored as A = S^H S (S upper: the
// Cholesky factor of the thin QR) by a blocked elimination of [A | I]. At
// block step K the threads that form the new pivot rows read the P x P pivot
// block and factor it in their own registers (the same instructions on the
// same data, so they take the same breakdown decision); the elimination
// leaves [S | S^{-H}], since S^{-H} A = S. The sequential chain is n / P
// steps of two barriers each, against 2n single-pivot steps for a Cholesky
// factorisation followed by an inversion.
// ---------------------------------------------------------------------------
constexpr double BREAKDOWN_EPS = 1e-12;
constexpr int SMALL_MAX = 32;

// pivot block size: 4 x 4 blocks factored in registers (n / 4 block steps;
// at n = 32 on a 1024-thread workgroup 76 registers, against 2 x 2 blocks
// and twice the steps 1.5 us faster per factorisation)
constexpr int SMALL_P = 4;
__host__ __device__ constexpr int small_pad(int n, int p) { return (n + p - 1) / p * p; }
__host__ __device__ constexpr int small_threads(int np) { return ((np * np + 63) / 64) * 64; }

struct SmallCtx {
    int n, np;  // live and padded order
    int i, j;   // this thread's entry
    bool on;    // i < np
};

template <int P>
__device__ __forceinline__ SmallCtx small_ctx(int n) {
    SmallCtx c;
    c.n = n;
    c.np = small_pad(n, P);
    c.i = (int)threadIdx.x / c.np;
    c.j = (int)threadIdx.x - c.i * c.np;
    c.on = c.i < c.np;
    return c;
}

// A = Hermitian part of the reduced n x n Gram G with identity padding; R = I.
__device__ inline void load_gram(double2 *A, double2 *R, const double2 *G, const SmallCtx &c) {
    if (c.on) {
        double2 a = make_double2(c.i == c.j ? 1.0 : 0.0, 0.0);
        if (c.i < c.n && c.j < c.n) {
            const double2 v = G[c.i * c.n + c.j], vt = G[c.j * c.n + c.i];
            a = make_double2(0.5 * (v.x + vt.x), 0.5 * (v.y - vt.y));
        }
        A[c.i * c.np + c.j] = a;
        R[c.i * c.np + c.j] = make_double2(c.i == c.j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
}

// Sum of the real diagonal of the live block and an all-finite flag (wave 0).
__device__ inline void trace_finite(const double2 *A, const SmallCtx &c, double *scratch) {
    if (threadIdx.x < 64) {
        double tr = 0;
        int fin = 1;
        for (int r = threadIdx.x; r < c.n * c.n; r += 64) {
            const int i = r / c.n, j = r - i * c.n;
            const double2 v = A[i * c.np + j];
            fin &= (isfinite(v.x) && isfinite(v.y)) ? 1 : 0;
            if (i == j) tr += v.x;
        }
        for (int m = 32; m > 0; m >>= 1) {
            tr += __shfl_xor(tr, m);
            fin &= __shfl_xor(fin, m);
        }
        if (threadIdx.x == 0) {
            scratch[0] = tr;
            scratch[1] = fin ? 1.0 : 0.0;
        }
    }
    __syncthreads();
}

// 1/sqrt(d) for d > 0: the hardware estimate (relative error below 2^-22)
// refined by two Newton steps y <- y (3 - d y^2) / 2, each of which squares the
// relative error, so the result is within a few ulp. On the dependent chain of
// the pivots this is far shorter than a correctly rounded sqrt and divide.
__device__ __forceinline__ double rsqrt_nr(double d) {
    double y = __builtin_amdgcn_rsq(d);
    const double h = 0.5 * d;
    y = y * fma(-h, y * y, 1.5);
    y = y * fma(-h, y * y, 1.5);
    return y;
}

// Upper Cholesky factor S of the P x P Hermitian block of A at (k0, k0) (upper
// triangle read) and T = S^{-H} (lower triangular), in registers. The first
// `live` pivots are tested against thr: returns 1, 0 (a pivot not above thr)
// or 2 (a pivot not finite).
template <int P>
__device__ __forceinline__ int factor_pivot(const double2 *A, int np, int k0, int live, double thr,
                                            double2 (&S)[P][P], double2 (&T)[P][P]) {
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int q = p; q < P; ++q) S[p][q] = A[(k0 + p) * np + k0 + q];
    int ok = 1;
    double rs[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        double d = S[p][p].x;
#pragma unroll
        for (int m = 0; m < p; ++m) d -= S[m][p].x * S[m][p].x + S[m][p].y * S[m][p].y;
        if (p < live && ok == 1 && !(d > thr)) ok = isfinite(d) ? 0 : 2;
        const double r = rsqrt_nr(d);
        rs[p] = r;
        S[p][p] = make_double2(d * r, 0.0);
#pragma unroll
        for (int q = p + 1; q < P; ++q) {
            double2 v = S[p][q];
#pragma unroll
            for (int m = 0; m < p; ++m) v = csub(v, cmulc(S[m][p], S[m][q]));
            S[p][q] = make_double2(v.x * rs[p], v.y * rs[p]);
        }
    }
    // forward substitution on L = S^H (L[p][m] = conj(S[m][p])): L T = I
#pragma unroll
    for (int q = 0; q < P; ++q) {
        T[q][q] = make_double2(rs[q], 0.0);
#pragma unroll
        for (int p = q + 1; p < P; ++p) {
            double2 v = make_double2(0, 0);
#pragma unroll
            for (int m = q; m < p; ++m) v = cadd(v, cmulc(S[m][p], T[m][q]));
            T[p][q] = make_double2(-v.x * rs[p], -v.y * rs[p]);
        }
    }
    return ok;
}

// In place: [A | R] (A Hermitian positive definite, R = I) -> [S | S^{-H}],
// S upper with exact zeros below the diagonal. tr = trace of the live block
// (the breakdown threshold's scale). Returns 1, or the failing pivot's code,
// the same in every thread.
//
// Block step k0: the pivot rows of [A | R] after the step are
// V = T [A | R](k0 .. k0 + P - 1, :), T = S_kk^{-H} of the pivot block; each
// entry of V is formed once (by the first P * 2 np threads, which factor the
// pivot block in registers) and kept in LDS, and every trailing entry then
// takes its rank-P update from V alone:
//   [A | R](i, j) -= sum_p conj(V(p, i)) [V | VR](p, j),  i >= k0 + P,
// since column i of the pivot rows after the step is V(:, i). Each thread
// reads and writes only its own entry in the update, so a step costs two
// barriers.
template <int P>
__device__ int chol_elim(double2 *A, double2 *R, const SmallCtx &c, double tr) {
    __shared__ double2 Vb[P * 2 * SMALL_MAX];  // the pivot rows of [A | R] after the step
    __shared__ int okb;
    const int np = c.np, w2 = 2 * np;
    const double thr = BREAKDOWN_EPS * tr;
    const int t = (int)threadIdx.x;
    const double2 zero = make_double2(0, 0);
    for (int k0 = 0; k0 < np; k0 += P) {
        if (t < P * w2) {
            double2 S[P][P], T[P][P];
            const int ok = factor_pivot<P>(A, np, k0, c.n - k0, thr, S, T);
            if (t == 0) okb = ok;
            const int p = t / w2, col = t - p * w2;
            const double2 *X = col < np ? A + col : R + (col - np);
            double2 xq[P];
#pragma unroll
            for (int q = 0; q < P; ++q) xq[q] = X[(k0 + q) * np];
            double2 v = zero;
#pragma unroll
            for (int pp = 0; pp < P; ++pp)
                if (p == pp) {
#pragma unroll
                    for (int q = 0; q <= pp; ++q) v = cadd(v, cmul(T[pp][q], xq[q]));
                }
            Vb[t] = v;
        }
        __syncthreads();
        const int ok = okb;
        if (ok != 1) return ok;
        if (c.on && c.i >= k0) {  // rows above the pivot block are final
            const int i = c.i, j = c.j;
            double2 na, nr;
            if (i < k0 + P) {
                na = j < i ? zero : Vb[(i - k0) * w2 + j];
                nr = Vb[(i - k0) * w2 + np + j];
            } else {
                na = A[i * np + j];
                nr = R[i * np + j];
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    const double2 u = Vb[p * w2 + i];
                    na = csub(na, cmulc(u, Vb[p * w2 + j]));
                    nr = csub(nr, cmulc(u, Vb[p * w2 + np + j]));
                }
                if (j < k0 + P) na = zero;
            }
            A[i * np + j] = na;
            R[i * np + j] = nr;
        }
        __syncthreads();
    }
    return 1;
}

// Out = op(A) op(B) over the live n x n block (conjA: A^H B; conjB: A B^H).
// Out may alias an operand (the products are formed before the barrier).
__device__ inline void small_mm(const double2 *A, const double2 *B, double2 *Out, const SmallCtx &c, bool conjA = false,
                         bool conjB = false) {
    const int np = c.np;
    const bool live = c.on && c.i < c.n && c.j < c.n;
    double2 s = make_double2(0, 0);
    if (live) {
        for (int k = 0; k < c.n; ++k) {
            const double2 a = conjA ? A[k * np + c.i] : A[c.i * np + k];
            const double2 b = conjB ? B[c.j * np + k] : B[k * np + c.j];
            const double2 a2 = conjA ? make_double2(a.x, -a.y) : a;
            const double2 b2 = conjB ? make_double2(b.x, -b.y) : b;
            s = cadd(s, cmul(a2, b2));
        }
    }
    __syncthreads();
    if (live) Out[c.i * np + c.j] = s;
    __syncthreads();
}

// Live n x n block into the global n x n complex64 matrix (optionally src^H).
__device__ inline void store_c64(float2 *dst, const double2 *src, const SmallCtx &c, bool conj_transpose = false) {
    if (c.on && c.i < c.n && c.j < c.n) {
        const double2 v = conj_transpose ? make_double2(src[c.j * c.np + c.i].x, -src[c.j * c.np + c.i].y)
                                         : src[c.i * c.np + c.j];
        dst[c.i * c.n + c.j] = make_float2((float)v.x, (float)v.y);
    }
}

// Global n x n matrix into the live block of an LDS matrix (zero padding).
__device__ inline void load_small(double2 *dst, const double2 *src, const SmallCtx &c) {
    if (c.on) dst[c.i * c.np + c.j] = (c.i < c.n && c.j < c.n) ? src[c.i * c.n + c.j] : make_double2(0, 0);
}

// ||C e_j|| / base_j into state->relres[j]; scratch[2] = max, scratch[3] = all
// finite. base_j is state->norm0[j], or is set here when set_base >= 0: to
// ||C e_j|| itself (1, the start of a relative stop test) or to 1 (0).
__device__ inline void column_norms(const double2 *C, const SmallCtx &c, SolverState *state, double *scratch,
                                    int set_base = -1) {
    if (threadIdx.x < 64) {
        double s = 0;
        const int j = threadIdx.x;
        if (j < c.n) {
            for (int i = 0; i < c.n; ++i) {
                const double2 v = C[i * c.np + j];
                s += v.x * v.x + v.y * v.y;
            }
            s = sqrt(s);
            double base;
            if (set_base >= 0) {
                base = set_base ? s : 1.0;
                state->norm0[j] = base;
            } else {
                base = state->norm0[j];
            }
            s = s / base;
            state->relres[j] = s;
        }
        double m = (j < c.n) ? s : 0.0;
        int fin = (j < c.n) ? (isfinite(s) ? 1 : 0) : 1;
        for (int k = 32; k > 0; k >>= 1) {
            m = fmax(m, __shfl_xor(m, k));
            fin &= __shfl_xor(fin, k);
        }
        if (threadIdx.x == 0) {
            scratch[2] = m;
            scratch[3] = fin ? 1.0 : 0.0;
        }
    }
    __syncthreads();
}

// Failure flags, set by thread 0 of the writer workgroup.
__device__ inline void fail(SolverState *state, int code, bool writer = true) {
    if (writer && threadIdx.x == 0) {
        if (code == 2)
            state->nonfinite = 1;
        else
            state->breakdown = 1;
        state->active = 0;
    }
}

constexpr int SMALL_INACTIVE = -1;  // the inner iteration had already stopped

// Loads of one inner step: the reduced Gram m.G (Hermitian part, identity
// padding; R = I) and, when `with_c`, C. The active flag is read beside them
// and tested after, so the two global round trips overlap. Returns 1, or
// SMALL_INACTIVE (the same in every thread).
__device__ __forceinline__ int step_load(const SmallMats &m, const SolverState *state, const SmallCtx &c, double2 *A,
                                         double2 *R, double2 *Cm, bool with_c) {
    const int live = state->active;
    if (with_c) load_small(Cm, m.C, c);
    load_gram(A, R, m.G, c);  // ends with a barrier
    return live == 0 ? SMALL_INACTIVE : 1;
}

// Cholesky factorisation of the loaded Gram with the finiteness and trace
// tests in front: 1, 0 (breakdown) or 2 (not finite).
template <int P>
__device__ __forceinline__ int step_factor(double2 *A, double2 *R, const SmallCtx &c, double *scratch) {
    trace_finite(A, c, scratch);
    if (scratch[1] == 0.0) return 2;
    if (!(scratch[0] > 0.0)) return 0;
    return chol_elim<P>(A, R, c, scratch[0]);
}

// Inner step after the Gram D^H Z: D^H Z = S^H S (Hermitian positive definite
// for an HPD operator and full-rank D), N = (D^H Z)^{-1} = S^{-1} S^{-H} into A
// and W = N C into R. On failure the writer sets the flags.
template <int P>
__device__ int step1_body(const SmallMats &m, SolverState *state, const SmallCtx &c, double2 *A, double2 *R,
                          double2 *Cm, double *scratch, bool writer) {
    const int live = step_load(m, state, c, A, R, Cm, true);
    if (live != 1) return live;
    const int ok = step_factor<P>(A, R, c, scratch);
    if (ok != 1) {
        fail(state, ok, writer);
        return ok;
    }
    small_mm(R, R, A, c, true);  // N = R^H R with R = S^{-H}
    small_mm(A, Cm, R, c);       // W = N C
    return 1;
}

// Inner step after the Gram T^H T: T^H T = S^H S, S into A and S^{-H} into R.
// The writer also forms C <- S C, the residual norms ||C e_j|| and the stop
// flags, and counts the iteration (also when the factorisation fails: the
// iteration's X update is in by then).
template <int P>
__device__ int step2_body(const SmallMats &m, SolverState *state, const SmallCtx &c, double2 *A, double2 *R,
                          double2 *Cm, double *scratch, bool writer) {
    const int live = step_load(m, state, c, A, R, Cm, writer);
    if (live != 1) return live;
    const int ok = step_factor<P>(A, R, c, scratch);
    if (ok != 1) {
        if (writer && threadIdx.x == 0) state->iters += 1;
        fail(state, ok, writer);
        return ok;
    }
    if (writer) {
        small_mm(A, Cm, Cm, c);  // C_new = S C (in place through the barrier)
        if (c.on && c.i < c.n && c.j < c.n) m.C[c.i * c.n + c.j] = Cm[c.i * c.np + c.j];
        column_norms(Cm, c, state, scratch);
        if (threadIdx.x == 0) {
            state->iters += 1;
            if (scratch[3] == 0.0) {
                state->nonfinite = 1;
                state->active = 0;
            } else if (scratch[2] <= state->tol) {
                state->done = 1;
                state->active = 0;
            } else if (state->iters >= state->max_inner) {
                state->active = 0;
            }
        }
    }
    return 1;
}

}  // namespace coarse
