// Block-CG linear algebra of BlockCGrQ (Fig. 2, left) on the device.
//
// * Gram matrices A^H B of two tall-skinny (rows x nrhs) blocks: split-K over a
//   fixed number of workgroups, double accumulation (a complex64 product is
//   exact in double), then a second pass that sums the partials in a fixed
//   order, so results are bitwise reproducible. This is the "many short-K
//   products summed by hand" treatment the paper found necessary for ThinQR
//   (Sec. 3.5), done as one split-K reduction.
// * Small nrhs x nrhs steps in double on one workgroup: Cholesky (the thin QR
//   kept explicit, Sec. 2.2), triangular inverses and products, the residual
//   column norms ||C e_j||, convergence and breakdown flags.
// * Block-vector updates X += D (N C), T = Q - Z N, Q = T S^{-1},
//   D = Q + D S^H, rows staged in LDS so updates are done in place.
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
// Gram reduction
// ---------------------------------------------------------------------------
constexpr int GRAM_TILE = 32;

template <typename T2>
__global__ __launch_bounds__(256) void gram_partial_kernel(const T2 *__restrict__ a, const T2 *__restrict__ b,
                                                           long long rows, int nr, double2 *__restrict__ partials,
                                                           const int *__restrict__ active) {
    __shared__ T2 as[GRAM_TILE * 32];
    __shared__ T2 bs[GRAM_TILE * 32];
    __shared__ double2 red[256];
    if (active != nullptr && *active == 0) return;
    const int tid = threadIdx.x;
    const int ne = nr * nr;
    const int groups = ne >= 256 ? 1 : 256 / ne;
    const int grp = tid / (ne < 256 ? ne : 256);
    const bool busy = grp < groups;
    const long long chunk = (rows + gridDim.x - 1) / gridDim.x;
    const long long r0 = blockIdx.x * chunk;
    long long r1 = r0 + chunk;
    if (r1 > rows) r1 = rows;
    double2 acc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = make_double2(0, 0);
    for (long long t0 = r0; t0 < r1; t0 += GRAM_TILE) {
        const int tr = (int)((r1 - t0) < GRAM_TILE ? (r1 - t0) : GRAM_TILE);
        for (int e = tid; e < tr * nr; e += 256) {
            as[e] = a[t0 * nr + e];
            bs[e] = b[t0 * nr + e];
        }
        __syncthreads();
        if (busy) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int ent = (ne >= 256) ? tid + 256 * k : tid - grp * ne;
                if (ent < ne && (k == 0 || ne >= 256)) {
                    const int ia = ent / nr, ic = ent - ia * nr;
                    double2 s = acc[k];
                    for (int rr = grp; rr < tr; rr += groups)
                        s = cadd(s, cmulc(to_d2(as[rr * nr + ia]), to_d2(bs[rr * nr + ic])));
                    acc[k] = s;
                }
            }
        }
        __syncthreads();
    }
    double2 *out = partials + (size_t)blockIdx.x * ne;
    if (ne >= 256) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int ent = tid + 256 * k;
            if (ent < ne) out[ent] = acc[k];
        }
    } else {
        red[tid] = busy ? acc[0] : make_double2(0, 0);
        __syncthreads();
        if (tid < ne) {
            double2 s = make_double2(0, 0);
            for (int gg = 0; gg < groups; ++gg) s = cadd(s, red[gg * ne + tid]);
            out[tid] = s;
        }
    }
}

__global__ __launch_bounds__(256) void gram_reduce_kernel(const double2 *__restrict__ partials, int nparts, int ne,
                                                          double2 *__restrict__ g, const int *__restrict__ active) {
    __shared__ double2 red[256];
    if (active != nullptr && *active == 0) return;
    const int e = blockIdx.x;
    double2 s = make_double2(0, 0);
    for (int k = threadIdx.x; k < nparts; k += 256) s = cadd(s, partials[(size_t)k * ne + e]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) g[e] = red[0];
}

template <typename T2>
void gram(const T2 *a, const T2 *b, long long rows, int nr, double2 *partials, double2 *g, const int *active,
          hipStream_t st) {
    hipLaunchKernelGGL(gram_partial_kernel<T2>, dim3(GRAM_BLOCKS), dim3(256), 0, st, a, b, rows, nr, partials,
                       active);
    hipLaunchKernelGGL(gram_reduce_kernel, dim3(nr * nr), dim3(256), 0, st, partials, GRAM_BLOCKS, nr * nr, g,
                       active);
}
template void gram<float2>(const float2 *, const float2 *, long long, int, double2 *, double2 *, const int *,
                           hipStream_t);
template void gram<double2>(const double2 *, const double2 *, long long, int, double2 *, double2 *, const int *,
                            hipStream_t);

// ---------------------------------------------------------------------------
// Outer-loop vector kernels (double)
// ---------------------------------------------------------------------------
__global__ void normalize_kernel(const double2 *__restrict__ r, const double2 *__restrict__ gdiag, long long rows,
                                 int nr, float2 *__restrict__ q, float2 *__restrict__ e) {
    const long long total = rows * nr;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < total;
         k += (long long)gridDim.x * blockDim.x) {
        const int col = (int)(k % nr);
        const double rn = sqrt(gdiag[col * nr + col].x);
        const double inv = rn > 0 ? 1.0 / rn : 0.0;
        const double2 v = r[k];
        q[k] = make_float2((float)(v.x * inv), (float)(v.y * inv));
        e[k] = make_float2(0.f, 0.f);
    }
}

__global__ void outer_update_kernel(double2 *__restrict__ x, const float2 *__restrict__ e,
                                    const double2 *__restrict__ gdiag, long long rows, int nr) {
    const long long total = rows * nr;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < total;
         k += (long long)gridDim.x * blockDim.x) {
        const int col = (int)(k % nr);
        const double rn = sqrt(gdiag[col * nr + col].x);
        const float2 v = e[k];
        double2 xv = x[k];
        xv.x += (double)v.x * rn;
        xv.y += (double)v.y * rn;
        x[k] = xv;
    }
}

static unsigned grid_for(long long total) {
    long long b = (total + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (unsigned)b;
}

void normalize_residual(const double2 *r, const double2 *gdiag, long long rows, int nr, float2 *q, float2 *e,
                        hipStream_t st) {
    hipLaunchKernelGGL(normalize_kernel, dim3(grid_for(rows * nr)), dim3(256), 0, st, r, gdiag, rows, nr, q, e);
}

void outer_update(double2 *x, const float2 *e, const double2 *gres, long long rows, int nr, hipStream_t st) {
    hipLaunchKernelGGL(outer_update_kernel, dim3(grid_for(rows * nr)), dim3(256), 0, st, x, e, gres, rows, nr);
}

// ---------------------------------------------------------------------------
// Small dense double-precision steps (one workgroup of 256 threads)
// ---------------------------------------------------------------------------
constexpr double BREAKDOWN_EPS = 1e-12;

__device__ void load_hermitian(double2 *A, const double2 *G, int n) {
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e - i * n;
        const double2 a = G[i * n + j], b = G[j * n + i];
        A[e] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    }
    __syncthreads();
}

// In place: A (Hermitian, upper part used) -> upper triangular C with C^H C = A.
// Returns 1 on success, 0 on a pivot <= eps*trace, 2 on a non-finite entry.
__device__ int chol_upper(double2 *A, int n, double *scratch) {
    if (threadIdx.x == 0) {
        double tr = 0;
        bool fin = true;
        for (int k = 0; k < n; ++k) tr += A[k * n + k].x;
        for (int e = 0; e < n * n; ++e) fin = fin && isfinite(A[e].x) && isfinite(A[e].y);
        scratch[0] = tr;
        scratch[1] = fin ? 1.0 : 0.0;
    }
    __syncthreads();
    const double tr = scratch[0];
    if (scratch[1] == 0.0) return 2;
    for (int k = 0; k < n; ++k) {
        const double piv = A[k * n + k].x;
        __syncthreads();
        if (!(piv > BREAKDOWN_EPS * tr)) return isfinite(piv) ? 0 : 2;
        const double d = sqrt(piv);
        for (int j = k + 1 + threadIdx.x; j < n; j += blockDim.x) {
            const double2 v = A[k * n + j];
            A[k * n + j] = make_double2(v.x / d, v.y / d);
        }
        if (threadIdx.x == 0) A[k * n + k] = make_double2(d, 0);
        __syncthreads();
        const int m = n - k - 1;
        for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
            const int i = k + 1 + idx / m, j = k + 1 + idx % m;
            if (j >= i) A[i * n + j] = csub(A[i * n + j], cmulc(A[k * n + i], A[k * n + j]));
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e - i * n;
        if (i > j) A[e] = make_double2(0, 0);
    }
    __syncthreads();
    return 1;
}

// Ci = C^{-1} for upper triangular C (column-wise back substitution).
__device__ void tri_inv_upper(const double2 *C, double2 *Ci, int n) {
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        for (int i = n - 1; i > j; --i) Ci[i * n + j] = make_double2(0, 0);
        for (int i = j; i >= 0; --i) {
            double2 s = make_double2(i == j ? 1.0 : 0.0, 0);
            for (int k = i + 1; k <= j; ++k) s = csub(s, cmul(C[i * n + k], Ci[k * n + j]));
            const double2 dd = C[i * n + i];  // real positive
            Ci[i * n + j] = make_double2(s.x / dd.x, s.y / dd.x);
        }
    }
    __syncthreads();
}

// Out = op(A) B, op = identity or conjugate transpose.
__device__ void small_mm(const double2 *A, const double2 *B, double2 *Out, int n, bool conjA) {
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e - i * n;
        double2 s = make_double2(0, 0);
        for (int k = 0; k < n; ++k)
            s = cadd(s, conjA ? cmulc(A[k * n + i], B[k * n + j]) : cmul(A[i * n + k], B[k * n + j]));
        Out[e] = s;
    }
    __syncthreads();
}

// Out = A B^H
__device__ void small_mm_bh(const double2 *A, const double2 *B, double2 *Out, int n) {
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e - i * n;
        double2 s = make_double2(0, 0);
        for (int k = 0; k < n; ++k) s = cadd(s, cmulc(B[j * n + k], A[i * n + k]));
        Out[e] = s;
    }
    __syncthreads();
}

__device__ void store_c64(float2 *dst, const double2 *src, int n, bool conj_transpose) {
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e - i * n;
        const double2 v = conj_transpose ? make_double2(src[j * n + i].x, -src[j * n + i].y) : src[e];
        dst[e] = make_float2((float)v.x, (float)v.y);
    }
}

__device__ void column_norms(const double2 *C, int n, SolverState *state, double *scratch) {
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        double s = 0;
        for (int i = 0; i < n; ++i) s += C[i * n + j].x * C[i * n + j].x + C[i * n + j].y * C[i * n + j].y;
        state->relres[j] = sqrt(s);
        scratch[4 + j] = sqrt(s);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0;
        bool fin = true;
        for (int j = 0; j < n; ++j) {
            m = fmax(m, scratch[4 + j]);
            fin = fin && isfinite(scratch[4 + j]);
        }
        scratch[2] = m;
        scratch[3] = fin ? 1.0 : 0.0;
    }
    __syncthreads();
}

__device__ void fail(SolverState *state, int code) {
    if (threadIdx.x == 0) {
        if (code == 2)
            state->nonfinite = 1;
        else
            state->breakdown = 1;
        state->active = 0;
    }
}

__global__ __launch_bounds__(256) void small_init_kernel(SmallMats m, SolverState *state, int n, double tol,
                                                         int max_inner) {
    __shared__ double2 A[32 * 32], Ci[32 * 32];
    __shared__ double scratch[40];
    if (threadIdx.x == 0) {
        state->active = 0;
        state->done = 0;
        state->breakdown = 0;
        state->nonfinite = 0;
        state->iters = 0;
        state->max_inner = max_inner;
        state->tol = tol;
    }
    load_hermitian(A, m.G, n);
    const int ok = chol_upper(A, n, scratch);
    if (ok != 1) {
        fail(state, ok);
        return;
    }
    tri_inv_upper(A, Ci, n);
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) m.C[e] = A[e];
    store_c64(m.Sinv, Ci, n, false);
    column_norms(A, n, state, scratch);
    if (threadIdx.x == 0) {
        if (scratch[2] <= tol)
            state->done = 1;
        else
            state->active = max_inner > 0 ? 1 : 0;
    }
}

// After G = D^H Z: N = G^{-1} = C1^{-1} C1^{-H} (C1^H C1 = G), W = N C.
__global__ __launch_bounds__(256) void small_step1_kernel(SmallMats m, SolverState *state, int n) {
    __shared__ double2 A[32 * 32], Ci[32 * 32], Nm[32 * 32];
    __shared__ double scratch[40];
    if (state->active == 0) return;
    load_hermitian(A, m.G, n);
    const int ok = chol_upper(A, n, scratch);
    if (ok != 1) {
        fail(state, ok);
        return;
    }
    tri_inv_upper(A, Ci, n);
    small_mm_bh(Ci, Ci, Nm, n);  // N = Ci Ci^H
    store_c64(m.N, Nm, n, false);
    // W = N C  (C from global, complex128)
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) A[e] = m.C[e];
    __syncthreads();
    small_mm(Nm, A, Ci, n, false);
    store_c64(m.W, Ci, n, false);
}

// After G = T^H T: S^H S = G, Sinv = S^{-1}, SH = S^H, C <- S C, residual norms, stop tests.
__global__ __launch_bounds__(256) void small_step2_kernel(SmallMats m, SolverState *state, int n) {
    __shared__ double2 A[32 * 32], Ci[32 * 32], Cc[32 * 32];
    __shared__ double scratch[40];
    if (state->active == 0) return;
    load_hermitian(A, m.G, n);
    const int ok = chol_upper(A, n, scratch);
    if (ok != 1) {
        if (threadIdx.x == 0) state->iters += 1;  // this iteration's X update is in
        fail(state, ok);
        return;
    }
    tri_inv_upper(A, Ci, n);
    store_c64(m.Sinv, Ci, n, false);
    store_c64(m.SH, A, n, true);
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) Cc[e] = m.C[e];
    __syncthreads();
    small_mm(A, Cc, Ci, n, false);  // C_new = S C
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) m.C[e] = Ci[e];
    column_norms(Ci, n, state, scratch);
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

void small_init(SmallMats m, SolverState *state, int nr, double tol, int max_inner, hipStream_t st) {
    hipLaunchKernelGGL(small_init_kernel, dim3(1), dim3(256), 0, st, m, state, nr, tol, max_inner);
}
void small_step1(SmallMats m, SolverState *state, int nr, hipStream_t st) {
    hipLaunchKernelGGL(small_step1_kernel, dim3(1), dim3(256), 0, st, m, state, nr);
}
void small_step2(SmallMats m, SolverState *state, int nr, hipStream_t st) {
    hipLaunchKernelGGL(small_step2_kernel, dim3(1), dim3(256), 0, st, m, state, nr);
}

// ---------------------------------------------------------------------------
// Tall-skinny block updates (rows of nrhs complex64 entries)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 fcmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__global__ __launch_bounds__(256) void update_xt_kernel(float2 *__restrict__ e, float2 *__restrict__ q,
                                                        const float2 *__restrict__ d, const float2 *__restrict__ z,
                                                        const float2 *__restrict__ w, const float2 *__restrict__ nm,
                                                        long long rows, int nr, const int *__restrict__ active) {
    __shared__ float2 Ws[32 * 32], Ns[32 * 32], Ds[256], Zs[256];
    if (active != nullptr && *active == 0) return;
    for (int k = threadIdx.x; k < nr * nr; k += 256) {
        Ws[k] = w[k];
        Ns[k] = nm[k];
    }
    const int rp = 256 / nr;
    const int rl = threadIdx.x / nr, r = threadIdx.x - rl * nr;
    const bool lane_ok = rl < rp;
    for (long long row0 = (long long)blockIdx.x * rp; row0 < rows; row0 += (long long)gridDim.x * rp) {
        const long long row = row0 + rl;
        const bool ok = lane_ok && row < rows;
        __syncthreads();
        if (ok) {
            Ds[rl * nr + r] = d[row * nr + r];
            Zs[rl * nr + r] = z[row * nr + r];
        }
        __syncthreads();
        if (ok) {
            float2 ea = make_float2(0.f, 0.f), ta = make_float2(0.f, 0.f);
            for (int c = 0; c < nr; ++c) {
                const float2 dv = Ds[rl * nr + c], zv = Zs[rl * nr + c];
                const float2 wv = Ws[c * nr + r], nv = Ns[c * nr + r];
                ea.x += dv.x * wv.x - dv.y * wv.y;
                ea.y += dv.x * wv.y + dv.y * wv.x;
                ta.x += zv.x * nv.x - zv.y * nv.y;
                ta.y += zv.x * nv.y + zv.y * nv.x;
            }
            const long long k = row * nr + r;
            float2 ev = e[k], qv = q[k];
            e[k] = make_float2(ev.x + ea.x, ev.y + ea.y);
            q[k] = make_float2(qv.x - ta.x, qv.y - ta.y);
        }
    }
}

__global__ __launch_bounds__(256) void update_qd_kernel(float2 *__restrict__ q, float2 *__restrict__ d,
                                                        const float2 *__restrict__ sinv, const float2 *__restrict__ sh,
                                                        long long rows, int nr, int init,
                                                        const int *__restrict__ active) {
    __shared__ float2 Si[32 * 32], Sh[32 * 32], Qs[256], Ds[256];
    if (active != nullptr && *active == 0) return;
    for (int k = threadIdx.x; k < nr * nr; k += 256) {
        Si[k] = sinv[k];
        Sh[k] = init ? make_float2(0.f, 0.f) : sh[k];
    }
    const int rp = 256 / nr;
    const int rl = threadIdx.x / nr, r = threadIdx.x - rl * nr;
    const bool lane_ok = rl < rp;
    for (long long row0 = (long long)blockIdx.x * rp; row0 < rows; row0 += (long long)gridDim.x * rp) {
        const long long row = row0 + rl;
        const bool ok = lane_ok && row < rows;
        __syncthreads();
        if (ok) {
            Qs[rl * nr + r] = q[row * nr + r];
            Ds[rl * nr + r] = init ? make_float2(0.f, 0.f) : d[row * nr + r];
        }
        __syncthreads();
        if (ok) {
            float2 qa = make_float2(0.f, 0.f), da = make_float2(0.f, 0.f);
            for (int c = 0; c < nr; ++c) {
                const float2 qv = Qs[rl * nr + c], dv = Ds[rl * nr + c];
                const float2 sv = Si[c * nr + r], hv = Sh[c * nr + r];
                qa.x += qv.x * sv.x - qv.y * sv.y;
                qa.y += qv.x * sv.y + qv.y * sv.x;
                da.x += dv.x * hv.x - dv.y * hv.y;
                da.y += dv.x * hv.y + dv.y * hv.x;
            }
            const long long k = row * nr + r;
            q[k] = qa;
            d[k] = make_float2(qa.x + da.x, qa.y + da.y);
        }
    }
}

static unsigned update_grid(long long rows, int nr) {
    const long long rp = 256 / nr;
    long long b = (rows + rp - 1) / rp;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (unsigned)b;
}

void update_xt(float2 *e, float2 *q, const float2 *d, const float2 *z, const float2 *w, const float2 *n,
               long long rows, int nr, const int *active, hipStream_t st) {
    hipLaunchKernelGGL(update_xt_kernel, dim3(update_grid(rows, nr)), dim3(256), 0, st, e, q, d, z, w, n, rows, nr,
                       active);
}

void update_qd(float2 *q, float2 *d, const float2 *sinv, const float2 *sh, long long rows, int nr, int init,
               const int *active, hipStream_t st) {
    hipLaunchKernelGGL(update_qd_kernel, dim3(update_grid(rows, nr)), dim3(256), 0, st, q, d, sinv, sh, rows, nr,
                       init, active);
}

}  // namespace coarse
