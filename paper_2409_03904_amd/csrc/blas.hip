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
#include <type_traits>

#include "blas.hpp"
#include "small.hpp"

namespace coarse {


// ---------------------------------------------------------------------------
// Gram reduction
//
// Workgroup b owns a fixed contiguous range of rows. Its four waves take
// every fourth row of each LDS-staged 64-row tile; inside a wave the 64 lanes
// form an 8 x 8 grid and lane (ta, tc) accumulates the BS x BS entries
// (ta + 8u, tc + 8v) of G in double (BS = ceil(nr/8)), i.e. 2*BS LDS reads
// per BS*BS complex multiply-adds. The four waves' sums are added in LDS in a
// fixed order and written as the workgroup's partial.
// ---------------------------------------------------------------------------
constexpr int GRAM_TILE = 32;

template <typename T2, int BS>
__global__ __launch_bounds__(256) void gram_partial_kernel(const T2 *__restrict__ a, const T2 *__restrict__ b,
                                                           long long rows, int nr, double2 *__restrict__ partials,
                                                           const int *__restrict__ active) {
    // two double-buffered tile pairs during the sweep, then the four waves' sums
    constexpr int TILE_T2 = GRAM_TILE * 32;
    constexpr int RAW = (4 * TILE_T2 * (int)sizeof(T2)) > 65536 ? (4 * TILE_T2 * (int)sizeof(T2)) : 65536;
    __shared__ __align__(16) unsigned char raw[RAW];
    T2 *tiles = reinterpret_cast<T2 *>(raw);
    double2 *red = reinterpret_cast<double2 *>(raw);
    if (active != nullptr && *active == 0) return;
    const int tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63, ta = lane >> 3, tc = lane & 7;
    const long long chunk = (rows + gridDim.x - 1) / gridDim.x;
    const long long r0 = blockIdx.x * chunk;
    long long r1 = r0 + chunk;
    if (r1 > rows) r1 = rows;
    double2 acc[BS][BS];
#pragma unroll
    for (int u = 0; u < BS; ++u)
#pragma unroll
        for (int v = 0; v < BS; ++v) acc[u][v] = make_double2(0, 0);
    const int per = GRAM_TILE * nr;       // elements per tile
    const int nld = (per + 255) / 256;    // <= 4
    // staging registers as native vectors (HIP's struct vector types in an
    // array are not split into registers and would live in scratch)
    typedef typename std::conditional<sizeof(T2) == 16, double, float>::type E;
    typedef E NV __attribute__((ext_vector_type(2)));
    const NV *av2 = reinterpret_cast<const NV *>(a), *bv2 = reinterpret_cast<const NV *>(b);
    NV ra[4], rb[4];
    const long long total = r1 > r0 ? (r1 - r0) * nr : 0;
    auto fetch = [&](long long t0) {      // tile starting at row t0 into registers (index clamped)
        const long long base = (t0 - r0) * nr;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k < nld) {
                long long e = base + tid + 256 * k;
                e = e < total ? e : total - 1;
                ra[k] = av2[r0 * nr + e];
                rb[k] = bv2[r0 * nr + e];
            }
        }
    };
    auto stash = [&](int buf) {
        NV *as = reinterpret_cast<NV *>(tiles + buf * 2 * TILE_T2), *bs = as + TILE_T2;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int e = tid + 256 * k;
            if (k < nld && e < per) {
                as[e] = ra[k];
                bs[e] = rb[k];
            }
        }
    };
    if (total > 0) {
        fetch(r0);
        stash(0);
    }
    __syncthreads();
    int buf = 0;
    for (long long t0 = r0; t0 < r1; t0 += GRAM_TILE) {
        const int tr = (int)((r1 - t0) < GRAM_TILE ? (r1 - t0) : GRAM_TILE);
        const bool more = t0 + GRAM_TILE < r1;
        if (more) fetch(t0 + GRAM_TILE);
        const T2 *as = tiles + buf * 2 * TILE_T2, *bs = as + TILE_T2;
        for (int rr = w; rr < tr; rr += 4) {
            double2 av[BS], bv[BS];
#pragma unroll
            for (int u = 0; u < BS; ++u) {
                const int ia = ta + 8 * u, ic = tc + 8 * u;
                av[u] = ia < nr ? to_d2(as[rr * nr + ia]) : make_double2(0, 0);
                bv[u] = ic < nr ? to_d2(bs[rr * nr + ic]) : make_double2(0, 0);
            }
#pragma unroll
            for (int u = 0; u < BS; ++u)
#pragma unroll
                for (int v = 0; v < BS; ++v) acc[u][v] = cadd(acc[u][v], cmulc(av[u], bv[v]));
        }
        if (more) stash(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    const int ne = nr * nr;
#pragma unroll
    for (int u = 0; u < BS; ++u)
#pragma unroll
        for (int v = 0; v < BS; ++v) {
            const int ia = ta + 8 * u, ic = tc + 8 * v;
            if (ia < nr && ic < nr) red[w * ne + ia * nr + ic] = acc[u][v];
        }
    __syncthreads();
    double2 *out = partials + (size_t)blockIdx.x * ne;
    for (int e = tid; e < ne; e += 256)
        out[e] = cadd(cadd(red[e], red[ne + e]), cadd(red[2 * ne + e], red[3 * ne + e]));
}

// Lane l of each entry of G sums partials l, l + 64, ... in order; then a fixed
// butterfly (pairs 32, 16, 8, 4, 2, 1 apart) adds the 64 lane sums: the
// summation order is fixed, so the result is reproducible bit for bit. A
// workgroup of eight waves takes eight consecutive entries: thread (el, pl),
// el = tid % 8, pl = tid / 8, holds lane pl of entry 8 b + el, so one load
// instruction reads eight whole 128-byte lines (eight partials x eight
// entries) instead of 64 lines from 64 partials. The butterfly's first three
// levels cross waves (through LDS, wave 0 finishing them), the last three run
// by shuffles inside wave 0. The partials are always valid memory (entries
// past ne are clamped), so their loads go out beside the flag's and only the
// store waits for it. count: partials, a multiple of 64 (GRAM_BLOCKS for the
// split-K Gram kernels, 256 for the fused step-1 update, one per workgroup of
// the Gram-fused apply).
constexpr int REDUCE_ENTRIES = 8;
__global__ __launch_bounds__(64 * REDUCE_ENTRIES) void gram_reduce_kernel(const double2 *__restrict__ partials,
                                                                          int ne, int count,
                                                                          double2 *__restrict__ g,
                                                                          const int *__restrict__ active) {
    static_assert(GRAM_BLOCKS % 64 == 0, "whole rounds of 64 partials");
    __shared__ double2 ls[64 * REDUCE_ENTRIES];
    const int el = threadIdx.x % REDUCE_ENTRIES, pl = threadIdx.x / REDUCE_ENTRIES;
    const int e = blockIdx.x * REDUCE_ENTRIES + el;
    const int ec = e < ne ? e : ne - 1;
    // unconditional load (a load under a branch is waited for at the join):
    // without a flag it reads a word of the partials and ignores it
    const int flag = *(active != nullptr ? active : reinterpret_cast<const int *>(partials));
    const int live = active != nullptr ? flag : 1;
    const int rounds = count / 64;
    double2 s = partials[(size_t)pl * ne + ec];
    for (int k0 = 1; k0 < rounds; k0 += 8) {
        double2 v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int kk = k0 + k < rounds ? k0 + k : rounds - 1;  // clamped: loaded, not added
            v[k] = partials[(size_t)(pl + 64 * kk) * ne + ec];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (k0 + k < rounds) s = cadd(s, v[k]);
    }
    ls[pl * REDUCE_ENTRIES + el] = s;
    __syncthreads();
    if (threadIdx.x < 64) {  // wave 0: lane = el + 8 pl, pl < 8
        auto at = [&](int q) { return ls[q * REDUCE_ENTRIES + el]; };
        // levels 32, 16, 8 of the butterfly, for lane sums pl < 8
        const double2 a0 = cadd(at(pl), at(pl + 32)), a1 = cadd(at(pl + 16), at(pl + 48));
        const double2 a2 = cadd(at(pl + 8), at(pl + 40)), a3 = cadd(at(pl + 24), at(pl + 56));
        double2 c = cadd(cadd(a0, a1), cadd(a2, a3));
        // levels 4, 2, 1: pl xor 4, 2, 1 is lane xor 32, 16, 8
#pragma unroll
        for (int m = 32; m >= 8; m >>= 1) {
            c.x += __shfl_xor(c.x, m);
            c.y += __shfl_xor(c.y, m);
        }
        if (live != 0 && pl == 0 && e < ne) g[e] = c;
    }
}

template <typename T2>
void gram_partials(const T2 *a, const T2 *b, long long rows, int nr, double2 *partials, const int *active,
                   hipStream_t st) {
    const int bsz = (nr + 7) / 8;
    switch (bsz) {
        case 1: hipLaunchKernelGGL((gram_partial_kernel<T2, 1>), dim3(GRAM_BLOCKS), dim3(256), 0, st, a, b, rows, nr, partials, active); break;
        case 2: hipLaunchKernelGGL((gram_partial_kernel<T2, 2>), dim3(GRAM_BLOCKS), dim3(256), 0, st, a, b, rows, nr, partials, active); break;
        case 3: hipLaunchKernelGGL((gram_partial_kernel<T2, 3>), dim3(GRAM_BLOCKS), dim3(256), 0, st, a, b, rows, nr, partials, active); break;
        default: hipLaunchKernelGGL((gram_partial_kernel<T2, 4>), dim3(GRAM_BLOCKS), dim3(256), 0, st, a, b, rows, nr, partials, active); break;
    }
}

void gram_reduce(const double2 *partials, int nr, double2 *g, const int *active, hipStream_t st) {
    gram_reduce_n(partials, GRAM_BLOCKS, nr, g, active, st);
}

void gram_reduce_n(const double2 *partials, int count, int nr, double2 *g, const int *active, hipStream_t st) {
    const int ne = nr * nr;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3((ne + REDUCE_ENTRIES - 1) / REDUCE_ENTRIES), dim3(64 * REDUCE_ENTRIES),
                       0, st, partials, ne, count, g, active);
}

template <typename T2>
void gram(const T2 *a, const T2 *b, long long rows, int nr, double2 *partials, double2 *g, const int *active,
          hipStream_t st) {
    gram_partials<T2>(a, b, rows, nr, partials, active, st);
    gram_reduce(partials, nr, g, active, st);
}
template void gram<float2>(const float2 *, const float2 *, long long, int, double2 *, double2 *, const int *,
                           hipStream_t);
template void gram<double2>(const double2 *, const double2 *, long long, int, double2 *, double2 *, const int *,
                            hipStream_t);
template void gram_partials<float2>(const float2 *, const float2 *, long long, int, double2 *, const int *,
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

// One workgroup of np^2 threads (rounded up to whole waves): BOUND 256 for
// n <= 16, 1024 up to n = 32; pivot blocks of SMALL_P = 4 either way.

// Q_0 C_0 = R^: C_0 = S from R^H R = S^H S, C_0^{-1} = S^{-1} for Q_0 = R S^{-1}.
template <int BOUND>
__global__ __launch_bounds__(BOUND) void small_init_kernel(SmallMats m, SolverState *state, int n, double tol,
                                                           int max_inner, int relative) {
    __shared__ double2 A[SMALL_MAX * SMALL_MAX], R[SMALL_MAX * SMALL_MAX];
    __shared__ double scratch[8];
    const SmallCtx c = small_ctx<SMALL_P>(n);
    if (threadIdx.x == 0) {
        state->active = 0;
        state->done = 0;
        state->breakdown = 0;
        state->nonfinite = 0;
        state->iters = 0;
        state->max_inner = max_inner;
        state->tol = tol;
    }
    load_gram(A, R, m.G, c);
    const int ok = step_factor<SMALL_P>(A, R, c, scratch);
    if (ok != 1) {
        fail(state, ok);
        return;
    }
    if (c.on && c.i < c.n && c.j < c.n) m.C[c.i * n + c.j] = A[c.i * c.np + c.j];
    store_c64(m.Sinv, R, c, true);  // S^{-1} = (S^{-H})^H
    column_norms(A, c, state, scratch, relative ? 1 : 0);
    if (threadIdx.x == 0) {
        if (scratch[2] <= tol)
            state->done = 1;
        else
            state->active = max_inner > 0 ? 1 : 0;
    }
}

// After the Gram D^H Z: N = (D^H Z)^{-1}, W = N C, stored for the block update.
template <int BOUND>
__global__ __launch_bounds__(BOUND) void small_step1_kernel(SmallMats m, SolverState *state, int n) {
    __shared__ double2 A[SMALL_MAX * SMALL_MAX], R[SMALL_MAX * SMALL_MAX], Cm[SMALL_MAX * SMALL_MAX];
    __shared__ double scratch[8];
    const SmallCtx c = small_ctx<SMALL_P>(n);
    if (step1_body<SMALL_P>(m, state, c, A, R, Cm, scratch, true) != 1) return;
    store_c64(m.N, A, c);
    store_c64(m.W, R, c);
}

// After the Gram T^H T: S^H S = T^H T, C <- S C, ||C e_j||, stop tests; S^{-1}
// and S^H stored for the block update.
template <int BOUND>
__global__ __launch_bounds__(BOUND) void small_step2_kernel(SmallMats m, SolverState *state, int n) {
    __shared__ double2 A[SMALL_MAX * SMALL_MAX], R[SMALL_MAX * SMALL_MAX], Cm[SMALL_MAX * SMALL_MAX];
    __shared__ double scratch[8];
    const SmallCtx c = small_ctx<SMALL_P>(n);
    if (step2_body<SMALL_P>(m, state, c, A, R, Cm, scratch, true) != 1) return;
    store_c64(m.SH, A, c, true);
    store_c64(m.Sinv, R, c, true);  // S^{-1} = (S^{-H})^H
}

#define SMALL_LAUNCH(KERNEL, ...)                                                                          \
    do {                                                                                                   \
        const int nt_ = small_threads(small_pad(nr, SMALL_P));                                             \
        if (nt_ <= 256)                                                                                    \
            hipLaunchKernelGGL(KERNEL<256>, dim3(1), dim3(nt_), 0, st, __VA_ARGS__);                       \
        else                                                                                               \
            hipLaunchKernelGGL(KERNEL<1024>, dim3(1), dim3(nt_), 0, st, __VA_ARGS__);                      \
    } while (0)

void small_init(SmallMats m, SolverState *state, int nr, double tol, int max_inner, hipStream_t st, int relative) {
    SMALL_LAUNCH(small_init_kernel, m, state, nr, tol, max_inner, relative);
}
void small_step1(SmallMats m, SolverState *state, int nr, hipStream_t st) {
    SMALL_LAUNCH(small_step1_kernel, m, state, nr);
}
void small_step2(SmallMats m, SolverState *state, int nr, hipStream_t st) {
    SMALL_LAUNCH(small_step2_kernel, m, state, nr);
}
#undef SMALL_LAUNCH

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

// Preconditioned iteration, after N = (D^H z)^{-1} and W = N C:
// E += D W; t = q - z N; T = qp - zp N (t, T in place of q, qp). One row of
// nrhs entries per nrhs lanes; D, z, zp rows staged in LDS.
__global__ __launch_bounds__(256) void update_pxt_kernel(float2 *__restrict__ e, float2 *__restrict__ q,
                                                         float2 *__restrict__ qp, const float2 *__restrict__ d,
                                                         const float2 *__restrict__ z, const float2 *__restrict__ zp,
                                                         const float2 *__restrict__ w, const float2 *__restrict__ nm,
                                                         long long rows, int nr, const int *__restrict__ active) {
    __shared__ float2 Ws[32 * 32], Ns[32 * 32], Ds[256], Zs[256], Ps[256];
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
            Ps[rl * nr + r] = zp[row * nr + r];
        }
        __syncthreads();
        if (ok) {
            float2 ea = make_float2(0.f, 0.f), ta = make_float2(0.f, 0.f), pa = make_float2(0.f, 0.f);
            for (int c = 0; c < nr; ++c) {
                const float2 wv = Ws[c * nr + r], nv = Ns[c * nr + r];
                const float2 dv = Ds[rl * nr + c], zv = Zs[rl * nr + c], pv = Ps[rl * nr + c];
                const float2 dw = fcmul(dv, wv), zn = fcmul(zv, nv), pn = fcmul(pv, nv);
                ea.x += dw.x;
                ea.y += dw.y;
                ta.x += zn.x;
                ta.y += zn.y;
                pa.x += pn.x;
                pa.y += pn.y;
            }
            const long long k = row * nr + r;
            const float2 ev = e[k], qv = q[k], pv = qp[k];
            e[k] = make_float2(ev.x + ea.x, ev.y + ea.y);
            q[k] = make_float2(qv.x - ta.x, qv.y - ta.y);
            qp[k] = make_float2(pv.x - pa.x, pv.y - pa.y);
        }
    }
}

// Preconditioned iteration, after S^H S = T^H t:
// q = t S^{-1}; qp = T S^{-1}; D = qp + D S^H (D = qp when init).
__global__ __launch_bounds__(256) void update_pqd_kernel(float2 *__restrict__ q, float2 *__restrict__ qp,
                                                         float2 *__restrict__ d, const float2 *__restrict__ sinv,
                                                         const float2 *__restrict__ sh, long long rows, int nr,
                                                         int init, const int *__restrict__ active) {
    __shared__ float2 Si[32 * 32], Sh[32 * 32], Qs[256], Ps[256], Ds[256];
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
            Ps[rl * nr + r] = qp[row * nr + r];
            Ds[rl * nr + r] = init ? make_float2(0.f, 0.f) : d[row * nr + r];
        }
        __syncthreads();
        if (ok) {
            float2 qa = make_float2(0.f, 0.f), pa = make_float2(0.f, 0.f), da = make_float2(0.f, 0.f);
            for (int c = 0; c < nr; ++c) {
                const float2 sv = Si[c * nr + r], hv = Sh[c * nr + r];
                const float2 qs = fcmul(Qs[rl * nr + c], sv), ps = fcmul(Ps[rl * nr + c], sv);
                const float2 dh = fcmul(Ds[rl * nr + c], hv);
                qa.x += qs.x;
                qa.y += qs.y;
                pa.x += ps.x;
                pa.y += ps.y;
                da.x += dh.x;
                da.y += dh.y;
            }
            const long long k = row * nr + r;
            q[k] = qa;
            qp[k] = pa;
            d[k] = make_float2(pa.x + da.x, pa.y + da.y);
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

void update_pxt(float2 *e, float2 *q, float2 *qp, const float2 *d, const float2 *z, const float2 *zp,
                const float2 *w, const float2 *n, long long rows, int nr, const int *active, hipStream_t st) {
    hipLaunchKernelGGL(update_pxt_kernel, dim3(update_grid(rows, nr)), dim3(256), 0, st, e, q, qp, d, z, zp, w, n,
                       rows, nr, active);
}

void update_pqd(float2 *q, float2 *qp, float2 *d, const float2 *sinv, const float2 *sh, long long rows, int nr,
                int init, const int *active, hipStream_t st) {
    hipLaunchKernelGGL(update_pqd_kernel, dim3(update_grid(rows, nr)), dim3(256), 0, st, q, qp, d, sinv, sh, rows,
                       nr, init, active);
}

void update_qd(float2 *q, float2 *d, const float2 *sinv, const float2 *sh, long long rows, int nr, int init,
               const int *active, hipStream_t st) {
    hipLaunchKernelGGL(update_qd_kernel, dim3(update_grid(rows, nr)), dim3(256), 0, st, q, d, sinv, sh, rows, nr,
                       init, active);
}

}  // namespace coarse
