// Multi-RHS deflation (Sec. 2.3, in the multi-RHS BLAS form of Sec. 2.5):
// for n_ev vectors |i> (the columns of V) with values lambda_i and a block X
// of right-hand sides,
//
//   c = V^H X  (n_ev x nrhs),   Defl(X) = V diag(1/lambda) c,   X_perp = X - V c,
//
// and the two-part stationary coarse solve Q X = Defl(X) + P(M) X_perp with P
// the Chebyshev approximation to 1/x (chebyshev.hip).
//
// Layout: V is [rows][n_ev] complex64 (row r = site * nbasis + basis index, as
// the vectors; one row holds the n_ev vectors' entries side by side), X and
// the outputs are [rows][nrhs] complex64, lambda is n_ev doubles on the device.
//
// Both products stream V from HBM once each and run on 16x16x4 f32 MFMA (a
// complex product as four real ones). The coefficient product is split over
// row ranges (split-K); the partial tiles are summed in double in a fixed
// order, so results are reproducible.
#include <cmath>
#include <cstdint>

#include "apply.hpp"

namespace coarse {

namespace {

constexpr int DEFL_SPLIT_MAX = 256;  // row ranges of the coefficient product
constexpr int DEFL_NEV_MAX = 4096;

__host__ __device__ inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

struct DeflLayout {
    int split, nev_pad, nr_pad;
    size_t partials, coef, coef_s, total;
};

DeflLayout defl_layout(long long rows, int nev, int nr) {
    DeflLayout l;
    l.nev_pad = round_up(nev > 0 ? nev : 1, 64);
    l.nr_pad = round_up(nr, 16);
    // enough workgroups to cover the chip several times, at least 64 rows each
    const long long tiles = (long long)(l.nev_pad / 64) * (l.nr_pad / 16);
    long long s = (2048 + tiles - 1) / tiles;
    const long long smax = (rows + 63) / 64;
    if (s > smax) s = smax;
    if (s > DEFL_SPLIT_MAX) s = DEFL_SPLIT_MAX;
    if (s < 1) s = 1;
    l.split = (int)s;
    l.partials = 0;
    l.coef = align256((size_t)l.split * l.nev_pad * l.nr_pad * 8);
    l.coef_s = l.coef + align256((size_t)l.nev_pad * l.nr_pad * 8);
    l.total = l.coef_s + align256((size_t)l.nev_pad * l.nr_pad * 8);
    return l;
}

}  // namespace

// partial[s][i][j] = sum over the rows of range s of conj(V[r][i]) X[r][j].
// Workgroup: four waves, wave w the 16 vectors 64 bx + 16 w, rhs 16 bz .. +15,
// rows of range by. Lane (c, g): A[i = c][k = g] = conj V[r + g][i0 + c],
// B[k = g][j = c] = X[r + g][j0 + c]; four row-steps in flight.
__global__ __launch_bounds__(256) void defl_coef_kernel(const float2 *__restrict__ v, const float2 *__restrict__ x,
                                                        long long rows, int nev, int nr, int split, int nev_pad,
                                                        int nr_pad, float2 *__restrict__ partial) {
    const int w = threadIdx.x >> 6, t = threadIdx.x & 63, c = t & 15, g = t >> 4;
    const int i0 = blockIdx.x * 64 + 16 * w, j0 = blockIdx.z * 16;
    const long long per = ((rows + split - 1) / split + 3) / 4 * 4;
    const long long r0 = (long long)blockIdx.y * per;
    long long r1 = r0 + per;
    if (r1 > rows) r1 = rows;
    const bool iv = i0 + c < nev, jv = j0 + c < nr;
    f32x4 re = f32x4{0, 0, 0, 0}, im = f32x4{0, 0, 0, 0};
    constexpr int U = 4;
    for (long long r = r0; r < r1; r += 4 * U) {
        float2 a[U], b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long row = r + 4 * u + g;
            const bool ok = row < r1;
            a[u] = (ok && iv) ? v[row * nev + i0 + c] : make_float2(0.f, 0.f);
            b[u] = (ok && jv) ? x[row * nr + j0 + c] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // (vr - i vi)(br + i bi): re = vr br + vi bi, im = vr bi - vi br
            re = mfma16x16x4(a[u].x, b[u].x, re);
            re = mfma16x16x4(a[u].y, b[u].y, re);
            im = mfma16x16x4(a[u].x, b[u].y, im);
            im = mfma16x16x4(-a[u].y, b[u].x, im);
        }
    }
    float2 *out = partial + ((size_t)blockIdx.y * nev_pad + i0) * nr_pad + j0 + c;
#pragma unroll
    for (int k = 0; k < 4; ++k) out[(size_t)(4 * g + k) * nr_pad] = make_float2(re[k], im[k]);
}

// c[i][j] = sum_s partial[s][i][j] (double, fixed order); c_s = c / lambda_i.
__global__ __launch_bounds__(256) void defl_reduce_kernel(const float2 *__restrict__ partial, int split, int nev,
                                                          int nr, int nev_pad, int nr_pad,
                                                          const double *__restrict__ lam, float2 *__restrict__ coef,
                                                          float2 *__restrict__ coef_s) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nev_pad * nr_pad) return;
    const int i = e / nr_pad, j = e - i * nr_pad;
    if (i >= nev || j >= nr) {
        coef[e] = make_float2(0.f, 0.f);
        coef_s[e] = make_float2(0.f, 0.f);
        return;
    }
    double sr = 0, si = 0;
    for (int s = 0; s < split; ++s) {
        const float2 p = partial[(size_t)s * nev_pad * nr_pad + e];
        sr += p.x;
        si += p.y;
    }
    const double li = 1.0 / lam[i];
    coef[e] = make_float2((float)sr, (float)si);
    coef_s[e] = make_float2((float)(sr * li), (float)(si * li));
}

// out[r][j] = base[r][j] + sign * sum_i V[r][i] coef[i][j] (base may be out or
// null). Wave: 16 rows x 16 rhs. The contraction index is assigned so that
// lane (c, g) reads four consecutive vectors 4g .. 4g+3 of row r0 + c (two
// 16-byte loads; a row's 16 entries per chunk come from one wave
// instruction pair), with the matching coefficient rows for the B operand;
// D[i = 4g + k][j = c] is row r0 + 4g + k, rhs j0 + c.
__global__ __launch_bounds__(256) void defl_promote_kernel(const float2 *__restrict__ v,
                                                           const float2 *__restrict__ coef, const float2 *base,
                                                           float2 *out, long long rows, int nev, int nr, int nr_pad,
                                                           float sign, int vec4) {
    const int w = threadIdx.x >> 6, t = threadIdx.x & 63, c = t & 15, g = t >> 4;
    const long long r0 = ((long long)blockIdx.x * 4 + w) * 16;
    if (r0 >= rows) return;  // wave-uniform; no barrier in this kernel
    const int j0 = blockIdx.y * 16;
    const long long ra = r0 + c;
    const bool rv = ra < rows;
    f32x4 re = f32x4{0, 0, 0, 0}, im = f32x4{0, 0, 0, 0};
    const float2 *vrow = v + (rv ? ra : 0) * nev;
    for (int k0 = 0; k0 < nev; k0 += 16) {
        const int kb = k0 + 4 * g;
        float2 a[4];
        if (vec4 && kb + 3 < nev) {
            const float4 p0 = *reinterpret_cast<const float4 *>(vrow + kb);
            const float4 p1 = *reinterpret_cast<const float4 *>(vrow + kb + 2);
            a[0] = make_float2(p0.x, p0.y);
            a[1] = make_float2(p0.z, p0.w);
            a[2] = make_float2(p1.x, p1.y);
            a[3] = make_float2(p1.z, p1.w);
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] = (kb + u < nev) ? vrow[kb + u] : make_float2(0.f, 0.f);
        }
        if (!rv) {
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] = make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            // coefficient rows past n_ev are zero in the workspace (nev_pad rows)
            const float2 b = coef[(size_t)(kb + u) * nr_pad + j0 + c];
            // (vr + i vi)(cr + i ci): re = vr cr - vi ci, im = vr ci + vi cr
            re = mfma16x16x4(a[u].x, b.x, re);
            re = mfma16x16x4(-a[u].y, b.y, re);
            im = mfma16x16x4(a[u].x, b.y, im);
            im = mfma16x16x4(a[u].y, b.x, im);
        }
    }
    if (j0 + c >= nr) return;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const long long row = r0 + 4 * g + k;
        if (row < rows) {
            const size_t e = (size_t)row * nr + j0 + c;
            float2 o = make_float2(sign * re[k], sign * im[k]);
            if (base) {
                const float2 bv = base[e];
                o.x += bv.x;
                o.y += bv.y;
            }
            out[e] = o;
        }
    }
}

namespace {

int32_t check_defl(const Geom &d, const void *v, int32_t nev, const double *lam, int nr) {
    (void)d;
    (void)nr;
    if (nev < 1 || nev > DEFL_NEV_MAX) {
        set_error("nev = %d out of range [1, %d]", nev, DEFL_NEV_MAX);
        return CG_INVALID_ARG;
    }
    if (!v || !lam) {
        set_error("v or lambda is NULL");
        return CG_INVALID_ARG;
    }
    return CG_OK;
}

// c, c_s of x into the workspace (the coefficient rows past n_ev zeroed).
void defl_coefficients(const Geom &d, const float2 *v, int nev, const double *lam, const float2 *x, int nr,
                       char *ws, const DeflLayout &l, hipStream_t st) {
    const long long rows = (long long)d.V * d.nb;
    float2 *partial = reinterpret_cast<float2 *>(ws + l.partials);
    float2 *coef = reinterpret_cast<float2 *>(ws + l.coef), *coef_s = reinterpret_cast<float2 *>(ws + l.coef_s);
    hipLaunchKernelGGL(defl_coef_kernel, dim3(l.nev_pad / 64, l.split, l.nr_pad / 16), dim3(256), 0, st, v, x, rows,
                       nev, nr, l.split, l.nev_pad, l.nr_pad, partial);
    const int ne = l.nev_pad * l.nr_pad;
    hipLaunchKernelGGL(defl_reduce_kernel, dim3((ne + 255) / 256), dim3(256), 0, st, partial, l.split, nev, nr,
                       l.nev_pad, l.nr_pad, lam, coef, coef_s);
}

void defl_promote(const Geom &d, const float2 *v, int nev, const float2 *coef, const float2 *base, float2 *out,
                  int nr, const DeflLayout &l, float sign, hipStream_t st) {
    const long long rows = (long long)d.V * d.nb;
    const long long waves = (rows + 15) / 16;
    // 16-byte loads of V need every row to start 16-byte aligned
    const int vec4 = (nev % 2 == 0 && (reinterpret_cast<uintptr_t>(v) & 15) == 0) ? 1 : 0;
    hipLaunchKernelGGL(defl_promote_kernel, dim3((unsigned)((waves + 3) / 4), l.nr_pad / 16), dim3(256), 0, st, v,
                       coef, base, out, rows, nev, nr, l.nr_pad, sign, vec4);
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    const char *pa = reinterpret_cast<const char *>(a), *pb = reinterpret_cast<const char *>(b);
    return pa < pb + nb && pb < pa + na;
}

}  // namespace

}  // namespace coarse

using namespace coarse;

extern "C" int32_t coarse_deflation_workspace_bytes(const coarse_geom *g, int32_t nev, int32_t nrhs, size_t *out) {
    clear_error();
    Geom d;
    int32_t rc = make_geom(g, &d);
    if (rc) return rc;
    if ((rc = check_nrhs(nrhs))) return rc;
    if (nev < 1 || nev > DEFL_NEV_MAX) {
        set_error("nev = %d out of range [1, %d]", nev, DEFL_NEV_MAX);
        return CG_INVALID_ARG;
    }
    if (!out) {
        set_error("out is NULL");
        return CG_INVALID_ARG;
    }
    *out = defl_layout((long long)d.V * d.nb, nev, nrhs).total;
    return CG_OK;
}

extern "C" int32_t coarse_deflate(const coarse_geom *g, const void *v, int32_t nev, const double *lam, const void *x,
                                  void *y, void *x_perp, int32_t nrhs, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    Geom d;
    int32_t rc = make_geom(g, &d);
    if (rc) return rc;
    if ((rc = check_nrhs(nrhs))) return rc;
    if ((rc = check_defl(d, v, nev, lam, nrhs))) return rc;
    if (!x || !y) {
        set_error("x or y is NULL");
        return CG_INVALID_ARG;
    }
    const long long rows = (long long)d.V * d.nb;
    const DeflLayout l = defl_layout(rows, nev, nrhs);
    if (!ws || ws_bytes < l.total) {
        set_error("workspace %zu bytes, need %zu", ws ? ws_bytes : (size_t)0, l.total);
        return CG_WORKSPACE_TOO_SMALL;
    }
    const size_t vb = (size_t)rows * nrhs * 8, bb = (size_t)rows * nev * 8;
    if (overlaps(x, vb, y, vb) || overlaps(y, vb, v, bb) || overlaps(ws, l.total, x, vb) ||
        overlaps(ws, l.total, y, vb) || overlaps(ws, l.total, v, bb) ||
        (x_perp && (overlaps(x_perp, vb, y, vb) || overlaps(x_perp, vb, v, bb) ||
                    overlaps(x_perp, vb, ws, l.total)))) {
        set_error("outputs, inputs and workspace must not overlap (x_perp may equal x)");
        return CG_INVALID_ARG;
    }
    if (x_perp && x_perp != x && overlaps(x_perp, vb, x, vb)) {
        set_error("x_perp must be x itself or not overlap it");
        return CG_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    char *w = reinterpret_cast<char *>(ws);
    const float2 *vv = reinterpret_cast<const float2 *>(v), *xx = reinterpret_cast<const float2 *>(x);
    defl_coefficients(d, vv, nev, lam, xx, nrhs, w, l, st);
    defl_promote(d, vv, nev, reinterpret_cast<const float2 *>(w + l.coef_s), nullptr,
                 reinterpret_cast<float2 *>(y), nrhs, l, 1.f, st);
    if (x_perp)
        defl_promote(d, vv, nev, reinterpret_cast<const float2 *>(w + l.coef), xx,
                     reinterpret_cast<float2 *>(x_perp), nrhs, l, -1.f, st);
    COARSE_HIP(hipGetLastError());
    return CG_OK;
}

extern "C" int32_t coarse_deflated_chebyshev_workspace_bytes(const coarse_geom *g, int32_t link_dtype, int32_t nev,
                                                             int32_t nrhs, size_t *out) {
    clear_error();
    Geom d;
    int32_t rc = make_geom(g, &d);
    if (rc) return rc;
    if ((rc = check_nrhs(nrhs))) return rc;
    if (nev < 1 || nev > DEFL_NEV_MAX) {
        set_error("nev = %d out of range [1, %d]", nev, DEFL_NEV_MAX);
        return CG_INVALID_ARG;
    }
    if (!out) {
        set_error("out is NULL");
        return CG_INVALID_ARG;
    }
    const long long rows = (long long)d.V * d.nb;
    const bool lowp = link_dtype == COARSE_BF16 || link_dtype == COARSE_FP16;
    const size_t vb = align256((size_t)rows * nrhs * 8);
    *out = defl_layout(rows, nev, nrhs).total + 4 * vb + ((lowp && d.nb % 16 == 0) ? align256(lowp_ws_bytes(d, nrhs)) : 0);
    return CG_OK;
}

extern "C" int32_t coarse_deflated_chebyshev_apply(const coarse_geom *g, const void *packed, int32_t link_dtype,
                                                   const void *v, int32_t nev, const double *lam, const void *x,
                                                   void *y, int32_t nrhs, double lo, double hi, int32_t order,
                                                   void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    Geom d;
    int32_t rc = make_geom(g, &d);
    if (rc) return rc;
    if ((rc = check_nrhs(nrhs))) return rc;
    if ((rc = check_defl(d, v, nev, lam, nrhs))) return rc;
    if ((rc = check_chebyshev(lo, hi, order))) return rc;
    if (!packed || !x || !y) {
        set_error("packed, x or y is NULL");
        return CG_INVALID_ARG;
    }
    if (link_dtype != COARSE_C64 && link_dtype != COARSE_C64_3M && link_dtype != COARSE_BF16 &&
        link_dtype != COARSE_FP16) {
        set_error("link_dtype %d not one of C64, C64_3M, BF16, FP16", link_dtype);
        return CG_INVALID_ARG;
    }
    if (link_dtype != COARSE_C64 && d.nb % 16) {
        set_error("16-bit and 3M links need nbasis %% 16 == 0 (got %d)", d.nb);
        return CG_UNSUPPORTED;
    }
    size_t need = 0;
    if ((rc = coarse_deflated_chebyshev_workspace_bytes(g, link_dtype, nev, nrhs, &need))) return rc;
    if (!ws || ws_bytes < need) {
        set_error("workspace %zu bytes, need %zu", ws ? ws_bytes : (size_t)0, need);
        return CG_WORKSPACE_TOO_SMALL;
    }
    const long long rows = (long long)d.V * d.nb;
    const size_t vb = (size_t)rows * nrhs * 8, bb = (size_t)rows * nev * 8;
    if (overlaps(x, vb, y, vb) || overlaps(y, vb, v, bb) || overlaps(ws, need, x, vb) || overlaps(ws, need, y, vb) ||
        overlaps(ws, need, v, bb) || packed == x || packed == y || packed == ws) {
        set_error("inputs, output and workspace must not overlap");
        return CG_INVALID_ARG;
    }
    const DeflLayout l = defl_layout(rows, nev, nrhs);
    char *w = reinterpret_cast<char *>(ws);
    const size_t va = align256(vb);
    char *xp = w + l.total;
    const ChebBuffers cb{xp + va, xp + 2 * va, xp + 3 * va, xp + 4 * va};
    hipStream_t st = (hipStream_t)stream;
    const float2 *vv = reinterpret_cast<const float2 *>(v);
    // c = V^H x; x_perp = x - V c; y = P(M) x_perp; y += V diag(1/lambda) c
    defl_coefficients(d, vv, nev, lam, reinterpret_cast<const float2 *>(x), nrhs, w, l, st);
    defl_promote(d, vv, nev, reinterpret_cast<const float2 *>(w + l.coef), reinterpret_cast<const float2 *>(x),
                 reinterpret_cast<float2 *>(xp), nrhs, l, -1.f, st);
    COARSE_HIP(hipGetLastError());
    if ((rc = chebyshev_poly(d, packed, link_dtype, xp, y, nrhs, lo, hi, order, cb, nullptr, st))) return rc;
    defl_promote(d, vv, nev, reinterpret_cast<const float2 *>(w + l.coef_s), reinterpret_cast<const float2 *>(y),
                 reinterpret_cast<float2 *>(y), nrhs, l, 1.f, st);
    COARSE_HIP(hipGetLastError());
    return CG_OK;
}
