// Tall-skinny and per-site batched complex products: multi-RHS deflation and
// the block project / promote between grids.
//
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
//
// Block project / promote (Sec. 2.5): per coarse site x_c with basis block
// B(x_c) (V_block x N_basis), C(x_c) = B(x_c)^H F(x_c) and F(x_c) = B(x_c) C(x_c)
// - the same two products with one row range per coarse site and the
// coefficient block of each site (basis [V][V_block][N_basis], fine vectors
// [V][V_block][N_rhs] grouped by coarse block, coarse vectors
// [V][N_basis][N_rhs]; all complex64).
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <vector>

#include "apply.hpp"
#include "blas.hpp"

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
// Workgroup: the 64 vectors 64 bx .. +63, rhs 16 bz .. +15, rows of range by;
// its four waves take interleaved 4-row steps and their sums meet in LDS. Four
// MFMA tiles per wave share the X operand: lane (c, g) reads vectors
// 4c .. 4c+3 of row r + g (two 16-byte loads; the 16 lanes of a k-group read
// the row's 512 contiguous bytes) and feeds vector 4c + t to tile t, so tile
// t's row i = c is vector 4c + t and its output row 4g + k is vector
// 4 (4g + k) + t. B[k = g][j = c] = X[r + g][j0 + c].
// DIRECT (block project): range by is coarse site by, and the sums go
// straight to out[by][i][j] (n_ev x nr, unpadded) instead of a padded partial.
template <bool DIRECT>
__global__ __launch_bounds__(256) void defl_coef_kernel(const float2 *__restrict__ v, const float2 *__restrict__ x,
                                                        long long rows, long long per, int nev, int nr, int nev_pad,
                                                        int nr_pad, int vec4, float2 *__restrict__ partial,
                                                        long long ldv) {
    __shared__ float red[4][2][4][4][64];  // wave, re/im, tile, k, lane
    const int w = threadIdx.x >> 6, t = threadIdx.x & 63, c = t & 15, g = t >> 4;
    const int i0 = blockIdx.x * 64, j0 = blockIdx.z * 16;
    const long long r0 = (long long)blockIdx.y * per;
    long long r1 = r0 + per;
    if (r1 > rows) r1 = rows;
    const int ib = i0 + 4 * c;  // this lane's four vectors
    const bool jv = j0 + c < nr;
    f32x4 re[4], im[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        re[q] = f32x4{0, 0, 0, 0};
        im[q] = f32x4{0, 0, 0, 0};
    }
    constexpr int U = 2;
    for (long long r = r0 + 4 * w; r < r1; r += 16 * U) {
        float2 a[U][4], b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long row = r + 16 * u + g;
            const bool ok = row < r1;
            const float2 *vr = v + (ok ? row : 0) * ldv;
            if (ok && vec4 && ib + 3 < nev) {
                const float4 p0 = *reinterpret_cast<const float4 *>(vr + ib);
                const float4 p1 = *reinterpret_cast<const float4 *>(vr + ib + 2);
                a[u][0] = make_float2(p0.x, p0.y);
                a[u][1] = make_float2(p0.z, p0.w);
                a[u][2] = make_float2(p1.x, p1.y);
                a[u][3] = make_float2(p1.z, p1.w);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) a[u][q] = (ok && ib + q < nev) ? vr[ib + q] : make_float2(0.f, 0.f);
            }
            b[u] = (ok && jv) ? x[row * nr + j0 + c] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // (vr - i vi)(br + i bi): re = vr br + vi bi, im = vr bi - vi br
                re[q] = mfma16x16x4(a[u][q].x, b[u].x, re[q]);
                re[q] = mfma16x16x4(a[u][q].y, b[u].y, re[q]);
                im[q] = mfma16x16x4(a[u][q].x, b[u].y, im[q]);
                im[q] = mfma16x16x4(-a[u][q].y, b[u].x, im[q]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            red[w][0][q][k][t] = re[q][k];
            red[w][1][q][k][t] = im[q][k];
        }
    __syncthreads();
    // 1024 outputs (64 vectors x 16 rhs, re and im interleaved per entry): thread
    // e takes entries e, e + 256, e + 512, e + 768; waves summed in fixed order
    for (int e = threadIdx.x; e < 1024; e += 256) {
        const int q = e >> 8, k = (e >> 6) & 3, l = e & 63;
        const float sr = (red[0][0][q][k][l] + red[1][0][q][k][l]) + (red[2][0][q][k][l] + red[3][0][q][k][l]);
        const float si = (red[0][1][q][k][l] + red[1][1][q][k][l]) + (red[2][1][q][k][l] + red[3][1][q][k][l]);
        const int lc = l & 15, lg = l >> 4;
        const int i = i0 + 4 * (4 * lg + k) + q;  // vector of tile q, output row 4 lg + k
        if (DIRECT) {
            if (i < nev && j0 + lc < nr) partial[((size_t)blockIdx.y * nev + i) * nr + j0 + lc] = make_float2(sr, si);
        } else {
            partial[((size_t)blockIdx.y * nev_pad + i) * nr_pad + j0 + lc] = make_float2(sr, si);
        }
    }
}

// c[i][j] = sum_s partial[s][i][j] (double; lane l of an entry sums ranges
// l, l + 16, ... in order, then a fixed butterfly over the 16 lane sums, pairs
// 8, 4, 2, 1 apart); c_s = c / lambda_i. Workgroup: 16 consecutive entries,
// thread (el, l) = (tid % 16, tid / 16) holding lane l of entry el, so one
// load instruction reads four whole 128-byte lines (four ranges x 16 entries);
// the butterfly's first two levels go through LDS, the last two are shuffles
// in wave 0.
__global__ __launch_bounds__(256) void defl_reduce_kernel(const float2 *__restrict__ partial, int split, int nev,
                                                          int nr, int nev_pad, int nr_pad,
                                                          const double *__restrict__ lam, float2 *__restrict__ coef,
                                                          float2 *__restrict__ coef_s) {
    __shared__ double2 ls[256];
    const int el = threadIdx.x & 15, l = threadIdx.x >> 4;
    const int e = blockIdx.x * 16 + el;
    const int ne = nev_pad * nr_pad;
    const bool live = e < ne;
    const int i = live ? e / nr_pad : 0, j = live ? e - i * nr_pad : 0;
    double sr = 0, si = 0;
    if (live && i < nev && j < nr) {
        for (int s = l; s < split; s += 16) {
            const float2 p = partial[(size_t)s * ne + e];
            sr += p.x;
            si += p.y;
        }
    }
    ls[l * 16 + el] = make_double2(sr, si);
    __syncthreads();
    if (threadIdx.x >= 64) return;  // wave 0: lane = el + 16 l, l < 4
    {
        auto at = [&](int q) { return ls[q * 16 + el]; };
        // levels 8 and 4 of the butterfly for lane sums l < 4
        const double2 a0 = at(l), a1 = at(l + 8), a2 = at(l + 4), a3 = at(l + 12);
        sr = (a0.x + a1.x) + (a2.x + a3.x);
        si = (a0.y + a1.y) + (a2.y + a3.y);
    }
    // levels 2 and 1: l xor 2, 1 is lane xor 32, 16
#pragma unroll
    for (int m = 32; m >= 16; m >>= 1) {
        sr += __shfl_xor(sr, m);
        si += __shfl_xor(si, m);
    }
    if (!live || l != 0) return;
    if (i >= nev || j >= nr) {
        coef[e] = make_float2(0.f, 0.f);
        coef_s[e] = make_float2(0.f, 0.f);
        return;
    }
    // a vector whose value is not positive and finite (a zero Ritz pair past an
    // exhausted Krylov space, say) is left out of both outputs
    const double lv = lam ? lam[i] : 1.0;
    const bool use = lv > 0.0 && lv <= 1.7976931348623157e308;
    const double li = use ? 1.0 / lv : 0.0;
    coef[e] = use ? make_float2((float)sr, (float)si) : make_float2(0.f, 0.f);
    coef_s[e] = make_float2((float)(sr * li), (float)(si * li));
}

// out1[r][j] = base1[r][j] + sign1 * sum_i V[r][i] coef1[i][j] and, with TWO,
// out2[r][j] = base2[r][j] + sum_i V[r][i] coef2[i][j] from the same reads of V
// (a base may be its output or null). Wave: RT tiles of 16 rows x 16 rhs
// sharing every coefficient load. The contraction index is assigned so that
// lane (c, g) reads four consecutive vectors 4g .. 4g+3 of row c of a tile
// (two 16-byte loads; a row's 16 entries per chunk come from one wave
// instruction pair), with the matching coefficient rows for the B operand;
// D[i = 4g + k][j = c] is the tile's row 4g + k, rhs j0 + c. The next chunk's
// V loads are issued before this chunk's products. Complex products in the 3M
// form (three real MFMA products each).
// vblock > 0 (block promote): the coefficients differ per coarse site, rows
// r .. r + vblock - 1 belonging to site r / vblock with its n_ev x nr block at
// coef + site * n_ev * nr_ld (vblock a multiple of 16 RT, so a wave's rows
// share one site).
template <bool TWO, int RT>
__global__ __launch_bounds__(256) void defl_promote_kernel(const float2 *__restrict__ v,
                                                           const float2 *__restrict__ coef1,
                                                           const float2 *__restrict__ coef2, const float2 *base1,
                                                           float2 *out1, const float2 *base2, float2 *out2,
                                                           long long rows, int nev, int nr, int nr_ld, float sign1,
                                                           int vec4, int vblock, long long ldv) {
    const int w = threadIdx.x >> 6, t = threadIdx.x & 63, c = t & 15, g = t >> 4;
    const long long r0 = ((long long)blockIdx.x * 4 + w) * 16 * RT;
    if (r0 >= rows) return;  // wave-uniform; no barrier in this kernel
    const int j0 = blockIdx.y * 16;
    if (vblock > 0) {
        const size_t off = (size_t)(r0 / vblock) * nev * nr_ld;
        coef1 += off;
        coef2 += off;
    }
    const bool jv = j0 + c < nr;
    // 3M: t1 = sum vr cr, t2 = sum vi ci, t3 = sum (vr + vi)(cr + ci);
    // re = t1 - t2, im = t3 - t1 - t2 (three real products per complex one)
    f32x4 t1a[RT], t2a[RT], t3a[RT], t1b[RT], t2b[RT], t3b[RT];
    const float2 *vrow[RT];
    bool rv[RT];
#pragma unroll
    for (int q = 0; q < RT; ++q) {
        t1a[q] = f32x4{0, 0, 0, 0};
        t2a[q] = f32x4{0, 0, 0, 0};
        t3a[q] = f32x4{0, 0, 0, 0};
        t1b[q] = f32x4{0, 0, 0, 0};
        t2b[q] = f32x4{0, 0, 0, 0};
        t3b[q] = f32x4{0, 0, 0, 0};
        const long long ra = r0 + 16 * q + c;
        rv[q] = ra < rows;
        vrow[q] = v + (rv[q] ? ra : 0) * ldv;
    }
    auto load = [&](int k0, float2 (&a)[RT][4]) {
        const int kb = k0 + 4 * g;
#pragma unroll
        for (int q = 0; q < RT; ++q) {
            if (rv[q] && vec4 && kb + 3 < nev) {
                const float4 p0 = *reinterpret_cast<const float4 *>(vrow[q] + kb);
                const float4 p1 = *reinterpret_cast<const float4 *>(vrow[q] + kb + 2);
                a[q][0] = make_float2(p0.x, p0.y);
                a[q][1] = make_float2(p0.z, p0.w);
                a[q][2] = make_float2(p1.x, p1.y);
                a[q][3] = make_float2(p1.z, p1.w);
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    a[q][u] = (rv[q] && kb + u < nev) ? vrow[q][kb + u] : make_float2(0.f, 0.f);
            }
        }
    };
    float2 an[RT][4];
    load(0, an);
    for (int k0 = 0; k0 < nev; k0 += 16) {
        float2 a[RT][4];
#pragma unroll
        for (int q = 0; q < RT; ++q)
#pragma unroll
            for (int u = 0; u < 4; ++u) a[q][u] = an[q][u];
        if (k0 + 16 < nev) load(k0 + 16, an);
        const int kb = k0 + 4 * g;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool cv = jv && kb + u < nev;
            const size_t ci = (size_t)(kb + u) * nr_ld + j0 + c;
            const float2 b = cv ? coef1[ci] : make_float2(0.f, 0.f);
            const float2 b2 = (TWO && cv) ? coef2[ci] : make_float2(0.f, 0.f);
            const float bs = b.x + b.y, bs2 = b2.x + b2.y;
#pragma unroll
            for (int q = 0; q < RT; ++q) {
                const float as = a[q][u].x + a[q][u].y;
                t1a[q] = mfma16x16x4(a[q][u].x, b.x, t1a[q]);
                t2a[q] = mfma16x16x4(a[q][u].y, b.y, t2a[q]);
                t3a[q] = mfma16x16x4(as, bs, t3a[q]);
                if (TWO) {
                    t1b[q] = mfma16x16x4(a[q][u].x, b2.x, t1b[q]);
                    t2b[q] = mfma16x16x4(a[q][u].y, b2.y, t2b[q]);
                    t3b[q] = mfma16x16x4(as, bs2, t3b[q]);
                }
            }
        }
    }
    if (!jv) return;
#pragma unroll
    for (int q = 0; q < RT; ++q)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const long long row = r0 + 16 * q + 4 * g + k;
            if (row < rows) {
                const size_t e = (size_t)row * nr + j0 + c;
                const float r1 = t1a[q][k] - t2a[q][k], i1 = t3a[q][k] - t1a[q][k] - t2a[q][k];
                float2 o = make_float2(sign1 * r1, sign1 * i1);
                if (base1) {
                    const float2 bv = base1[e];
                    o.x += bv.x;
                    o.y += bv.y;
                }
                out1[e] = o;
                if (TWO) {
                    float2 o2 = make_float2(t1b[q][k] - t2b[q][k], t3b[q][k] - t1b[q][k] - t2b[q][k]);
                    if (base2) {
                        const float2 bv = base2[e];
                        o2.x += bv.x;
                        o2.y += bv.y;
                    }
                    out2[e] = o2;
                }
            }
        }
}

// y += a (complex64 entries).
__global__ __launch_bounds__(256) void defl_add_kernel(const float2 *__restrict__ a, float2 *__restrict__ y,
                                                       long long n) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float2 av = a[i], yv = y[i];
        y[i] = make_float2(yv.x + av.x, yv.y + av.y);
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
    const int vec4 = (nev % 2 == 0 && (reinterpret_cast<uintptr_t>(v) & 15) == 0) ? 1 : 0;
    const long long per = ((rows + l.split - 1) / l.split + 15) / 16 * 16;
    hipLaunchKernelGGL(defl_coef_kernel<false>, dim3(l.nev_pad / 64, l.split, l.nr_pad / 16), dim3(256), 0, st, v, x,
                       rows, per, nev, nr, l.nev_pad, l.nr_pad, vec4, partial, (long long)nev);
    const int ne = l.nev_pad * l.nr_pad;
    hipLaunchKernelGGL(defl_reduce_kernel, dim3((ne + 15) / 16), dim3(256), 0, st, partial, l.split, nev, nr,
                       l.nev_pad, l.nr_pad, lam, coef, coef_s);
}

// out1 = base1 + sign1 V coef1 and, if out2 is not null, out2 = base2 + V coef2
// in the same pass over V.
void defl_promote(const Geom &d, const float2 *v, int nev, const float2 *coef1, const float2 *base1, float2 *out1,
                  float sign1, const float2 *coef2, const float2 *base2, float2 *out2, int nr, const DeflLayout &l,
                  hipStream_t st) {
    const long long rows = (long long)d.V * d.nb;
    // 16-byte loads of V need every row to start 16-byte aligned
    const int vec4 = (nev % 2 == 0 && (reinterpret_cast<uintptr_t>(v) & 15) == 0) ? 1 : 0;
    // two 16-row tiles per wave halve the coefficient loads per byte of V
    const long long waves2 = (rows + 31) / 32;
    const dim3 grid((unsigned)((waves2 + 3) / 4), l.nr_pad / 16);
    if (out2)
        hipLaunchKernelGGL((defl_promote_kernel<true, 2>), grid, dim3(256), 0, st, v, coef1, coef2, base1, out1, base2,
                           out2, rows, nev, nr, l.nr_pad, sign1, vec4, 0, (long long)nev);
    else
        hipLaunchKernelGGL((defl_promote_kernel<false, 2>), grid, dim3(256), 0, st, v, coef1, coef1, base1, out1,
                           (const float2 *)nullptr, (float2 *)nullptr, rows, nev, nr, l.nr_pad, sign1, vec4, 0,
                           (long long)nev);
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
    const float2 *cf = reinterpret_cast<const float2 *>(w + l.coef), *cs = reinterpret_cast<const float2 *>(w + l.coef_s);
    if (x_perp)  // y = V c_s and x_perp = x - V c from one pass over V
        defl_promote(d, vv, nev, cf, xx, reinterpret_cast<float2 *>(x_perp), -1.f, cs, nullptr,
                     reinterpret_cast<float2 *>(y), nrhs, l, st);
    else
        defl_promote(d, vv, nev, cs, nullptr, reinterpret_cast<float2 *>(y), 1.f, nullptr, nullptr, nullptr, nrhs, l,
                     st);
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
    *out = defl_layout(rows, nev, nrhs).total + 5 * vb + ((lowp && d.nb % 16 == 0) ? align256(lowp_ws_bytes(d, nrhs)) : 0);
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
    char *xp = w + l.total, *yd = xp + va;
    const ChebBuffers cb{yd + va, yd + 2 * va, yd + 3 * va, yd + 4 * va};
    hipStream_t st = (hipStream_t)stream;
    const float2 *vv = reinterpret_cast<const float2 *>(v);
    // c = V^H x; x_perp = x - V c and y_d = V diag(1/lambda) c in one pass over V;
    // y = P(M) x_perp; y += y_d
    defl_coefficients(d, vv, nev, lam, reinterpret_cast<const float2 *>(x), nrhs, w, l, st);
    defl_promote(d, vv, nev, reinterpret_cast<const float2 *>(w + l.coef), reinterpret_cast<const float2 *>(x),
                 reinterpret_cast<float2 *>(xp), -1.f, reinterpret_cast<const float2 *>(w + l.coef_s), nullptr,
                 reinterpret_cast<float2 *>(yd), nrhs, l, st);
    COARSE_HIP(hipGetLastError());
    if ((rc = chebyshev_poly(d, packed, link_dtype, xp, y, nrhs, lo, hi, order, cb, nullptr, st))) return rc;
    const long long n2 = rows * nrhs;
    hipLaunchKernelGGL(defl_add_kernel, dim3((unsigned)std::min<long long>((n2 + 255) / 256, 8192)), dim3(256), 0, st,
                       reinterpret_cast<const float2 *>(yd), reinterpret_cast<float2 *>(y), n2);
    COARSE_HIP(hipGetLastError());
    return CG_OK;
}

// ---- block project / promote between grids (Sec. 2.5) ---------------------

namespace {

int32_t check_transfer(const coarse_geom *g, Geom *d, int32_t vblock, int32_t nrhs, const void *basis,
                       const void *a, const void *b) {
    int32_t rc = make_geom(g, d);
    if (rc) return rc;
    if ((rc = check_nrhs(nrhs))) return rc;
    if (vblock < 16 || vblock % 16 || vblock > 65536) {
        set_error("vblock = %d must be a multiple of 16 in [16, 65536]", vblock);
        return CG_UNSUPPORTED;
    }
    if (d->V > 65535) {
        set_error("block transfer takes at most 65535 coarse sites (one grid row per site), got %d", d->V);
        return CG_UNSUPPORTED;
    }
    if ((long long)d->V * vblock * (d->nb > nrhs ? d->nb : nrhs) >= (1LL << 31)) {
        set_error("V * vblock * max(nbasis, nrhs) must stay below 2^31");
        return CG_INVALID_ARG;
    }
    if (!basis || !a || !b) {
        set_error("basis, input or output is NULL");
        return CG_INVALID_ARG;
    }
    if (a == b || a == basis || b == basis) {
        set_error("basis, input and output must not alias");
        return CG_INVALID_ARG;
    }
    return CG_OK;
}

}  // namespace

extern "C" int32_t coarse_block_project(const coarse_geom *g, int32_t vblock, const void *basis, const void *fine,
                                        void *coarse_out, int32_t nrhs, void *stream) {
    clear_error();
    Geom d;
    int32_t rc = check_transfer(g, &d, vblock, nrhs, basis, fine, coarse_out);
    if (rc) return rc;
    const long long rows = (long long)d.V * vblock;
    const int nb = d.nb;
    const int vec4 = (nb % 2 == 0 && (reinterpret_cast<uintptr_t>(basis) & 15) == 0) ? 1 : 0;
    hipLaunchKernelGGL(defl_coef_kernel<true>, dim3(round_up(nb, 64) / 64, d.V, round_up(nrhs, 16) / 16), dim3(256),
                       0, (hipStream_t)stream, reinterpret_cast<const float2 *>(basis),
                       reinterpret_cast<const float2 *>(fine), rows, (long long)vblock, nb, nrhs, round_up(nb, 64),
                       round_up(nrhs, 16), vec4, reinterpret_cast<float2 *>(coarse_out), (long long)nb);
    COARSE_HIP(hipGetLastError());
    return CG_OK;
}

extern "C" int32_t coarse_block_promote(const coarse_geom *g, int32_t vblock, const void *basis,
                                        const void *coarse_in, void *fine, int32_t nrhs, void *stream) {
    clear_error();
    Geom d;
    int32_t rc = check_transfer(g, &d, vblock, nrhs, basis, coarse_in, fine);
    if (rc) return rc;
    const long long rows = (long long)d.V * vblock;
    const int nb = d.nb;
    const int vec4 = (nb % 2 == 0 && (reinterpret_cast<uintptr_t>(basis) & 15) == 0) ? 1 : 0;
    const auto *bp = reinterpret_cast<const float2 *>(basis);
    const auto *cp = reinterpret_cast<const float2 *>(coarse_in);
    auto *fp = reinterpret_cast<float2 *>(fine);
    const unsigned gy = (unsigned)(round_up(nrhs, 16) / 16);
    if (vblock % 32 == 0) {  // two 16-row tiles of one site per wave
        const long long waves = rows / 32;
        hipLaunchKernelGGL((defl_promote_kernel<false, 2>), dim3((unsigned)((waves + 3) / 4), gy), dim3(256), 0,
                           (hipStream_t)stream, bp, cp, cp, (const float2 *)nullptr, fp, (const float2 *)nullptr,
                           (float2 *)nullptr, rows, nb, nrhs, nrhs, 1.f, vec4, vblock, (long long)nb);
    } else {
        const long long waves = rows / 16;
        hipLaunchKernelGGL((defl_promote_kernel<false, 1>), dim3((unsigned)((waves + 3) / 4), gy), dim3(256), 0,
                           (hipStream_t)stream, bp, cp, cp, (const float2 *)nullptr, fp, (const float2 *)nullptr,
                           (float2 *)nullptr, rows, nb, nrhs, nrhs, 1.f, vec4, vblock, (long long)nb);
    }
    COARSE_HIP(hipGetLastError());
    return CG_OK;
}

// ---- block Lanczos for the deflation vectors --------------------------------
//
// Block Lanczos with full reorthogonalisation on the coarse operator: the
// O(n) work (applies, reorthogonalisation against every earlier block with the
// products above, the Gram matrices of the thin QR steps, the Ritz vectors)
// runs on the device; the small dense steps (Cholesky factors of block x block
// Gram matrices, the Rayleigh-Ritz eigenproblem of the K x K projected matrix by
// Householder tridiagonalisation and QL) run on the host in double, between
// synchronisations.

// dst[r][col0 + j] = src[r][j] (j < b) for a row-major destination of ld columns.
__global__ __launch_bounds__(256) void lanczos_put_kernel(const float2 *__restrict__ src, float2 *__restrict__ dst,
                                                          long long rows, int b, long long ld, int col0) {
    const long long n = rows * b, stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        const long long r = e / b;
        dst[r * ld + col0 + (e - r * b)] = src[e];
    }
}

namespace {

constexpr int LANCZOS_MAX_K = 512;

typedef std::complex<double> cd;

// Upper-triangular R with R^H R = G (G Hermitian, n x n row-major); false when
// a pivot is not above rel * ref, ref being the trace of G unless a positive
// reference is given (rank-deficient block).
bool host_chol(const std::vector<cd> &G, int n, std::vector<cd> &R, double rel, double ref = 0.0) {
    std::vector<cd> A(G);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) A[i * n + j] = 0.5 * (G[i * n + j] + std::conj(G[j * n + i]));
    double tr = 0;
    for (int i = 0; i < n; ++i) tr += A[i * n + i].real();
    if (ref > 0.0) tr = ref;
    R.assign((size_t)n * n, cd(0, 0));
    for (int k = 0; k < n; ++k) {
        const double piv = A[k * n + k].real();
        if (!(piv > rel * tr) || !std::isfinite(piv)) return false;
        const double d = std::sqrt(piv);
        R[k * n + k] = d;
        for (int j = k + 1; j < n; ++j) R[k * n + j] = A[k * n + j] / d;
        for (int i = k + 1; i < n; ++i)
            for (int j = k + 1; j < n; ++j) A[i * n + j] -= std::conj(R[k * n + i]) * R[k * n + j];
    }
    return true;
}

// Inverse of an upper-triangular n x n matrix (back substitution per column).
std::vector<cd> host_tri_inv(const std::vector<cd> &R, int n) {
    std::vector<cd> X((size_t)n * n, cd(0, 0));
    for (int c = 0; c < n; ++c) {
        for (int i = n - 1; i >= 0; --i) {
            cd s = (i == c) ? cd(1, 0) : cd(0, 0);
            for (int k = i + 1; k < n; ++k) s -= R[i * n + k] * X[k * n + c];
            X[i * n + c] = s / R[i * n + i];
        }
    }
    return X;
}

// Hermitian eigendecomposition by Householder reduction to a real symmetric
// tridiagonal matrix and implicit QL iterations (host, double).
// Reduction: for column k a reflector H = I - 2 v v^H maps A[k+1:, k] to
// alpha e_1 (alpha of the column's first entry's phase, opposite sign), applied
// to the trailing block as B <- B - v u^H - u v^H with w = B v, K = v^H w,
// u = 2 (w - K v), and accumulated into Q. A diagonal unitary D then turns the
// complex subdiagonal e_i into |e_i| (phase_{i+1} = phase_i e_i / |e_i|). QL with
// Wilkinson-type shifts diagonalises the real tridiagonal T_r = Z diag(w) Z^T
// (the implicit QL method of Bowdler, Martin, Reinsch and Wilkinson, Numer. Math.
// 11 (1968), as published in the Handbook for Automatic Computation vol. II and
// EISPACK's imtql2, restated here for complex128 input after the phase step);
// the eigenvectors of A are Q D Z. Eigenvalues ascending into w, eigenvectors
// into the columns of Zc (n x n row-major).
void host_eigh(std::vector<cd> A, int n, std::vector<double> &w, std::vector<cd> &Zc) {
    std::vector<cd> Q((size_t)n * n, cd(0, 0));
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
    std::vector<cd> v(n), wv(n), u(n), qv(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1, o = k + 1;
        double xn = 0;
        for (int i = 0; i < m; ++i) xn += std::norm(A[(size_t)(o + i) * n + k]);
        xn = std::sqrt(xn);
        if (xn == 0) continue;
        const cd x0 = A[(size_t)o * n + k];
        const cd ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cd(1, 0);
        const cd alpha = -ph * xn;
        for (int i = 0; i < m; ++i) v[i] = A[(size_t)(o + i) * n + k];
        v[0] -= alpha;
        double vn = 0;
        for (int i = 0; i < m; ++i) vn += std::norm(v[i]);
        vn = std::sqrt(vn);
        if (vn == 0) continue;
        for (int i = 0; i < m; ++i) v[i] /= vn;
        // w = B v, K = v^H w
        cd K = 0;
        for (int i = 0; i < m; ++i) {
            cd sacc = 0;
            for (int j = 0; j < m; ++j) sacc += A[(size_t)(o + i) * n + o + j] * v[j];
            wv[i] = sacc;
            K += std::conj(v[i]) * sacc;
        }
        for (int i = 0; i < m; ++i) u[i] = 2.0 * (wv[i] - K.real() * v[i]);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j)
                A[(size_t)(o + i) * n + o + j] -= v[i] * std::conj(u[j]) + u[i] * std::conj(v[j]);
        A[(size_t)o * n + k] = alpha;
        A[(size_t)k * n + o] = std::conj(alpha);
        for (int i = 1; i < m; ++i) A[(size_t)(o + i) * n + k] = A[(size_t)k * n + o + i] = 0;
        // Q[:, o:] <- Q[:, o:] (I - 2 v v^H)
        for (int r = 0; r < n; ++r) {
            cd sacc = 0;
            for (int j = 0; j < m; ++j) sacc += Q[(size_t)r * n + o + j] * v[j];
            for (int j = 0; j < m; ++j) Q[(size_t)r * n + o + j] -= 2.0 * sacc * std::conj(v[j]);
        }
    }
    // real tridiagonal: d, e (e[i] couples i and i+1), phases
    std::vector<double> d(n), e(n, 0.0);
    std::vector<cd> phase(n, cd(1, 0));
    for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i].real();
    for (int i = 0; i + 1 < n; ++i) {
        const cd ei = A[(size_t)(i + 1) * n + i];
        const double ae = std::abs(ei);
        e[i] = ae;
        phase[i + 1] = ae > 0 ? phase[i] * ei / ae : phase[i];
    }
    std::vector<double> Z((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
    for (int l = 0; l < n; ++l) {
        for (int iter = 0; iter < 200; ++iter) {
            int m = l;
            for (; m + 1 < n; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= 1e-15 * dd) break;
            }
            if (m == l) break;
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
            double sn = 1, cs = 1, pp = 0;
            int i = m - 1;
            bool early = false;
            for (; i >= l; --i) {
                const double f = sn * e[i], b = cs * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0) {
                    d[i + 1] -= pp;
                    e[m] = 0;
                    early = true;
                    break;
                }
                sn = f / r;
                cs = g / r;
                g = d[i + 1] - pp;
                r = (d[i] - g) * sn + 2.0 * cs * b;
                pp = sn * r;
                d[i + 1] = g + pp;
                g = cs * r - b;
                for (int k = 0; k < n; ++k) {
                    const double zf = Z[(size_t)k * n + i + 1];
                    Z[(size_t)k * n + i + 1] = sn * Z[(size_t)k * n + i] + cs * zf;
                    Z[(size_t)k * n + i] = cs * Z[(size_t)k * n + i] - sn * zf;
                }
            }
            if (early) continue;
            d[l] -= pp;
            e[l] = g;
            e[m] = 0;
        }
    }
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] < d[y]; });
    w.resize(n);
    Zc.assign((size_t)n * n, cd(0, 0));
    // eigenvector j of A: Q D Z[:, idx[j]]
    for (int j = 0; j < n; ++j) {
        w[j] = d[idx[j]];
        for (int k = 0; k < n; ++k) qv[k] = phase[k] * Z[(size_t)k * n + idx[j]];
        for (int r = 0; r < n; ++r) {
            cd sacc = 0;
            for (int k = 0; k < n; ++k) sacc += Q[(size_t)r * n + k] * qv[k];
            Zc[(size_t)r * n + j] = sacc;
        }
    }
}

struct LanczosLayout {
    size_t Q, cur, W, tmp, defl, gp, G, sinv, Y, lowp, total;
    DeflLayout dl;
};

LanczosLayout lanczos_layout(const Geom &d, int32_t link_dtype, int b, int K, int nev) {
    const long long rows = (long long)d.V * d.nb;
    LanczosLayout l;
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    l.dl = defl_layout(rows, K, b);
    l.Q = carve((size_t)rows * K * 8);
    l.cur = carve((size_t)rows * b * 8);
    l.W = carve((size_t)rows * b * 8);
    l.tmp = carve((size_t)rows * b * 8);
    l.defl = carve(l.dl.total);
    l.gp = carve((size_t)GRAM_BLOCKS * b * b * 16);
    l.G = carve((size_t)b * b * 16);
    l.sinv = carve((size_t)2 * b * b * 8);
    l.Y = carve((size_t)K * nev * 8);
    const bool lowp = link_dtype == COARSE_BF16 || link_dtype == COARSE_FP16;
    l.lowp = carve((lowp && d.nb % 16 == 0) ? lowp_ws_bytes(d, b) : 0);
    l.total = off;
    return l;
}

int32_t check_lanczos(const Geom &d, int32_t link_dtype, int32_t b, int32_t steps, int32_t nev) {
    int32_t rc = check_nrhs(b);
    if (rc) return rc;
    if (steps < 1 || (long long)steps * b > LANCZOS_MAX_K) {
        set_error("steps * block = %lld must lie in [1, %d]", (long long)steps * b, LANCZOS_MAX_K);
        return CG_INVALID_ARG;
    }
    if ((long long)steps * b > (long long)d.V * d.nb) {
        set_error("steps * block exceeds the number of unknowns");
        return CG_INVALID_ARG;
    }
    if (nev < 1 || nev > steps * b) {
        set_error("nev = %d must lie in [1, steps * block]", nev);
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
    return CG_OK;
}

}  // namespace

extern "C" int32_t coarse_block_lanczos_workspace_bytes(const coarse_geom *g, int32_t link_dtype, int32_t block,
                                                        int32_t steps, int32_t nev, size_t *out) {
    clear_error();
    Geom d;
    int32_t rc = make_geom(g, &d);
    if (rc) return rc;
    if ((rc = check_lanczos(d, link_dtype, block, steps, nev))) return rc;
    if (!out) {
        set_error("out is NULL");
        return CG_INVALID_ARG;
    }
    *out = lanczos_layout(d, link_dtype, block, steps * block, nev).total;
    return CG_OK;
}

extern "C" int32_t coarse_block_lanczos(const coarse_geom *g, const void *packed, int32_t link_dtype, const void *x0,
                                        int32_t block, int32_t steps, int32_t nev, void *v_out, double *lam_out,
                                        double *res_out, int32_t *k_out, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    Geom d;
    int32_t rc = make_geom(g, &d);
    if (rc) return rc;
    if ((rc = check_lanczos(d, link_dtype, block, steps, nev))) return rc;
    if (!packed || !x0 || !v_out || !lam_out) {
        set_error("packed, x0, v_out or lam_out is NULL");
        return CG_INVALID_ARG;
    }
    const int b = block, K = steps * block;
    const LanczosLayout l = lanczos_layout(d, link_dtype, b, K, nev);
    if (!ws || ws_bytes < l.total) {
        set_error("workspace %zu bytes, need %zu", ws ? ws_bytes : (size_t)0, l.total);
        return CG_WORKSPACE_TOO_SMALL;
    }
    const long long rows = (long long)d.V * d.nb;
    const size_t vb = (size_t)rows * b * 8, ob = (size_t)rows * nev * 8;
    if (overlaps(ws, l.total, x0, vb) || overlaps(ws, l.total, v_out, ob) || overlaps(v_out, ob, x0, vb) ||
        packed == ws || packed == v_out) {
        set_error("x0, v_out and the workspace must not overlap");
        return CG_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    char *w = reinterpret_cast<char *>(ws);
    float2 *Q = reinterpret_cast<float2 *>(w + l.Q), *cur = reinterpret_cast<float2 *>(w + l.cur);
    float2 *W = reinterpret_cast<float2 *>(w + l.W), *tmp = reinterpret_cast<float2 *>(w + l.tmp);
    double2 *gp = reinterpret_cast<double2 *>(w + l.gp), *G = reinterpret_cast<double2 *>(w + l.G);
    float2 *sinv = reinterpret_cast<float2 *>(w + l.sinv), *Y = reinterpret_cast<float2 *>(w + l.Y);
    void *lowp = (link_dtype == COARSE_BF16 || link_dtype == COARSE_FP16) ? w + l.lowp : nullptr;
    char *dw = w + l.defl;
    float2 *coef = reinterpret_cast<float2 *>(dw + l.dl.coef);
    const DeflLayout &dl = l.dl;
    const dim3 pgrid((unsigned)std::min<long long>((rows * b + 255) / 256, 8192));
    std::vector<double2> gh((size_t)b * b);
    std::vector<cd> Gh((size_t)b * b), R, Tm((size_t)(K + b) * K, cd(0, 0)), Rlast;
    std::vector<float2> cbuf((size_t)dl.nev_pad * dl.nr_pad), sbuf((size_t)b * b);

    // Gram X^H X to the host (into Gh)
    auto gram_host = [&](const float2 *X) -> int32_t {
        gram<float2>(X, X, rows, b, gp, G, nullptr, st);
        COARSE_HIP(hipMemcpyAsync(gh.data(), G, gh.size() * 16, hipMemcpyDeviceToHost, st));
        COARSE_HIP(hipStreamSynchronize(st));
        for (size_t i = 0; i < gh.size(); ++i) Gh[i] = cd(gh[i].x, gh[i].y);
        return CG_OK;
    };
    // The Cholesky factor of the Gram X^H X; false on a rank-deficient block: a
    // pivot not above 1e-10 of ref (the squared norm of the block before it was
    // orthogonalised; ref = 0: of X's own), i.e. a new direction below 1e-5 of
    // the applied block, which single precision cannot tell from rounding
    auto qr_factor = [&](const float2 *X, std::vector<cd> &Rf, bool &ok, double ref) -> int32_t {
        int32_t r = gram_host(X);
        if (r) return r;
        ok = host_chol(Gh, b, Rf, 1e-10, ref);
        return CG_OK;
    };
    // X <- X Rf^{-1} in place (tmp receives a copy)
    auto normalise = [&](float2 *X, const std::vector<cd> &Rf) -> int32_t {
        const std::vector<cd> Ri = host_tri_inv(Rf, b);
        for (int i = 0; i < b * b; ++i) sbuf[i] = make_float2((float)Ri[i].real(), (float)Ri[i].imag());
        COARSE_HIP(hipMemcpyAsync(sinv, sbuf.data(), sbuf.size() * 8, hipMemcpyHostToDevice, st));
        update_qd(X, tmp, sinv, sinv, rows, b, 1, nullptr, st);
        COARSE_HIP(hipGetLastError());
        return CG_OK;
    };

    COARSE_HIP(hipMemcpyAsync(cur, x0, vb, hipMemcpyDeviceToDevice, st));
    bool ok = true;
    if ((rc = qr_factor(cur, R, ok, 0.0))) return rc;
    if (!ok) {
        set_error("the start block is rank deficient");
        return CG_BREAKDOWN;
    }
    if ((rc = normalise(cur, R))) return rc;
    hipLaunchKernelGGL(lanczos_put_kernel, pgrid, dim3(256), 0, st, cur, Q, rows, b, (long long)K, 0);
    int m = K;  // columns of the final basis
    bool broke = false;
    for (int j = 0; j < steps; ++j) {
        if ((rc = launch_apply(d, packed, link_dtype, cur, W, b, COARSE_C64, nullptr, nullptr, st, 0, -1, lowp)))
            return rc;
        const int nj = (j + 1) * b;
        const int vec4 = (K % 2 == 0 && (reinterpret_cast<uintptr_t>(Q) & 15) == 0) ? 1 : 0;
        // squared norm of M Q_j before the reorthogonalisation (the rank test's scale)
        if ((rc = gram_host(W))) return rc;
        double wnorm2 = 0;
        for (int i = 0; i < b; ++i) wnorm2 += Gh[i * b + i].real();
        for (int pass = 0; pass < 2; ++pass) {
            // c = Q_{0..j}^H W; W -= Q_{0..j} c
            const long long per = ((rows + dl.split - 1) / dl.split + 15) / 16 * 16;
            hipLaunchKernelGGL(defl_coef_kernel<false>, dim3(round_up(nj, 64) / 64, dl.split, dl.nr_pad / 16),
                               dim3(256), 0, st, Q, W, rows, per, nj, b, dl.nev_pad, dl.nr_pad, vec4,
                               reinterpret_cast<float2 *>(dw + dl.partials), (long long)K);
            const int ne = dl.nev_pad * dl.nr_pad;
            hipLaunchKernelGGL(defl_reduce_kernel, dim3((ne + 15) / 16), dim3(256), 0, st,
                               reinterpret_cast<const float2 *>(dw + dl.partials), dl.split, nj, b, dl.nev_pad,
                               dl.nr_pad, (const double *)nullptr, coef, reinterpret_cast<float2 *>(dw + dl.coef_s));
            const long long waves2 = (rows + 31) / 32;
            hipLaunchKernelGGL((defl_promote_kernel<false, 2>), dim3((unsigned)((waves2 + 3) / 4), dl.nr_pad / 16),
                               dim3(256), 0, st, Q, coef, coef, W, W, (const float2 *)nullptr, (float2 *)nullptr,
                               rows, nj, b, dl.nr_pad, -1.f, vec4, 0, (long long)K);
            COARSE_HIP(hipGetLastError());
            COARSE_HIP(hipMemcpyAsync(cbuf.data(), coef, (size_t)nj * dl.nr_pad * 8, hipMemcpyDeviceToHost, st));
            COARSE_HIP(hipStreamSynchronize(st));
            for (int i = 0; i < nj; ++i)
                for (int c = 0; c < b; ++c) {
                    const float2 v = cbuf[(size_t)i * dl.nr_pad + c];
                    Tm[(size_t)i * K + j * b + c] += cd(v.x, v.y);
                }
        }
        std::vector<cd> Bj;
        if ((rc = qr_factor(W, Bj, ok, wnorm2))) return rc;
        if (!ok) {  // the Krylov space is exhausted (or numerically rank deficient)
            m = nj;
            broke = true;
            break;
        }
        for (int i = 0; i < b; ++i)
            for (int c = 0; c < b; ++c) Tm[(size_t)(nj + i) * K + j * b + c] = Bj[i * b + c];
        Rlast = Bj;
        if (j + 1 < steps) {
            if ((rc = normalise(W, Bj))) return rc;
            std::swap(cur, W);
            hipLaunchKernelGGL(lanczos_put_kernel, pgrid, dim3(256), 0, st, cur, Q, rows, b, (long long)K, nj);
            COARSE_HIP(hipGetLastError());
        }
    }
    // Rayleigh-Ritz on the Hermitian part of the leading m x m block
    std::vector<cd> A((size_t)m * m);
    for (int i = 0; i < m; ++i)
        for (int c = 0; c < m; ++c)
            A[(size_t)i * m + c] = 0.5 * (Tm[(size_t)i * K + c] + std::conj(Tm[(size_t)c * K + i]));
    std::vector<double> theta;
    std::vector<cd> Z;
    host_eigh(A, m, theta, Z);
    const int k = std::min(nev, m);
    std::vector<float2> yb((size_t)m * nev, make_float2(0.f, 0.f));
    for (int i = 0; i < m; ++i)
        for (int c = 0; c < k; ++c) yb[(size_t)i * nev + c] = make_float2((float)Z[(size_t)i * m + c].real(),
                                                                          (float)Z[(size_t)i * m + c].imag());
    COARSE_HIP(hipMemcpyAsync(Y, yb.data(), yb.size() * 8, hipMemcpyHostToDevice, st));
    // V = Q Y: the promotion with the m basis columns contracted, nev output columns
    {
        const int vec4 = (K % 2 == 0 && (reinterpret_cast<uintptr_t>(Q) & 15) == 0) ? 1 : 0;
        const long long waves2 = (rows + 31) / 32;
        hipLaunchKernelGGL((defl_promote_kernel<false, 2>), dim3((unsigned)((waves2 + 3) / 4), round_up(nev, 16) / 16),
                           dim3(256), 0, st, Q, Y, Y, (const float2 *)nullptr, reinterpret_cast<float2 *>(v_out),
                           (const float2 *)nullptr, (float2 *)nullptr, rows, m, nev, nev, 1.f, vec4, 0, (long long)K);
        COARSE_HIP(hipGetLastError());
    }
    COARSE_HIP(hipStreamSynchronize(st));
    for (int c = 0; c < nev; ++c) {
        lam_out[c] = c < k ? theta[c] : 0.0;
        if (res_out) {
            // M Q y - theta Q y = W_last z, z the last block of the Ritz vector y:
            // ||R_last z|| from the last factor, or on a break (no factor: W_last is
            // rank deficient but not necessarily zero) sqrt(z^H G z) from its Gram G
            double r2 = 0;
            if (c < k && !broke)
                for (int i = 0; i < b; ++i) {
                    cd s = 0;
                    for (int q = 0; q < b; ++q) s += Rlast[i * b + q] * Z[(size_t)(m - b + q) * m + c];
                    r2 += std::norm(s);
                }
            else if (c < k)
                for (int i = 0; i < b; ++i) {
                    cd s = 0;
                    for (int q = 0; q < b; ++q) s += Gh[i * b + q] * Z[(size_t)(m - b + q) * m + c];
                    r2 += (std::conj(Z[(size_t)(m - b + i) * m + c]) * s).real();
                }
            res_out[c] = std::sqrt(std::max(r2, 0.0));
        }
    }
    if (k_out) *k_out = m;
    return CG_OK;
}

// Host utility (no device work): eigenvalues (ascending) and eigenvectors of a
// Hermitian n x n matrix, interleaved complex128 row-major in and out.
extern "C" int32_t coarse_hermitian_eigh(int32_t n, const double *a, double *w, double *z) {
    clear_error();
    if (n < 1 || n > 4096 || !a || !w || !z) {
        set_error("need 1 <= n <= 4096 and non-NULL a, w, z");
        return CG_INVALID_ARG;
    }
    std::vector<cd> A((size_t)n * n);
    for (size_t i = 0; i < A.size(); ++i) A[i] = cd(a[2 * i], a[2 * i + 1]);
    std::vector<double> wv;
    std::vector<cd> Z;
    host_eigh(A, n, wv, Z);
    for (int i = 0; i < n; ++i) w[i] = wv[i];
    for (size_t i = 0; i < Z.size(); ++i) {
        z[2 * i] = Z[i].real();
        z[2 * i + 1] = Z[i].imag();
    }
    return CG_OK;
}
