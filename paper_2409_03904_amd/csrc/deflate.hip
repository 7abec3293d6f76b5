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
                                                        int nr_pad, int vec4, float2 *__restrict__ partial) {
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
            const float2 *vr = v + (ok ? row : 0) * nev;
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

// c[i][j] = sum_s partial[s][i][j] (double; each of 16 lanes sums every 16th
// range, then a fixed butterfly); c_s = c / lambda_i. Workgroup: 16 entries.
__global__ __launch_bounds__(256) void defl_reduce_kernel(const float2 *__restrict__ partial, int split, int nev,
                                                          int nr, int nev_pad, int nr_pad,
                                                          const double *__restrict__ lam, float2 *__restrict__ coef,
                                                          float2 *__restrict__ coef_s) {
    const int e = blockIdx.x * 16 + (threadIdx.x >> 4), l = threadIdx.x & 15;
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
#pragma unroll
    for (int m = 8; m > 0; m >>= 1) {
        sr += __shfl_xor(sr, m, 16);
        si += __shfl_xor(si, m, 16);
    }
    if (!live || l != 0) return;
    if (i >= nev || j >= nr) {
        coef[e] = make_float2(0.f, 0.f);
        coef_s[e] = make_float2(0.f, 0.f);
        return;
    }
    const double li = 1.0 / lam[i];
    coef[e] = make_float2((float)sr, (float)si);
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
                                                           int vec4, int vblock) {
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
        vrow[q] = v + (rv[q] ? ra : 0) * nev;
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
                       rows, per, nev, nr, l.nev_pad, l.nr_pad, vec4, partial);
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
                           out2, rows, nev, nr, l.nr_pad, sign1, vec4, 0);
    else
        hipLaunchKernelGGL((defl_promote_kernel<false, 2>), grid, dim3(256), 0, st, v, coef1, coef1, base1, out1,
                           (const float2 *)nullptr, (float2 *)nullptr, rows, nev, nr, l.nr_pad, sign1, vec4, 0);
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
                       round_up(nrhs, 16), vec4, reinterpret_cast<float2 *>(coarse_out));
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
                           (float2 *)nullptr, rows, nb, nrhs, nrhs, 1.f, vec4, vblock);
    } else {
        const long long waves = rows / 16;
        hipLaunchKernelGGL((defl_promote_kernel<false, 1>), dim3((unsigned)((waves + 3) / 4), gy), dim3(256), 0,
                           (hipStream_t)stream, bp, cp, cp, (const float2 *)nullptr, fp, (const float2 *)nullptr,
                           (float2 *)nullptr, rows, nb, nrhs, nrhs, 1.f, vec4, vblock);
    }
    COARSE_HIP(hipGetLastError());
    return CG_OK;
}
