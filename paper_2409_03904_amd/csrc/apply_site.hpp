// Per-site body of the float32/float64 MFMA coarse apply (shared by the
// one-site-per-workgroup kernel and the persistent batched kernel).
#pragma once
#include "common.hpp"
#include <type_traits>

namespace coarse {

// ---------------------------------------------------------------------------
// float32 / float64 MFMA kernel, complex64 links in the tiled layout.
// T = float: complex64 vectors, 16x16x4 f32 MFMA.
// T = double: complex128 vectors, 16x16x4 f64 MFMA on exact float->double links.
// NT: number of 16-column tiles of the 2*nrhs real output columns.
// ---------------------------------------------------------------------------
template <typename T, int NT>
__device__ __forceinline__ void site_apply_mfma(const Geom &g, const float *__restrict__ links,
                                                const T *__restrict__ x, T *__restrict__ y, int nr,
                                                const T *__restrict__ sub, int s, unsigned char *smem_raw) {
    typedef typename std::conditional<sizeof(T) == 4, f32x4, f64x4>::type AccT;
    const int nb = g.nb;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int w = tid >> 6, t = tid & 63, il = t & 15, q = t >> 4;
    const int nmt = (nb + 15) >> 4;
    const bool wave_on = w < nmt;     // waves beyond the row tiles only help staging
    const int rows = wave_on ? min(16, nb - 16 * w) : 0;
    const bool row_ok = il < rows;
    const int nch = nb >> 3;          // 16-wide k' chunks per link block
    const int xblk = nb * nr * 2;     // T elements per neighbour block
    T *xb0 = reinterpret_cast<T *>(smem_raw);
    T *xb1 = xb0 + xblk;

    // B operand of lane (il, q) at step st: X'[4st + q][16nt + il].
    // h = q & 1 picks Re/Im of X(j = 2st + q/2, r); column part 0 = Yr, 1 = Yi.
    int boff[NT];
    T bsg[NT];
    {
        const int h = q & 1;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int n = 16 * nt + il;
            const int part = n / nr, r = n - part * nr;
            if (part >= 2) {
                boff[nt] = 0;
                bsg[nt] = T(0);
            } else {
                const int comp = (part == 0) ? h : 1 - h;
                boff[nt] = 2 * r + comp;
                bsg[nt] = (part == 0 && h) ? T(-1) : T(1);
            }
        }
    }
    const int jq = q >> 1;

    int c[4];
    site_coords(g, s, c);

    // neighbour block staging: float4 units, at most 8 per thread
    const int nvec = (xblk * (int)sizeof(T)) >> 4;
    float4 xr[8];
    auto load_x = [&](int p) {
        const int z = displaced(g, c, p, 1);
        const float4 *src = reinterpret_cast<const float4 *>(x + (size_t)z * xblk);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int e = tid + k * nthr;
            if (e < nvec) xr[k] = src[e];
        }
    };
    auto store_x = [&](T *dst) {
        float4 *d4 = reinterpret_cast<float4 *>(dst);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int e = tid + k * nthr;
            if (e < nvec) d4[e] = xr[k];
        }
    };

    const size_t blk_floats = (size_t)nb * nb * 2;
    const float *lsite = links + (size_t)s * g.np * blk_floats;
    const int lane_off = 16 * w * 16 + (q * rows + il) * 4;
    float4 a_cur[8], a_nxt[8];
    auto load_a = [&](float4 *a, int p) {
        const float *lb = lsite + (size_t)p * blk_floats + lane_off;
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
            if (cc < nch) a[cc] = row_ok ? *reinterpret_cast<const float4 *>(lb + cc * nb * 16)
                                         : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };

    load_x(0);
    load_a(a_cur, 0);
    store_x(xb0);
    __syncthreads();

    AccT acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = AccT{0, 0, 0, 0};

    for (int p = 0; p < g.np; ++p) {
        const bool more = (p + 1) < g.np;
        if (more) {
            load_x(p + 1);
            load_a(a_nxt, p + 1);
        }
        const T *xc = (p & 1) ? xb1 : xb0;
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
            if (wave_on && cc < nch) {
                const float av4[4] = {a_cur[cc].x, a_cur[cc].y, a_cur[cc].z, a_cur[cc].w};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int j = 8 * cc + 2 * u + jq;
                    const T *xrow = xc + j * nr * 2;
                    const T av = (T)av4[u];
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        const T bv = bsg[nt] * xrow[boff[nt]];
                        acc[nt] = mfma16x16x4(av, bv, acc[nt]);
                    }
                }
            }
        }
        if (more) {
            store_x((p & 1) ? xb0 : xb1);
#pragma unroll
            for (int cc = 0; cc < 8; ++cc) a_cur[cc] = a_nxt[cc];
        }
        __syncthreads();
    }

    // epilogue: D tiles -> LDS [row][2*nr] -> complex output
    T *out = xb0;
    const int two_nr = 2 * nr;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int n = 16 * nt + il;
        if (wave_on && n < two_nr) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // accumulator layout: lane group q holds rows 4q..4q+3 (f32) but
                // rows q, q+4, q+8, q+12 (f64) of the 16x16 tile, column il
                const int row = 16 * w + (sizeof(T) == 8 ? q + 4 * v : 4 * q + v);
                if (row < nb) out[row * two_nr + n] = acc[nt][v];
            }
        }
    }
    __syncthreads();
    T *yo = y + (size_t)s * xblk;
    const T *so = sub ? sub + (size_t)s * xblk : nullptr;
    for (int e = tid; e < nb * nr; e += nthr) {
        const int i = e / nr, r = e - i * nr;
        T re = out[i * two_nr + r], im = out[i * two_nr + nr + r];
        if (so) {
            re = so[2 * e] - re;
            im = so[2 * e + 1] - im;
        }
        yo[2 * e] = re;
        yo[2 * e + 1] = im;
    }
    __syncthreads();  // LDS free for the next site
}

}  // namespace coarse
