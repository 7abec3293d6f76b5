// Per-site body of the float32/float64 MFMA coarse apply (shared by the
// one-site-per-workgroup kernel and the persistent batched kernel).
//
// One workgroup computes y(s) = sum_p A_p(s) X(s + delta_p) for one site s:
// wave w owns output rows 16w..16w+15 and streams those rows of every link
// block straight into the MFMA A operand (16-byte non-temporal loads, the
// links are read exactly once per apply); the neighbour block X(s + delta_p)
// is staged in LDS once per point and shared by the waves. Link loads run
// PD points ahead of the MFMAs in a ring of register buffers (indices fixed
// at compile time by unrolling the point loop over the ring), the next
// neighbour block one point ahead.
#pragma once
#include <type_traits>

#include "common.hpp"

namespace coarse {

typedef float fvec4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ fvec4 stream_load(const float *p) {
    return __builtin_nontemporal_load(reinterpret_cast<const fvec4 *>(p));
}

// NCH: 16-wide k' chunks per link block (= nbasis/8); 0 = runtime value up to 8.
// PD: link prefetch depth in stencil points.
template <typename T, int NT, int NCH, int PD>
__device__ __forceinline__ void site_apply_mfma(const Geom &g, const float *__restrict__ links,
                                                const T *__restrict__ x, T *__restrict__ y, int nr,
                                                const T *__restrict__ sub, int s, unsigned char *smem_raw) {
    typedef typename std::conditional<sizeof(T) == 4, f32x4, f64x4>::type AccT;
    constexpr int MAXCH = NCH ? NCH : 8;
    constexpr int XV = sizeof(T) == 4 ? 4 : 8;  // max float4 of a neighbour block per thread
    constexpr int RING = PD + 1;
    const int nb = g.nb;
    const int nch = NCH ? NCH : (nb >> 3);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int w = tid >> 6, t = tid & 63, il = t & 15, q = t >> 4;
    const int nmt = (nb + 15) >> 4;
    const bool wave_on = w < nmt;     // waves beyond the row tiles only help staging
    const int rows = wave_on ? min(16, nb - 16 * w) : 0;
    const bool row_ok = il < rows;
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

    // Staging loads are unconditional (index clamped into the block) so the
    // staging registers stay registers; only the LDS stores are predicated.
    const int nvec = (xblk * (int)sizeof(T)) >> 4;
    const int xv = (nvec + nthr - 1) / nthr;  // <= XV
    fvec4 xr[XV];
    auto load_x = [&](int p) {
        const int z = displaced(g, c, p, 1);
        const fvec4 *src = reinterpret_cast<const fvec4 *>(x + (size_t)z * xblk);
#pragma unroll
        for (int k = 0; k < XV; ++k) {
            if (k < xv) xr[k] = src[min(tid + k * nthr, nvec - 1)];
        }
    };
    auto store_x = [&](T *dst) {
        fvec4 *d4 = reinterpret_cast<fvec4 *>(dst);
#pragma unroll
        for (int k = 0; k < XV; ++k) {
            const int e = tid + k * nthr;
            if (k < xv && e < nvec) d4[e] = xr[k];
        }
    };

    const size_t blk_floats = (size_t)nb * nb * 2;
    const float *lsite = links + (size_t)s * g.np * blk_floats;
    const int lane_off = 16 * w * 16 + (q * rows + il) * 4;
    fvec4 ring[RING][MAXCH];
    auto load_a = [&](fvec4 *a, int p) {
        const float *lb = lsite + (size_t)p * blk_floats + lane_off;
#pragma unroll
        for (int cc = 0; cc < MAXCH; ++cc) {
            if (NCH || cc < nch) a[cc] = row_ok ? stream_load(lb + cc * nb * 16) : fvec4{0.f, 0.f, 0.f, 0.f};
        }
    };

    AccT acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = AccT{0, 0, 0, 0};

    const int np = g.np;
    load_x(0);
#pragma unroll
    for (int k = 0; k < PD; ++k)
        if (k < np) load_a(ring[k], k);
    store_x(xb0);
    __syncthreads();

    for (int p0 = 0; p0 < np; p0 += RING) {
#pragma unroll
        for (int k = 0; k < RING; ++k) {
            const int p = p0 + k;
            if (p < np) {
                if (p + PD < np) load_a(ring[(k + PD) % RING], p + PD);
                const bool more = (p + 1) < np;
                if (more) load_x(p + 1);
                const T *xc = (p & 1) ? xb1 : xb0;
                if (wave_on) {
#pragma unroll
                    for (int cc = 0; cc < MAXCH; ++cc) {
                        if (NCH || cc < nch) {
                            const fvec4 a4 = ring[k][cc];
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const int j = 8 * cc + 2 * u + jq;
                                const T *xrow = xc + j * nr * 2;
                                const T av = (T)a4[u];
#pragma unroll
                                for (int nt = 0; nt < NT; ++nt)
                                    acc[nt] = mfma16x16x4(av, bsg[nt] * xrow[boff[nt]], acc[nt]);
                            }
                            // long blocks: keep the LDS reads of later chunks from
                            // being hoisted (register pressure, occupancy)
                            if (MAXCH > 4) __builtin_amdgcn_sched_barrier(0);
                        }
                    }
                }
                if (more) store_x((p & 1) ? xb0 : xb1);
                __syncthreads();
            }
        }
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
