// The Gram D^H Z of BlockCGrQ (Fig. 2, the matrix inverted after the
// operator application) fused into the epilogue of an apply kernel: the
// product splits into one short-K product per site (K = the nbasis rows of
// the site's block) plus a sum over sites, the scheme Sec. 3.5 uses for its
// Gram and thin-QR products.
//
// Workgroup b of the fused launch applies the operator at the sites of
// blocks b, b + nblk, b + 2 nblk, ... (nblk a multiple of 8, so all of them
// fall in the same XCD's slab of sites), adds each site's D^H Z to an
// accumulator in LDS and finally writes it as partial b, so that nblk partials
// (not one per site) are summed afterwards in a fixed order.
#pragma once
#include "common.hpp"

namespace coarse {

struct GramEpi {
    double2 *partials;  // nblk x nr x nr complex128
    int nblk;           // workgroups of the launch (a multiple of 64)
};

// Workgroups of a Gram-fused apply over V sites: V / S for the smallest power
// of two S with V / S <= cap (cap: the resident workgroups the kernel needs,
// and the partials kept within 8 MiB), or 0 when V does not split into a
// multiple of 64 workgroups.
inline int gram_fused_blocks(int V, int nr, int cap) {
    const long long bytes_cap = (8ll << 20) / ((long long)nr * nr * 16);
    long long lim = cap < bytes_cap ? cap : bytes_cap;
    if (lim < 64) return 0;
    for (int s = 1; s <= V; s *= 2) {
        if (V % s) return 0;
        const int n = V / s;
        if (n <= lim) return n % 64 == 0 ? n : 0;
    }
    return 0;
}

// One site's D^H Z added to acc (nr x nr complex128 in LDS, as (Re, Im)
// pairs). Each wave takes its own 16 rows of the site's block: lane (c, g)
// holds D and Z at rows 4 g + v (v < 4) of the wave's row tile, columns
// 16 k + c (k < NT3) -- the layout of the apply's accumulators, so Z needs no
// data movement -- and forms the 16 x 16 output tiles over those rows with
// f64 MFMA, K = the row index:
//   Re G = Dr^T Zr + Di^T Zi,  Im G = Dr^T Zi - Di^T Zr
// (every product of two float32 parts is exact in double). The waves form
// their tiles at the same time, then add them to acc in turn, wave 0 first,
// each turn closed by a barrier: with the sites added in a fixed order the
// sum is reproducible bit for bit.
template <int NT3>
__device__ __forceinline__ void gram_rows(const float2 (&dv)[NT3][4], const float2 (&zv)[NT3][4], int nr,
                                          LDS_AS double *acc, int w, int nw) {
    const int t = threadIdx.x & 63, c = t & 15, g = t >> 4;
    f64x4 gr[NT3][NT3], gi[NT3][NT3];
#pragma unroll
    for (int mt = 0; mt < NT3; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT3; ++nt) {
            gr[mt][nt] = f64x4{0, 0, 0, 0};
            gi[mt][nt] = gr[mt][nt];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double ar = dv[mt][v].x, ai = dv[mt][v].y;
                const double br = zv[nt][v].x, bi = zv[nt][v].y;
                gr[mt][nt] = mfma16x16x4(ar, br, gr[mt][nt]);
                gr[mt][nt] = mfma16x16x4(ai, bi, gr[mt][nt]);
                gi[mt][nt] = mfma16x16x4(ar, bi, gi[mt][nt]);
                gi[mt][nt] = mfma16x16x4(-ai, br, gi[mt][nt]);
            }
        }
    // f64 accumulator layout: lane (c, g) register u holds tile row g + 4 u, column c
    for (int turn = 0; turn < nw; ++turn) {
        if (turn == w) {
#pragma unroll
            for (int mt = 0; mt < NT3; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT3; ++nt) {
                    const int b = 16 * nt + c;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int a = 16 * mt + g + 4 * u;
                        if (a < nr && b < nr) {
                            LDS_AS double *s = acc + 2 * (a * nr + b);
                            s[0] = s[0] + gr[mt][nt][u];
                            s[1] = s[1] + gi[mt][nt][u];
                        }
                    }
                }
        }
        __syncthreads();
    }
}

}  // namespace coarse
