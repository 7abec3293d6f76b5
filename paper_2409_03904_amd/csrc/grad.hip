// Link gradient of a real loss through y = M x:
//   dA_p(x) (+)= alpha * G(x) . X(x + delta_p)^H,
// an nb x nb block per (site, point), each the sum over the nrhs columns of
// outer products (K = nrhs).
//
// MFMA form (nbasis % 16 == 0), three real products per complex
// multiply-add (3M):
//   T1 = Gr Xr^T,  T2 = Gi Xi^T,  T3 = (Gr + Gi)(Xr - Xi)^T,
//   Re dA = T1 + T2,  Im dA = T3 - T1 + T2,
// on 16x16x4 float32 MFMA with K = the RHS index r. One workgroup per site,
// wave w owns the 16-column tile j = 16 w .. 16 w + 15 of every output block
// and all its row tiles. The contraction order is free, so each lane's
// operands are pairs of consecutive entries of one row of G or of X, read
// with 16-byte loads straight from the [site][nbasis][nrhs] vectors (no LDS,
// no barrier). G's operands stay in registers for the site; X(x + delta_p)'s
// for the next point are loaded while the current one is multiplied. In the output
// layout of the MFMA, lane (column l, k-group q) holds rows 4 q + v of column
// l: for each v the 64 lanes write four whole 128-byte rows of 16 complex
// entries, with non-temporal stores (the output is never re-read here and
// would push the neighbour blocks of X out of L2).
//
// VALU form (other nbasis): one workgroup per (site, point), thread per
// output entry, operands in LDS with a padded row stride.
#include "common.hpp"

namespace coarse {

namespace {

// padded LDS row stride (floats) of an nr-column complex block: keeps float2
// alignment and spreads consecutive rows over the banks
__host__ __device__ inline int grad_row_stride(int nr) { return 2 * nr + 4; }

typedef float f2n __attribute__((ext_vector_type(2)));
typedef float f4n __attribute__((ext_vector_type(4)));

// Sites of one XCD form a contiguous slab (workgroups are dealt round-robin
// to the 8 XCDs), so neighbour blocks of X mostly stay in that XCD's L2.
__device__ __forceinline__ int grad_site_of_block(int b, int V) {
    return (V % 8 == 0) ? ((b & 7) * (V >> 3) + (b >> 3)) : b;
}

}  // namespace

// Entries r = 16 kg + 8 h + 2 q and r + 1 of one row (nr columns) of a
// [rows][nr] complex64 block, zero past nr: one 16-byte load when nr is even
// (then the pair is all in or all out), two guarded 8-byte loads otherwise.
template <bool EVEN>
__device__ __forceinline__ f4n load_pair(const float2 *row, int r, int nr) {
    if (EVEN) {
        const f4n v = *reinterpret_cast<const f4n *>(row + min(r, nr - 2));
        return r < nr ? v : f4n{0.f, 0.f, 0.f, 0.f};
    }
    const float2 a = row[min(r, nr - 1)], b = row[min(r + 1, nr - 1)];
    return f4n{r < nr ? a.x : 0.f, r < nr ? a.y : 0.f, r + 1 < nr ? b.x : 0.f, r + 1 < nr ? b.y : 0.f};
}

// NST = nbasis / 16 (waves, and row and column tiles per block);
// KG = ceil(nrhs / 16); EVEN: nrhs % 2 == 0.
// Wave w owns output column tile j = 16 w + l and walks its row tiles rt
// (one tile's three accumulators live at a time): each X entry it loads
// feeds 3 NST MFMAs, and the workgroup reads each neighbour block of X once. K order: lane k-group q at step s of group kg takes
// r = 16 kg + 8 (s >> 1) + 2 q + (s & 1), so its operands are two pairs of
// consecutive entries of one row of G or X (16-byte loads).
template <int NST, int KG, bool EVEN>
__global__ __launch_bounds__(256) void link_grad_3m_kernel(Geom g, const float2 *__restrict__ gy,
                                                           const float2 *__restrict__ x, float2 *__restrict__ dl,
                                                           float alpha, int accumulate, int nr) {
    constexpr int NB = 16 * NST;
    const int np = g.np;
    const int s = grad_site_of_block(blockIdx.x, g.V);
    const int w = threadIdx.x >> 6, t = threadIdx.x & 63, l = t & 15, q = t >> 4;

    // A operands: row i = 16 rt + l of G(x) (Gr + Gi formed per use)
    float gr[NST][KG][4], gi[NST][KG][4];
#pragma unroll
    for (int rt = 0; rt < NST; ++rt) {
        const float2 *grow = gy + ((size_t)s * NB + 16 * rt + l) * nr;
#pragma unroll
        for (int kg = 0; kg < KG; ++kg)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const f4n v = load_pair<EVEN>(grow, 16 * kg + 8 * h + 2 * q, nr);
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    gr[rt][kg][2 * h + e] = v[2 * e];
                    gi[rt][kg][2 * h + e] = v[2 * e + 1];
                }
            }
    }
    int cs[4];
    site_coords(g, s, cs);

    // B operands of point p: row j = 16 w + l of X(x + delta_p)
    const size_t xblk = (size_t)NB * nr;
    auto load_b = [&](f4n (&v)[KG][2], int p) {
        const float2 *xrow = x + (size_t)displaced(g, cs, p, 1) * xblk + (size_t)(16 * w + l) * nr;
#pragma unroll
        for (int kg = 0; kg < KG; ++kg)
#pragma unroll
            for (int h = 0; h < 2; ++h) v[kg][h] = load_pair<EVEN>(xrow, 16 * kg + 8 * h + 2 * q, nr);
    };

    f4n cur[KG][2], nxt[KG][2];
    load_b(cur, 0);
    for (int p = 0; p < np; ++p) {
        if (p + 1 < np) load_b(nxt, p + 1);
        // lane (column l, k-group q) holds rows 16 rt + 4 q + v of column 16 w + l
        float2 *ob = dl + ((size_t)s * np + p) * NB * NB + 16 * w + l;
#pragma unroll
        for (int rt = 0; rt < NST; ++rt) {
            f32x4 t1 = f32x4{0, 0, 0, 0}, t2 = t1, t3 = t1;
#pragma unroll
            for (int kg = 0; kg < KG; ++kg)
#pragma unroll
                for (int st = 0; st < 4; ++st) {
                    const f4n v = cur[kg][st >> 1];
                    const float xr = v[2 * (st & 1)], xi = v[2 * (st & 1) + 1];
                    t1 = mfma16x16x4(gr[rt][kg][st], xr, t1);
                    t2 = mfma16x16x4(gi[rt][kg][st], xi, t2);
                    t3 = mfma16x16x4(gr[rt][kg][st] + gi[rt][kg][st], xr - xi, t3);
                }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                float2 *o = ob + (size_t)(16 * rt + 4 * q + v) * NB;
                float re = alpha * (t1[v] + t2[v]), im = alpha * (t3[v] - t1[v] + t2[v]);
                if (accumulate) {
                    const float2 old = *o;
                    re += old.x;
                    im += old.y;
                }
                __builtin_nontemporal_store(f2n{re, im}, reinterpret_cast<f2n *>(o));
            }
        }
#pragma unroll
        for (int kg = 0; kg < KG; ++kg)
#pragma unroll
            for (int h = 0; h < 2; ++h) cur[kg][h] = nxt[kg][h];
    }
}

__global__ __launch_bounds__(256) void link_grad_kernel(Geom g, const float2 *__restrict__ gy,
                                                        const float2 *__restrict__ x, float2 *__restrict__ dl,
                                                        float alpha, int accumulate, int nr) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int nb = g.nb;
    const int blk = blockIdx.x;  // s * np + p
    const int s = blk / g.np, p = blk - s * g.np;
    int c[4];
    site_coords(g, s, c);
    const int z = displaced(g, c, p, 1);
    const int rs = grad_row_stride(nr);
    LDS_AS float *gs = lds_ptr<float>(smem_raw);  // [nb][rs]
    LDS_AS float *xs = gs + nb * rs;              // [nb][rs]
    const float2 *gsrc = gy + (size_t)s * nb * nr;
    const float2 *xsrc = x + (size_t)z * nb * nr;
    for (int e = threadIdx.x; e < nb * nr; e += blockDim.x) {
        const int j = e / nr, r = e - j * nr;
        const float2 gv = gsrc[e], xv = xsrc[e];
        gs[j * rs + 2 * r] = gv.x;
        gs[j * rs + 2 * r + 1] = gv.y;
        xs[j * rs + 2 * r] = xv.x;
        xs[j * rs + 2 * r + 1] = xv.y;
    }
    __syncthreads();
    float2 *out = dl + (size_t)blk * nb * nb;
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
        const int i = e / nb, j = e - i * nb;
        float re = 0.f, im = 0.f;
        for (int r = 0; r < nr; ++r) {
            const float ar = gs[i * rs + 2 * r], ai = gs[i * rs + 2 * r + 1];
            const float br = xs[j * rs + 2 * r], bi = xs[j * rs + 2 * r + 1];
            // a * conj(b)
            re += ar * br + ai * bi;
            im += ai * br - ar * bi;
        }
        re *= alpha;
        im *= alpha;
        if (accumulate) {
            const float2 o = out[e];
            re += o.x;
            im += o.y;
        }
        out[e] = make_float2(re, im);
    }
}

}  // namespace coarse

using namespace coarse;

extern "C" int32_t coarse_link_grad(const coarse_geom *g, const void *gy, const void *x, void *dlinks, float alpha,
                                    int32_t accumulate, int32_t nrhs, void *stream) {
    clear_error();
    Geom d;
    int32_t rc = make_geom(g, &d);
    if (rc) return rc;
    if ((rc = check_nrhs(nrhs))) return rc;
    if (!gy || !x || !dlinks) {
        set_error("gy, x or dlinks is NULL");
        return CG_INVALID_ARG;
    }
    if (dlinks == gy || dlinks == x) {
        set_error("dlinks must not alias the inputs");
        return CG_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    const size_t lds = ((size_t)2 * d.nb * grad_row_stride(nrhs) + 2) * sizeof(float);
    if (d.nb % 16 == 0) {
        const dim3 grid((unsigned)d.V), block(64 * (d.nb / 16));
        const float2 *g2 = (const float2 *)gy, *x2 = (const float2 *)x;
        float2 *o2 = (float2 *)dlinks;
#define GL(NST_, KG_, EV_)                                                                                   \
    hipLaunchKernelGGL((link_grad_3m_kernel<NST_, KG_, EV_>), grid, block, 0, st, d, g2, x2, o2, alpha,       \
                       accumulate, nrhs)
#define GL_NST(KG_, EV_)                  \
    switch (d.nb / 16) {                  \
        case 1: GL(1, KG_, EV_); break;   \
        case 2: GL(2, KG_, EV_); break;   \
        case 3: GL(3, KG_, EV_); break;   \
        default: GL(4, KG_, EV_); break;  \
    }
        const bool even = nrhs % 2 == 0;
        if (nrhs <= 16) {
            if (even) GL_NST(1, true) else GL_NST(1, false)
        } else {
            if (even) GL_NST(2, true) else GL_NST(2, false)
        }
#undef GL_NST
#undef GL
    } else {
        hipLaunchKernelGGL(link_grad_kernel, dim3((unsigned)(d.V * d.np)), dim3(256), lds, st, d,
                           (const float2 *)gy, (const float2 *)x, (float2 *)dlinks, alpha, accumulate, nrhs);
    }
    COARSE_HIP(hipGetLastError());
    return CG_OK;
}
