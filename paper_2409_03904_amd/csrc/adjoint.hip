// Adjoint coarse apply on MFMA: y(x) = sum_p A_p(x - delta_p)^H X(x - delta_p).
//
// The adjoint contracts over the ROW index of each link block, while the
// packed layout hands each lane a row. So each block is staged once in LDS
// (coalesced 16-byte loads by the whole workgroup, double-buffered with the
// next point's loads in flight) and every lane reads the transposed entries
// it needs. In the 4M real embedding of A^H the signs move to the input
// operand: [Yr | Yi] = [Ar^T Ai^T] . [[Xr  Xi], [Xi  -Xr]] with k' = 2j + h.
// One workgroup per output site, one wave per 16-row tile, as in the forward
// kernel; every link block is still read from HBM exactly once per apply.
#include <type_traits>

#include "apply.hpp"

namespace coarse {

// native 4-wide vector: unlike HIP's float4 struct, arrays of it stay in registers
typedef float av4 __attribute__((ext_vector_type(4)));

// row stride (floats) of a link block staged row-major in LDS: 2 nb + 2 makes
// both the staging writes (rows 2 banks apart) and the transposed reads (one
// link row per half-wave, consecutive columns) free of bank conflicts
__host__ __device__ inline int adj_row_stride(int nb) { return 2 * nb + 2; }

// NB: nbasis fixed at compile time (16, 24, 32, 48, 64: the k-step loop unrolls
// and the staging loads per thread are exact), or 0 for any multiple of 8.
template <typename T, int NT, int NB>
__global__ __launch_bounds__(256) void adjoint_mfma_kernel(Geom g, const float *__restrict__ links,
                                                            const T *__restrict__ x, T *__restrict__ y, int nr) {
    typedef typename std::conditional<sizeof(T) == 4, f32x4, f64x4>::type AccT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int nb = NB > 0 ? NB : g.nb;
    // float4 loads per thread per point: link block, vector block (nr <= 8 NT)
    constexpr int NTHR = 64 * ((NB + 15) / 16);
    constexpr int LV = NB > 0 ? (NB * NB / 2 + NTHR - 1) / NTHR : 8;
    constexpr int XV = NB > 0 ? (NB * NT * (int)sizeof(T) + NTHR - 1) / NTHR : 8;
    const int V = g.V;
    const int b = blockIdx.x;
    const int s = (V % 8 == 0) ? ((b & 7) * (V >> 3) + (b >> 3)) : b;
    const int tid = threadIdx.x, nthr = NB > 0 ? NTHR : (int)blockDim.x;
    const int w = tid >> 6, t = tid & 63, il = t & 15, q = t >> 4;
    const int i = 16 * w + il;           // output row = column of the link block
    const int ic = min(i, nb - 1);       // rows past nbasis read a valid column (results unused)
    const int h = q & 1, jq = q >> 1;
    const int blk = 2 * nb * nb;         // floats per link block
    const int rs = adj_row_stride(nb);
    const int ablk = nb * rs;            // floats per staged block
    const int xblk = nb * nr * 2;        // T per vector block
    // LDS: [link block 0 | link block 1 | X block 0 | X block 1]
    LDS_AS float *lbase = lds_ptr<float>(smem_raw);
    LDS_AS T *xbase = reinterpret_cast<LDS_AS T *>(lbase + 2 * ablk + (2 * ablk) % 4);

    // B operand: part 0 (Yr): +Xr, +Xi for h = 0, 1; part 1 (Yi): +Xi, -Xr.
    int boff[NT];
    T bsg[NT];
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
            bsg[nt] = (part == 1 && h) ? T(-1) : T(1);
        }
    }

    int c[4];
    site_coords(g, s, c);

    const int lvec = blk >> 2;                          // float4 per link block
    const int xvec = (xblk * (int)sizeof(T)) >> 4;      // float4 per vector block
    // Loads are branch-free (indices clamped; surplus lanes re-read the last
    // float4): a load under a branch makes the wait-count insertion drain the
    // prefetch at the join.
    av4 lr[LV], xr[XV];
#define ADJ_LOAD(P)                                                                                     \
    {                                                                                                   \
        const int p_ = min((P), g.np - 1);                                                              \
        const int z_ = displaced(g, c, p_, -1);                                                         \
        const av4 *ls_ = reinterpret_cast<const av4 *>(links + ((size_t)z_ * g.np + p_) * blk);         \
        const av4 *xs_ = reinterpret_cast<const av4 *>(x + (size_t)z_ * xblk);                          \
        _Pragma("unroll") for (int k = 0; k < LV; ++k) lr[k] = ls_[min(tid + k * nthr, lvec - 1)];      \
        _Pragma("unroll") for (int k = 0; k < XV; ++k) xr[k] = xs_[min(tid + k * nthr, xvec - 1)];      \
    }
    // packed float4 e holds A'[16 mt + il'][16 cc + 4u + q'] (u = 0..3) of the
    // tiled layout (full 16-row tiles; partial tiles have `rows` rows); it goes
    // to the row-major block, row i', column k' (= 2j + Re/Im)
#define ADJ_STORE(BUF)                                                                                  \
    {                                                                                                   \
        LDS_AS float *ld_ = lbase + (BUF) * ablk;                                                       \
        LDS_AS av4 *x4_ = reinterpret_cast<LDS_AS av4 *>(xbase + (BUF) * xblk);                         \
        _Pragma("unroll") for (int k = 0; k < LV; ++k) {                                                \
            const int e = tid + k * nthr;                                                               \
            if (e < lvec) {                                                                             \
                const int f = 4 * e;                      /* float offset in the packed block */        \
                const int cc = f / (16 * nb), rem = f - cc * 16 * nb;                                   \
                const int mt = rem >> 8, in_tile = rem - (mt << 8);                                     \
                const int rows = min(16, nb - 16 * mt);                                                 \
                const int qq = (in_tile >> 2) / rows, ii = 16 * mt + (in_tile >> 2) - qq * rows;        \
                LDS_AS float *dst = ld_ + ii * rs + 16 * cc + qq;                                       \
                dst[0] = lr[k].x;                                                                       \
                dst[4] = lr[k].y;                                                                       \
                dst[8] = lr[k].z;                                                                       \
                dst[12] = lr[k].w;                                                                      \
            }                                                                                           \
        }                                                                                               \
        _Pragma("unroll") for (int k = 0; k < XV; ++k) {                                                \
            const int e = tid + k * nthr;                                                               \
            if (e < xvec) x4_[e] = xr[k];                                                               \
        }                                                                                               \
    }

    ADJ_LOAD(0)
    ADJ_STORE(0)
    __syncthreads();

    AccT acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = AccT{0, 0, 0, 0};
    const int nsteps = nb >> 1;  // k' = 2nb per block, 4 per step

    for (int p = 0; p < g.np; ++p) {
        ADJ_LOAD(p + 1)  // the last point re-reads itself (clamped), branch-free
        const LDS_AS float *lc_ = lbase + (p & 1) * ablk;
        const LDS_AS T *xc = xbase + (p & 1) * xblk;
        // lane (il, q), step st: component h of A[j][i] with j = 2 st + jq
        const LDS_AS float *acol = lc_ + jq * rs + 2 * ic + h;
#pragma unroll
        for (int st = 0; st < nsteps; ++st) {
            const int j = 2 * st + jq;
            const float av = acol[2 * st * rs];
            const LDS_AS T *xrow = xc + j * nr * 2;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[nt] = mfma16x16x4((T)av, bsg[nt] * xrow[boff[nt]], acc[nt]);
        }
        ADJ_STORE((p + 1) & 1)
        __syncthreads();
    }

#undef ADJ_LOAD
#undef ADJ_STORE
    LDS_AS T *out = lds_ptr<T>(smem_raw);
    const int two_nr = 2 * nr;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int n = 16 * nt + il;
        if (n < two_nr) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * w + (sizeof(T) == 8 ? q + 4 * v : 4 * q + v);
                if (row < nb) out[row * two_nr + n] = acc[nt][v];
            }
        }
    }
    __syncthreads();
    T *yo = y + (size_t)s * xblk;
    for (int e = tid; e < nb * nr; e += nthr) {
        const int ii = e / nr, r = e - ii * nr;
        yo[2 * e] = out[ii * two_nr + r];
        yo[2 * e + 1] = out[ii * two_nr + nr + r];
    }
}

// Dynamic LDS above the default 64 KB needs a per-kernel opt-in (gfx950 has
// 160 KB per CU). Returns false when the runtime refuses it.
template <typename T, int NT, int NB>
static bool lds_opt_in(size_t lds) {
    static size_t granted = 64 * 1024;
    if (lds <= granted) return true;
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(&adjoint_mfma_kernel<T, NT, NB>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    granted = lds;
    return true;
}

template <typename T, int NT, int NB>
static bool launch_adj_nb(const Geom &g, const float *links, const T *x, T *y, int nr, hipStream_t st) {
    const int waves = (g.nb + 15) / 16;
    const size_t ablk = (size_t)g.nb * adj_row_stride(g.nb);
    const size_t lds = (2 * ablk + (2 * ablk) % 4) * sizeof(float) + (size_t)2 * g.nb * nr * 2 * sizeof(T);
    if (!lds_opt_in<T, NT, NB>(lds)) return false;
    hipLaunchKernelGGL((adjoint_mfma_kernel<T, NT, NB>), dim3(g.V), dim3(64 * waves), lds, st, g, links, x, y, nr);
    return true;
}

template <typename T, int NT>
static bool launch_adj_t(const Geom &g, const float *links, const T *x, T *y, int nr, hipStream_t st) {
    switch (g.nb) {
        case 16: return launch_adj_nb<T, NT, 16>(g, links, x, y, nr, st);
        case 24: return launch_adj_nb<T, NT, 24>(g, links, x, y, nr, st);
        case 32: return launch_adj_nb<T, NT, 32>(g, links, x, y, nr, st);
        case 48: return launch_adj_nb<T, NT, 48>(g, links, x, y, nr, st);
        case 64: return launch_adj_nb<T, NT, 64>(g, links, x, y, nr, st);
        default: return launch_adj_nb<T, NT, 0>(g, links, x, y, nr, st);
    }
}

template <typename T>
static bool launch_adj(const Geom &g, const float *links, const T *x, T *y, int nr, hipStream_t st) {
    switch ((2 * nr + 15) / 16) {
        case 1: return launch_adj_t<T, 1>(g, links, x, y, nr, st);
        case 2: return launch_adj_t<T, 2>(g, links, x, y, nr, st);
        case 3: return launch_adj_t<T, 3>(g, links, x, y, nr, st);
        default: return launch_adj_t<T, 4>(g, links, x, y, nr, st);
    }
}

// Returns true when the MFMA adjoint took the call.
bool launch_adjoint_mfma(const Geom &g, const void *packed, int32_t link_dtype, const void *x, void *y, int nr,
                         int32_t vec_dtype, hipStream_t st) {
    if (link_dtype != COARSE_C64 || !tiled_c64(g.nb) || nr < 1 || nr > 32) return false;
    const size_t vbytes = vec_dtype == COARSE_C128 ? 16 : 8;
    const size_t ablk = (size_t)g.nb * adj_row_stride(g.nb);
    const size_t lds = (2 * ablk + 4) * 4 + (size_t)2 * g.nb * nr * vbytes;
    if (lds > 160 * 1024) return false;
    if (vec_dtype == COARSE_C64) return launch_adj<float>(g, (const float *)packed, (const float *)x, (float *)y, nr, st);
    if (vec_dtype == COARSE_C128)
        return launch_adj<double>(g, (const float *)packed, (const double *)x, (double *)y, nr, st);
    return false;
}

}  // namespace coarse

// ---- links of the adjoint operator ------------------------------------------
//
// M^H is itself a stencil operator: (M^H X)(x) = sum_p A_p(x - delta_p)^H
// X(x - delta_p), i.e. links B_p(x) = A_p(x - delta_p)^H at displacements
// -delta_p. Writing B once (public layout) lets a caller pack it in any link
// layout, the 3M one included, and apply M^H with the forward kernels.
namespace coarse {

__global__ __launch_bounds__(256) void adjoint_links_kernel(Geom g, const float2 *__restrict__ a,
                                                            float2 *__restrict__ b) {
    const int nb = g.nb, np = g.np;
    const long long blk = (long long)nb * nb, per_site = np * blk;
    const long long n = (long long)g.V * per_site, stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        const int x = (int)(e / per_site);
        const long long rem = e - (long long)x * per_site;
        const int p = (int)(rem / blk);
        const int ij = (int)(rem - (long long)p * blk), i = ij / nb, j = ij - i * nb;
        int c[4];
        site_coords(g, x, c);
        const int src = displaced(g, c, p, -1);
        const float2 v = a[(((long long)src * np + p) * nb + j) * nb + i];
        b[e] = make_float2(v.x, -v.y);
    }
}

}  // namespace coarse

using namespace coarse;

extern "C" int32_t coarse_adjoint_links(const coarse_geom *g, const void *links, void *links_adj, void *stream) {
    coarse::clear_error();
    coarse::Geom d;
    int32_t rc = coarse::make_geom(g, &d);
    if (rc) return rc;
    if (!links || !links_adj) {
        coarse::set_error("links or links_adj is NULL");
        return CG_INVALID_ARG;
    }
    const long long n = (long long)d.V * d.np * d.nb * d.nb;
    const char *pa = reinterpret_cast<const char *>(links), *pb = reinterpret_cast<const char *>(links_adj);
    if (pa < pb + n * 8 && pb < pa + n * 8) {
        coarse::set_error("links and links_adj must not overlap");
        return CG_INVALID_ARG;
    }
    const long long blocks = (n + 255) / 256;
    hipLaunchKernelGGL(coarse::adjoint_links_kernel, dim3((unsigned)(blocks < 16384 ? blocks : 16384)), dim3(256), 0,
                       (hipStream_t)stream, d, reinterpret_cast<const float2 *>(links),
                       reinterpret_cast<float2 *>(links_adj));
    COARSE_HIP(hipGetLastError());
    return CG_OK;
}
