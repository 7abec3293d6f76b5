// Link import: repack the public complex64 links into the kernel layouts and,
// for 16-bit storage, quantise every non-self block with one power-of-two
// scale (the operator's coefficients kept inside the library in a
// compute-ready layout, Sec. 2.5).
#include "common.hpp"

namespace coarse {

// One thread per complex entry; writes the two floats of the real embedding.
__global__ void pack_c64_kernel(int nb, size_t nblocks, const float2 *__restrict__ src,
                                float *__restrict__ dst) {
    size_t per = (size_t)nb * nb;
    size_t total = nblocks * per;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        size_t blk = e / per;
        int ij = (int)(e - blk * per);
        int i = ij / nb, j = ij - i * nb;
        float2 v = src[e];
        float *b = dst + blk * per * 2;
        b[c64_block_offset(nb, i, 2 * j)] = v.x;
        b[c64_block_offset(nb, i, 2 * j + 1)] = v.y;
    }
}

// 3M layout: one thread per complex entry.
__global__ void pack_c64_3m_kernel(int nb, size_t nblocks, const float2 *__restrict__ src,
                                   float *__restrict__ dst) {
    size_t per = (size_t)nb * nb;
    size_t total = nblocks * per;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        size_t blk = e / per;
        int ij = (int)(e - blk * per);
        int i = ij / nb, j = ij - i * nb;
        float2 v = src[e];
        float *b = dst + blk * per * 2;
        b[c64_3m_block_offset(nb, i, j, 0)] = v.x;
        b[c64_3m_block_offset(nb, i, j, 1)] = v.y;
    }
}

// One workgroup per (site, point) block. Self blocks go to the complex64
// region in the tiled layout; every other block is scaled and rounded.
template <int KIND>  // 0 = bf16, 1 = fp16
__global__ __launch_bounds__(256) void pack_lowp_kernel(Geom g, const float2 *__restrict__ src,
                                                         uint16_t *__restrict__ q16,
                                                         float *__restrict__ self_c64,
                                                         float *__restrict__ scales) {
    __shared__ float red[256];
    const int blk = blockIdx.x;  // s * np + p
    const int s = blk / g.np, p = blk - s * g.np;
    const int nb = g.nb, per = nb * nb;
    const float2 *a = src + (size_t)blk * per;
    if (p == g.self_p) {
        float *b = self_c64 + (size_t)s * per * 2;
        for (int e = threadIdx.x; e < per; e += blockDim.x) {
            int i = e / nb, j = e - i * nb;
            float2 v = a[e];
            b[c64_block_offset(nb, i, 2 * j)] = v.x;
            b[c64_block_offset(nb, i, 2 * j + 1)] = v.y;
        }
        if (threadIdx.x == 0) scales[blk] = 1.f;
        return;
    }
    float m = 0.f;
    for (int e = threadIdx.x; e < per; e += blockDim.x) {
        float2 v = a[e];
        m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    const float sc = pow2_ceil(red[0]);
    const float inv = 1.f / sc;  // exact: power of two
    uint16_t *b = q16 + (size_t)blk * per * 2;
    for (int e = threadIdx.x; e < per; e += blockDim.x) {
        int i = e / nb, j = e - i * nb;
        float2 v = a[e];
        float re = v.x * inv, im = v.y * inv;
        b[h16_block_offset(nb, i, 2 * j)] = KIND == 0 ? to_bf16_bits(re) : to_f16_bits(re);
        b[h16_block_offset(nb, i, 2 * j + 1)] = KIND == 0 ? to_bf16_bits(im) : to_f16_bits(im);
    }
    if (threadIdx.x == 0) scales[blk] = sc;
}

}  // namespace coarse

using namespace coarse;

extern "C" int32_t coarse_packed_bytes(const coarse_geom *g, int32_t link_dtype, size_t *out) {
    clear_error();
    Geom d;
    int32_t rc = make_geom(g, &d);
    if (rc) return rc;
    if (!out) {
        set_error("out is NULL");
        return CG_INVALID_ARG;
    }
    if (link_dtype == COARSE_C64) {
        *out = (size_t)d.V * d.np * d.nb * d.nb * 8;
        return CG_OK;
    }
    if (link_dtype == COARSE_C64_3M) {
        if (d.nb % 16) {
            set_error("3M links need nbasis %% 16 == 0 (got %d)", d.nb);
            return CG_UNSUPPORTED;
        }
        *out = (size_t)d.V * d.np * d.nb * d.nb * 8;
        return CG_OK;
    }
    if (link_dtype == COARSE_BF16 || link_dtype == COARSE_FP16) {
        if (d.nb % 16) {
            set_error("16-bit links need nbasis %% 16 == 0 (got %d)", d.nb);
            return CG_UNSUPPORTED;
        }
        *out = lowp_layout(d.V, d.np, d.nb, d.self_p >= 0).total;
        return CG_OK;
    }
    set_error("link_dtype %d not one of C64, C64_3M, BF16, FP16", link_dtype);
    return CG_INVALID_ARG;
}

extern "C" int32_t coarse_pack_links(const coarse_geom *g, const void *links_c64, int32_t link_dtype,
                                     void *packed, void *stream) {
    size_t bytes;
    int32_t rc = coarse_packed_bytes(g, link_dtype, &bytes);
    if (rc) return rc;
    if (!links_c64 || !packed) {
        set_error("links or packed is NULL");
        return CG_INVALID_ARG;
    }
    if (links_c64 == packed) {
        set_error("packed must not alias the source links");
        return CG_INVALID_ARG;
    }
    Geom d;
    make_geom(g, &d);
    hipStream_t st = (hipStream_t)stream;
    if (link_dtype == COARSE_C64 || link_dtype == COARSE_C64_3M) {
        size_t nblocks = (size_t)d.V * d.np;
        size_t total = nblocks * d.nb * d.nb;
        int threads = 256;
        size_t blocks = (total + threads - 1) / threads;
        if (blocks > 65536) blocks = 65536;
        if (link_dtype == COARSE_C64)
            hipLaunchKernelGGL(pack_c64_kernel, dim3((unsigned)blocks), dim3(threads), 0, st, d.nb, nblocks,
                               (const float2 *)links_c64, (float *)packed);
        else
            hipLaunchKernelGGL(pack_c64_3m_kernel, dim3((unsigned)blocks), dim3(threads), 0, st, d.nb, nblocks,
                               (const float2 *)links_c64, (float *)packed);
    } else {
        LowpLayout l = lowp_layout(d.V, d.np, d.nb, d.self_p >= 0);
        char *base = (char *)packed;
        uint16_t *q16 = (uint16_t *)base;
        float *self_c64 = (float *)(base + l.self_off);
        float *scales = (float *)(base + l.scale_off);
        dim3 grid((unsigned)(d.V * d.np));
        if (link_dtype == COARSE_BF16)
            hipLaunchKernelGGL(pack_lowp_kernel<0>, grid, dim3(256), 0, st, d, (const float2 *)links_c64, q16,
                               self_c64, scales);
        else
            hipLaunchKernelGGL(pack_lowp_kernel<1>, grid, dim3(256), 0, st, d, (const float2 *)links_c64, q16,
                               self_c64, scales);
    }
    COARSE_HIP(hipGetLastError());
    return CG_OK;
}
