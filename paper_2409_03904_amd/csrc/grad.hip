// Link gradient of a real loss through y = M x:
//   dA_p(x) (+)= alpha * G(x) . X(x + delta_p)^H,
// an nb x nb block per (site, point), each the sum over the nrhs columns of
// outer products (K = nrhs).
//
// MFMA form (nbasis % 16 == 0): one workgroup per site, one wave per 16-row
// tile of the output. In the 4M real embedding with k' = 2r + h and output
// column n' = 2j + part,
//   A[i][k']        = component h of G[i][r]                 (fixed per site)
//   B[k'][2j]       = component h of X[j][r]                 (Re-part column)
//   B[k'][2j + 1]   = component 1-h of conj(X[j][r])         (Im-part column)
// so D[i][2j] = Re dA[i][j] and D[i][2j+1] = Im dA[i][j]: the columns are
// already the interleaved complex64 public layout. The MFMA is issued with
// its two operands exchanged, which yields the transposed tile, so each lane
// holds four consecutive columns of one row and stores them at once. G's row tile sits in registers for all points; each neighbour
// block X(x + delta_p) and its conjugate are staged once in LDS (row stride
// padded against bank conflicts), the next one prefetched into registers.
// The output (the dominant traffic) is written once per entry.
//
// VALU form (other nbasis): one workgroup per (site, point), thread per
// output entry, operands in LDS with a padded row stride.
#include "common.hpp"

namespace coarse {

namespace {

// padded LDS row stride (floats) of an nr-column complex block: keeps float2
// alignment and spreads consecutive rows over the banks
__host__ __device__ inline int grad_row_stride(int nr) { return 2 * nr + 4; }

}  // namespace

template <int KS>
__global__ __launch_bounds__(256) void link_grad_mfma_kernel(Geom g, const float2 *__restrict__ gy,
                                                             const float2 *__restrict__ x, float *__restrict__ dl,
                                                             float alpha, int accumulate, int nr) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int nb = g.nb, np = g.np;
    const int s = blockIdx.x;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int w = tid >> 6, t = tid & 63, c = t & 15, q = t >> 4;
    const int rs = grad_row_stride(nr);
    LDS_AS float *xp = lds_ptr<float>(smem_raw);  // X(z), padded rows
    LDS_AS float *xc = xp + nb * rs + 2;          // conj X(z), two banks over from xp's rows
    const int nto = nb / 8;                        // 16-column output tiles (2 nb real columns)

    // A operand: lane (row c, k-group q) of the wave's 16 rows, step st: k' = 4 st + q
    float a[KS];
    {
        const float *grow = reinterpret_cast<const float *>(gy + ((size_t)s * nb + 16 * w + c) * nr);
#pragma unroll
        for (int st = 0; st < KS; ++st) {
            const int k = 4 * st + q;
            a[st] = (k < 2 * nr) ? grow[k] : 0.f;  // component k & 1 of G[i][k >> 1]
        }
    }
    int cs[4];
    site_coords(g, s, cs);

    const int nel = nb * nr;                       // complex elements of a block
    const int per = (nel + nthr - 1) / nthr;       // <= 8
    float2 pre[8];
    auto load_x = [&](int p) {
        const float2 *src = x + (size_t)displaced(g, cs, p, 1) * nel;
#pragma unroll
        for (int k = 0; k < 8; ++k) pre[k] = src[min(tid + k * nthr, nel - 1)];
    };
    auto store_x = [&]() {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int e = tid + k * nthr;
            if (k < per && e < nel) {
                const int j = e / nr, r = e - j * nr;
                const float2 v = pre[k];
                LDS_AS float *dp = xp + j * rs + 2 * r, *dc = xc + j * rs + 2 * r;
                dp[0] = v.x;
                dp[1] = v.y;
                dc[0] = v.x;
                dc[1] = -v.y;
            }
        }
    };

    load_x(0);
    for (int p = 0; p < np; ++p) {
        store_x();
        __syncthreads();
        if (p + 1 < np) load_x(p + 1);
        float *out = dl + ((size_t)s * np + p) * nb * nb * 2 + (size_t)(16 * w + c) * (2 * nb);
        for (int nt = 0; nt < nto; ++nt) {
            // X-side lane (column c, k-group q): n' = 16 nt + c -> j = 8 nt + c/2, part = c & 1
            const int j = 8 * nt + (c >> 1), part = c & 1;
            const LDS_AS float *brow = (part ? xc : xp) + j * rs;
            f32x4 acc = f32x4{0, 0, 0, 0};
#pragma unroll
            for (int st = 0; st < KS; ++st) {
                const int k = 4 * st + q;
                const int kk = part ? (k ^ 1) : k;  // Im column takes component 1 - h of conj X
                const float b = (k < 2 * nr) ? brow[kk] : 0.f;
                // operands swapped: the MFMA forms the transposed tile, so lane
                // (c, q) holds row c, columns 16 nt + 4q .. + 3 -- (Re, Im) of
                // two consecutive dA entries, one 16-byte store
                acc = mfma16x16x4(b, a[st], acc);
            }
            f32x4 val = f32x4{alpha * acc[0], alpha * acc[1], alpha * acc[2], alpha * acc[3]};
            f32x4 *o = reinterpret_cast<f32x4 *>(out + 16 * nt + 4 * q);
            if (accumulate) val += *o;
            *o = val;
        }
        __syncthreads();
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
        switch ((2 * nrhs + 3) / 4) {  // k' steps of 4
#define GL(KS_)                                                                                                 \
    case KS_:                                                                                                   \
        hipLaunchKernelGGL(link_grad_mfma_kernel<KS_>, grid, block, lds, st, d, (const float2 *)gy,            \
                           (const float2 *)x, (float *)dlinks, alpha, accumulate, nrhs);                        \
        break;
            GL(1) GL(2) GL(3) GL(4) GL(5) GL(6) GL(7) GL(8) GL(9) GL(10) GL(11) GL(12) GL(13) GL(14) GL(15) GL(16)
#undef GL
            default: break;
        }
    } else {
        hipLaunchKernelGGL(link_grad_kernel, dim3((unsigned)(d.V * d.np)), dim3(256), lds, st, d,
                           (const float2 *)gy, (const float2 *)x, (float2 *)dlinks, alpha, accumulate, nrhs);
    }
    COARSE_HIP(hipGetLastError());
    return CG_OK;
}
