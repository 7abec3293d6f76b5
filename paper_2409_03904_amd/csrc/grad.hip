// Link gradient of a real loss through y = M x:
//   dA_p(x) (+)= alpha * G(x) . X(x + delta_p)^H,
// an nb x nb block per (site, point), each the sum over the nrhs columns of
// outer products (K = nrhs). The two operand blocks are staged in LDS once per
// workgroup; the output is written once, coalesced, in the public layout.
#include "common.hpp"

namespace coarse {

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
    float2 *gs = reinterpret_cast<float2 *>(smem_raw);  // [nb][nr]
    float2 *xs = gs + nb * nr;                           // [nb][nr]
    const float2 *gsrc = gy + (size_t)s * nb * nr;
    const float2 *xsrc = x + (size_t)z * nb * nr;
    for (int e = threadIdx.x; e < nb * nr; e += blockDim.x) {
        gs[e] = gsrc[e];
        xs[e] = xsrc[e];
    }
    __syncthreads();
    float2 *out = dl + (size_t)blk * nb * nb;
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
        const int i = e / nb, j = e - i * nb;
        float re = 0.f, im = 0.f;
        for (int r = 0; r < nr; ++r) {
            const float2 a = gs[i * nr + r], b = xs[j * nr + r];
            // a * conj(b)
            re += a.x * b.x + a.y * b.y;
            im += a.y * b.x - a.x * b.y;
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
    const size_t lds = (size_t)2 * d.nb * nrhs * sizeof(float2);
    hipLaunchKernelGGL(link_grad_kernel, dim3((unsigned)(d.V * d.np)), dim3(256), lds, (hipStream_t)stream, d,
                       (const float2 *)gy, (const float2 *)x, (float2 *)dlinks, alpha, accumulate, nrhs);
    COARSE_HIP(hipGetLastError());
    return CG_OK;
}
