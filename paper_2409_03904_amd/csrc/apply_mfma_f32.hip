// float32 MFMA coarse apply: instantiations and launcher.
#include "apply.hpp"
#include "apply_site.hpp"

namespace coarse {

// XCD-aware site order: sites of one XCD form a contiguous slab (workgroups
// are dealt round-robin to the 8 XCDs), so a slab's neighbour blocks stay in
// that XCD's L2.
__device__ __forceinline__ int site_of_block(int b, int V) {
    return (V % 8 == 0) ? ((b & 7) * (V >> 3) + (b >> 3)) : b;
}

// One coarse site per workgroup.
template <typename T, int NR, int NT, int NCH, int PD, int PS>
__global__ __launch_bounds__(256) void apply_mfma_kernel(Geom g, const float *__restrict__ links,
                                                          const T *__restrict__ x, T *__restrict__ y, int nr,
                                                          const T *__restrict__ sub,
                                                          const int *__restrict__ active) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (active != nullptr && *active == 0) return;
    site_apply_mfma<T, NR, NT, NCH, PD, PS>(g, (const GLOBAL_AS float *)links, (const GLOBAL_AS T *)x,
                                            (GLOBAL_AS T *)y, nr, (const GLOBAL_AS T *)sub,
                                            site_of_block(blockIdx.x, g.V), smem_raw);
}

template <typename T, int NR, int NT, int NCH, int PS, int PD = 2>
static bool launch_one(const Geom &g, const float *links, const T *x, T *y, int nr, const T *sub, const int *active,
                       hipStream_t st) {
    const int waves = (g.nb + 15) / 16;
    if (!site_apply_staging_fits<T, NT>(g.nb, nr, 64 * waves)) {
        set_error("apply: nbasis %d, nrhs %d exceed the staging bound of the selected kernel", g.nb, nr);
        return false;
    }
    const size_t lds = site_apply_lds_elems<T>(g.nb, nr, PS) * sizeof(T);
    if (lds > 64 * 1024) {  // complex128 staging at large nbasis * nrhs: up to 128 KB of the 160 KB
        static size_t granted = 64 * 1024;
        if (lds > granted) {
            (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&apply_mfma_kernel<T, NR, NT, NCH, PD, PS>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            granted = lds;
        }
    }
    hipLaunchKernelGGL((apply_mfma_kernel<T, NR, NT, NCH, PD, PS>), dim3(g.V), dim3(64 * waves * PS), lds, st, g,
                       links, x, y, nr, sub, active);
    return true;
}

// compile-time chunk count for the workload shapes' nbasis (8, 24, 32, 48, 64), runtime otherwise
template <typename T, int NR, int NT, int PS, int PD = 2>
static bool launch_nch(const Geom &g, const float *links, const T *x, T *y, int nr, const T *sub, const int *active,
                       hipStream_t st) {
    switch (g.nb >> 3) {
        case 1: return launch_one<T, NR, NT, 1, PS, PD>(g, links, x, y, nr, sub, active, st);
        case 3: return launch_one<T, NR, NT, 3, PS, PD>(g, links, x, y, nr, sub, active, st);
        case 4: return launch_one<T, NR, NT, 4, PS, PD>(g, links, x, y, nr, sub, active, st);
        case 6: return launch_one<T, NR, NT, 6, PS, PD>(g, links, x, y, nr, sub, active, st);
        case 8: return launch_one<T, NR, NT, 8, PS, PD>(g, links, x, y, nr, sub, active, st);
        default: return launch_one<T, NR, NT, 0, PS, PD>(g, links, x, y, nr, sub, active, st);
    }
}

template <int NR, int NT>
static bool launch_ps(const Geom &g, const float *links, const float *x, float *y, int nr, const float *sub,
                      const int *active, hipStream_t st, int variant) {
    // variants 0 .. max_variant(nb): point split 1, 2, 4 with two points of
    // link prefetch (the split needs PS * 64 * ceil(nb/16) <= 256); variant
    // max_variant(nb) + 1: no split, one point of prefetch (fewer registers,
    // more waves per SIMD)
    if (variant == max_variant(g.nb) + 1) return launch_nch<float, NR, NT, 1, 1>(g, links, x, y, nr, sub, active, st);
    if (variant >= 2 && g.nb <= 16) {
        return launch_nch<float, NR, NT, 4>(g, links, x, y, nr, sub, active, st);
    } else if (variant >= 1 && g.nb <= 32) {
        return launch_nch<float, NR, NT, 2>(g, links, x, y, nr, sub, active, st);
    } else {
        return launch_nch<float, NR, NT, 1>(g, links, x, y, nr, sub, active, st);
    }
}

bool launch_mfma_f32(const Geom &g, const float *links, const float *x, float *y, int nr, const float *sub,
                     const int *active, hipStream_t st, int variant) {
    switch (nr) {
        case 4: return launch_ps<4, 1>(g, links, x, y, nr, sub, active, st, variant);
        case 8: return launch_ps<8, 1>(g, links, x, y, nr, sub, active, st, variant);
        case 16: return launch_ps<16, 2>(g, links, x, y, nr, sub, active, st, variant);
        case 32: return launch_ps<32, 4>(g, links, x, y, nr, sub, active, st, variant);
        default: break;
    }
    switch ((2 * nr + 15) / 16) {
        case 1: return launch_nch<float, 0, 1, 1>(g, links, x, y, nr, sub, active, st);
        case 2: return launch_nch<float, 0, 2, 1>(g, links, x, y, nr, sub, active, st);
        case 3: return launch_nch<float, 0, 3, 1>(g, links, x, y, nr, sub, active, st);
        default: return launch_nch<float, 0, 4, 1>(g, links, x, y, nr, sub, active, st);
    }
}

}  // namespace coarse
