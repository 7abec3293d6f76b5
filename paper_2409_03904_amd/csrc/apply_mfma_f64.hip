// float64-accumulation MFMA coarse apply (complex128 vectors, exact float->double
// links; the residual of the outer defect-correction loop): instantiations and launcher.
#include "apply.hpp"
#include "apply_site.hpp"

namespace coarse {

// XCD-aware site order: sites of one XCD form a contiguous slab (workgroups
// are dealt round-robin to the 8 XCDs), so a slab's neighbour blocks stay in
// that XCD's L2.
__device__ __forceinline__ int site_of_block(int b, int V) {
    return (V % 8 == 0) ? ((b & 7) * (V >> 3) + (b >> 3)) : b;
}

// One coarse site per workgroup, two workgroups per CU asked of the compiler
// (with X staged without its conjugate they fit the LDS at nbasis 64,
// nrhs 32; left to itself the compiler gives that instance 285 registers and
// one wave per SIMD, and its f64 MFMA chains then stall).
template <typename T, int NR, int NT, int NCH, int PD, int PS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void apply_mfma_kernel(Geom g, const float *__restrict__ links,
                                                          const T *__restrict__ x, T *__restrict__ y, int nr,
                                                          const T *__restrict__ sub,
                                                          const int *__restrict__ active) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (active != nullptr && *active == 0) return;
    site_apply_mfma<T, NR, NT, NCH, PD, PS>(g, (const GLOBAL_AS float *)links, (const GLOBAL_AS T *)x,
                                            (GLOBAL_AS T *)y, nr, (const GLOBAL_AS T *)sub,
                                            site_of_block(blockIdx.x, g.V), smem_raw);
}

template <typename T, int NR, int NT, int NCH, int PS>
static bool launch_one(const Geom &g, const float *links, const T *x, T *y, int nr, const T *sub, const int *active,
                       hipStream_t st) {
    constexpr int PD = 1;  // 2-slot ring
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
template <typename T, int NR, int NT, int PS>
static bool launch_nch(const Geom &g, const float *links, const T *x, T *y, int nr, const T *sub, const int *active,
                       hipStream_t st) {
    switch (g.nb >> 3) {
        case 1: return launch_one<T, NR, NT, 1, PS>(g, links, x, y, nr, sub, active, st);
        case 3: return launch_one<T, NR, NT, 3, PS>(g, links, x, y, nr, sub, active, st);
        case 4: return launch_one<T, NR, NT, 4, PS>(g, links, x, y, nr, sub, active, st);
        case 6: return launch_one<T, NR, NT, 6, PS>(g, links, x, y, nr, sub, active, st);
        case 8: return launch_one<T, NR, NT, 8, PS>(g, links, x, y, nr, sub, active, st);
        default: return launch_one<T, NR, NT, 0, PS>(g, links, x, y, nr, sub, active, st);
    }
}

bool launch_mfma_f64(const Geom &g, const float *links, const double *x, double *y, int nr, const double *sub,
                     const int *active, hipStream_t st) {
    switch ((2 * nr + 15) / 16) {
        case 1: return launch_nch<double, 0, 1, 1>(g, links, x, y, nr, sub, active, st);
        case 2: return launch_nch<double, 0, 2, 1>(g, links, x, y, nr, sub, active, st);
        case 3: return launch_nch<double, 0, 3, 1>(g, links, x, y, nr, sub, active, st);
        default: return launch_nch<double, 0, 4, 1>(g, links, x, y, nr, sub, active, st);
    }
}

}  // namespace coarse
