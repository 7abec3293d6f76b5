// Several independent coarse systems (different lattices, nbasis and nrhs)
// applied in ONE persistent kernel launch.
//
// A device work queue hands out (system, site) items, largest link block
// first (longest-processing-time order), to a fixed grid of resident
// workgroups; each workgroup applies the whole fused stencil GEMM of one site
// (the same per-site MFMA body as the single-system kernel) and fetches the
// next item. Every workgroup leaves the loop once the queue is exhausted.
#include <algorithm>
#include <vector>

#include "apply.hpp"
#include "apply_site.hpp"

namespace coarse {

constexpr int MAX_BATCH = 8;

struct BatchSys {
    Geom g;
    const float *links;
    const float *x;
    float *y;
    int nr;
    int nt;
    int ps;          // point split: 4 / row tiles, so all four waves work
    int item_base;
    int items;
};

struct BatchArgs {
    int nsys;
    int total;
    BatchSys sys[MAX_BATCH];
};

// Workspace: [0, 256) the queue counter, then the descriptor table.
constexpr size_t DESC_OFFSET = 256;
constexpr size_t WS_BYTES = DESC_OFFSET + ((sizeof(BatchArgs) + 255) / 256) * 256;

// Publish the descriptor (a kernel argument, copied by value at launch) to the
// workspace and reset the queue: stream-ordered, so back-to-back launches on
// one workspace never see each other's tables.
__global__ void batch_setup_kernel(BatchArgs a, BatchArgs *__restrict__ desc, int *__restrict__ counter) {
    if (threadIdx.x == 0) {
        *desc = a;
        *counter = 0;
    }
}

__global__ __launch_bounds__(256) void apply_batched_kernel(const BatchArgs *__restrict__ a,
                                                             int *__restrict__ counter) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int item_s;
    const int nsys = a->nsys, total = a->total;
    for (;;) {
        if (threadIdx.x == 0) item_s = atomicAdd(counter, 1);
        __syncthreads();
        // wave-uniform: the descriptor reads below become scalar loads
        const int item = __builtin_amdgcn_readfirstlane(item_s);
        __syncthreads();
        if (item >= total) break;
        int k = 0;
        while (k + 1 < nsys && item >= a->sys[k + 1].item_base) ++k;
        const BatchSys &S = a->sys[k];
        const int site = item - S.item_base;
        const GLOBAL_AS float *links = (const GLOBAL_AS float *)S.links, *x = (const GLOBAL_AS float *)S.x;
        GLOBAL_AS float *y = (GLOBAL_AS float *)S.y;
#define SITE(NT_, PS_) site_apply_mfma<float, 0, NT_, 0, 1, PS_>(S.g, links, x, y, S.nr, nullptr, site, smem_raw)
#define BY_PS(NT_)                    \
    if (S.ps == 4)                    \
        SITE(NT_, 4);                 \
    else if (S.ps == 2)               \
        SITE(NT_, 2);                 \
    else                              \
        SITE(NT_, 1);
        switch (S.nt) {
            case 1: BY_PS(1) break;
            case 2: BY_PS(2) break;
            case 3: BY_PS(3) break;
            default: BY_PS(4) break;
        }
#undef BY_PS
#undef SITE
    }
}

static int g_cu_count = 0;

static int cu_count() {
    if (g_cu_count == 0) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            g_cu_count = n;
        else
            g_cu_count = 256;
    }
    return g_cu_count;
}

// Validate the systems and build the queue description (largest items first).
static int32_t build_batch(const coarse_system *sys, int32_t nsys, BatchArgs *out, size_t *lds) {
    if (!sys || nsys < 1 || nsys > MAX_BATCH) {
        set_error("nsys = %d out of range [1, %d]", nsys, MAX_BATCH);
        return CG_INVALID_ARG;
    }
    std::vector<int> order(nsys);
    std::vector<BatchSys> bs(nsys);
    size_t need = 0;
    for (int i = 0; i < nsys; ++i) {
        Geom d;
        int32_t rc = make_geom(&sys[i].geom, &d);
        if (rc) return rc;
        if ((rc = check_nrhs(sys[i].nrhs))) return rc;
        if (!tiled_c64(d.nb)) {
            set_error("batched apply needs nbasis %% 8 == 0 (system %d has %d)", i, d.nb);
            return CG_UNSUPPORTED;
        }
        if (!sys[i].packed || !sys[i].x || !sys[i].y || sys[i].x == sys[i].y) {
            set_error("system %d: NULL or aliased pointers", i);
            return CG_INVALID_ARG;
        }
        bs[i].g = d;
        bs[i].links = (const float *)sys[i].packed;
        bs[i].x = (const float *)sys[i].x;
        bs[i].y = (float *)sys[i].y;
        bs[i].nr = sys[i].nrhs;
        bs[i].nt = (2 * sys[i].nrhs + 15) / 16;
        const int nmt = (d.nb + 15) / 16;
        bs[i].ps = nmt == 1 ? 4 : (nmt == 2 ? 2 : 1);
        bs[i].items = d.V;
        // every group of 64 * nmt threads stages a whole neighbour block (PS == 1: all 256 threads)
        const int group = bs[i].ps == 1 ? 256 : 64 * nmt;
        const bool fits = bs[i].nt == 1   ? site_apply_staging_fits<float, 1>(d.nb, bs[i].nr, group)
                          : bs[i].nt == 2 ? site_apply_staging_fits<float, 2>(d.nb, bs[i].nr, group)
                          : bs[i].nt == 3 ? site_apply_staging_fits<float, 3>(d.nb, bs[i].nr, group)
                                          : site_apply_staging_fits<float, 4>(d.nb, bs[i].nr, group);
        if (!fits) {
            set_error("system %d: nbasis %d, nrhs %d exceed the staging bound", i, d.nb, bs[i].nr);
            return CG_UNSUPPORTED;
        }
        need = std::max(need, site_apply_lds_elems(d.nb, sys[i].nrhs, bs[i].ps) * sizeof(float));
        order[i] = i;
    }
    // longest items first: link bytes per site, then nrhs
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const long long ca = (long long)bs[a].g.np * bs[a].g.nb * bs[a].g.nb, cb = (long long)bs[b].g.np * bs[b].g.nb * bs[b].g.nb;
        if (ca != cb) return ca > cb;
        return bs[a].nr > bs[b].nr;
    });
    out->nsys = nsys;
    int base = 0;
    for (int k = 0; k < nsys; ++k) {
        out->sys[k] = bs[order[k]];
        out->sys[k].item_base = base;
        base += out->sys[k].items;
    }
    out->total = base;
    *lds = need;
    return CG_OK;
}

int32_t launch_batched(const BatchArgs &a, size_t lds, int *counter, int wg_per_cu, hipStream_t st) {
    BatchArgs *desc = reinterpret_cast<BatchArgs *>(reinterpret_cast<char *>(counter) + DESC_OFFSET);
    hipLaunchKernelGGL(batch_setup_kernel, dim3(1), dim3(64), 0, st, a, desc, counter);
    const int grid = cu_count() * wg_per_cu;
    hipLaunchKernelGGL(apply_batched_kernel, dim3(grid), dim3(256), lds, st, desc, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "batched apply launch");
    return CG_OK;
}

}  // namespace coarse

using namespace coarse;

extern "C" int32_t coarse_batched_workspace_bytes(const coarse_system *sys, int32_t nsys, size_t *out) {
    clear_error();
    BatchArgs a;
    size_t lds;
    int32_t rc = build_batch(sys, nsys, &a, &lds);
    if (rc) return rc;
    if (!out) {
        set_error("out is NULL");
        return CG_INVALID_ARG;
    }
    *out = WS_BYTES;  // queue counter + descriptor table
    return CG_OK;
}

static int g_wg_per_cu = 4;

// Workgroups per CU of the persistent grid (the autotuner's knob); 0 keeps the current value.
extern "C" int32_t coarse_batched_set_occupancy(int32_t wg_per_cu) {
    if (wg_per_cu < 0 || wg_per_cu > 16) {
        set_error("wg_per_cu = %d out of range [0, 16]", wg_per_cu);
        return CG_INVALID_ARG;
    }
    if (wg_per_cu > 0) g_wg_per_cu = wg_per_cu;
    return g_wg_per_cu;
}

extern "C" int32_t coarse_apply_batched(const coarse_system *sys, int32_t nsys, void *ws, size_t ws_bytes,
                                        void *stream) {
    clear_error();
    BatchArgs a;
    size_t lds;
    int32_t rc = build_batch(sys, nsys, &a, &lds);
    if (rc) return rc;
    if (!ws) {
        set_error("ws is NULL");
        return CG_INVALID_ARG;
    }
    if (ws_bytes < WS_BYTES) {
        set_error("workspace %zu bytes, need %zu", ws_bytes, WS_BYTES);
        return CG_WORKSPACE_TOO_SMALL;
    }
    return launch_batched(a, lds, (int *)ws, g_wg_per_cu, (hipStream_t)stream);
}
