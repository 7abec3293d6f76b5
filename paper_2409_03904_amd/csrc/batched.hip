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
    int waves;    // waves per workgroup of the persistent grid
    int generic;  // some nrhs not in {4, 8, 16, 32}: runtime-nrhs bodies
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

// One kernel per body family: the compile-time-nrhs bodies (nrhs 4, 8, 16, 32)
// keep every LDS offset an immediate and the register budget low; the
// runtime-nrhs bodies (any nrhs) live in their own kernel so that they do not
// set the budget of the first.
template <bool GENERIC>
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
#define SITE(NR_, NT_, NCH_, PS_) \
    site_apply_mfma<float, NR_, NT_, NCH_, 1, PS_>(S.g, links, x, y, S.nr, nullptr, site, smem_raw)
#define BY_PS(NR_, NT_)               \
    if (S.ps == 4)                    \
        SITE(NR_, NT_, 0, 4);         \
    else if (S.ps == 2)               \
        SITE(NR_, NT_, 0, 2);         \
    else                              \
        SITE(NR_, NT_, 0, 1);
        // fixed-shape bodies: nbasis 24 / 32 (two row tiles, split 1 or 2) and
        // 48 (three row tiles, no split), nrhs 4, 8, 16, 32
#define BY_NCH(NR_, NT_)                                        \
    switch (S.g.nb >> 3) {                                      \
        case 3:                                                 \
            if (S.ps == 2) SITE(NR_, NT_, 3, 2);                \
            else SITE(NR_, NT_, 3, 1);                          \
            break;                                              \
        case 4:                                                 \
            if (S.ps == 2) SITE(NR_, NT_, 4, 2);                \
            else SITE(NR_, NT_, 4, 1);                          \
            break;                                              \
        default: SITE(NR_, NT_, 6, 1); break;                   \
    }
        if (GENERIC) {
            switch (S.nt) {
                case 1: BY_PS(0, 1) break;
                case 2: BY_PS(0, 2) break;
                case 3: BY_PS(0, 3) break;
                default: BY_PS(0, 4) break;
            }
        } else {
            switch (S.nr) {
                case 4: BY_NCH(4, 1) break;
                case 8: BY_NCH(8, 1) break;
                case 16: BY_NCH(16, 2) break;
                default: BY_NCH(32, 4) break;
            }
        }
#undef BY_NCH
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
        bs[i].items = d.V;
        order[i] = i;
    }
    // Waves per workgroup: the choice with the fewest byte-weighted idle waves.
    // A system with nmt row tiles splits its points over ps = waves / nmt groups
    // when that is 1, 2 or 4 (every wave busy); otherwise ps = 1 and the extra
    // waves only help staging.
    auto split = [](int waves, int nmt) {
        const int q = waves / nmt;
        return (waves % nmt == 0 && (q == 1 || q == 2 || q == 4)) ? q : 1;
    };
    int max_nmt = 1;
    for (int i = 0; i < nsys; ++i) max_nmt = std::max(max_nmt, (bs[i].g.nb + 15) / 16);
    int best_w = 4;
    double best_cost = 1e300;
    for (int wv = max_nmt; wv <= 4; ++wv) {
        double cost = 0;
        for (int i = 0; i < nsys; ++i) {
            const int nmt = (bs[i].g.nb + 15) / 16;
            const double bytes = (double)bs[i].items * bs[i].g.np * bs[i].g.nb * bs[i].g.nb;
            cost += bytes * wv / (double)(split(wv, nmt) * nmt);
        }
        if (cost <= best_cost * (1 + 1e-12)) {  // ties: the larger workgroup (the grid counts workgroups)
            best_cost = std::min(best_cost, cost);
            best_w = wv;
        }
    }
    out->waves = best_w;
    out->generic = 0;
    for (int i = 0; i < nsys; ++i) {
        const Geom &d = bs[i].g;
        const int nmt = (d.nb + 15) / 16;
        bs[i].ps = split(best_w, nmt);
        const int nr = bs[i].nr;
        // the fixed-shape kernel covers nrhs 4/8/16/32 with nbasis 24 or 32
        // (split 1 or 2) or 48 (no split); anything else takes the generic one
        const bool fixed_nr = nr == 4 || nr == 8 || nr == 16 || nr == 32;
        const bool fixed_nb = ((d.nb == 24 || d.nb == 32) && bs[i].ps <= 2) || (d.nb == 48 && bs[i].ps == 1);
        if (!fixed_nr || !fixed_nb) out->generic = 1;
        // every group of 64 * nmt threads stages a whole neighbour block (PS == 1: the whole workgroup)
        const int group = bs[i].ps == 1 ? 64 * best_w : 64 * nmt;
        const bool fits = bs[i].nt == 1   ? site_apply_staging_fits<float, 1>(d.nb, bs[i].nr, group)
                          : bs[i].nt == 2 ? site_apply_staging_fits<float, 2>(d.nb, bs[i].nr, group)
                          : bs[i].nt == 3 ? site_apply_staging_fits<float, 3>(d.nb, bs[i].nr, group)
                                          : site_apply_staging_fits<float, 4>(d.nb, bs[i].nr, group);
        if (!fits) {
            set_error("system %d: nbasis %d, nrhs %d exceed the staging bound", i, d.nb, bs[i].nr);
            return CG_UNSUPPORTED;
        }
        need = std::max(need, site_apply_lds_elems<float>(d.nb, sys[i].nrhs, bs[i].ps) * sizeof(float));
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
    if (lds > 64 * 1024) {
        static size_t granted[2] = {64 * 1024, 64 * 1024};
        const void *fn = a.generic ? reinterpret_cast<const void *>(&apply_batched_kernel<true>)
                                   : reinterpret_cast<const void *>(&apply_batched_kernel<false>);
        if (lds > granted[a.generic]) {
            (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            granted[a.generic] = lds;
        }
    }
    if (a.generic)
        hipLaunchKernelGGL(apply_batched_kernel<true>, dim3(grid), dim3(64 * a.waves), lds, st, desc, counter);
    else
        hipLaunchKernelGGL(apply_batched_kernel<false>, dim3(grid), dim3(64 * a.waves), lds, st, desc, counter);
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
