// Host-side argument validation and error text of the C ABI.
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "common.hpp"

namespace coarse {

static thread_local char g_last_error[512] = {0};

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
}

void clear_error() { g_last_error[0] = 0; }

int32_t hip_fail(hipError_t e, const char *what) {
    set_error("%s failed: %s", what, hipGetErrorString(e));
    return CG_HIP_ERROR;
}

int32_t make_geom(const coarse_geom *g, Geom *out) {
    if (!g) {
        set_error("geometry is NULL");
        return CG_INVALID_ARG;
    }
    long long V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (g->dims[mu] < 1 || g->dims[mu] > 4096) {
            set_error("dims[%d] = %d out of range [1, 4096]", mu, g->dims[mu]);
            return CG_INVALID_ARG;
        }
        V *= g->dims[mu];
    }
    if (V > (1LL << 26)) {
        set_error("volume %lld too large", V);
        return CG_INVALID_ARG;
    }
    if (g->nbasis < 1 || g->nbasis > 64) {
        set_error("nbasis = %d out of range [1, 64]", g->nbasis);
        return CG_INVALID_ARG;
    }
    if (g->npoint < 1 || g->npoint > 81) {
        set_error("npoint = %d out of range [1, 81]", g->npoint);
        return CG_INVALID_ARG;
    }
    if (!g->offsets) {
        set_error("offsets is NULL");
        return CG_INVALID_ARG;
    }
    Geom d;
    memset(&d, 0, sizeof(d));
    bool seen[81] = {false};
    d.self_p = -1;
    for (int p = 0; p < g->npoint; ++p) {
        int canon = 0, mul = 1;
        for (int mu = 0; mu < 4; ++mu) {
            int v = g->offsets[4 * p + mu];
            if (v < -1 || v > 1) {
                set_error("offset %d component %d = %d not in {-1,0,1}", p, mu, v);
                return CG_INVALID_ARG;
            }
            d.off[p][mu] = (int8_t)v;
            canon += mul * (v + 1);
            mul *= 3;
        }
        if (seen[canon]) {
            set_error("offset %d repeats an earlier displacement", p);
            return CG_INVALID_ARG;
        }
        seen[canon] = true;
        if (canon == 40) d.self_p = p;
    }
    for (int mu = 0; mu < 4; ++mu) d.L[mu] = g->dims[mu];
    d.V = (int)V;
    d.nb = g->nbasis;
    d.np = g->npoint;
    *out = d;
    return CG_OK;
}

int32_t check_nrhs(int32_t nrhs) {
    if (nrhs < 1 || nrhs > 32) {
        set_error("nrhs = %d out of range [1, 32]", nrhs);
        return CG_INVALID_ARG;
    }
    return CG_OK;
}

}  // namespace coarse

using namespace coarse;

extern "C" const char *cg_status_string(int32_t status) {
    switch (status) {
        case CG_OK: return "ok";
        case CG_NOT_CONVERGED: return "not converged";
        case CG_INVALID_ARG: return "invalid argument";
        case CG_UNSUPPORTED: return "unsupported shape or type";
        case CG_HIP_ERROR: return "HIP error";
        case CG_BREAKDOWN: return "block breakdown (Gram matrix not positive definite)";
        case CG_NONFINITE: return "non-finite value";
        case CG_WORKSPACE_TOO_SMALL: return "workspace too small";
        default: return "unknown status";
    }
}

extern "C" const char *cg_last_error(void) { return g_last_error; }
