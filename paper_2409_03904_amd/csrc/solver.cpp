// Block-CG solve of M X = B: double precision defect correction around
// BlockCGrQ (Fig. 2, left) run in single (or 16-bit link) precision.
//
// Per outer cycle, in double: R = B - M X (complex64 links, double
// accumulation), column norms from the diagonal of R^H R, stop test,
// R^ = R diag(1/||r_j||) rounded to complex64.
// Inner BlockCGrQ from E = 0 on M~, every Gram accumulated in double and
// every small step in double on the device:
//   Q_0 C_0 = R^;  D_0 = Q_0;
//   Z = M~ D;  N = (D^H Z)^{-1};  E += D (N C);  T = Q - Z N;
//   S^H S = T^H T;  Q = T S^{-1};  D = Q + D S^H;  C = S C.
// (The figure's iterate update omits C_k; with R_k = Q_k C_k the step that
// zeroes D_k^H R_{k+1} is D_k N_k C_k.) Residual norms ||C e_j|| come free
// from C. The iteration sequence is captured once into a hipGraph of
// `check_every` iterations and replayed; a device flag turns the remaining
// kernels of a replay into no-ops once the inner tolerance, the iteration
// limit or a breakdown is reached, and the host reads the flag between
// replays (the only device-to-host synchronisation of the inner loop).
// Then X += E diag(||r_j||) in double.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "apply.hpp"
#include "blas.hpp"

namespace coarse {

struct Workspace {
    double2 *r128;     // outer residual
    float2 *e, *d, *z, *q;
    double2 *partials;
    double2 *g_res, *g_b;  // Gram of the outer residual and of B (diagonals used)
    SmallMats m;
    SolverState *state;
    void *lowp;        // prepared 16-bit input operands of the two-pass 16-bit apply
    size_t bytes;
};

static size_t carve(char *base, size_t off, size_t bytes, void **out) {
    off = align256(off);
    if (out) *out = base ? base + off : nullptr;
    return off + bytes;
}

static size_t layout_ws(char *base, const Geom &g, int nr, Workspace *w) {
    const long long rows = (long long)g.V * g.nb;
    size_t off = 0;
    const size_t v128 = (size_t)rows * nr * 16, v64 = (size_t)rows * nr * 8, sm = (size_t)nr * nr;
    off = carve(base, off, v128, (void **)&w->r128);
    off = carve(base, off, v64, (void **)&w->e);
    off = carve(base, off, v64, (void **)&w->d);
    off = carve(base, off, v64, (void **)&w->z);
    off = carve(base, off, v64, (void **)&w->q);
    off = carve(base, off, (size_t)GRAM_BLOCKS * sm * 16, (void **)&w->partials);
    off = carve(base, off, sm * 16, (void **)&w->g_res);
    off = carve(base, off, sm * 16, (void **)&w->g_b);
    off = carve(base, off, sm * 16, (void **)&w->m.G);
    off = carve(base, off, sm * 16, (void **)&w->m.C);
    off = carve(base, off, sm * 8, (void **)&w->m.W);
    off = carve(base, off, sm * 8, (void **)&w->m.N);
    off = carve(base, off, sm * 8, (void **)&w->m.Sinv);
    off = carve(base, off, sm * 8, (void **)&w->m.SH);
    off = carve(base, off, sizeof(SolverState), (void **)&w->state);
    off = carve(base, off, g.nb % 16 == 0 ? lowp_ws_bytes(g, nr) : 0, &w->lowp);
    w->m.partials = w->partials;
    w->bytes = align256(off);
    return w->bytes;
}

static int32_t check_params(const cg_solve_params *p) {
    if (!p) {
        set_error("params is NULL");
        return CG_INVALID_ARG;
    }
    if (!(p->tol > 0) || !(p->inner_tol > 0) || p->max_outer < 0 || p->max_inner < 1 || p->check_every < 1 ||
        p->check_every > 1000) {
        set_error("invalid solver parameters (tol %g, inner_tol %g, max_outer %d, max_inner %d, check_every %d)", p->tol,
                  p->inner_tol, p->max_outer, p->max_inner, p->check_every);
        return CG_INVALID_ARG;
    }
    return CG_OK;
}

// One inner iteration's launches (all no-ops once state->active == 0).
static int32_t inner_iteration(const Geom &g, const void *packed, int32_t dtype, Workspace &w, long long rows, int nr,
                               hipStream_t st) {
    const int *active = &w.state->active;
    const bool lowp = dtype == COARSE_BF16 || dtype == COARSE_FP16;
    int32_t rc = launch_apply(g, packed, dtype, w.d, w.z, nr, COARSE_C64, nullptr, active, st, 0, -1,
                              lowp ? w.lowp : nullptr);
    if (rc) return rc;
    if (blas_mfma_supported(nr)) {
        gram_mfma(w.d, w.z, rows, nr, w.partials, w.m.G, active, st);
        small_step1(w.m, w.state, nr, st);
        update_xt_gram_mfma(w.e, w.q, w.d, w.z, w.m.W, w.m.N, rows, nr, w.partials, w.m.G, active, st);
        small_step2(w.m, w.state, nr, st);
        update_qd_mfma(w.q, w.d, w.m.Sinv, w.m.SH, rows, nr, 0, active, st);
    } else {
        gram<float2>(w.d, w.z, rows, nr, w.partials, w.m.G, active, st);
        small_step1(w.m, w.state, nr, st);
        update_xt(w.e, w.q, w.d, w.z, w.m.W, w.m.N, rows, nr, active, st);
        gram<float2>(w.q, w.q, rows, nr, w.partials, w.m.G, active, st);
        small_step2(w.m, w.state, nr, st);
        update_qd(w.q, w.d, w.m.Sinv, w.m.SH, rows, nr, 0, active, st);
    }
    return CG_OK;
}

static double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace coarse

using namespace coarse;

extern "C" int32_t coarse_bcg_workspace_bytes(const coarse_geom *g, int32_t nrhs, const cg_solve_params *p,
                                              size_t *out) {
    clear_error();
    Geom d;
    int32_t rc = make_geom(g, &d);
    if (rc) return rc;
    if ((rc = check_nrhs(nrhs))) return rc;
    (void)p;
    if (!out) {
        set_error("out is NULL");
        return CG_INVALID_ARG;
    }
    Workspace w;
    *out = layout_ws(nullptr, d, nrhs, &w);
    return CG_OK;
}

extern "C" int32_t coarse_bcg_solve(const coarse_geom *g, const void *packed_outer, const void *packed_inner,
                                    int32_t inner_dtype, const void *b, void *x, int32_t nrhs,
                                    const cg_solve_params *p, cg_solve_stats *st_out, void *ws, size_t ws_bytes,
                                    void *stream) {
    clear_error();
    cg_solve_stats stats;
    memset(&stats, 0, sizeof(stats));
    stats.nrhs = nrhs;
    auto finish = [&](int32_t rc) {
        stats.status = rc;
        if (st_out) *st_out = stats;
        return rc;
    };
    Geom d;
    int32_t rc = make_geom(g, &d);
    if (rc) return finish(rc);
    if ((rc = check_nrhs(nrhs))) return finish(rc);
    if ((rc = check_params(p))) return finish(rc);
    if (!packed_outer || !b || !x || !ws) {
        set_error("packed_outer, b, x or ws is NULL");
        return finish(CG_INVALID_ARG);
    }
    if (b == x || x == packed_outer || b == packed_outer) {
        set_error("b, x and the links must not alias");
        return finish(CG_INVALID_ARG);
    }
    if (!packed_inner) {
        packed_inner = packed_outer;
        inner_dtype = COARSE_C64;
    }
    if (inner_dtype != COARSE_C64 && inner_dtype != COARSE_BF16 && inner_dtype != COARSE_FP16 &&
        inner_dtype != COARSE_C64_3M) {
        set_error("inner_dtype %d not one of C64, C64_3M, BF16, FP16", inner_dtype);
        return finish(CG_INVALID_ARG);
    }
    if (inner_dtype != COARSE_C64 && d.nb % 16) {
        set_error("16-bit and 3M inner links need nbasis %% 16 == 0");
        return finish(CG_UNSUPPORTED);
    }
    const long long rows = (long long)d.V * d.nb;
    Workspace w;
    const size_t need = layout_ws(nullptr, d, nrhs, &w);
    if (ws_bytes < need) {
        set_error("workspace %zu bytes, need %zu", ws_bytes, need);
        return finish(CG_WORKSPACE_TOO_SMALL);
    }
    layout_ws((char *)ws, d, nrhs, &w);

    const double t_start = now_s();
    hipStream_t user = (hipStream_t)stream;
    hipStream_t st;
    COARSE_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    hipEvent_t ev;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    int32_t result = CG_NOT_CONVERGED;
    auto cleanup = [&]() {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        hipStreamDestroy(st);
    };
#define SOLVE_HIP(call)                      \
    do {                                     \
        hipError_t _e = (call);              \
        if (_e != hipSuccess) {              \
            int32_t _r = hip_fail(_e, #call); \
            cleanup();                       \
            return finish(_r);               \
        }                                    \
    } while (0)
    SOLVE_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    SOLVE_HIP(hipEventRecord(ev, user));
    SOLVE_HIP(hipStreamWaitEvent(st, ev, 0));
    hipEventDestroy(ev);

    const double2 *b2 = (const double2 *)b;
    double2 *x2 = (double2 *)x;
    const int nr = nrhs;

    // ||b_j||
    std::vector<double2> gh((size_t)nr * nr);
    std::vector<double> bn(nr), rn(nr);
    gram<double2>(b2, b2, rows, nr, w.partials, w.g_b, nullptr, st);
    SOLVE_HIP(hipMemcpyAsync(gh.data(), w.g_b, gh.size() * 16, hipMemcpyDeviceToHost, st));
    SOLVE_HIP(hipStreamSynchronize(st));
    for (int j = 0; j < nr; ++j) {
        bn[j] = std::sqrt(gh[(size_t)j * nr + j].x);
        if (!std::isfinite(bn[j])) {
            set_error("right-hand side column %d is not finite", j);
            cleanup();
            return finish(CG_NONFINITE);
        }
        if (bn[j] == 0.0) bn[j] = 1.0;
    }

    double t_inner = 0, t_outer = 0;
    SolverState hs;
    for (int cycle = 0;; ++cycle) {
        const double t0 = now_s();
        // R = B - M X (double accumulation), norms
        rc = launch_apply(d, packed_outer, COARSE_C64, x2, w.r128, nr, COARSE_C128, b2, nullptr, st);
        if (rc) {
            cleanup();
            return finish(rc);
        }
        gram<double2>(w.r128, w.r128, rows, nr, w.partials, w.g_res, nullptr, st);
        SOLVE_HIP(hipMemcpyAsync(gh.data(), w.g_res, gh.size() * 16, hipMemcpyDeviceToHost, st));
        SOLVE_HIP(hipStreamSynchronize(st));
        double mx = 0;
        bool fin = true;
        for (int j = 0; j < nr; ++j) {
            rn[j] = std::sqrt(gh[(size_t)j * nr + j].x);
            stats.relres[j] = rn[j] / bn[j];
            fin = fin && std::isfinite(rn[j]);
            mx = std::max(mx, stats.relres[j]);
        }
        stats.relres_max = mx;
        stats.cycles = cycle;
        t_outer += now_s() - t0;
        if (!fin) {
            set_error("non-finite residual in cycle %d", cycle);
            result = CG_NONFINITE;
            break;
        }
        if (mx <= p->tol) {
            result = CG_OK;
            break;
        }
        if (cycle >= p->max_outer) {
            result = CG_NOT_CONVERGED;
            break;
        }
        // inner solve
        const double t1 = now_s();
        normalize_residual(w.r128, w.g_res, rows, nr, w.q, w.e, st);
        if (blas_mfma_supported(nr)) {
            gram_mfma(w.q, w.q, rows, nr, w.partials, w.m.G, nullptr, st);
            small_init(w.m, w.state, nr, p->inner_tol, p->max_inner, st);
            update_qd_mfma(w.q, w.d, w.m.Sinv, w.m.SH, rows, nr, 1, &w.state->active, st);
        } else {
            gram<float2>(w.q, w.q, rows, nr, w.partials, w.m.G, nullptr, st);
            small_init(w.m, w.state, nr, p->inner_tol, p->max_inner, st);
            update_qd(w.q, w.d, w.m.Sinv, w.m.SH, rows, nr, 1, &w.state->active, st);
        }
        const int m = p->check_every;
        if (p->use_graph && !exec) {
            SOLVE_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            int32_t crc = CG_OK;
            for (int k = 0; k < m && crc == CG_OK; ++k) crc = inner_iteration(d, packed_inner, inner_dtype, w, rows, nr, st);
            hipError_t ce = hipStreamEndCapture(st, &graph);
            if (crc) {
                cleanup();
                return finish(crc);
            }
            SOLVE_HIP(ce);
            SOLVE_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        }
        // every replay advances the iteration count unless the flag is down, so
        // more replays than max_inner/m + 1 means the device never reported back
        const long long max_replays = (long long)p->max_inner / m + 2;
        long long replays = 0;
        for (;;) {
            if (++replays > max_replays) {
                set_error("inner iteration did not report completion after %lld replays", replays - 1);
                cleanup();
                return finish(CG_HIP_ERROR);
            }
            if (p->use_graph) {
                SOLVE_HIP(hipGraphLaunch(exec, st));
            } else {
                for (int k = 0; k < m; ++k) {
                    rc = inner_iteration(d, packed_inner, inner_dtype, w, rows, nr, st);
                    if (rc) {
                        cleanup();
                        return finish(rc);
                    }
                }
            }
            SOLVE_HIP(hipMemcpyAsync(&hs, w.state, sizeof(hs), hipMemcpyDeviceToHost, st));
            SOLVE_HIP(hipStreamSynchronize(st));
            if (!hs.active) break;
        }
        stats.iterations += hs.iters;
        t_inner += now_s() - t1;
        const double t2 = now_s();
        outer_update(x2, w.e, w.g_res, rows, nr, st);
        t_outer += now_s() - t2;
        if (hs.nonfinite) {
            set_error("non-finite value in the inner iteration (cycle %d)", cycle);
            SOLVE_HIP(hipStreamSynchronize(st));
            result = CG_NONFINITE;
            break;
        }
        if (hs.breakdown && hs.iters == 0) {
            set_error("block breakdown: the residual block is rank deficient (cycle %d)", cycle);
            SOLVE_HIP(hipStreamSynchronize(st));
            result = CG_BREAKDOWN;
            break;
        }
    }
    SOLVE_HIP(hipStreamSynchronize(st));
    stats.seconds_inner = t_inner;
    stats.seconds_outer = t_outer;
    stats.seconds_total = now_s() - t_start;
    cleanup();
    return finish(result);
#undef SOLVE_HIP
}
