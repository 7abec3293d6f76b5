// Block-CG solve of M X = B: double precision defect correction around
// BlockCGrQ (Fig. 2, left) run in single (or 16-bit link) precision.
//
// Per outer cycle, in double: R = B - M X (complex64 links in the 4M or the
// 3M layout, double accumulation), column norms from the diagonal of R^H R, stop test,
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
//
// With a Chebyshev preconditioner (Fig. 2, right; Sec. 2.2 and 2.3) the inner
// iteration is Preconditioned BlockCGrQ on M~ with M^{-1} = P(M~), the
// degree-n interpolant of 1/x on [lo, hi]: residual-space blocks q, z and
// their images Q = P q, Z = P z are rotated side by side,
//   z_0 = R^;  Z_0 = P z_0;  C_0^H C_0 = Z_0^H z_0;  q_0 = z_0 C_0^{-1};
//   Q_0 = Z_0 C_0^{-1};  D_0 = Q_0;  then per iteration
//   z = M~ D;  Z = P z;  N = (D^H z)^{-1};  E += D (N C);
//   t = q - z N;  T = Q - Z N;  S^H S = T^H t;  q = t S^{-1};  Q = T S^{-1};
//   D = Q + D S^H;  C = S C,
// and ||C e_j|| is the P-norm of the residual column, tested relative to its
// value at the start of the cycle.
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "apply.hpp"
#include "blas.hpp"

namespace coarse {

// Chebyshev preconditioner of the inner iteration (on == 0: plain BlockCGrQ).
struct Precond {
    int on = 0;
    double lo = 0, hi = 0;
    int order = 0;
};

struct Workspace {
    double2 *r128;     // outer residual
    float2 *e, *d, *z, *q;
    float2 *qp, *zp;          // preconditioned images of q and z (preconditioned solve only)
    float2 *ta, *tb, *zc;     // Chebyshev recurrence scratch (preconditioned solve only)
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

static size_t layout_ws(char *base, const Geom &g, int nr, Workspace *w, bool prec = false) {
    const long long rows = (long long)g.V * g.nb;
    size_t off = 0;
    const size_t v128 = (size_t)rows * nr * 16, v64 = (size_t)rows * nr * 8, sm = (size_t)nr * nr;
    off = carve(base, off, v128, (void **)&w->r128);
    off = carve(base, off, v64, (void **)&w->e);
    off = carve(base, off, v64, (void **)&w->d);
    off = carve(base, off, v64, (void **)&w->z);
    off = carve(base, off, v64, (void **)&w->q);
    // split-K partials: GRAM_BLOCKS of the Gram kernels (the fused step-1
    // update writes fewer), or the workgroups of the Gram-fused 3M apply when
    // that is more
    const int gfb = apply_3m_gram_blocks(g, nr);
    off = carve(base, off, (size_t)(gfb > GRAM_BLOCKS ? gfb : GRAM_BLOCKS) * sm * 16, (void **)&w->partials);
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
    const size_t pv = prec ? v64 : 0;
    off = carve(base, off, pv, (void **)&w->qp);
    off = carve(base, off, pv, (void **)&w->zp);
    off = carve(base, off, pv, (void **)&w->ta);
    off = carve(base, off, pv, (void **)&w->tb);
    off = carve(base, off, pv, (void **)&w->zc);
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
    if (p->outer_dtype != COARSE_C64 && p->outer_dtype != COARSE_C64_3M) {
        set_error("outer_dtype %d not one of C64, C64_3M", p->outer_dtype);
        return CG_INVALID_ARG;
    }
    return CG_OK;
}

// Gram a^H b into m.G (MFMA where the shape allows).
static void inner_gram(const float2 *a, const float2 *b, Workspace &w, long long rows, int nr, const int *active,
                       hipStream_t st) {
    if (blas_mfma_supported(nr))
        gram_mfma(a, b, rows, nr, w.partials, w.m.G, active, st);
    else
        gram<float2>(a, b, rows, nr, w.partials, w.m.G, active, st);
}

// One inner iteration's launches (all no-ops once state->active == 0).
static int32_t inner_iteration(const Geom &g, const void *packed, int32_t dtype, Workspace &w, long long rows, int nr,
                               const Precond &pc, hipStream_t st) {
    const int *active = &w.state->active;
    const bool lowp = dtype == COARSE_BF16 || dtype == COARSE_FP16;
    // 3M links at nrhs 2..32: Z = M D with D^H Z fused into the apply's epilogue
    const int gfb = (dtype == COARSE_C64_3M && !pc.on && blas_mfma_supported(nr) && mfma_supported(g.nb, nr, dtype,
                                                                                                  COARSE_C64))
                        ? apply_3m_gram_blocks(g, nr)
                        : 0;
    if (gfb > 0) {
        launch_apply_3m_gram(g, (const float *)packed, (const float *)w.d, (float *)w.z, nr, w.partials, gfb, active,
                             st, tuned_variant(g.nb, nr, g.np, dtype, COARSE_C64));
        gram_reduce_n(w.partials, gfb, nr, w.m.G, active, st);
    } else {
        int32_t rc = launch_apply(g, packed, dtype, w.d, w.z, nr, COARSE_C64, nullptr, active, st, 0, -1,
                                  lowp ? w.lowp : nullptr);
        if (rc) return rc;
    }
    int32_t rc;
    if (pc.on) {
        const ChebBuffers cb{w.ta, w.tb, w.zc, w.lowp};
        if ((rc = chebyshev_poly(g, packed, dtype, w.z, w.zp, nr, pc.lo, pc.hi, pc.order, cb, active, st)))
            return rc;
        inner_gram(w.d, w.z, w, rows, nr, active, st);  // D^H z
        small_step1(w.m, w.state, nr, st);
        update_pxt(w.e, w.q, w.qp, w.d, w.z, w.zp, w.m.W, w.m.N, rows, nr, active, st);
        inner_gram(w.qp, w.q, w, rows, nr, active, st);  // T^H t
        small_step2(w.m, w.state, nr, st);
        update_pqd(w.q, w.qp, w.d, w.m.Sinv, w.m.SH, rows, nr, 0, active, st);
        return CG_OK;
    }
    if (small_fused_supported(nr)) {
        if (gfb == 0) gram_mfma(w.d, w.z, rows, nr, w.partials, w.m.G, active, st);
        step1_update_xt_gram_mfma(w.m, w.state, w.e, w.q, w.d, w.z, rows, nr, st);
        step2_update_qd_mfma(w.m, w.state, w.q, w.d, rows, nr, st);
    } else if (blas_mfma_supported(nr)) {
        if (gfb == 0) gram_mfma(w.d, w.z, rows, nr, w.partials, w.m.G, active, st);
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

static int32_t check_prec(const cg_chebyshev_prec *prec) {
    if (!prec) {
        set_error("prec is NULL");
        return CG_INVALID_ARG;
    }
    return check_chebyshev(prec->lo, prec->hi, prec->order);
}

extern "C" int32_t coarse_pbcg_workspace_bytes(const coarse_geom *g, int32_t nrhs, const cg_solve_params *p,
                                               const cg_chebyshev_prec *prec, size_t *out) {
    clear_error();
    Geom d;
    int32_t rc = make_geom(g, &d);
    if (rc) return rc;
    if ((rc = check_nrhs(nrhs))) return rc;
    if ((rc = check_prec(prec))) return rc;
    (void)p;
    if (!out) {
        set_error("out is NULL");
        return CG_INVALID_ARG;
    }
    Workspace w;
    *out = layout_ws(nullptr, d, nrhs, &w, true);
    return CG_OK;
}

namespace coarse {

// One system of a (possibly batched) solve.
struct SolveJob {
    Geom d;
    const void *packed_outer = nullptr, *packed_inner = nullptr;
    int32_t outer_dtype = COARSE_C64;
    int32_t inner_dtype = COARSE_C64;
    const double2 *b = nullptr;
    double2 *x = nullptr;
    int nr = 0;
    long long rows = 0;
    Workspace w;
    Precond pc;
    hipStream_t st = nullptr;
    std::vector<double> bn, rn;
    std::vector<double2> gh;
    cg_solve_stats stats;
    int32_t result = CG_NOT_CONVERGED;
    bool finished = false;   // outer loop over for this system
    bool inner_on = false;   // running inner iterations in the current cycle
    bool x0_zero = false;    // X_0 == 0: the first residual is B itself (no apply)
    std::vector<double2> gx; // host copy of X_0^H X_0
    SolverState hs;
};

// Validate one system and lay out its workspace at `base` (nullptr: size only).
static int32_t prepare_job(SolveJob &j, const coarse_geom *g, int32_t outer_dtype, const void *packed_outer,
                           const void *packed_inner, int32_t inner_dtype, const void *b, void *x, int32_t nrhs,
                           char *base, size_t *bytes, const cg_chebyshev_prec *prec = nullptr) {
    int32_t rc = make_geom(g, &j.d);
    if (rc) return rc;
    if ((rc = check_nrhs(nrhs))) return rc;
    if (!packed_outer || !b || !x) {
        set_error("packed_outer, b or x is NULL");
        return CG_INVALID_ARG;
    }
    if (b == x || x == packed_outer || b == packed_outer) {
        set_error("b, x and the links must not alias");
        return CG_INVALID_ARG;
    }
    if (outer_dtype == COARSE_C64_3M && j.d.nb % 16) {
        set_error("3M outer links need nbasis %% 16 == 0");
        return CG_UNSUPPORTED;
    }
    if (!packed_inner) {
        packed_inner = packed_outer;
        inner_dtype = outer_dtype;
    }
    if (inner_dtype != COARSE_C64 && inner_dtype != COARSE_BF16 && inner_dtype != COARSE_FP16 &&
        inner_dtype != COARSE_C64_3M) {
        set_error("inner_dtype %d not one of C64, C64_3M, BF16, FP16", inner_dtype);
        return CG_INVALID_ARG;
    }
    if (inner_dtype != COARSE_C64 && j.d.nb % 16) {
        set_error("16-bit and 3M inner links need nbasis %% 16 == 0");
        return CG_UNSUPPORTED;
    }
    j.packed_outer = packed_outer;
    j.outer_dtype = outer_dtype;
    j.packed_inner = packed_inner;
    j.inner_dtype = inner_dtype;
    j.b = (const double2 *)b;
    j.x = (double2 *)x;
    j.nr = nrhs;
    j.rows = (long long)j.d.V * j.d.nb;
    if (prec) {
        j.pc.on = 1;
        j.pc.lo = prec->lo;
        j.pc.hi = prec->hi;
        j.pc.order = prec->order;
    }
    *bytes = layout_ws(base, j.d, nrhs, &j.w, j.pc.on != 0);
    memset(&j.stats, 0, sizeof(j.stats));
    j.stats.nrhs = nrhs;
    j.bn.assign(nrhs, 1.0);
    j.rn.assign(nrhs, 0.0);
    j.gh.assign((size_t)nrhs * nrhs, make_double2(0, 0));
    return CG_OK;
}

// Instantiated inner-iteration graphs, reused by later solves that would
// capture exactly the same work (a coarse solve is typically called again and
// again with one operator and one workspace). The key holds every value the
// captured kernels take: device, iterations per graph, and per system the
// geometry with its offsets, nrhs, the inner links and their type, the tuned
// apply variant and the workspace pointers. At most GRAPH_CACHE graphs are
// kept, the least recently used one is destroyed first.
constexpr size_t GRAPH_CACHE = 8;

// One instantiated graph; destroyed when the last holder lets go (the cache,
// or a solve still replaying it after another thread evicted it).
struct GraphHolder {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    GraphHolder(hipGraph_t g, hipGraphExec_t e) : graph(g), exec(e) {}
    GraphHolder(const GraphHolder &) = delete;
    GraphHolder &operator=(const GraphHolder &) = delete;
    ~GraphHolder() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};
struct GraphEntry {
    std::vector<uint64_t> key;
    std::shared_ptr<GraphHolder> held;
};
static std::mutex g_graph_mu;
// most recently used last; never destroyed: graphs must not be torn down
// during static destruction, after the HIP runtime may have shut down
static std::vector<GraphEntry> &g_graphs = *new std::vector<GraphEntry>();

static std::vector<uint64_t> graph_key(const std::vector<SolveJob> &jobs, int m) {
    std::vector<uint64_t> k;
    int dev = 0;
    (void)hipGetDevice(&dev);
    k.push_back((uint64_t)dev);
    k.push_back((uint64_t)m);
    k.push_back(jobs.size());
    auto ptr = [&](const void *q) { k.push_back((uint64_t)(uintptr_t)q); };
    for (const SolveJob &j : jobs) {
        const Geom &g = j.d;
        for (int mu = 0; mu < 4; ++mu) k.push_back((uint64_t)g.L[mu]);
        k.push_back((uint64_t)g.nb);
        k.push_back((uint64_t)g.np);
        k.push_back((uint64_t)(uint32_t)g.self_p);
        for (int p = 0; p < g.np; ++p) {
            uint32_t o;
            std::memcpy(&o, g.off[p], 4);
            k.push_back(o);
        }
        k.push_back((uint64_t)j.nr);
        k.push_back((uint64_t)j.rows);
        k.push_back((uint64_t)(uint32_t)j.inner_dtype);
        k.push_back((uint64_t)(uint32_t)tuned_variant(g.nb, j.nr, g.np, j.inner_dtype, COARSE_C64));
        ptr(j.packed_inner);
        k.push_back((uint64_t)j.pc.on);
        uint64_t lo, hi;
        std::memcpy(&lo, &j.pc.lo, 8);
        std::memcpy(&hi, &j.pc.hi, 8);
        k.push_back(lo);
        k.push_back(hi);
        k.push_back((uint64_t)(uint32_t)j.pc.order);
        const Workspace &w = j.w;
        for (const void *q : {(const void *)w.e, (const void *)w.d, (const void *)w.z, (const void *)w.q,
                              (const void *)w.partials, (const void *)w.m.G, (const void *)w.m.C, (const void *)w.m.W,
                              (const void *)w.m.N, (const void *)w.m.Sinv, (const void *)w.m.SH, (const void *)w.state,
                              (const void *)w.lowp, (const void *)w.qp, (const void *)w.zp, (const void *)w.ta,
                              (const void *)w.tb, (const void *)w.zc})
            ptr(q);
    }
    return k;
}

// The cached graph for this key, or null; a hit becomes the most recently
// used entry.
static std::shared_ptr<GraphHolder> graph_lookup(const std::vector<uint64_t> &key) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (size_t i = 0; i < g_graphs.size(); ++i) {
        if (g_graphs[i].key == key) {
            GraphEntry e = g_graphs[i];
            g_graphs.erase(g_graphs.begin() + (long)i);
            g_graphs.push_back(e);
            return e.held;
        }
    }
    return nullptr;
}

static void graph_insert(std::vector<uint64_t> key, const std::shared_ptr<GraphHolder> &held) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    if (g_graphs.size() >= GRAPH_CACHE) g_graphs.erase(g_graphs.begin());
    g_graphs.push_back(GraphEntry{std::move(key), held});
}

// Inner stop of a cycle: max(inner_tol, kFinalCycleMargin * tol / relres),
// relres being the true relative residual the cycle starts from.
static constexpr double kFinalCycleMargin = 0.25;

__global__ void reset_state_kernel(SolverState *s) {
    if (threadIdx.x == 0) s->active = 0;
}

// The defect-correction loop for every job at once. Per cycle: the double
// residuals of all unfinished systems (each on its own stream), then the
// inner BlockCGrQ of those that continue, as one captured graph holding one
// branch per system (a single system captures on its own stream), replayed
// until every system's device flag is down.
static int32_t run_solves(std::vector<SolveJob> &jobs, const cg_solve_params *p, hipStream_t user) {
    const double t_start = now_s();
    const int n = (int)jobs.size();
    hipStream_t main = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::shared_ptr<GraphHolder> held;  // keeps exec alive while this solve replays it
    std::vector<hipEvent_t> evs;
    auto cleanup = [&]() {
        // exec belongs to `held`; graph is set only while a capture has not
        // reached a holder
        if (graph) (void)hipGraphDestroy(graph);
        for (auto e : evs) hipEventDestroy(e);
        for (auto &j : jobs)
            if (j.st) hipStreamDestroy(j.st);
        if (main) hipStreamDestroy(main);
    };
    int32_t hip_rc = CG_OK;
#define SOLVE_HIP(call)                       \
    do {                                      \
        hipError_t _e = (call);               \
        if (_e != hipSuccess) {               \
            hip_rc = hip_fail(_e, #call);     \
            goto fail;                        \
        }                                     \
    } while (0)
#define SOLVE_RC(expr)                        \
    do {                                      \
        int32_t _r = (expr);                  \
        if (_r != CG_OK) {                    \
            hip_rc = _r;                      \
            goto fail;                        \
        }                                     \
    } while (0)
    {
        // streams: every job waits for the caller's stream
        const int nev = 2 * n + 3;  // user, fork, per-job ready, per-job done, join
        evs.assign(nev, nullptr);
        for (int k = 0; k < nev; ++k) SOLVE_HIP(hipEventCreateWithFlags(&evs[k], hipEventDisableTiming));
        hipEvent_t ev_user = evs[0], ev_fork = evs[1];
        SOLVE_HIP(hipEventRecord(ev_user, user));
        SOLVE_HIP(hipStreamCreateWithFlags(&main, hipStreamNonBlocking));
        SOLVE_HIP(hipStreamWaitEvent(main, ev_user, 0));
        for (auto &j : jobs) {
            SOLVE_HIP(hipStreamCreateWithFlags(&j.st, hipStreamNonBlocking));
            SOLVE_HIP(hipStreamWaitEvent(j.st, ev_user, 0));
        }
        // ||b_j||, and every device flag down until a system starts its inner solve
        // ... and X_0^H X_0: a zero start (the usual case) makes the first
        // residual B itself, a copy instead of a double-precision apply
        for (auto &j : jobs) {
            hipLaunchKernelGGL(reset_state_kernel, dim3(1), dim3(64), 0, j.st, j.w.state);
            gram<double2>(j.b, j.b, j.rows, j.nr, j.w.partials, j.w.g_b, nullptr, j.st);
            SOLVE_HIP(hipMemcpyAsync(j.gh.data(), j.w.g_b, j.gh.size() * 16, hipMemcpyDeviceToHost, j.st));
            j.gx.assign(j.gh.size(), make_double2(0, 0));
            gram<double2>(j.x, j.x, j.rows, j.nr, j.w.partials, j.w.g_res, nullptr, j.st);
            SOLVE_HIP(hipMemcpyAsync(j.gx.data(), j.w.g_res, j.gx.size() * 16, hipMemcpyDeviceToHost, j.st));
        }
        for (auto &j : jobs) {
            SOLVE_HIP(hipStreamSynchronize(j.st));
            double xtr = 0;
            for (int c = 0; c < j.nr; ++c) xtr += j.gx[(size_t)c * j.nr + c].x;
            j.x0_zero = (xtr == 0.0);  // a non-finite X_0 goes through the apply and is reported there
            for (int c = 0; c < j.nr; ++c) {
                j.bn[c] = std::sqrt(j.gh[(size_t)c * j.nr + c].x);
                if (!std::isfinite(j.bn[c])) {
                    set_error("right-hand side column %d is not finite", c);
                    j.result = CG_NONFINITE;
                    j.finished = true;
                }
                if (j.bn[c] == 0.0) j.bn[c] = 1.0;
            }
        }

        const int m = p->check_every;
        for (int cycle = 0;; ++cycle) {
            // ---- residuals R = B - M X (double accumulation), norms, stop tests ----
            const double t0 = now_s();
            hipEvent_t ev_join = evs[2 * n + 2];
            bool any = false;
            for (auto &j : jobs) {
                j.inner_on = false;
                if (j.finished) continue;
                if (cycle == 0 && j.x0_zero)
                    SOLVE_HIP(hipMemcpyAsync(j.w.r128, j.b, (size_t)j.rows * j.nr * sizeof(double2),
                                             hipMemcpyDeviceToDevice, j.st));
                else
                    SOLVE_RC(launch_apply(j.d, j.packed_outer, j.outer_dtype, j.x, j.w.r128, j.nr, COARSE_C128, j.b,
                                          nullptr, j.st));
                gram<double2>(j.w.r128, j.w.r128, j.rows, j.nr, j.w.partials, j.w.g_res, nullptr, j.st);
                SOLVE_HIP(hipMemcpyAsync(j.gh.data(), j.w.g_res, j.gh.size() * 16, hipMemcpyDeviceToHost, j.st));
            }
            for (auto &j : jobs) {
                if (j.finished) continue;
                SOLVE_HIP(hipStreamSynchronize(j.st));
                j.stats.seconds_outer += now_s() - t0;
                double mx = 0;
                bool fin = true;
                for (int c = 0; c < j.nr; ++c) {
                    j.rn[c] = std::sqrt(j.gh[(size_t)c * j.nr + c].x);
                    j.stats.relres[c] = j.rn[c] / j.bn[c];
                    fin = fin && std::isfinite(j.rn[c]);
                    mx = std::max(mx, j.stats.relres[c]);
                }
                j.stats.relres_max = mx;
                j.stats.cycles = cycle;
                if (!fin) {
                    set_error("non-finite residual in cycle %d", cycle);
                    j.result = CG_NONFINITE;
                    j.finished = true;
                } else if (mx <= p->tol) {
                    j.result = CG_OK;
                    j.finished = true;
                } else if (cycle >= p->max_outer) {
                    j.result = CG_NOT_CONVERGED;
                    j.finished = true;
                } else {
                    j.inner_on = true;
                    any = true;
                }
            }
            if (!any) break;

            // ---- inner start: Q_0 C_0 = R^, D_0 = Q_0 ----
            const double t1 = now_s();
            for (auto &j : jobs) {
                if (!j.inner_on) continue;
                // a cycle need not reduce the residual further than the outer
                // target asks: the last cycle stops at a quarter of that factor
                const double itol = std::max(p->inner_tol, kFinalCycleMargin * p->tol / j.stats.relres_max);
                normalize_residual(j.w.r128, j.w.g_res, j.rows, j.nr, j.w.q, j.w.e, j.st);
                if (j.pc.on) {
                    // z_0 = R^ (in q); Z_0 = P z_0; C_0^H C_0 = Z_0^H z_0; q_0, Q_0, D_0
                    const ChebBuffers cb{j.w.ta, j.w.tb, j.w.zc, j.w.lowp};
                    SOLVE_RC(chebyshev_poly(j.d, j.packed_inner, j.inner_dtype, j.w.q, j.w.qp, j.nr, j.pc.lo,
                                            j.pc.hi, j.pc.order, cb, nullptr, j.st));
                    inner_gram(j.w.qp, j.w.q, j.w, j.rows, j.nr, nullptr, j.st);
                    small_init(j.w.m, j.w.state, j.nr, itol, p->max_inner, j.st, 1);
                    update_pqd(j.w.q, j.w.qp, j.w.d, j.w.m.Sinv, j.w.m.SH, j.rows, j.nr, 1, &j.w.state->active,
                               j.st);
                } else if (blas_mfma_supported(j.nr)) {
                    gram_mfma(j.w.q, j.w.q, j.rows, j.nr, j.w.partials, j.w.m.G, nullptr, j.st);
                    small_init(j.w.m, j.w.state, j.nr, itol, p->max_inner, j.st);
                    update_qd_mfma(j.w.q, j.w.d, j.w.m.Sinv, j.w.m.SH, j.rows, j.nr, 1, &j.w.state->active, j.st);
                } else {
                    gram<float2>(j.w.q, j.w.q, j.rows, j.nr, j.w.partials, j.w.m.G, nullptr, j.st);
                    small_init(j.w.m, j.w.state, j.nr, itol, p->max_inner, j.st);
                    update_qd(j.w.q, j.w.d, j.w.m.Sinv, j.w.m.SH, j.rows, j.nr, 1, &j.w.state->active, j.st);
                }
            }
            // the replays run on `main` (batched) or on the job's stream (single)
            hipStream_t rs = n == 1 ? jobs[0].st : main;
            if (n > 1) {
                for (int k = 0; k < n; ++k) {
                    SOLVE_HIP(hipEventRecord(evs[2 + k], jobs[k].st));
                    SOLVE_HIP(hipStreamWaitEvent(main, evs[2 + k], 0));
                }
            }
            if (p->use_graph && !exec) {
                held = graph_lookup(graph_key(jobs, m));
                if (held) exec = held->exec;
            }
            if (p->use_graph && !exec) {
                // every system's branch is captured, finished ones included (their
                // flag is down, so their kernels return at once)
                SOLVE_HIP(hipStreamBeginCapture(rs, hipStreamCaptureModeThreadLocal));
                int32_t crc = CG_OK;
                if (n == 1) {
                    for (int k = 0; k < m && crc == CG_OK; ++k)
                        crc = inner_iteration(jobs[0].d, jobs[0].packed_inner, jobs[0].inner_dtype, jobs[0].w,
                                              jobs[0].rows, jobs[0].nr, jobs[0].pc, rs);
                } else {
                    hipError_t fe = hipEventRecord(ev_fork, main);
                    for (int k = 0; k < n && crc == CG_OK && fe == hipSuccess; ++k) {
                        SolveJob &j = jobs[k];
                        fe = hipStreamWaitEvent(j.st, ev_fork, 0);
                        for (int it = 0; it < m && crc == CG_OK && fe == hipSuccess; ++it)
                            crc = inner_iteration(j.d, j.packed_inner, j.inner_dtype, j.w, j.rows, j.nr, j.pc, j.st);
                        if (fe == hipSuccess) fe = hipEventRecord(evs[2 + n + k], j.st);
                        if (fe == hipSuccess) fe = hipStreamWaitEvent(main, evs[2 + n + k], 0);
                    }
                    if (fe != hipSuccess && crc == CG_OK) crc = hip_fail(fe, "graph fork/join");
                }
                hipError_t ce = hipStreamEndCapture(rs, &graph);
                SOLVE_RC(crc);
                SOLVE_HIP(ce);
                SOLVE_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
                held = std::make_shared<GraphHolder>(graph, exec);  // owns both from here
                graph = nullptr;
                graph_insert(graph_key(jobs, m), held);
            }
            // every replay advances the iteration count of an active system unless
            // its flag is down, so more replays than max_inner/m + 1 means a device
            // flag never came back
            const long long max_replays = (long long)p->max_inner / m + 2;
            long long replays = 0;
            for (;;) {
                if (++replays > max_replays) {
                    set_error("inner iteration did not report completion after %lld replays", replays - 1);
                    hip_rc = CG_HIP_ERROR;
                    goto fail;
                }
                if (p->use_graph) {
                    SOLVE_HIP(hipGraphLaunch(exec, rs));
                } else {
                    for (auto &j : jobs) {
                        if (!j.inner_on) continue;
                        for (int k = 0; k < m; ++k)
                            SOLVE_RC(inner_iteration(j.d, j.packed_inner, j.inner_dtype, j.w, j.rows, j.nr, j.pc, rs));
                    }
                }
                for (auto &j : jobs)
                    if (j.inner_on) SOLVE_HIP(hipMemcpyAsync(&j.hs, j.w.state, sizeof(SolverState),
                                                              hipMemcpyDeviceToHost, rs));
                SOLVE_HIP(hipStreamSynchronize(rs));
                bool running = false;
                for (auto &j : jobs) running = running || (j.inner_on && j.hs.active);
                if (!running) break;
            }
            if (n > 1) {
                SOLVE_HIP(hipEventRecord(ev_join, main));
                for (auto &j : jobs) SOLVE_HIP(hipStreamWaitEvent(j.st, ev_join, 0));
            }
            const double t_in = now_s() - t1;
            // ---- X += E diag(||r_j||), per-system outcome of the cycle ----
            for (auto &j : jobs) {
                if (!j.inner_on) continue;
                j.stats.seconds_inner += t_in;
                j.stats.iterations += j.hs.iters;
                outer_update(j.x, j.w.e, j.w.g_res, j.rows, j.nr, j.st);
                if (j.hs.nonfinite) {
                    set_error("non-finite value in the inner iteration (cycle %d)", cycle);
                    j.result = CG_NONFINITE;
                    j.finished = true;
                } else if (j.hs.breakdown && j.hs.iters == 0) {
                    set_error("block breakdown: the residual block is rank deficient (cycle %d)", cycle);
                    j.result = CG_BREAKDOWN;
                    j.finished = true;
                }
            }
        }
        for (auto &j : jobs) SOLVE_HIP(hipStreamSynchronize(j.st));
        const double total = now_s() - t_start;
        for (auto &j : jobs) j.stats.seconds_total = total;
        cleanup();
        return CG_OK;
    }
fail:
    for (auto &j : jobs) {
        if (j.st) (void)hipStreamSynchronize(j.st);
        j.result = hip_rc;
    }
    if (main) (void)hipStreamSynchronize(main);
    cleanup();
    return hip_rc;
#undef SOLVE_HIP
#undef SOLVE_RC
}

}  // namespace coarse

namespace coarse {

static int32_t solve_one(const coarse_geom *g, const void *packed_outer, const void *packed_inner, int32_t inner_dtype,
                         const void *b, void *x, int32_t nrhs, const cg_solve_params *p,
                         const cg_chebyshev_prec *prec, cg_solve_stats *st_out, void *ws, size_t ws_bytes,
                         void *stream) {
    std::vector<SolveJob> jobs(1);
    SolveJob &j = jobs[0];
    auto finish = [&](int32_t rc) {
        j.stats.status = rc;
        j.stats.nrhs = nrhs;
        if (st_out) *st_out = j.stats;
        return rc;
    };
    memset(&j.stats, 0, sizeof(j.stats));
    int32_t rc = check_params(p);
    if (rc) return finish(rc);
    size_t need = 0;
    if ((rc = prepare_job(j, g, p->outer_dtype, packed_outer, packed_inner, inner_dtype, b, x, nrhs, nullptr, &need,
                          prec)))
        return finish(rc);
    if (!ws) {
        set_error("ws is NULL");
        return finish(CG_INVALID_ARG);
    }
    if (ws_bytes < need) {
        set_error("workspace %zu bytes, need %zu", ws_bytes, need);
        return finish(CG_WORKSPACE_TOO_SMALL);
    }
    prepare_job(j, g, p->outer_dtype, packed_outer, packed_inner, inner_dtype, b, x, nrhs, (char *)ws, &need, prec);
    rc = run_solves(jobs, p, (hipStream_t)stream);
    return finish(rc ? rc : j.result);
}

}  // namespace coarse

extern "C" int32_t coarse_bcg_solve(const coarse_geom *g, const void *packed_outer, const void *packed_inner,
                                    int32_t inner_dtype, const void *b, void *x, int32_t nrhs,
                                    const cg_solve_params *p, cg_solve_stats *st_out, void *ws, size_t ws_bytes,
                                    void *stream) {
    clear_error();
    return solve_one(g, packed_outer, packed_inner, inner_dtype, b, x, nrhs, p, nullptr, st_out, ws, ws_bytes,
                     stream);
}

extern "C" int32_t coarse_pbcg_solve(const coarse_geom *g, const void *packed_outer, const void *packed_inner,
                                     int32_t inner_dtype, const void *b, void *x, int32_t nrhs,
                                     const cg_solve_params *p, const cg_chebyshev_prec *prec,
                                     cg_solve_stats *st_out, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int32_t rc = check_prec(prec);
    if (rc) {
        if (st_out) {
            memset(st_out, 0, sizeof(*st_out));
            st_out->status = rc;
            st_out->nrhs = nrhs;
        }
        return rc;
    }
    return solve_one(g, packed_outer, packed_inner, inner_dtype, b, x, nrhs, p, prec, st_out, ws, ws_bytes, stream);
}

// Workspaces of a batch: each system's, 256-byte aligned, back to back.
static int32_t batch_layout(const coarse_solve_system *sys, int32_t nsys, int32_t outer_dtype,
                            std::vector<SolveJob> &jobs, char *base, size_t *total) {
    if (!sys || nsys < 1 || nsys > 64) {
        set_error("nsys = %d out of range [1, 64]", nsys);
        return CG_INVALID_ARG;
    }
    jobs.resize(nsys);
    size_t off = 0;
    for (int k = 0; k < nsys; ++k) {
        size_t bytes = 0;
        int32_t rc = prepare_job(jobs[k], &sys[k].geom, outer_dtype, sys[k].packed_outer, sys[k].packed_inner,
                                 sys[k].inner_dtype, sys[k].b, sys[k].x, sys[k].nrhs, base ? base + off : nullptr,
                                 &bytes);
        if (rc) {
            char msg[512];
            snprintf(msg, sizeof(msg), "system %d: %s", k, cg_last_error());
            set_error("%s", msg);
            return rc;
        }
        off = align256(off + bytes);
    }
    *total = off;
    return CG_OK;
}

extern "C" int32_t coarse_bcg_batched_workspace_bytes(const coarse_solve_system *sys, int32_t nsys,
                                                      const cg_solve_params *p, size_t *out) {
    clear_error();
    if (!out) {
        set_error("out is NULL");
        return CG_INVALID_ARG;
    }
    std::vector<SolveJob> jobs;
    // the layout does not depend on the outer link type (a zeroed or absent
    // p means C64 links; an invalid one is reported by the solve)
    const int32_t od = (p && p->outer_dtype == COARSE_C64_3M) ? COARSE_C64_3M : COARSE_C64;
    return batch_layout(sys, nsys, od, jobs, nullptr, out);
}

extern "C" int32_t coarse_bcg_solve_batched(const coarse_solve_system *sys, int32_t nsys, const cg_solve_params *p,
                                            cg_solve_stats *st_out, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int32_t rc = check_params(p);
    std::vector<SolveJob> jobs;
    size_t need = 0;
    if (!rc) rc = batch_layout(sys, nsys, p->outer_dtype, jobs, nullptr, &need);
    if (!rc && !ws) {
        set_error("ws is NULL");
        rc = CG_INVALID_ARG;
    }
    if (!rc && ws_bytes < need) {
        set_error("workspace %zu bytes, need %zu", ws_bytes, need);
        rc = CG_WORKSPACE_TOO_SMALL;
    }
    for (int k = 0; k < (int)jobs.size() && k < nsys; ++k) {
        for (int i = k + 1; i < nsys && !rc; ++i)
            if (sys[k].x == sys[i].x) {
                set_error("systems %d and %d share x", k, i);
                rc = CG_INVALID_ARG;
            }
    }
    if (rc) {
        if (st_out && nsys > 0 && nsys <= 64)
            for (int k = 0; k < nsys; ++k) {
                memset(&st_out[k], 0, sizeof(cg_solve_stats));
                st_out[k].status = rc;
            }
        return rc;
    }
    batch_layout(sys, nsys, p->outer_dtype, jobs, (char *)ws, &need);
    rc = run_solves(jobs, p, (hipStream_t)stream);
    int32_t overall = rc;
    for (int k = 0; k < nsys; ++k) {
        jobs[k].stats.status = rc ? rc : jobs[k].result;
        if (st_out) st_out[k] = jobs[k].stats;
        if (!overall && jobs[k].result != CG_OK) overall = jobs[k].result;
    }
    return overall;
}
