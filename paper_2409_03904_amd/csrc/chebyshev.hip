// Stationary Chebyshev approximation to 1/x applied to the coarse operator
// (Sec. 2.3): the paper replaces the data-dependent CG polynomial of the
// coarse solve by the degree-n Chebyshev interpolant of 1/x on [lo, hi],
//
//   P(x) = sum_{k=0}^{n} c_k T_k(y(x)),   y(x) = (2x - (hi + lo)) / (hi - lo),
//
// with the coefficients taken from 1/x at the n + 1 Chebyshev points. P(M) x is
// formed by the three-term recurrence T_0 = x, T_1 = Y x,
// T_{k+1} = 2 Y T_k - T_{k-1} (Y = y(M)): one apply of M per degree, each
// followed by one elementwise pass that forms T_{k+1} from M T_k, T_k and
// T_{k-1} and adds c_{k+1} T_{k+1} into the output (the recurrence and the
// accumulation fused, so every vector is touched once per degree). With 3M
// links that pass is the epilogue of the apply itself.
#include <cmath>
#include <vector>

#include "apply.hpp"

namespace coarse {

// (the kernels sit in the named namespace so that profiles show their names)

// VT: four floats (two complex64 entries) per element, or two for an odd
// count of entries
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));

// Degree 1: t1 = a z - d x, y = c0 x + c1 t1 (z = M x).
// (every kernel returns at once when `active` points at 0: inside the
// preconditioned block CG the polynomial stops with the iteration)
template <typename VT>
__global__ __launch_bounds__(256) void cheb_first_kernel(const VT *__restrict__ z, const VT *__restrict__ x,
                                                         VT *__restrict__ t1, VT *__restrict__ y, long long n, float a,
                                                         float d, float c0, float c1, const int *active) {
    if (active != nullptr && *active == 0) return;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const VT xv = x[i];
        const VT t = a * z[i] - d * xv;
        t1[i] = t;
        y[i] = c0 * xv + c1 * t;
    }
}

// Degree k + 1: t_next = 2a z - 2d t - t_prev (z = M t), y += c t_next;
// t_next may be t_prev's buffer: each element is read before the same thread
// writes it.
template <typename VT>
__global__ __launch_bounds__(256) void cheb_step_kernel(const VT *__restrict__ z, const VT *__restrict__ t,
                                                        const VT *t_prev, VT *t_next, VT *__restrict__ y, long long n,
                                                        float a2, float d2, float c, const int *active) {
    if (active != nullptr && *active == 0) return;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const VT tn = a2 * z[i] - d2 * t[i] - t_prev[i];
        t_next[i] = tn;
        y[i] = y[i] + c * tn;
    }
}

// Degree 0: y = c0 x.
template <typename VT>
__global__ __launch_bounds__(256) void cheb_scale_kernel(const VT *__restrict__ x, VT *__restrict__ y, long long n,
                                                         float c0, const int *active) {
    if (active != nullptr && *active == 0) return;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = c0 * x[i];
}

namespace {

constexpr int CHEB_MAX_ORDER = 1000;

int32_t check_cheb(double lo, double hi, int32_t order) {
    if (!(lo > 0.0) || !(hi > lo) || !std::isfinite(hi)) {
        set_error("need 0 < lo < hi (got lo %g, hi %g)", lo, hi);
        return CG_INVALID_ARG;
    }
    if (order < 0 || order > CHEB_MAX_ORDER) {
        set_error("order %d out of range [0, %d]", order, CHEB_MAX_ORDER);
        return CG_INVALID_ARG;
    }
    return CG_OK;
}

// The interpolation coefficients (host, double): with theta_j = pi (j + 1/2) / (n + 1)
// and x_j = (hi - lo)/2 cos(theta_j) + (hi + lo)/2,
// c_k = 2/(n + 1) sum_j cos(k theta_j) / x_j, c_0 halved.
void cheb_coefficients(double lo, double hi, int order, double *c) {
    const double pi = 3.14159265358979323846;
    const int m = order + 1;
    std::vector<double> theta(m), f(m);
    for (int j = 0; j < m; ++j) {
        theta[j] = pi * (j + 0.5) / m;
        f[j] = 1.0 / (0.5 * (hi - lo) * std::cos(theta[j]) + 0.5 * (hi + lo));
    }
    for (int k = 0; k < m; ++k) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s += f[j] * std::cos(k * theta[j]);
        c[k] = s * 2.0 / m;
    }
    c[0] *= 0.5;
}

struct ChebLayout {
    size_t ta, tb, z, lowp, total;
};

ChebLayout cheb_layout(const Geom &g, int32_t link_dtype, int nr) {
    const size_t v = (size_t)g.V * g.nb * nr * 8;  // one complex64 block vector
    const bool lowp = link_dtype == COARSE_BF16 || link_dtype == COARSE_FP16;
    ChebLayout l;
    l.ta = 0;
    l.tb = align256(v);
    l.z = l.tb + align256(v);
    l.lowp = l.z + align256(v);
    l.total = l.lowp + ((lowp && g.nb % 16 == 0) ? align256(lowp_ws_bytes(g, nr)) : 0);
    return l;
}

dim3 stream_grid(long long n) {
    const long long b = (n + 255) / 256;
    return dim3((unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192));
}

template <typename VT>
int32_t cheb_run(const Geom &d, const void *packed, int32_t link_dtype, const void *x, void *y, int nrhs, double lo,
                 double hi, int order, const ChebBuffers &b, long long n, const int *active, hipStream_t st) {
    std::vector<double> c(order + 1);
    cheb_coefficients(lo, hi, order, c.data());
    const VT *xv = reinterpret_cast<const VT *>(x);
    VT *yv = reinterpret_cast<VT *>(y);
    const dim3 grid = stream_grid(n), block(256);
    if (order == 0) {
        hipLaunchKernelGGL(cheb_scale_kernel<VT>, grid, block, 0, st, xv, yv, n, (float)c[0], active);
        COARSE_HIP(hipGetLastError());
        return CG_OK;
    }
    VT *ta = reinterpret_cast<VT *>(b.ta), *tb = reinterpret_cast<VT *>(b.tb);
    VT *z = reinterpret_cast<VT *>(b.z);
    void *lowp = (link_dtype == COARSE_BF16 || link_dtype == COARSE_FP16) ? b.lowp : nullptr;
    const double a = 2.0 / (hi - lo), dd = (hi + lo) / (hi - lo);
    int32_t rc;
    if (link_dtype == COARSE_C64_3M && sizeof(VT) == 16) {
        // the recurrence and the accumulation run in the epilogue of the 3M
        // apply: no separate pass and no M t round trip through memory
        const float *links = reinterpret_cast<const float *>(packed);
        const int variant = tuned_variant(d.nb, nrhs, d.np, COARSE_C64_3M, COARSE_C64);
        ChebEpi e1{nullptr, reinterpret_cast<float *>(ta), reinterpret_cast<float *>(y),
                   (float)a, (float)(-dd), 0.f, 0.f, (float)c[1], (float)c[0]};
        launch_apply_3m_cheb(d, links, reinterpret_cast<const float *>(x), e1, nrhs, active, st, variant);
        COARSE_HIP(hipGetLastError());
        const VT *t_prev = xv;
        VT *t = ta;
        for (int k = 2; k <= order; ++k) {
            VT *t_next = (t_prev == xv) ? tb : const_cast<VT *>(t_prev);
            ChebEpi ek{reinterpret_cast<const float *>(t_prev), reinterpret_cast<float *>(t_next),
                       reinterpret_cast<float *>(y), (float)(2.0 * a), (float)(-2.0 * dd), -1.f, 1.f, (float)c[k], 0.f};
            launch_apply_3m_cheb(d, links, reinterpret_cast<const float *>(t), ek, nrhs, active, st, variant);
            COARSE_HIP(hipGetLastError());
            t_prev = t;
            t = t_next;
        }
        return CG_OK;
    }
    // degree 1
    if ((rc = launch_apply(d, packed, link_dtype, x, z, nrhs, COARSE_C64, nullptr, active, st, 0, -1, lowp)))
        return rc;
    hipLaunchKernelGGL(cheb_first_kernel<VT>, grid, block, 0, st, z, xv, ta, yv, n, (float)a, (float)dd,
                       (float)c[0], (float)c[1], active);
    COARSE_HIP(hipGetLastError());
    // degrees 2 .. order: t_prev is x (read only) at degree 2, then the two
    // workspace buffers alternate
    const VT *t_prev = xv;
    VT *t = ta;
    for (int k = 2; k <= order; ++k) {
        if ((rc = launch_apply(d, packed, link_dtype, t, z, nrhs, COARSE_C64, nullptr, active, st, 0, -1, lowp)))
            return rc;
        VT *t_next = (t_prev == xv) ? tb : const_cast<VT *>(t_prev);
        hipLaunchKernelGGL(cheb_step_kernel<VT>, grid, block, 0, st, z, t, t_prev, t_next, yv, n, (float)(2.0 * a),
                           (float)(2.0 * dd), (float)c[k], active);
        COARSE_HIP(hipGetLastError());
        t_prev = t;
        t = t_next;
    }
    return CG_OK;
}

}  // namespace

int32_t chebyshev_poly(const Geom &d, const void *packed, int32_t link_dtype, const void *x, void *y, int nrhs,
                       double lo, double hi, int order, const ChebBuffers &b, const int *active, hipStream_t st) {
    const long long entries = (long long)d.V * d.nb * nrhs;
    // 16-byte vectors (and the fused 3M epilogue, which reads and writes x's
    // and y's site blocks as float4) need x and y 16-byte aligned; a view that
    // starts at an odd complex64 entry takes the 8-byte passes
    const bool al16 = ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 15) == 0;
    if (entries % 2 == 0 && al16)
        return cheb_run<f4v>(d, packed, link_dtype, x, y, nrhs, lo, hi, order, b, entries / 2, active, st);
    return cheb_run<f2v>(d, packed, link_dtype, x, y, nrhs, lo, hi, order, b, entries, active, st);
}

int32_t check_chebyshev(double lo, double hi, int32_t order) { return check_cheb(lo, hi, order); }

}  // namespace coarse

using namespace coarse;

extern "C" int32_t coarse_chebyshev_coefficients(double lo, double hi, int32_t order, double *c) {
    clear_error();
    int32_t rc = check_cheb(lo, hi, order);
    if (rc) return rc;
    if (!c) {
        set_error("c is NULL");
        return CG_INVALID_ARG;
    }
    cheb_coefficients(lo, hi, order, c);
    return CG_OK;
}

extern "C" int32_t coarse_chebyshev_workspace_bytes(const coarse_geom *g, int32_t link_dtype, int32_t nrhs,
                                                    size_t *out) {
    clear_error();
    Geom d;
    int32_t rc = make_geom(g, &d);
    if (rc) return rc;
    if ((rc = check_nrhs(nrhs))) return rc;
    if (!out) {
        set_error("out is NULL");
        return CG_INVALID_ARG;
    }
    if (link_dtype != COARSE_C64 && link_dtype != COARSE_C64_3M && link_dtype != COARSE_BF16 &&
        link_dtype != COARSE_FP16) {
        set_error("link_dtype %d not one of C64, C64_3M, BF16, FP16", link_dtype);
        return CG_INVALID_ARG;
    }
    *out = cheb_layout(d, link_dtype, nrhs).total;
    return CG_OK;
}

extern "C" int32_t coarse_chebyshev_apply(const coarse_geom *g, const void *packed, int32_t link_dtype, const void *x,
                                          void *y, int32_t nrhs, double lo, double hi, int32_t order, void *ws,
                                          size_t ws_bytes, void *stream) {
    clear_error();
    Geom d;
    int32_t rc = make_geom(g, &d);
    if (rc) return rc;
    if ((rc = check_nrhs(nrhs))) return rc;
    if ((rc = check_cheb(lo, hi, order))) return rc;
    if (!packed || !x || !y) {
        set_error("packed, x or y is NULL");
        return CG_INVALID_ARG;
    }
    if (link_dtype != COARSE_C64 && link_dtype != COARSE_C64_3M && link_dtype != COARSE_BF16 &&
        link_dtype != COARSE_FP16) {
        set_error("link_dtype %d not one of C64, C64_3M, BF16, FP16", link_dtype);
        return CG_INVALID_ARG;
    }
    if (link_dtype != COARSE_C64 && d.nb % 16) {
        set_error("16-bit and 3M links need nbasis %% 16 == 0 (got %d)", d.nb);
        return CG_UNSUPPORTED;
    }
    const ChebLayout l = cheb_layout(d, link_dtype, nrhs);
    if (order > 0 && (!ws || ws_bytes < l.total)) {
        set_error("workspace %zu bytes, need %zu", ws ? ws_bytes : (size_t)0, l.total);
        return CG_WORKSPACE_TOO_SMALL;
    }
    if (x == y || packed == x || packed == y || (order > 0 && (ws == x || ws == y || ws == packed))) {
        set_error("inputs, output and workspace must not alias");
        return CG_INVALID_ARG;
    }
    char *base = reinterpret_cast<char *>(ws);
    ChebBuffers b{nullptr, nullptr, nullptr, nullptr};
    if (order > 0) b = ChebBuffers{base + l.ta, base + l.tb, base + l.z, base + l.lowp};
    return chebyshev_poly(d, packed, link_dtype, x, y, nrhs, lo, hi, order, b, nullptr, (hipStream_t)stream);
}
