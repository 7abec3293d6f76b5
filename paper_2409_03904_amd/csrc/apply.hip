// Coarse-operator apply kernels for gfx950.
//
// The operator of Sec. 2.6, y(x) = sum_p A_p(x) X(x + delta_p), evaluated as
// ONE per-site complex GEMM of shape nb x nrhs x (npoint*nb) per coarse site,
// fused over every stencil point (the paper issues one batched GEMM per
// point; fusing removes the per-point launches and synchronisations).
//
// Complex arithmetic goes to the real MFMA units in the "4M" real embedding
//   [Yr | Yi] = [Ar Ai] . [[ Xr  Xi ]
//                          [-Xi  Xr ]]
// where [Ar Ai] interleaves real and imaginary parts along k' = 2j + h. That
// is exactly the complex64 memory order of a link row, so the links stream
// from HBM straight into the MFMA A operand; the sign pattern lives in the
// small, LDS-staged input operand.
//
// Work split: one workgroup per coarse site, one wave per 16-row tile of the
// nb output rows; every wave streams its own rows of each link block (read
// once per apply) while the neighbour block X(x + delta_p) is staged in LDS
// once per point and shared by the waves (double-buffered, the next
// neighbour's loads in flight while the current one is consumed).
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>

#include "apply.hpp"
#include "apply_site.hpp"
#include "blas.hpp"

namespace coarse {

// Sites of one XCD form a contiguous slab (workgroups are dealt round-robin
// to the 8 XCDs), so a slab's neighbour blocks stay in that XCD's L2.
__device__ __forceinline__ int site_of_block(int b, int V) {
    return (V % 8 == 0) ? ((b & 7) * (V >> 3) + (b >> 3)) : b;
}

// ---------------------------------------------------------------------------
// 16-bit link kernel (BF16 or FP16 storage, per-(site, point) power-of-two
// scales), complex64 vectors, 16x16x32 MFMA with float32 accumulation.
// The self block stays complex64 and goes through the float32 MFMA.
// Neighbour blocks are converted once, at staging time, into the ready-made
// 16-bit B operand [step][tile][lane][8] in LDS (one 16-byte LDS read per
// MFMA); FP16 inputs carry one power-of-two scale per (site, rhs column).
// ---------------------------------------------------------------------------
template <int KIND, int NT>
__global__ __launch_bounds__(256) void apply_lowp_kernel(Geom g, const uint16_t *__restrict__ q16,
                                                          const float *__restrict__ self_c64,
                                                          const float *__restrict__ lscale,
                                                          const float *__restrict__ x, float *__restrict__ y,
                                                          int nr, const float *__restrict__ sub,
                                                          const int *__restrict__ active) {
    typedef typename std::conditional<KIND == 0, bf16x8, f16x8>::type OpT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (active != nullptr && *active == 0) return;

    const int nb = g.nb;
    const int nst = nb >> 4;  // 32-wide k' steps per block == number of waves
    const int s = site_of_block(blockIdx.x, g.V);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int w = tid >> 6, t = tid & 63, il = t & 15, q = t >> 4;
    const int two_nr = 2 * nr;
    const int xblk = nb * nr * 2;

    // LDS: two 16-bit operand buffers, then per-wave column maxima (FP16 scales)
    const int hbuf_u4 = nst * NT * 64;  // uint4 entries per buffer
    uint4 *hb0 = reinterpret_cast<uint4 *>(smem_raw);
    uint4 *hb1 = hb0 + hbuf_u4;
    float *cmax = reinterpret_cast<float *>(hb1 + hbuf_u4);  // [2][4 waves][32 cols]
    float *fx = reinterpret_cast<float *>(smem_raw);          // aliases hb0/hb1 (self phase, epilogue)

    int part_[NT], r_[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int n = 16 * nt + il;
        part_[nt] = n / nr;
        r_[nt] = n - part_[nt] * nr;
    }

    int c[4];
    site_coords(g, s, c);

    f32x4 acc[NT], accp[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = f32x4{0, 0, 0, 0};

    // ---- self point: complex64 links, float32 input, float32 MFMA ----
    if (g.self_p >= 0) {
        const int nvec = (xblk * 4) >> 4;
        const float4 *src = reinterpret_cast<const float4 *>(x + (size_t)s * xblk);
        float4 *d4 = reinterpret_cast<float4 *>(fx);
        for (int e = tid; e < nvec; e += nthr) d4[e] = src[e];
        __syncthreads();
        const int h = q & 1, jq = q >> 1;
        int boff[NT];
        float bsg[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            if (part_[nt] >= 2) {
                boff[nt] = 0;
                bsg[nt] = 0.f;
            } else {
                const int comp = (part_[nt] == 0) ? h : 1 - h;
                boff[nt] = 2 * r_[nt] + comp;
                bsg[nt] = (part_[nt] == 0 && h) ? -1.f : 1.f;
            }
        }
        const float *lb = self_c64 + (size_t)s * nb * nb * 2 + 16 * w * 16 + (q * 16 + il) * 4;
        const int nch = nb >> 3;
        for (int cc = 0; cc < nch; ++cc) {
            const float4 a = *reinterpret_cast<const float4 *>(lb + cc * nb * 16);
            const float av4[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = 8 * cc + 2 * u + jq;
                const float *xrow = fx + j * two_nr;
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[nt] = mfma16x16x4(av4[u], bsg[nt] * xrow[boff[nt]], acc[nt]);
            }
        }
        __syncthreads();
    }

    // ---- every other point: 16-bit links and inputs ----
    // staging thread (wave w, lane t) builds entry (st = w, nt, t) of the
    // operand: rows j = 16w + 4q + 0..3 of column r_[nt], pairs
    // part 0: (Re, -Im), part 1: (Im, Re), pad: 0.
    float2 xv[NT][4];
    auto load_x = [&](int p) {
        const int z = displaced(g, c, p, 1);
        const float2 *src = reinterpret_cast<const float2 *>(x + (size_t)z * xblk);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
            for (int e2 = 0; e2 < 4; ++e2) {
                const int j = 16 * w + 4 * q + e2;
                xv[nt][e2] = (part_[nt] < 2) ? src[j * nr + r_[nt]] : make_float2(0.f, 0.f);
            }
        }
    };
    // FP16: per-wave maxima of each column over this wave's 16 rows
    auto col_max = [&](int buf) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            float m = 0.f;
#pragma unroll
            for (int e2 = 0; e2 < 4; ++e2) m = fmaxf(m, fmaxf(fabsf(xv[nt][e2].x), fabsf(xv[nt][e2].y)));
            m = fmaxf(m, __shfl_xor(m, 16));
            m = fmaxf(m, __shfl_xor(m, 32));
            if (q == 0 && part_[nt] < 2) cmax[(buf * 4 + w) * 32 + r_[nt]] = m;
        }
    };
    auto col_scale = [&](int buf, int r) {
        float m = 0.f;
        for (int ww = 0; ww < nst; ++ww) m = fmaxf(m, cmax[(buf * 4 + ww) * 32 + r]);
        return pow2_ceil(m);
    };
    auto store_x = [&](uint4 *hb, int buf) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            float inv = 1.f;
            if (KIND == 1 && part_[nt] < 2) inv = 1.f / col_scale(buf, r_[nt]);
            uint32_t d[4];
#pragma unroll
            for (int e2 = 0; e2 < 4; ++e2) {
                float lo, hi;
                if (part_[nt] == 0) {
                    lo = xv[nt][e2].x;
                    hi = -xv[nt][e2].y;
                } else {
                    lo = xv[nt][e2].y;
                    hi = xv[nt][e2].x;
                }
                lo *= inv;
                hi *= inv;
                const uint16_t bl = KIND == 0 ? to_bf16_bits(lo) : to_f16_bits(lo);
                const uint16_t bh = KIND == 0 ? to_bf16_bits(hi) : to_f16_bits(hi);
                d[e2] = (uint32_t)bl | ((uint32_t)bh << 16);
            }
            hb[(w * NT + nt) * 64 + t] = make_uint4(d[0], d[1], d[2], d[3]);
        }
    };

    const int np = g.np;
    const size_t blk_h = (size_t)nb * nb * 2;
    const uint16_t *lsite = q16 + (size_t)s * np * blk_h;
    uint4 a_cur[4], a_nxt[4];
    auto load_a = [&](uint4 *a, int p) {
        const uint16_t *lb = lsite + (size_t)p * blk_h;
#pragma unroll
        for (int st = 0; st < 4; ++st)
            if (st < nst) a[st] = *reinterpret_cast<const uint4 *>(lb + ((size_t)(st * nst + w) * 64 + t) * 8);
    };

    int p = (g.self_p == 0) ? 1 : 0;
    int k = 0;
    if (p < np) {
        load_x(p);
        load_a(a_cur, p);
        if (KIND == 1) {
            col_max(0);
            __syncthreads();
        }
        store_x(hb0, 0);
        __syncthreads();
    }
    while (p < np) {
        int pn = p + 1;
        if (pn == g.self_p) ++pn;
        const bool more = pn < np;
        if (more) {
            load_x(pn);
            load_a(a_nxt, pn);
        }
        const uint4 *hc = (k & 1) ? hb1 : hb0;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) accp[nt] = f32x4{0, 0, 0, 0};
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            if (st < nst) {
                const OpT av = __builtin_bit_cast(OpT, a_cur[st]);
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const OpT bv = __builtin_bit_cast(OpT, hc[(st * NT + nt) * 64 + t]);
                    if (KIND == 0)
                        accp[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, accp[nt], 0, 0, 0);
                    else
                        accp[nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, accp[nt], 0, 0, 0);
                }
            }
        }
        const float ls = lscale[(size_t)s * np + p];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            float f = ls;
            if (KIND == 1 && part_[nt] < 2) f *= col_scale(k & 1, r_[nt]);
            acc[nt] += accp[nt] * f;
        }
        if (more) {
            if (KIND == 1) {
                col_max((k + 1) & 1);
                __syncthreads();
            }
            store_x((k & 1) ? hb0 : hb1, (k + 1) & 1);
#pragma unroll
            for (int st = 0; st < 4; ++st) a_cur[st] = a_nxt[st];
        }
        __syncthreads();
        p = pn;
        ++k;
    }

    // epilogue
    float *out = fx;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int n = 16 * nt + il;
        if (n < two_nr) {
#pragma unroll
            for (int v = 0; v < 4; ++v) out[(16 * w + 4 * q + v) * two_nr + n] = acc[nt][v];
        }
    }
    __syncthreads();
    float *yo = y + (size_t)s * xblk;
    const float *so = sub ? sub + (size_t)s * xblk : nullptr;
    for (int e = tid; e < nb * nr; e += nthr) {
        const int i = e / nr, r = e - i * nr;
        float re = out[i * two_nr + r], im = out[i * two_nr + nr + r];
        if (so) {
            re = so[2 * e] - re;
            im = so[2 * e + 1] - im;
        }
        yo[2 * e] = re;
        yo[2 * e + 1] = im;
    }
}

// ---------------------------------------------------------------------------
// Generic VALU kernel: any nbasis, forward or adjoint, any link storage.
// One thread per output entry (site, i, r). Same rounding of the input as
// the 16-bit MFMA kernel. Used where the MFMA tiling does not apply.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void apply_generic_kernel(Geom g, const float *__restrict__ lc64,
                                                             const uint16_t *__restrict__ q16,
                                                             const float *__restrict__ self_c64,
                                                             const float *__restrict__ lscale, int link_kind,
                                                             const T *__restrict__ x, T *__restrict__ y, int nr,
                                                             int adjoint, const T *__restrict__ sub,
                                                             const int *__restrict__ active) {
    if (active != nullptr && *active == 0) return;
    const int nb = g.nb;
    const size_t total = (size_t)g.V * nb * nr;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int s = (int)(e / ((size_t)nb * nr));
        const int rem = (int)(e - (size_t)s * nb * nr);
        const int i = rem / nr, r = rem - i * nr;
        int c[4];
        site_coords(g, s, c);
        T are = 0, aim = 0;
        for (int p = 0; p < g.np; ++p) {
            const int z = displaced(g, c, p, adjoint ? -1 : 1);
            const int ls = adjoint ? z : s;
            const bool lowp = (link_kind != COARSE_C64) && (p != g.self_p);
            float xsc = 1.f;
            if (lowp && link_kind == COARSE_FP16) {
                float m = 0.f;
                for (int j = 0; j < nb; ++j) {
                    const T *xp = x + (((size_t)z * nb + j) * nr + r) * 2;
                    m = fmaxf(m, fmaxf(fabsf((float)xp[0]), fabsf((float)xp[1])));
                }
                xsc = pow2_ceil(m);
            }
            const float lsc = lowp ? lscale[(size_t)ls * g.np + p] : 1.f;
            for (int j = 0; j < nb; ++j) {
                const int ai = adjoint ? j : i, aj = adjoint ? i : j;
                float lr, li;
                if (!lowp) {
                    const float *blk = (link_kind == COARSE_C64) ? lc64 + ((size_t)ls * g.np + p) * nb * nb * 2
                                                                 : self_c64 + (size_t)ls * nb * nb * 2;
                    lr = blk[c64_block_offset(nb, ai, 2 * aj)];
                    li = blk[c64_block_offset(nb, ai, 2 * aj + 1)];
                } else {
                    const uint16_t *blk = q16 + ((size_t)ls * g.np + p) * nb * nb * 2;
                    const uint16_t br = blk[h16_block_offset(nb, ai, 2 * aj)];
                    const uint16_t bi = blk[h16_block_offset(nb, ai, 2 * aj + 1)];
                    lr = (link_kind == COARSE_BF16 ? bf16_bits_to_float(br) : f16_bits_to_float(br)) * lsc;
                    li = (link_kind == COARSE_BF16 ? bf16_bits_to_float(bi) : f16_bits_to_float(bi)) * lsc;
                }
                if (adjoint) li = -li;
                const T *xp = x + (((size_t)z * nb + j) * nr + r) * 2;
                T xr = xp[0], xi = xp[1];
                if (lowp) {
                    if (link_kind == COARSE_BF16) {
                        xr = (T)bf16_bits_to_float(to_bf16_bits((float)xr));
                        xi = (T)bf16_bits_to_float(to_bf16_bits((float)xi));
                    } else {
                        xr = (T)(f16_bits_to_float(to_f16_bits((float)xr / xsc)) * xsc);
                        xi = (T)(f16_bits_to_float(to_f16_bits((float)xi / xsc)) * xsc);
                    }
                }
                are += (T)lr * xr - (T)li * xi;
                aim += (T)lr * xi + (T)li * xr;
            }
        }
        T *yo = y + e * 2;
        if (sub) {
            are = sub[e * 2] - are;
            aim = sub[e * 2 + 1] - aim;
        }
        yo[0] = are;
        yo[1] = aim;
    }
}

// ---------------------------------------------------------------------------
// Dispatch
// ---------------------------------------------------------------------------
bool mfma_supported(int nb, int nrhs, int32_t link_dtype, int32_t vec_dtype) {
    if (nrhs < 1 || nrhs > 32) return false;
    if (link_dtype == COARSE_C64_3M) return nb % 16 == 0 && (vec_dtype == COARSE_C64 || vec_dtype == COARSE_C128);
    if (link_dtype == COARSE_C64) return tiled_c64(nb) && (vec_dtype == COARSE_C64 || vec_dtype == COARSE_C128);
    return (nb % 16 == 0) && vec_dtype == COARSE_C64;
}

// ---------------------------------------------------------------------------
// Variant table (filled by coarse_tune_apply, optionally persisted).
// Variant v of the float32 kernel: point split PS = 1 << v (v = 0, 1, 2),
// allowed while 64 * row_tiles * PS <= 256.
// ---------------------------------------------------------------------------
struct TuneKey {
    int nb, nr, np, link, vec;
    bool operator<(const TuneKey &o) const {
        if (nb != o.nb) return nb < o.nb;
        if (nr != o.nr) return nr < o.nr;
        if (np != o.np) return np < o.np;
        if (link != o.link) return link < o.link;
        return vec < o.vec;
    }
};
static std::mutex g_tune_mu;
static std::map<TuneKey, int> g_tune;
static bool g_tune_loaded = false;

static void tune_load_env_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = getenv("COARSE_TUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    TuneKey k;
    int v;
    float us;
    while (fscanf(f, "%d %d %d %d %d %d %f", &k.nb, &k.nr, &k.np, &k.link, &k.vec, &v, &us) == 7) g_tune[k] = v;
    fclose(f);
}

int tuned_variant(int nb, int nr, int np, int link, int vec) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_env_locked();
    auto it = g_tune.find(TuneKey{nb, nr, np, link, vec});
    return it == g_tune.end() ? 0 : it->second;
}

int max_variant(int nb) {
    const int nmt = (nb + 15) / 16;
    return nmt == 1 ? 2 : (nmt == 2 ? 1 : 0);
}

template <int KIND, int NT>
static void launch_lowp_t(const Geom &g, const uint16_t *q16, const float *self_c64, const float *scales,
                          const float *x, float *y, int nr, const float *sub, const int *active, hipStream_t st) {
    const int waves = g.nb / 16;
    const size_t hbytes = (size_t)2 * waves * NT * 64 * 16;
    const size_t lds = hbytes + 2 * 4 * 32 * sizeof(float);
    hipLaunchKernelGGL((apply_lowp_kernel<KIND, NT>), dim3(g.V), dim3(64 * waves), lds, st, g, q16, self_c64,
                       scales, x, y, nr, sub, active);
}

template <int KIND>
static void launch_lowp(const Geom &g, const uint16_t *q16, const float *self_c64, const float *scales,
                        const float *x, float *y, int nr, const float *sub, const int *active, hipStream_t st) {
    const int nt = (2 * nr + 15) / 16;
    switch (nt) {
        case 1: launch_lowp_t<KIND, 1>(g, q16, self_c64, scales, x, y, nr, sub, active, st); break;
        case 2: launch_lowp_t<KIND, 2>(g, q16, self_c64, scales, x, y, nr, sub, active, st); break;
        case 3: launch_lowp_t<KIND, 3>(g, q16, self_c64, scales, x, y, nr, sub, active, st); break;
        default: launch_lowp_t<KIND, 4>(g, q16, self_c64, scales, x, y, nr, sub, active, st); break;
    }
}

static void lowp_parts(const Geom &g, const void *packed, const uint16_t **q16, const float **self_c64,
                       const float **scales) {
    LowpLayout l = lowp_layout(g.V, g.np, g.nb, g.self_p >= 0);
    const char *base = (const char *)packed;
    *q16 = (const uint16_t *)base;
    *self_c64 = (const float *)(base + l.self_off);
    *scales = (const float *)(base + l.scale_off);
}

template <typename T>
static void launch_generic(const Geom &g, const void *packed, int32_t link_dtype, const T *x, T *y, int nr,
                           int adjoint, const T *sub, const int *active, hipStream_t st) {
    const float *lc64 = nullptr;
    const uint16_t *q16 = nullptr;
    const float *self_c64 = nullptr, *scales = nullptr;
    if (link_dtype == COARSE_C64)
        lc64 = (const float *)packed;
    else
        lowp_parts(g, packed, &q16, &self_c64, &scales);
    const size_t total = (size_t)g.V * g.nb * nr;
    size_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(apply_generic_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, st, g, lc64, q16, self_c64,
                       scales, (int)link_dtype, x, y, nr, adjoint, sub, active);
}

int32_t launch_apply(const Geom &g, const void *packed, int32_t link_dtype, const void *x, void *y, int nrhs,
                     int32_t vec_dtype, const void *sub, const int *active, hipStream_t st, int force_generic,
                     int variant, void *lowp_ws) {
    const bool mfma = !force_generic && mfma_supported(g.nb, nrhs, link_dtype, vec_dtype);
    if (variant < 0) variant = tuned_variant(g.nb, nrhs, g.np, link_dtype, vec_dtype);
    if (vec_dtype == COARSE_C128) {
        if (link_dtype == COARSE_C64_3M) {
            if (!mfma) {
                set_error("3M links run on the MFMA kernel only");
                return CG_UNSUPPORTED;
            }
            launch_apply_3m_f64(g, (const float *)packed, (const double *)x, (double *)y, nrhs, (const double *)sub,
                                active, st);
        } else if (link_dtype != COARSE_C64) {
            set_error("complex128 vectors need complex64 links (4M or 3M layout)");
            return CG_UNSUPPORTED;
        } else if (mfma) {
            if (!launch_mfma_f64(g, (const float *)packed, (const double *)x, (double *)y, nrhs,
                                 (const double *)sub, active, st))
                return CG_UNSUPPORTED;
        }
        else
            launch_generic<double>(g, packed, link_dtype, (const double *)x, (double *)y, nrhs, 0,
                                   (const double *)sub, active, st);
    } else if (vec_dtype == COARSE_C64) {
        if (link_dtype == COARSE_C64_3M) {
            if (!mfma) {
                set_error("3M links run on the MFMA kernel only");
                return CG_UNSUPPORTED;
            }
            launch_apply_3m(g, (const float *)packed, (const float *)x, (float *)y, nrhs, (const float *)sub, active,
                            st, variant);
        } else if (link_dtype == COARSE_C64) {
            if (mfma) {
                if (!launch_mfma_f32(g, (const float *)packed, (const float *)x, (float *)y, nrhs,
                                     (const float *)sub, active, st, variant))
                    return CG_UNSUPPORTED;
            }
            else
                launch_generic<float>(g, packed, link_dtype, (const float *)x, (float *)y, nrhs, 0,
                                      (const float *)sub, active, st);
        } else {
            if (g.nb % 16) {
                set_error("16-bit links need nbasis %% 16 == 0");
                return CG_UNSUPPORTED;
            }
            if (mfma) {
                const uint16_t *q16;
                const float *self_c64, *scales;
                lowp_parts(g, packed, &q16, &self_c64, &scales);
                if (lowp_ws)
                    launch_lowp_ws(g, link_dtype == COARSE_BF16 ? 0 : 1, q16, self_c64, scales, (const float *)x,
                                   (float *)y, nrhs, (const float *)sub, active, lowp_ws, st);
                else if (link_dtype == COARSE_BF16)
                    launch_lowp<0>(g, q16, self_c64, scales, (const float *)x, (float *)y, nrhs, (const float *)sub,
                                   active, st);
                else
                    launch_lowp<1>(g, q16, self_c64, scales, (const float *)x, (float *)y, nrhs, (const float *)sub,
                                   active, st);
            } else {
                launch_generic<float>(g, packed, link_dtype, (const float *)x, (float *)y, nrhs, 0,
                                      (const float *)sub, active, st);
            }
        }
    } else {
        set_error("vec_dtype %d not one of C64, C128", vec_dtype);
        return CG_INVALID_ARG;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "apply kernel launch");
    return CG_OK;
}

int32_t launch_apply_adjoint(const Geom &g, const void *packed, int32_t link_dtype, const void *x, void *y,
                             int nrhs, int32_t vec_dtype, hipStream_t st, int force_generic) {
    if (link_dtype == COARSE_C64_3M) {
        if (force_generic || vec_dtype != COARSE_C64 || g.nb % 16) {
            set_error("3M links: the MFMA adjoint only (complex64 vectors, nbasis %% 16 == 0)");
            return CG_UNSUPPORTED;
        }
        launch_adjoint_3m(g, (const float *)packed, (const float *)x, (float *)y, nrhs, st, 0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "3M adjoint kernel launch");
        return CG_OK;
    }
    if (!force_generic && launch_adjoint_mfma(g, packed, link_dtype, x, y, nrhs, vec_dtype, st)) {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "adjoint kernel launch");
        return CG_OK;
    }
    if (vec_dtype == COARSE_C128) {
        if (link_dtype != COARSE_C64) {
            set_error("complex128 vectors need complex64 links");
            return CG_UNSUPPORTED;
        }
        launch_generic<double>(g, packed, link_dtype, (const double *)x, (double *)y, nrhs, 1, nullptr, nullptr,
                               st);
    } else if (vec_dtype == COARSE_C64) {
        if (link_dtype != COARSE_C64 && g.nb % 16) {
            set_error("16-bit links need nbasis %% 16 == 0");
            return CG_UNSUPPORTED;
        }
        launch_generic<float>(g, packed, link_dtype, (const float *)x, (float *)y, nrhs, 1, nullptr, nullptr, st);
    } else {
        set_error("vec_dtype %d not one of C64, C128", vec_dtype);
        return CG_INVALID_ARG;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "adjoint kernel launch");
    return CG_OK;
}

}  // namespace coarse

using namespace coarse;

static int32_t check_apply_args(const coarse_geom *g, const void *packed, int32_t link_dtype, const void *x,
                                void *y, int32_t nrhs, int32_t vec_dtype, Geom *d) {
    clear_error();
    int32_t rc = make_geom(g, d);
    if (rc) return rc;
    if ((rc = check_nrhs(nrhs))) return rc;
    if (!packed || !x || !y) {
        set_error("packed, x or y is NULL");
        return CG_INVALID_ARG;
    }
    if (x == y || packed == x || packed == y) {
        set_error("inputs and outputs must not alias");
        return CG_INVALID_ARG;
    }
    if (link_dtype != COARSE_C64 && link_dtype != COARSE_BF16 && link_dtype != COARSE_FP16 &&
        link_dtype != COARSE_C64_3M) {
        set_error("link_dtype %d not one of C64, C64_3M, BF16, FP16", link_dtype);
        return CG_INVALID_ARG;
    }
    if (vec_dtype != COARSE_C64 && vec_dtype != COARSE_C128) {
        set_error("vec_dtype %d not one of C64, C128", vec_dtype);
        return CG_INVALID_ARG;
    }
    if (link_dtype != COARSE_C64 && d->nb % 16) {
        set_error("16-bit and 3M links need nbasis %% 16 == 0 (got %d)", d->nb);
        return CG_UNSUPPORTED;
    }
    if ((link_dtype == COARSE_BF16 || link_dtype == COARSE_FP16) && vec_dtype != COARSE_C64) {
        set_error("16-bit links take complex64 vectors");
        return CG_UNSUPPORTED;
    }
    if ((size_t)d->V * d->nb * nrhs >= ((size_t)1 << 31)) {
        set_error("V*nbasis*nrhs too large");
        return CG_INVALID_ARG;
    }
    return CG_OK;
}

extern "C" int32_t coarse_apply(const coarse_geom *g, const void *packed, int32_t link_dtype, const void *x, void *y,
                                int32_t nrhs, int32_t vec_dtype, void *stream) {
    Geom d;
    int32_t rc = check_apply_args(g, packed, link_dtype, x, y, nrhs, vec_dtype, &d);
    if (rc) return rc;
    return launch_apply(d, packed, link_dtype, x, y, nrhs, vec_dtype, nullptr, nullptr, (hipStream_t)stream);
}

extern "C" int32_t coarse_apply_adjoint(const coarse_geom *g, const void *packed, int32_t link_dtype, const void *x,
                                        void *y, int32_t nrhs, int32_t vec_dtype, void *stream) {
    Geom d;
    int32_t rc = check_apply_args(g, packed, link_dtype, x, y, nrhs, vec_dtype, &d);
    if (rc) return rc;
    return launch_apply_adjoint(d, packed, link_dtype, x, y, nrhs, vec_dtype, (hipStream_t)stream);
}

extern "C" int32_t coarse_apply_workspace_bytes(const coarse_geom *g, int32_t link_dtype, int32_t nrhs,
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
    const bool lowp = link_dtype == COARSE_BF16 || link_dtype == COARSE_FP16;
    if (!lowp && link_dtype != COARSE_C64 && link_dtype != COARSE_C64_3M) {
        set_error("link_dtype %d not one of C64, C64_3M, BF16, FP16", link_dtype);
        return CG_INVALID_ARG;
    }
    *out = (lowp && d.nb % 16 == 0) ? lowp_ws_bytes(d, nrhs) : 0;
    return CG_OK;
}

extern "C" int32_t coarse_apply_ws(const coarse_geom *g, const void *packed, int32_t link_dtype, const void *x,
                                   void *y, int32_t nrhs, int32_t vec_dtype, void *ws, size_t ws_bytes,
                                   void *stream) {
    Geom d;
    int32_t rc = check_apply_args(g, packed, link_dtype, x, y, nrhs, vec_dtype, &d);
    if (rc) return rc;
    const bool lowp = link_dtype == COARSE_BF16 || link_dtype == COARSE_FP16;
    const size_t need = lowp ? lowp_ws_bytes(d, nrhs) : 0;
    if (need > 0 && (!ws || ws_bytes < need)) {
        set_error("workspace %zu bytes, need %zu", ws ? ws_bytes : (size_t)0, need);
        return CG_WORKSPACE_TOO_SMALL;
    }
    if (need > 0 && (ws == x || ws == y)) {
        set_error("workspace aliases x or y");
        return CG_INVALID_ARG;
    }
    return launch_apply(d, packed, link_dtype, x, y, nrhs, vec_dtype, nullptr, nullptr, (hipStream_t)stream, 0, -1,
                        need > 0 ? ws : nullptr);
}

// ---------------------------------------------------------------------------
// Apply with the Gram x^H y: the operator application of a BlockCGrQ
// iteration together with the matrix the iteration inverts next (Fig. 2), as
// the inner solve forms them. 3M links on a shape with a Gram-fused form
// accumulate the Gram in the apply's epilogue; every other case runs the
// apply and then the split-K Gram. The partials (and, for 16-bit links, the
// prepared operands of the two-pass apply) live in the caller's workspace.
// ---------------------------------------------------------------------------
static int gram_fused_for(const Geom &d, int32_t link_dtype, int nr) {
    return (link_dtype == COARSE_C64_3M && blas_mfma_supported(nr)) ? apply_3m_gram_blocks(d, nr) : 0;
}

static size_t apply_gram_ws(const Geom &d, int32_t link_dtype, int nr, size_t *lowp_off) {
    const int fb = gram_fused_for(d, link_dtype, nr);
    const size_t parts = align256((size_t)(fb > GRAM_BLOCKS ? fb : GRAM_BLOCKS) * nr * nr * sizeof(double2));
    *lowp_off = parts;
    const bool lowp = link_dtype == COARSE_BF16 || link_dtype == COARSE_FP16;
    return parts + (lowp && d.nb % 16 == 0 ? align256(lowp_ws_bytes(d, nr)) : 0);
}

extern "C" int32_t coarse_apply_gram_workspace_bytes(const coarse_geom *g, int32_t link_dtype, int32_t nrhs,
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
    if (link_dtype != COARSE_C64 && link_dtype != COARSE_BF16 && link_dtype != COARSE_FP16 &&
        link_dtype != COARSE_C64_3M) {
        set_error("link_dtype %d not one of C64, C64_3M, BF16, FP16", link_dtype);
        return CG_INVALID_ARG;
    }
    size_t off;
    *out = apply_gram_ws(d, link_dtype, nrhs, &off);
    return CG_OK;
}

extern "C" int32_t coarse_apply_gram(const coarse_geom *g, const void *packed, int32_t link_dtype, const void *x,
                                     void *y, int32_t nrhs, void *gram, void *ws, size_t ws_bytes, void *stream) {
    Geom d;
    int32_t rc = check_apply_args(g, packed, link_dtype, x, y, nrhs, COARSE_C64, &d);
    if (rc) return rc;
    if (!gram) {
        set_error("gram is NULL");
        return CG_INVALID_ARG;
    }
    size_t lowp_off;
    const size_t need = apply_gram_ws(d, link_dtype, nrhs, &lowp_off);
    if (!ws || ws_bytes < need) {
        set_error("workspace %zu bytes, need %zu", ws ? ws_bytes : (size_t)0, need);
        return CG_WORKSPACE_TOO_SMALL;
    }
    if (ws == x || ws == y || ws == gram || gram == x || gram == y || gram == packed) {
        set_error("workspace, gram, x and y must not alias");
        return CG_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    double2 *partials = static_cast<double2 *>(ws);
    double2 *gout = static_cast<double2 *>(gram);
    const long long rows = (long long)d.V * d.nb;
    const int fb = gram_fused_for(d, link_dtype, nrhs);
    if (fb > 0) {
        launch_apply_3m_gram(d, (const float *)packed, (const float *)x, (float *)y, nrhs, partials, fb, nullptr, st,
                             tuned_variant(d.nb, nrhs, d.np, link_dtype, COARSE_C64));
        gram_reduce_n(partials, fb, nrhs, gout, nullptr, st);
    } else {
        const bool lowp = link_dtype == COARSE_BF16 || link_dtype == COARSE_FP16;
        void *lws = lowp ? static_cast<char *>(ws) + lowp_off : nullptr;
        if ((rc = launch_apply(d, packed, link_dtype, x, y, nrhs, COARSE_C64, nullptr, nullptr, st, 0, -1, lws)))
            return rc;
        if (blas_mfma_supported(nrhs))
            gram_mfma((const float2 *)x, (const float2 *)y, rows, nrhs, partials, gout, nullptr, st);
        else
            coarse::gram<float2>((const float2 *)x, (const float2 *)y, rows, nrhs, partials, gout, nullptr, st);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "apply-Gram launch");
    return CG_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free apply: the two-pass 16-bit kernels take their prepared
// input operands from a file-scope device array instead of a caller
// workspace. Each GPU that loads the library holds its own copy of the array
// until the process ends. Host code never passes the array's name to a
// kernel (on the host that name is a stand-in, not a device address): the
// device address is looked up once per device with hipGetSymbolAddress and
// kept here.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[COARSE_APPLY_NOALLOC_SCRATCH_BYTES];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the device `stream` belongs to (which must
// be the current device: the symbol lookup is made with it current).
static int32_t scratch_for_stream(hipStream_t st, void **out) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipDevice_t sdev = cur;
    e = hipStreamGetDevice(st, &sdev);
    if (e != hipSuccess) return hip_fail(e, "hipStreamGetDevice");
    if ((int)sdev != cur) {
        set_error("stream belongs to device %d but device %d is current; make the stream's device current",
                  (int)sdev, cur);
        return CG_INVALID_ARG;
    }
    if (cur < 0 || cur >= kMaxDevices) {
        set_error("device ordinal %d beyond the %d devices the scratch table holds", cur, kMaxDevices);
        return CG_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[cur]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) {
            set_error("hipGetSymbolAddress(scratch) returned NULL on device %d", cur);
            return CG_HIP_ERROR;
        }
        g_scratch_ptr[cur] = p;
    }
    *out = g_scratch_ptr[cur];
    return CG_OK;
}

extern "C" int32_t coarse_apply_noalloc(const coarse_geom *g, const void *packed, int32_t link_dtype, const void *x,
                                        void *y, int32_t nrhs, int32_t vec_dtype, void *stream) {
    Geom d;
    int32_t rc = check_apply_args(g, packed, link_dtype, x, y, nrhs, vec_dtype, &d);
    if (rc) return rc;
    const bool lowp = link_dtype == COARSE_BF16 || link_dtype == COARSE_FP16;
    const size_t need = lowp ? lowp_ws_bytes(d, nrhs) : 0;
    if (need > (size_t)COARSE_APPLY_NOALLOC_SCRATCH_BYTES) {
        set_error("this apply needs %zu bytes of scratch; the allocation-free apply holds %zu "
                  "(use coarse_apply_ws with a workspace of coarse_apply_workspace_bytes)",
                  need, (size_t)COARSE_APPLY_NOALLOC_SCRATCH_BYTES);
        return CG_WORKSPACE_TOO_SMALL;
    }
    hipStream_t st = (hipStream_t)stream;
    void *ws = nullptr;
    if (need > 0 && (rc = scratch_for_stream(st, &ws))) return rc;
    return launch_apply(d, packed, link_dtype, x, y, nrhs, vec_dtype, nullptr, nullptr, st, 0, -1, ws);
}

// Test hook: force the VALU kernel (the MFMA and VALU paths are parity-tested separately).
extern "C" int32_t coarse_apply_generic(const coarse_geom *g, const void *packed, int32_t link_dtype, const void *x,
                                        void *y, int32_t nrhs, int32_t vec_dtype, void *stream) {
    Geom d;
    int32_t rc = check_apply_args(g, packed, link_dtype, x, y, nrhs, vec_dtype, &d);
    if (rc) return rc;
    if (link_dtype == COARSE_C64_3M) {
        set_error("the VALU kernels read the C64, BF16 and FP16 layouts only");
        return CG_UNSUPPORTED;
    }
    return launch_apply(d, packed, link_dtype, x, y, nrhs, vec_dtype, nullptr, nullptr, (hipStream_t)stream, 1);
}

// Test hook: the VALU adjoint.
extern "C" int32_t coarse_apply_adjoint_generic(const coarse_geom *g, const void *packed, int32_t link_dtype,
                                                const void *x, void *y, int32_t nrhs, int32_t vec_dtype, void *stream) {
    Geom d;
    int32_t rc = check_apply_args(g, packed, link_dtype, x, y, nrhs, vec_dtype, &d);
    if (rc) return rc;
    if (link_dtype == COARSE_C64_3M) {
        set_error("the VALU kernels read the C64, BF16 and FP16 layouts only");
        return CG_UNSUPPORTED;
    }
    return launch_apply_adjoint(d, packed, link_dtype, x, y, nrhs, vec_dtype, (hipStream_t)stream, 1);
}

// Time every kernel variant for this shape on the caller's buffers (y is
// overwritten), keep the fastest in the variant table, append it to the file
// named by COARSE_TUNE_CACHE if set. Synchronises the stream.
extern "C" int32_t coarse_tune_apply(const coarse_geom *g, const void *packed, int32_t link_dtype, const void *x,
                                     void *y, int32_t nrhs, int32_t vec_dtype, int32_t reps, void *stream,
                                     int32_t *best_variant, float *best_us) {
    Geom d;
    int32_t rc = check_apply_args(g, packed, link_dtype, x, y, nrhs, vec_dtype, &d);
    if (rc) return rc;
    if (reps < 1 || reps > 10000) {
        set_error("reps = %d out of range [1, 10000]", reps);
        return CG_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    int nv = 1;
    if (vec_dtype == COARSE_C64 && mfma_supported(d.nb, nrhs, link_dtype, vec_dtype)) {
        if (link_dtype == COARSE_C64) nv = max_variant(d.nb) + 2;  // point split 1, 2, 4; shallow prefetch
        if (link_dtype == COARSE_C64_3M) nv = 2;                    // prefetch depth 1, 2
    }
    hipEvent_t e0, e1;
    COARSE_HIP(hipEventCreate(&e0));
    COARSE_HIP(hipEventCreate(&e1));
    // the variants take turns over three rounds and each keeps its fastest
    // round: a slow drift of the clock under load (the 81-point applies run
    // between 2.05 and 2.3 GHz) then favours none of them
    constexpr int kRounds = 3;
    float vbest[8];
    for (int v = 0; v < 8; ++v) vbest[v] = 1e30f;
    for (int round = 0; round < kRounds && rc == CG_OK; ++round) {
        for (int v = 0; v < nv && rc == CG_OK; ++v) {
            rc = launch_apply(d, packed, link_dtype, x, y, nrhs, vec_dtype, nullptr, nullptr, st, 0, v);  // warm-up
            if (rc) break;
            hipEventRecord(e0, st);
            for (int r = 0; r < reps && rc == CG_OK; ++r)
                rc = launch_apply(d, packed, link_dtype, x, y, nrhs, vec_dtype, nullptr, nullptr, st, 0, v);
            hipEventRecord(e1, st);
            if (rc) break;
            hipError_t e = hipEventSynchronize(e1);
            if (e != hipSuccess) {
                rc = hip_fail(e, "hipEventSynchronize");
                break;
            }
            float ms = 0.f;
            hipEventElapsedTime(&ms, e0, e1);
            const float us = ms * 1000.f / reps;
            if (us < vbest[v]) vbest[v] = us;
        }
    }
    int best = 0;
    float best_t = 1e30f;
    for (int v = 0; v < nv; ++v)
        if (vbest[v] < best_t) {
            best_t = vbest[v];
            best = v;
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_env_locked();
        g_tune[TuneKey{d.nb, nrhs, d.np, link_dtype, vec_dtype}] = best;
        const char *path = getenv("COARSE_TUNE_CACHE");
        if (path) {
            FILE *f = fopen(path, "a");
            if (f) {
                fprintf(f, "%d %d %d %d %d %d %.3f\n", d.nb, nrhs, d.np, link_dtype, vec_dtype, best, best_t);
                fclose(f);
            }
        }
    }
    if (best_variant) *best_variant = best;
    if (best_us) *best_us = best_t;
    return CG_OK;
}

// Number of complex64 MFMA apply variants for this nbasis (point split 1, 2, 4).
extern "C" int32_t coarse_apply_variant_count(int32_t nbasis) {
    if (nbasis < 1 || nbasis > 64) {
        set_error("nbasis = %d out of range [1, 64]", nbasis);
        return CG_INVALID_ARG;
    }
    return max_variant(nbasis) + 2;
}

// Set (variant >= 0) or clear (variant < 0) the table entry of a shape.
extern "C" int32_t coarse_set_apply_variant(int32_t nbasis, int32_t nrhs, int32_t npoint, int32_t link_dtype,
                                            int32_t vec_dtype, int32_t variant) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_env_locked();
    const TuneKey k{nbasis, nrhs, npoint, link_dtype, vec_dtype};
    if (variant < 0)
        g_tune.erase(k);
    else
        g_tune[k] = variant;
    return CG_OK;
}
