// Coarse apply with 16-bit links (BF16 or FP16 storage, one power-of-two
// float32 scale per (site, point) block, complex64 self block), complex64
// vectors, 16x16x32 MFMA with float32 accumulation -- the two-pass form used
// when the caller provides a workspace.
//
// Pass 1 converts each site's X block ONCE into ready-made 16-bit B
// operands of the 16x16x32 MFMA (layout [site][step][column tile][lane][8
// halves]): each 32-bit word holds the pair (Re X, Im X) of one entry, with
// FP16 inputs scaled by one power of two per (site, rhs column). In the 4M
// real embedding (k' = 2j + h) the two output halves use one B operand and
// two A operands derived from each link word in registers:
//   Re Y = sum (Re A, -Im A) . (Re X, Im X)   (the word with its high sign flipped),
//   Im Y = sum (Im A,  Re A) . (Re X, Im X)   (the word with its halves swapped),
// so the operand that every neighbour reads is one 16-bit copy of X.
//
// Pass 2 streams the link blocks of every non-self point through a ring of
// register slots, PD points ahead of the MFMAs (16-byte non-temporal loads,
// each link read once), while the neighbour's operands are copied into a
// double-buffered LDS area shared by the row-tile waves. Each point's
// partial product is scaled (link scale x input column scale) into the
// float32 accumulator. The self point runs first on the float32 MFMA with the
// complex64 block and the unrounded input.
#include <type_traits>

#include "apply.hpp"

namespace coarse {

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32v4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int lowp_site_of_block(int b, int V) {
    return (V % 8 == 0) ? ((b & 7) * (V >> 3) + (b >> 3)) : b;
}

}  // namespace

// ---------------------------------------------------------------------------
// Pass 1: X -> 16-bit B operands (+ FP16 column scales). One workgroup per
// site, one wave per 32-wide k' step (16 rows of X). NBT: 16-column tiles of
// the nrhs columns.
// ---------------------------------------------------------------------------
template <int KIND, int NBT>
__global__ __launch_bounds__(256) void lowp_operand_kernel(const float *__restrict__ x, int nb, int nr,
                                                            u32x4 *__restrict__ xo, float *__restrict__ xs,
                                                            const int *__restrict__ active) {
    __shared__ __align__(16) float xb[64 * 32 * 2];
    __shared__ float inv_s[32];
    if (active != nullptr && *active == 0) return;
    const int s = blockIdx.x;
    const int nst = nb >> 4;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int st = tid >> 6, t = tid & 63, il = t & 15, q = t >> 4;
    const int xblk = nb * nr * 2;
    {
        const float4 *src = reinterpret_cast<const float4 *>(x + (size_t)s * xblk);
        float4 *dst = reinterpret_cast<float4 *>(xb);
        for (int e = tid; e < xblk / 4; e += nthr) dst[e] = src[e];
    }
    __syncthreads();
    if (tid < nr) {
        float sc = 1.f;
        if (KIND == 1) {  // FP16: smallest power of two >= the column's largest component
            float m = 0.f;
            for (int j = 0; j < nb; ++j)
                m = fmaxf(m, fmaxf(fabsf(xb[(j * nr + tid) * 2]), fabsf(xb[(j * nr + tid) * 2 + 1])));
            sc = pow2_ceil(m);
            xs[(size_t)s * nr + tid] = sc;
        }
        inv_s[tid] = 1.f / sc;
    }
    __syncthreads();
    u32x4 *out = xo + (size_t)s * nst * NBT * 64;
#pragma unroll
    for (int b = 0; b < NBT; ++b) {
        const int r = 16 * b + il;
        u32x4 d = u32x4{0, 0, 0, 0};
        if (r < nr) {
            const float inv = inv_s[r];
#pragma unroll
            for (int e2 = 0; e2 < 4; ++e2) {
                const int j = 16 * st + 4 * q + e2;
                const float re = xb[(j * nr + r) * 2] * inv, im = xb[(j * nr + r) * 2 + 1] * inv;
                const uint32_t bl = KIND == 0 ? to_bf16_bits(re) : to_f16_bits(re);
                const uint32_t bh = KIND == 0 ? to_bf16_bits(im) : to_f16_bits(im);
                d[e2] = bl | (bh << 16);
            }
        }
        out[(st * NBT + b) * 64 + t] = d;
    }
}

// ---------------------------------------------------------------------------
// Pass 2: the stencil apply on the prepared operands.
// NBT: 16-column tiles of the nrhs columns (each gives a Re Y and an Im Y
// accumulator tile); NST = nbasis / 16 (waves and k' steps); PD: link
// prefetch depth in points.
// ---------------------------------------------------------------------------
template <int KIND, int NBT, int NST, int PD>
__global__ __launch_bounds__(256) void apply_lowp2_kernel(Geom g, const uint16_t *__restrict__ q16,
                                                           const float *__restrict__ self_c64,
                                                           const float *__restrict__ lscale,
                                                           const float *__restrict__ x, const u32x4 *__restrict__ xo,
                                                           const float *__restrict__ xs, float *__restrict__ y,
                                                           int nr, const float *__restrict__ sub,
                                                           const int *__restrict__ active) {
    typedef typename std::conditional<KIND == 0, bf16x8, f16x8>::type OpT;
    constexpr int RING = PD + 1;
    constexpr int BOPS = NST * NBT * 64;  // u32x4 operands per neighbour
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (active != nullptr && *active == 0) return;

    const int nb = 16 * NST;
    const int s = lowp_site_of_block(blockIdx.x, g.V);
    const int tid = threadIdx.x;
    const int w = tid >> 6, t = tid & 63, il = t & 15, q = t >> 4;
    const int two_nr = 2 * nr;
    const int xblk = nb * nr * 2;
    LDS_AS u32x4 *bbuf = lds_ptr<u32x4>(smem_raw);  // [2][BOPS]
    LDS_AS float *fx = lds_ptr<float>(smem_raw);     // aliases bbuf: self phase, epilogue

    int c[4];
    site_coords(g, s, c);

    // acc[0][b]: Re Y, acc[1][b]: Im Y of columns 16 b + il
    f32x4 acc[2][NBT];
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int b = 0; b < NBT; ++b) acc[v][b] = f32x4{0, 0, 0, 0};

    // every point's neighbour site and link scale, gathered once: read per step
    // from LDS they cost no scalar memory round trip (a per-step scalar load
    // shares the wait counter with the LDS operand reads and stalls the step)
    __shared__ int zsite[81];
    __shared__ float lsc[81];
    for (int p = tid; p < g.np; p += 64 * NST) {
        zsite[p] = displaced(g, c, p, 1);
        lsc[p] = lscale[(size_t)s * g.np + p];
    }
    __syncthreads();

    // ---- self point: complex64 block, float32 input, float32 MFMA ----
    if (g.self_p >= 0) {
        const f32v4 *src = reinterpret_cast<const f32v4 *>(x + (size_t)s * xblk);
        LDS_AS f32v4 *d4 = reinterpret_cast<LDS_AS f32v4 *>(fx);
        for (int e = tid; e < xblk / 4; e += 64 * NST) d4[e] = src[e];
        __syncthreads();
        // B entry of lane (column il, k-group q) at k' = 2j + h, h = q & 1:
        // Re Y takes (Re X, -Im X), Im Y takes (Im X, Re X)
        const int h = q & 1, jq = q >> 1;
        int boff[2][NBT];
        float bsg[2][NBT];
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int b = 0; b < NBT; ++b) {
                const int r = 16 * b + il;
                if (r >= nr) {
                    boff[v][b] = 0;
                    bsg[v][b] = 0.f;
                } else {
                    const int comp = v == 0 ? h : 1 - h;
                    boff[v][b] = 2 * r + comp;
                    bsg[v][b] = (v == 0 && h) ? -1.f : 1.f;
                }
            }
        const float *lb = self_c64 + (size_t)s * nb * nb * 2 + 16 * w * 16 + (q * 16 + il) * 4;
#pragma unroll
        for (int cc = 0; cc < 2 * NST; ++cc) {
            const float4 a = *reinterpret_cast<const float4 *>(lb + cc * nb * 16);
            const float av4[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = 8 * cc + 2 * u + jq;
                const LDS_AS float *xrow = fx + j * two_nr;
#pragma unroll
                for (int v = 0; v < 2; ++v)
#pragma unroll
                    for (int b = 0; b < NBT; ++b)
                        acc[v][b] = mfma16x16x4(av4[u], bsg[v][b] * xrow[boff[v][b]], acc[v][b]);
            }
        }
        __syncthreads();
    }

    // ---- the other points, i = 0 .. np - 2 (p = i, skipping the self point) ----
    const int np = g.np;
    const int npts = (g.self_p >= 0) ? np - 1 : np;
    auto point = [&](int i) { return (g.self_p >= 0 && i >= g.self_p) ? i + 1 : i; };
    const size_t blk_h = (size_t)nb * nb * 2;
    const uint16_t *lsite = q16 + (size_t)s * np * blk_h;

    // loads are branch-free (indices clamped into range): a load under a
    // branch makes the wait-count insertion drain the whole prefetch
    u32x4 bx[NBT];
    float xsn[NBT];
    auto load_b = [&](int i) {
        const int z = zsite[point(min(i, npts - 1))];
        const u32x4 *src = xo + (size_t)z * BOPS;
#pragma unroll
        for (int k = 0; k < NBT; ++k) bx[k] = src[tid + k * 64 * NST];
        if (KIND == 1) {
#pragma unroll
            for (int b = 0; b < NBT; ++b) xsn[b] = xs[(size_t)z * nr + min(16 * b + il, nr - 1)];
        }
    };
    auto store_b = [&](int buf) {
#pragma unroll
        for (int k = 0; k < NBT; ++k) bbuf[buf * BOPS + tid + k * 64 * NST] = bx[k];
    };
    u32x4 ring[RING][NST];
    auto load_a = [&](u32x4 (&a)[NST], int i) {
        const uint16_t *lb = lsite + (size_t)point(min(i, npts - 1)) * blk_h;
#pragma unroll
        for (int st = 0; st < NST; ++st)
            a[st] = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(lb + ((size_t)(st * NST + w) * 64 + t) * 8));
    };

    float xsc[NBT];
#pragma unroll
    for (int b = 0; b < NBT; ++b) xsc[b] = 1.f;
    if (npts > 0) {
        load_b(0);
        load_a(ring[0], 0);
#pragma unroll
        for (int k = 1; k < PD; ++k) load_a(ring[k], k);
        store_b(0);
        if (KIND == 1) {
#pragma unroll
            for (int b = 0; b < NBT; ++b) xsc[b] = xsn[b];
        }
    }
    __syncthreads();

    auto step = [&](int i, u32x4 (&cur)[NST], u32x4 (&nxt)[NST], bool do_b, bool do_pref) {
        if (do_b) load_b(i + 1);
        if (do_pref) load_a(nxt, i + PD);
        const float ls = lsc[point(i)];
        const LDS_AS u32x4 *bc = bbuf + (i & 1) * BOPS;
        f32x4 accp[2][NBT];
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int b = 0; b < NBT; ++b) accp[v][b] = f32x4{0, 0, 0, 0};
#pragma unroll
        for (int st = 0; st < NST; ++st) {
            // each word (Re A, Im A): (Re A, -Im A) for Re Y, (Im A, Re A) for Im Y
            const u32x4 aw = cur[st];
            u32x4 ar, ai;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                ar[e] = aw[e] ^ 0x80000000u;
                ai[e] = __builtin_amdgcn_alignbit(aw[e], aw[e], 16);
            }
            const OpT avr = __builtin_bit_cast(OpT, ar), avi = __builtin_bit_cast(OpT, ai);
#pragma unroll
            for (int b = 0; b < NBT; ++b) {
                const OpT bv = __builtin_bit_cast(OpT, bc[(st * NBT + b) * 64 + t]);
                if (KIND == 0) {
                    accp[0][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(avr, bv, accp[0][b], 0, 0, 0);
                    accp[1][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(avi, bv, accp[1][b], 0, 0, 0);
                } else {
                    accp[0][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(avr, bv, accp[0][b], 0, 0, 0);
                    accp[1][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(avi, bv, accp[1][b], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int b = 0; b < NBT; ++b) {
            const float f = KIND == 1 ? ls * xsc[b] : ls;
            acc[0][b] += accp[0][b] * f;
            acc[1][b] += accp[1][b] * f;
        }
        if (do_b) {
            store_b((i + 1) & 1);
            if (KIND == 1) {
#pragma unroll
                for (int b = 0; b < NBT; ++b) xsc[b] = xsn[b];
            }
        }
        __syncthreads();
    };

    // steady state: whole ring rounds with every load in range (branch-free)
    int i0 = 0;
    for (; i0 + RING + PD <= npts; i0 += RING) {
#pragma unroll
        for (int k = 0; k < RING; ++k) step(i0 + k, ring[k], ring[(k + PD) % RING], true, true);
    }
    // tail: at most RING + PD - 1 steps, loads guarded
#pragma unroll
    for (int k = 0; k < RING + PD; ++k) {
        const int i = i0 + k;
        if (i < npts) step(i, ring[k % RING], ring[(k + PD) % RING], i + 1 < npts, i + PD < npts);
    }

    // epilogue: accumulators -> LDS ([row][Re Y | Im Y]) -> complex output
    LDS_AS float *out = fx;
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int b = 0; b < NBT; ++b) {
            const int r = 16 * b + il;
            if (r < nr) {
#pragma unroll
                for (int k = 0; k < 4; ++k) out[(16 * w + 4 * q + k) * two_nr + v * nr + r] = acc[v][b][k];
            }
        }
    __syncthreads();
    float *yo = y + (size_t)s * xblk;
    const float *so = sub ? sub + (size_t)s * xblk : nullptr;
    for (int e = tid; e < nb * nr; e += 64 * NST) {
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
// Host side
// ---------------------------------------------------------------------------
static int lowp_nbt(int nr) { return (nr + 15) / 16; }

size_t lowp_ws_bytes(const Geom &g, int nr) {
    const int nst = g.nb / 16, nbt = lowp_nbt(nr);
    return align256((size_t)g.V * nst * nbt * 64 * 16) + align256((size_t)g.V * nr * 4);
}

template <int KIND, int NBT, int NST>
static void launch_lowp2_t(const Geom &g, const uint16_t *q16, const float *self_c64, const float *scales,
                           const float *x, float *y, int nr, const float *sub, const int *active, void *ws,
                           hipStream_t st) {
    u32x4 *xo = reinterpret_cast<u32x4 *>(ws);
    float *xs = reinterpret_cast<float *>(reinterpret_cast<char *>(ws) +
                                          align256((size_t)g.V * NST * NBT * 64 * 16));
    hipLaunchKernelGGL((lowp_operand_kernel<KIND, NBT>), dim3(g.V), dim3(64 * NST), 0, st, x, g.nb, nr, xo, xs,
                       active);
    const size_t lds = (size_t)2 * NST * NBT * 64 * 16;
    hipLaunchKernelGGL((apply_lowp2_kernel<KIND, NBT, NST, 2>), dim3(g.V), dim3(64 * NST), lds, st, g, q16, self_c64,
                       scales, x, xo, xs, y, nr, sub, active);
}

template <int KIND, int NBT>
static void launch_lowp2_nst(const Geom &g, const uint16_t *q16, const float *self_c64, const float *scales,
                             const float *x, float *y, int nr, const float *sub, const int *active, void *ws,
                             hipStream_t st) {
    switch (g.nb / 16) {
        case 1: launch_lowp2_t<KIND, NBT, 1>(g, q16, self_c64, scales, x, y, nr, sub, active, ws, st); break;
        case 2: launch_lowp2_t<KIND, NBT, 2>(g, q16, self_c64, scales, x, y, nr, sub, active, ws, st); break;
        case 3: launch_lowp2_t<KIND, NBT, 3>(g, q16, self_c64, scales, x, y, nr, sub, active, ws, st); break;
        default: launch_lowp2_t<KIND, NBT, 4>(g, q16, self_c64, scales, x, y, nr, sub, active, ws, st); break;
    }
}

template <int KIND>
static void launch_lowp2_k(const Geom &g, const uint16_t *q16, const float *self_c64, const float *scales,
                           const float *x, float *y, int nr, const float *sub, const int *active, void *ws,
                           hipStream_t st) {
    switch (lowp_nbt(nr)) {
        case 1: launch_lowp2_nst<KIND, 1>(g, q16, self_c64, scales, x, y, nr, sub, active, ws, st); break;
        default: launch_lowp2_nst<KIND, 2>(g, q16, self_c64, scales, x, y, nr, sub, active, ws, st); break;
    }
}

void launch_lowp_ws(const Geom &g, int kind, const uint16_t *q16, const float *self_c64, const float *scales,
                    const float *x, float *y, int nr, const float *sub, const int *active, void *ws,
                    hipStream_t st) {
    if (kind == 0)
        launch_lowp2_k<0>(g, q16, self_c64, scales, x, y, nr, sub, active, ws, st);
    else
        launch_lowp2_k<1>(g, q16, self_c64, scales, x, y, nr, sub, active, ws, st);
}

}  // namespace coarse
