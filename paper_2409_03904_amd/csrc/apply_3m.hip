// Coarse apply in the 3M form: each complex multiply-add of the per-site GEMM
// Y(x) = sum_p A_p(x) X(x + delta_p) is computed from three real products,
//   T1 = Ar Xr,  T2 = Ai Xi,  T3 = (Ar + Ai)(Xr + Xi),
//   Re Y = T1 - T2,  Im Y = T3 - T1 - T2,
// on 16x16x4 float32 MFMA with the real K index = link column j. Against the
// 4M real embedding (one M x 2N x 2K product) this is 3/4 of the MFMA work at
// the same link bytes, for nrhs a multiple of 16 (the N tiles are nrhs wide,
// not 2 nrhs).
//
// Links (complex64, 3M layout, nbasis % 16 == 0; c64_3m_block_offset): lane
// (row il, k-group q) of a wave's 16-row tile reads with one 16-byte
// non-temporal load the (Re, Im) pairs of columns 8c + q and 8c + 4 + q -- the
// A operands of two k-steps;
// Ar + Ai is one add per step. The loads run PD points ahead in a register
// ring with compile-time slots, as in the 4M kernel. The neighbour block
// X(x + delta_p) is staged once per point in LDS as two planar real arrays
// Xr, Xi (row stride padded to whole 16-column tiles; with two column tiles
// the halves of odd rows are swapped, so the two k-groups that one LDS cycle
// serves, rows j and j + 1, fall in different banks), double buffered and
// shared by the waves; Xr + Xi is formed from the two values a lane reads for
// T1 and T2. A scheduling barrier after each eight-column chunk keeps the
// next chunk's operand reads behind its products (fewer live registers).
#include "apply.hpp"
#include "gram_epi.hpp"

namespace coarse {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int site3m_of_block(int b, int V) {
    return (V % 8 == 0) ? ((b & 7) * (V >> 3) + (b >> 3)) : b;
}

}  // namespace

// NT3 = nrhs / 16 rounded up (column tiles); NST = nbasis / 16 (waves);
// NCH = nbasis / 8 (chunks of eight link columns); PD = prefetch depth.
// CHEB: the epilogue runs one degree of a Chebyshev recurrence (ChebEpi)
// instead of storing y = M x (or sub - M x).
// GRAM: y = M x, and the Gram x^H y of the workgroup's sites (the blocks
// b, b + nblk, ... of the site order) accumulated in LDS and written as one
// partial (GramEpi); the site's own x block is staged beside the planes, and
// each wave forms the Gram of its own rows from its accumulators.
// Occupancy asked of the Gram-fused form: left to itself the compiler gives
// its one-column-tile instances 20-30 more registers than the plain apply
// (one wave per SIMD fewer); two column tiles keep the default (asking for
// more spills). The plain two-column-tile instance at nbasis 64 with one point
// of prefetch is held to three waves per SIMD (152 registers; the LDS allows
// three workgroups); with two points it keeps the default (two waves).
template <int NT3, int NST, int PD, bool GRAM>
constexpr int apply3m_min_waves() {
    return (GRAM && NT3 == 1) ? (NST <= 2 ? 4 : 3) : ((!GRAM && NT3 == 2 && NST == 4 && PD == 1) ? 3 : 1);
}

template <int NT3, int NST, int PD, bool CHEB, bool GRAM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(apply3m_min_waves<NT3, NST, PD, GRAM>())))
void apply_3m_kernel(Geom g, const float *__restrict__ links,
                                                        const float *__restrict__ x, float *__restrict__ y, int nr,
                                                        const float *__restrict__ sub,
                                                        const int *__restrict__ active, ChebEpi ce, GramEpi ge) {
    constexpr int NCH = 2 * NST;
    constexpr int RING = PD + 1;
    constexpr int RS = 16 * NT3;          // padded row stride of a staged plane
    constexpr int NB = 16 * NST;
    constexpr int PLANE = NB * RS;         // floats per plane
    constexpr int XV = (NT3 * 16 + 7) / 8;  // float4 staging loads per thread, bound (nr <= 16 NT3)
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (active != nullptr && *active == 0) return;
    // physical column of (row j, column r) in a staged plane
    auto pcol = [](int j, int r) { return NT3 == 2 ? (r ^ ((j & 1) << 4)) : r; };

    const int tid = threadIdx.x, nthr = 64 * NST;
    const int w = tid >> 6, t = tid & 63, il = t & 15, q = t >> 4;
    const int xblk = NB * nr * 2;  // floats of a complex block
    LDS_AS float *pl = lds_ptr<float>(smem_raw);  // [2 buffers][Xr | Xi]
    // GRAM: the site's x block and the Gram accumulator after the planes
    LDS_AS float *dsite = pl + 2 * 2 * PLANE;
    LDS_AS double *gacc = reinterpret_cast<LDS_AS double *>(dsite + NB * RS * 2);  // (Re, Im) pairs
    const int nvec = xblk >> 2;
    if (GRAM) {
        for (int e = tid; e < 2 * nr * nr; e += nthr) gacc[e] = 0.0;
        // (the first read of gacc follows the first site's barriers)
    }

    const int nsites = GRAM ? (g.V - (int)blockIdx.x + ge.nblk - 1) / ge.nblk : 1;
    for (int site_k = 0; site_k < nsites; ++site_k) {
    const int s = site3m_of_block(GRAM ? (int)blockIdx.x + site_k * ge.nblk : (int)blockIdx.x, g.V);

    int c[4];
    site_coords(g, s, c);

    // staging: float4 e of the complex block holds entries (j, r), (j, r + 1)
    f4v xr[XV];
    auto load_x = [&](int p) {
        const f4v *src = reinterpret_cast<const f4v *>(x + (size_t)displaced(g, c, p, 1) * xblk);
#pragma unroll
        for (int k = 0; k < XV; ++k) xr[k] = src[min(tid + k * nthr, nvec - 1)];
    };
    auto store_x = [&](int buf) {
        LDS_AS float *br = pl + buf * 2 * PLANE, *bi = br + PLANE;
#pragma unroll
        for (int k = 0; k < XV; ++k) {
            // no branch: a thread past the block re-writes the last float4
            // (loaded clamped, so the same values); a guard here lets the
            // compiler sink the staging load into it, after the link loads,
            // whose wait then exposes their latency every point
            const int e = min(tid + k * nthr, nvec - 1);
            const int f = 2 * e;  // first complex entry of the float4
            const int j = f / nr, r = f - j * nr;
            const f4v v = xr[k];
            const int o1 = j * RS + pcol(j, r);
            br[o1] = v.x;
            bi[o1] = v.y;
            // second entry: same row unless r + 1 == nr (odd nr only)
            const int j2 = (r + 1 < nr) ? j : j + 1, r2 = (r + 1 < nr) ? r + 1 : 0;
            const int o2 = j2 * RS + pcol(j2, r2);
            br[o2] = v.z;
            bi[o2] = v.w;
        }
    };

    const size_t blk_floats = (size_t)NB * NB * 2;
    const float *lsite = links + (size_t)s * g.np * blk_floats;
    const int lane_off = c64_3m_block_offset(NB, 16 * w + il, q, 0);  // entry (il, q) of chunk 0, tile w
    f4v ring[RING][NCH];
    auto load_a = [&](f4v (&a)[NCH], int p) {
        const float *lb = lsite + (size_t)p * blk_floats + lane_off;
#pragma unroll
        for (int cc = 0; cc < NCH; ++cc)
            a[cc] = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(lb + cc * NB * 16));
    };

    f32x4 t1[NT3], t2[NT3], t3[NT3];
#pragma unroll
    for (int nt = 0; nt < NT3; ++nt) t1[nt] = t2[nt] = t3[nt] = f32x4{0, 0, 0, 0};

    const int np = g.np;
    const size_t sx = (size_t)s * xblk;
    // GRAM: the site's own block as [row][column] complex64 (its self-point
    // staging, when the stencil has one, reads the same lines); loaded first,
    // so that storing it waits for nothing issued after it
    f4v dx[XV];
    if (GRAM) {
        const f4v *src = reinterpret_cast<const f4v *>(x + sx);
#pragma unroll
        for (int k = 0; k < XV; ++k) dx[k] = src[min(tid + k * nthr, nvec - 1)];
    }
    load_x(0);
#pragma unroll
    for (int k = 0; k < PD; ++k) load_a(ring[k], min(k, np - 1));
    if (GRAM) {
        LDS_AS f4v *dst = reinterpret_cast<LDS_AS f4v *>(dsite);
#pragma unroll
        for (int k = 0; k < XV; ++k) dst[min(tid + k * nthr, nvec - 1)] = dx[k];
    }
    store_x(0);
    __syncthreads();

    auto step = [&](int i, f4v (&cur)[NCH], f4v (&nxt)[NCH], bool do_x, bool do_pref) {
        if (do_x) load_x(i + 1);
        if (do_pref) load_a(nxt, i + PD);
        const LDS_AS float *br = pl + (i & 1) * 2 * PLANE, *bi = br + PLANE;
#pragma unroll
        for (int cc = 0; cc < NCH; ++cc) {
            const f4v a4 = cur[cc];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float ar = a4[2 * h], ai = a4[2 * h + 1], as = ar + ai;
                const int j = 8 * cc + 4 * h + q;  // B lane (k-group q, column il)
#pragma unroll
                for (int nt = 0; nt < NT3; ++nt) {
                    const int o = j * RS + pcol(j, 16 * nt + il);
                    const float xre = br[o], xim = bi[o];
                    t1[nt] = mfma16x16x4(ar, xre, t1[nt]);
                    t2[nt] = mfma16x16x4(ai, xim, t2[nt]);
                    t3[nt] = mfma16x16x4(as, xre + xim, t3[nt]);
                }
            }
            __builtin_amdgcn_sched_barrier(0);  // one chunk at a time
        }
        if (do_x) store_x((i + 1) & 1);
        __syncthreads();
    };

    // steady state without branches, then a guarded tail (as in the 4M kernel)
    int i0 = 0;
    for (; i0 + RING + PD <= np; i0 += RING) {
#pragma unroll
        for (int k = 0; k < RING; ++k) step(i0 + k, ring[k], ring[(k + PD) % RING], true, true);
    }
#pragma unroll
    for (int k = 0; k < RING + PD; ++k) {
        const int i = i0 + k;
        if (i < np) step(i, ring[k % RING], ring[(k + PD) % RING], i + 1 < np, i + PD < np);
    }

    if (CHEB) {
        // M t into LDS (free after the last point's barrier) as the site's
        // [row][column][re, im] block, then every thread takes whole float4
        // chunks: t, t_prev and y are read and t_next and y written with
        // coalesced 16-byte accesses
        LDS_AS float *zb = pl;
#pragma unroll
        for (int nt = 0; nt < NT3; ++nt) {
            const int r = 16 * nt + il;
            if (r < nr) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * w + 4 * q + v;
                    zb[(row * nr + r) * 2] = t1[nt][v] - t2[nt][v];
                    zb[(row * nr + r) * 2 + 1] = t3[nt][v] - t1[nt][v] - t2[nt][v];
                }
            }
        }
        __syncthreads();
        const LDS_AS f4v *z4 = reinterpret_cast<const LDS_AS f4v *>(zb);
        const f4v *tx = reinterpret_cast<const f4v *>(x + sx);
        const f4v *tp = reinterpret_cast<const f4v *>(ce.t_prev + sx);
        f4v *tn = reinterpret_cast<f4v *>(ce.t_next + sx);
        f4v *yy = reinterpret_cast<f4v *>(ce.y + sx);
        for (int e = tid; e < nvec; e += nthr) {
            const f4v tv = tx[e];
            f4v nv = ce.A * z4[e] + ce.B * tv;
            if (ce.C != 0.f) nv += ce.C * tp[e];
            tn[e] = nv;
            f4v yv = ce.E * nv + ce.F * tv;
            if (ce.D != 0.f) yv += ce.D * yy[e];
            yy[e] = yv;
        }
    } else {
        // epilogue: lane (il, q) holds rows 4q + v of column 16 nt + il
        float *yo = y + sx;
        const float *so = (!GRAM && sub) ? sub + sx : nullptr;  // the Gram-fused form stores M x
        float2 zv[NT3][4], dv[NT3][4];  // GRAM: Z and D of the lane's entries (0 past column nr)
#pragma unroll
        for (int nt = 0; nt < NT3; ++nt) {
            const int r = 16 * nt + il;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * w + 4 * q + v;
                float re = t1[nt][v] - t2[nt][v];
                float im = t3[nt][v] - t1[nt][v] - t2[nt][v];
                if (GRAM) {
                    const int rc = r < nr ? r : nr - 1;
                    const float dre = dsite[2 * (row * nr + rc)], dim = dsite[2 * (row * nr + rc) + 1];
                    zv[nt][v] = r < nr ? make_float2(re, im) : make_float2(0.f, 0.f);
                    dv[nt][v] = r < nr ? make_float2(dre, dim) : make_float2(0.f, 0.f);
                }
                if (r < nr) {
                    const size_t o = ((size_t)row * nr + r) * 2;
                    if (so) {
                        re = so[o] - re;
                        im = so[o + 1] - im;
                    }
                    yo[o] = re;
                    yo[o + 1] = im;
                }
            }
        }
        // the waves' turns end with barriers, after which the next site's
        // block may be staged over dsite
        if (GRAM) gram_rows<NT3>(dv, zv, nr, gacc, w, NST);
    }
    }  // sites

    if (GRAM) {
        double2 *out = ge.partials + (size_t)blockIdx.x * nr * nr;
        for (int e = tid; e < nr * nr; e += nthr) out[e] = make_double2(gacc[2 * e], gacc[2 * e + 1]);
    }
}

// ---------------------------------------------------------------------------
// Adjoint in the 3M form on the same packed links:
//   y(x) = sum_p A_p(x - delta_p)^H X(x - delta_p),
//   Re y = Ar^T Xr + Ai^T Xi = T1 + T2,
//   Im y = Ar^T Xi - Ai^T Xr = T3 - T1 + T2  with T3 = (Ar - Ai)^T (Xr + Xi).
// The contraction runs over the link ROW i, so a wave owns a 16-column tile j
// of the output and the A operand of lane (column il, k-group q) at k-step s
// is the entry (i = 4 s + q, j = 16 w + il) of the neighbour's link block:
// one 8-byte (Re, Im) load straight from the 3M layout, whose entry order
// makes the 64 lanes of a step read four whole 128-byte lines (an order in
// which they read half lines ran at 0.5 of the forward kernel's rate), no
// transpose through LDS. The input operand is the neighbour's X staged as in
// the forward kernel (there too the contraction index is the row of X): two
// planes Xr, Xi, the sum formed per read, a scheduling barrier every two
// k-steps.
// ---------------------------------------------------------------------------
template <int NT3, int NST, int PD>
__global__ __launch_bounds__(256) void adjoint_3m_kernel(Geom g, const float *__restrict__ links,
                                                          const float *__restrict__ x, float *__restrict__ y, int nr) {
    constexpr int RING = PD + 1;
    constexpr int RS = 16 * NT3;
    constexpr int NB = 16 * NST;
    constexpr int NSTEP = NB / 4;          // k-steps per point
    constexpr int PLANE = NB * RS;
    constexpr int XV = (NT3 * 16 + 7) / 8;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    auto pcol = [](int j, int r) { return NT3 == 2 ? (r ^ ((j & 1) << 4)) : r; };

    const int s = site3m_of_block(blockIdx.x, g.V);
    const int tid = threadIdx.x, nthr = 64 * NST;
    const int w = tid >> 6, t = tid & 63, il = t & 15, q = t >> 4;
    const int xblk = NB * nr * 2;
    LDS_AS float *pl = lds_ptr<float>(smem_raw);

    int c[4];
    site_coords(g, s, c);

    const int nvec = xblk >> 2;
    f4v xr[XV];
    auto load_x = [&](int src_site) {
        const f4v *src = reinterpret_cast<const f4v *>(x + (size_t)src_site * xblk);
#pragma unroll
        for (int k = 0; k < XV; ++k) xr[k] = src[min(tid + k * nthr, nvec - 1)];
    };
    auto store_x = [&](int buf) {
        LDS_AS float *br = pl + buf * 2 * PLANE, *bi = br + PLANE;
#pragma unroll
        for (int k = 0; k < XV; ++k) {
            const int e = min(tid + k * nthr, nvec - 1);  // branch-free, as in the forward kernel
            const int f = 2 * e;
            const int j = f / nr, r = f - j * nr;
            const f4v v = xr[k];
            const int o1 = j * RS + pcol(j, r);
            br[o1] = v.x;
            bi[o1] = v.y;
            const int j2 = (r + 1 < nr) ? j : j + 1, r2 = (r + 1 < nr) ? r + 1 : 0;
            const int o2 = j2 * RS + pcol(j2, r2);
            br[o2] = v.z;
            bi[o2] = v.w;
        }
    };

    // the point's source site x - delta_p: its links (point p) and its X
    const size_t blk_floats = (size_t)NB * NB * 2;
    const int lane_off = c64_3m_block_offset(NB, q, 16 * w + il, 0);
    f2v ring[RING][NSTEP];
    auto load_a = [&](f2v (&a)[NSTEP], int p) {
        const float *lb = links + ((size_t)displaced(g, c, p, -1) * g.np + p) * blk_floats + lane_off;
#pragma unroll
        for (int k = 0; k < NSTEP; ++k)
            a[k] = __builtin_nontemporal_load(reinterpret_cast<const f2v *>(lb + (k >> 2) * 256 + (k & 3) * 64));
    };

    f32x4 t1[NT3], t2[NT3], t3[NT3];
#pragma unroll
    for (int nt = 0; nt < NT3; ++nt) t1[nt] = t2[nt] = t3[nt] = f32x4{0, 0, 0, 0};

    const int np = g.np;
    load_x(displaced(g, c, 0, -1));
#pragma unroll
    for (int k = 0; k < PD; ++k) load_a(ring[k], min(k, np - 1));
    store_x(0);
    __syncthreads();

    auto step = [&](int i, f2v (&cur)[NSTEP], f2v (&nxt)[NSTEP], bool do_x, bool do_pref) {
        if (do_x) load_x(displaced(g, c, i + 1, -1));
        if (do_pref) load_a(nxt, i + PD);
        // keep the next point's loads in front of this point's products (left
        // to itself the scheduler sinks them behind the MFMAs, and the staging
        // wait after the products then exposes their whole latency)
        __builtin_amdgcn_sched_barrier(0);
        const LDS_AS float *br = pl + (i & 1) * 2 * PLANE, *bi = br + PLANE;
#pragma unroll
        for (int k = 0; k < NSTEP; ++k) {
            const float ar = cur[k].x, ai = cur[k].y, ad = ar - ai;
            const int row = 4 * k + q;  // B lane (k-group q, column il): X row i
#pragma unroll
            for (int nt = 0; nt < NT3; ++nt) {
                const int o = row * RS + pcol(row, 16 * nt + il);
                const float xre = br[o], xim = bi[o];
                t1[nt] = mfma16x16x4(ar, xre, t1[nt]);
                t2[nt] = mfma16x16x4(ai, xim, t2[nt]);
                t3[nt] = mfma16x16x4(ad, xre + xim, t3[nt]);
            }
            if (k & 1) __builtin_amdgcn_sched_barrier(0);  // two k-steps at a time
        }
        if (do_x) store_x((i + 1) & 1);
        __syncthreads();
    };

    int i0 = 0;
    for (; i0 + RING + PD <= np; i0 += RING) {
#pragma unroll
        for (int k = 0; k < RING; ++k) step(i0 + k, ring[k], ring[(k + PD) % RING], true, true);
    }
#pragma unroll
    for (int k = 0; k < RING + PD; ++k) {
        const int i = i0 + k;
        if (i < np) step(i, ring[k % RING], ring[(k + PD) % RING], i + 1 < np, i + PD < np);
    }

    // lane (il, q) holds output rows j = 16 w + 4 q + v of column 16 nt + il
    float *yo = y + (size_t)s * xblk;
#pragma unroll
    for (int nt = 0; nt < NT3; ++nt) {
        const int r = 16 * nt + il;
        if (r < nr) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * w + 4 * q + v;
                const size_t o = ((size_t)row * nr + r) * 2;
                yo[o] = t1[nt][v] + t2[nt][v];
                yo[o + 1] = t3[nt][v] - t1[nt][v] + t2[nt][v];
            }
        }
    }
}

template <int NT3, int NST>
static void launch_adjoint_3m_t(const Geom &g, const float *links, const float *x, float *y, int nr,
                                hipStream_t st, int variant) {
    const size_t lds = (size_t)2 * 2 * (16 * NST) * (16 * NT3) * sizeof(float);
    if (variant >= 1)
        hipLaunchKernelGGL((adjoint_3m_kernel<NT3, NST, 2>), dim3(g.V), dim3(64 * NST), lds, st, g, links, x, y, nr);
    else
        hipLaunchKernelGGL((adjoint_3m_kernel<NT3, NST, 1>), dim3(g.V), dim3(64 * NST), lds, st, g, links, x, y, nr);
}

template <int NT3>
static void launch_adjoint_3m_nst(const Geom &g, const float *links, const float *x, float *y, int nr,
                                  hipStream_t st, int variant) {
    switch (g.nb / 16) {
        case 1: launch_adjoint_3m_t<NT3, 1>(g, links, x, y, nr, st, variant); break;
        case 2: launch_adjoint_3m_t<NT3, 2>(g, links, x, y, nr, st, variant); break;
        case 3: launch_adjoint_3m_t<NT3, 3>(g, links, x, y, nr, st, variant); break;
        default: launch_adjoint_3m_t<NT3, 4>(g, links, x, y, nr, st, variant); break;
    }
}

void launch_adjoint_3m(const Geom &g, const float *links, const float *x, float *y, int nr, hipStream_t st,
                       int variant) {
    if (nr <= 16)
        launch_adjoint_3m_nst<1>(g, links, x, y, nr, st, variant);
    else
        launch_adjoint_3m_nst<2>(g, links, x, y, nr, st, variant);
}

// ---------------------------------------------------------------------------
// The forward 3M form with complex128 vectors and float64 accumulation, on the
// same 3M-layout links (the residual b - M x of the outer defect-correction
// loop): the link values are exact in double, T1, T2 and T3 run on 16x16x4
// f64 MFMA. The neighbour block is staged as two planes Xr, Xi of doubles
// (double-buffered, 64 KB at nbasis 64, nrhs 32, two workgroups per CU);
// Xr + Xi is formed from the two values a lane reads for T1 and T2. f64
// accumulator layout: lane (il, q) register u holds tile row q + 4 u.
// ---------------------------------------------------------------------------
template <int NT3, int NST>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void apply_3m_f64_kernel(Geom g, const float *__restrict__ links, const double *__restrict__ x,
                         double *__restrict__ y, int nr, const double *__restrict__ sub,
                         const int *__restrict__ active) {
    constexpr int NCH = 2 * NST;
    constexpr int RING = 2;               // one point of link prefetch
    constexpr int RS = 16 * NT3;          // padded row stride of a staged plane
    constexpr int NB = 16 * NST;
    constexpr int PLANE = NB * RS;        // doubles per plane
    constexpr int XV = 4 * NT3;           // complex128 staging loads per thread, bound (nr <= 16 NT3)
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (active != nullptr && *active == 0) return;
    auto pcol = [](int j, int r) { return NT3 == 2 ? (r ^ ((j & 1) << 4)) : r; };

    const int s = site3m_of_block(blockIdx.x, g.V);
    const int tid = threadIdx.x, nthr = 64 * NST;
    const int w = tid >> 6, t = tid & 63, il = t & 15, q = t >> 4;
    const int xblk = NB * nr;  // complex128 entries of a site block
    LDS_AS double *pl = lds_ptr<double>(smem_raw);  // [2 buffers][Xr | Xi]

    int c[4];
    site_coords(g, s, c);

    double2 xv[XV];
    auto load_x = [&](int p) {
        const double2 *src = reinterpret_cast<const double2 *>(x) + (size_t)displaced(g, c, p, 1) * xblk;
#pragma unroll
        for (int k = 0; k < XV; ++k) xv[k] = src[min(tid + k * nthr, xblk - 1)];
    };
    auto store_x = [&](int buf) {
        LDS_AS double *br = pl + buf * 2 * PLANE, *bi = br + PLANE;
#pragma unroll
        for (int k = 0; k < XV; ++k) {
            // branch-free: a thread past the block re-writes the last entry
            const int e = min(tid + k * nthr, xblk - 1);
            const int j = e / nr, r = e - j * nr;
            const int o = j * RS + pcol(j, r);
            br[o] = xv[k].x;
            bi[o] = xv[k].y;
        }
    };

    const size_t blk_floats = (size_t)NB * NB * 2;
    const float *lsite = links + (size_t)s * g.np * blk_floats;
    const int lane_off = c64_3m_block_offset(NB, 16 * w + il, q, 0);
    f4v ring[RING][NCH];
    auto load_a = [&](f4v (&a)[NCH], int p) {
        const float *lb = lsite + (size_t)p * blk_floats + lane_off;
#pragma unroll
        for (int cc = 0; cc < NCH; ++cc)
            a[cc] = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(lb + cc * NB * 16));
    };

    f64x4 t1[NT3], t2[NT3], t3[NT3];
#pragma unroll
    for (int nt = 0; nt < NT3; ++nt) t1[nt] = t2[nt] = t3[nt] = f64x4{0, 0, 0, 0};

    const int np = g.np;
    load_x(0);
    load_a(ring[0], 0);
    store_x(0);
    __syncthreads();

    auto step = [&](int i, f4v (&cur)[NCH], f4v (&nxt)[NCH], bool do_x, bool do_pref) {
        if (do_x) load_x(i + 1);
        if (do_pref) load_a(nxt, i + 1);
        const LDS_AS double *br = pl + (i & 1) * 2 * PLANE, *bi = br + PLANE;
#pragma unroll
        for (int cc = 0; cc < NCH; ++cc) {
            const f4v a4 = cur[cc];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const double ar = a4[2 * h], ai = a4[2 * h + 1], as = ar + ai;
                const int j = 8 * cc + 4 * h + q;  // B lane (k-group q, column il)
#pragma unroll
                for (int nt = 0; nt < NT3; ++nt) {
                    const int o = j * RS + pcol(j, 16 * nt + il);
                    const double xre = br[o], xim = bi[o];
                    t1[nt] = mfma16x16x4(ar, xre, t1[nt]);
                    t2[nt] = mfma16x16x4(ai, xim, t2[nt]);
                    t3[nt] = mfma16x16x4(as, xre + xim, t3[nt]);
                }
            }
            // one chunk at a time: hoisting every chunk's operand reads and
            // conversions ahead of the products would not fit the registers
            __builtin_amdgcn_sched_barrier(0);
        }
        if (do_x) store_x((i + 1) & 1);
        __syncthreads();
    };

    // steady state without branches, then a guarded tail (as in the float kernel)
    int i0 = 0;
    for (; i0 + RING + 1 <= np; i0 += RING) {
#pragma unroll
        for (int k = 0; k < RING; ++k) step(i0 + k, ring[k], ring[(k + 1) % RING], true, true);
    }
#pragma unroll
    for (int k = 0; k < RING + 1; ++k) {
        const int i = i0 + k;
        if (i < np) step(i, ring[k % RING], ring[(k + 1) % RING], i + 1 < np, i + 1 < np);
    }

    double2 *yo = reinterpret_cast<double2 *>(y) + (size_t)s * xblk;
    const double2 *so = sub ? reinterpret_cast<const double2 *>(sub) + (size_t)s * xblk : nullptr;
#pragma unroll
    for (int nt = 0; nt < NT3; ++nt) {
        const int r = 16 * nt + il;
        if (r < nr) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int row = 16 * w + q + 4 * u;
                const size_t o = (size_t)row * nr + r;
                double re = t1[nt][u] - t2[nt][u];
                double im = t3[nt][u] - t1[nt][u] - t2[nt][u];
                if (so) {
                    re = so[o].x - re;
                    im = so[o].y - im;
                }
                yo[o] = make_double2(re, im);
            }
        }
    }
}

template <int NT3, int NST>
static void launch_3m_f64_t(const Geom &g, const float *links, const double *x, double *y, int nr,
                            const double *sub, const int *active, hipStream_t st) {
    const size_t lds = (size_t)2 * 2 * (16 * NST) * (16 * NT3) * sizeof(double);  // at most 64 KB
    hipLaunchKernelGGL((apply_3m_f64_kernel<NT3, NST>), dim3(g.V), dim3(64 * NST), lds, st, g, links, x, y, nr, sub,
                       active);
}

template <int NT3>
static void launch_3m_f64_nst(const Geom &g, const float *links, const double *x, double *y, int nr,
                              const double *sub, const int *active, hipStream_t st) {
    switch (g.nb / 16) {
        case 1: launch_3m_f64_t<NT3, 1>(g, links, x, y, nr, sub, active, st); break;
        case 2: launch_3m_f64_t<NT3, 2>(g, links, x, y, nr, sub, active, st); break;
        case 3: launch_3m_f64_t<NT3, 3>(g, links, x, y, nr, sub, active, st); break;
        default: launch_3m_f64_t<NT3, 4>(g, links, x, y, nr, sub, active, st); break;
    }
}

void launch_apply_3m_f64(const Geom &g, const float *links, const double *x, double *y, int nr, const double *sub,
                         const int *active, hipStream_t st) {
    if (nr <= 16)
        launch_3m_f64_nst<1>(g, links, x, y, nr, sub, active, st);
    else
        launch_3m_f64_nst<2>(g, links, x, y, nr, sub, active, st);
}

// variant 0: prefetch one point ahead; variant 1: two points (more bytes in
// flight, more registers; at nbasis 64 and two column tiles it halves the
// occupancy). The autotuner times both.
template <int NT3, int NST, bool CHEB, bool GRAM>
static void launch_3m_t(const Geom &g, const float *links, const float *x, float *y, int nr, const float *sub,
                        const int *active, const ChebEpi &ce, const GramEpi &ge, hipStream_t st, int variant) {
    size_t lds = (size_t)2 * 2 * (16 * NST) * (16 * NT3) * sizeof(float);
    if (GRAM) lds += (size_t)(16 * NST) * (16 * NT3) * 2 * sizeof(float) + (size_t)nr * nr * sizeof(double2);
    const dim3 grid(GRAM ? ge.nblk : g.V);
    if (lds > 64 * 1024) {  // the Gram-fused form at nbasis 64, nrhs 32: 80 KB of the 160 KB
        static size_t granted[2] = {64 * 1024, 64 * 1024};
        const int pv = variant >= 1 ? 1 : 0;
        if (lds > granted[pv]) {
            const void *fn = pv ? reinterpret_cast<const void *>(&apply_3m_kernel<NT3, NST, 2, CHEB, GRAM>)
                                : reinterpret_cast<const void *>(&apply_3m_kernel<NT3, NST, 1, CHEB, GRAM>);
            (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            granted[pv] = lds;
        }
    }
    if (variant >= 1)
        hipLaunchKernelGGL((apply_3m_kernel<NT3, NST, 2, CHEB, GRAM>), grid, dim3(64 * NST), lds, st, g, links, x, y,
                           nr, sub, active, ce, ge);
    else
        hipLaunchKernelGGL((apply_3m_kernel<NT3, NST, 1, CHEB, GRAM>), grid, dim3(64 * NST), lds, st, g, links, x, y,
                           nr, sub, active, ce, ge);
}

template <int NT3, bool CHEB, bool GRAM>
static void launch_3m_nst(const Geom &g, const float *links, const float *x, float *y, int nr, const float *sub,
                          const int *active, const ChebEpi &ce, const GramEpi &ge, hipStream_t st, int variant) {
    switch (g.nb / 16) {
        case 1: launch_3m_t<NT3, 1, CHEB, GRAM>(g, links, x, y, nr, sub, active, ce, ge, st, variant); break;
        case 2: launch_3m_t<NT3, 2, CHEB, GRAM>(g, links, x, y, nr, sub, active, ce, ge, st, variant); break;
        case 3: launch_3m_t<NT3, 3, CHEB, GRAM>(g, links, x, y, nr, sub, active, ce, ge, st, variant); break;
        default: launch_3m_t<NT3, 4, CHEB, GRAM>(g, links, x, y, nr, sub, active, ce, ge, st, variant); break;
    }
}

void launch_apply_3m(const Geom &g, const float *links, const float *x, float *y, int nr, const float *sub,
                     const int *active, hipStream_t st, int variant) {
    const ChebEpi none{};
    const GramEpi nog{};
    if (nr <= 16)
        launch_3m_nst<1, false, false>(g, links, x, y, nr, sub, active, none, nog, st, variant);
    else
        launch_3m_nst<2, false, false>(g, links, x, y, nr, sub, active, none, nog, st, variant);
}

void launch_apply_3m_cheb(const Geom &g, const float *links, const float *t, const ChebEpi &ce, int nr,
                          const int *active, hipStream_t st, int variant) {
    const GramEpi nog{};
    if (nr <= 16)
        launch_3m_nst<1, true, false>(g, links, t, nullptr, nr, nullptr, active, ce, nog, st, variant);
    else
        launch_3m_nst<2, true, false>(g, links, t, nullptr, nr, nullptr, active, ce, nog, st, variant);
}

// Workgroups of the Gram-fused 3M apply (0: use the apply and the Gram
// kernel). Up to 2048 of the two-wave workgroups (nbasis <= 32) and 512 of
// the larger ones keep the chip's resident slots filled. Fused only for one
// column tile (nrhs <= 16): at 8^4 / 32 / 16 the fused kernel takes 8 us more
// than the plain apply against the 9 us Gram pass it replaces; with two
// column tiles (nrhs 32) it runs at two waves per SIMD against the plain
// apply's three and loses 300 us on a 2.5 ms apply to save a 46 us Gram.
int apply_3m_gram_blocks(const Geom &g, int nr) {
    if (g.nb % 16 || g.V % 8 || nr > 16) return 0;
    return gram_fused_blocks(g.V, nr, g.nb <= 32 ? 2048 : 512);
}

void launch_apply_3m_gram(const Geom &g, const float *links, const float *x, float *y, int nr, double2 *partials,
                          int nblk, const int *active, hipStream_t st, int variant) {
    const ChebEpi none{};
    const GramEpi ge{partials, nblk};
    if (nr <= 16)
        launch_3m_nst<1, false, true>(g, links, x, y, nr, nullptr, active, none, ge, st, variant);
    else
        launch_3m_nst<2, false, true>(g, links, x, y, nr, nullptr, active, none, ge, st, variant);
}

}  // namespace coarse
