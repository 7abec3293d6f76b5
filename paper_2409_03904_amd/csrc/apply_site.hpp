// Per-site body of the float32/float64 MFMA coarse apply (shared by the
// one-site-per-workgroup kernel and the persistent batched kernel).
//
// One workgroup computes y(s) = sum_p A_p(s) X(s + delta_p) for one site s:
// wave w owns output rows 16w..16w+15 and streams those rows of every link
// block straight into the MFMA A operand (16-byte non-temporal loads, the
// links are read exactly once per apply). The neighbour block X(s + delta_p)
// is staged in LDS once per point and shared by the waves: in the 4M
// embedding the Yr columns consume (Re X, -Im X) and the Yi columns
// (Im X, Re X); for float32 the conjugate is staged beside X, so every
// B-operand value is a plain LDS read from one of the two copies, for float64
// the sign bit is flipped in the register. Link loads run PD points ahead of the MFMAs in a ring
// of register buffers (ring indices fixed at compile time), the next
// neighbour block one point ahead.
#pragma once
#include <type_traits>

#include "common.hpp"

namespace coarse {

typedef float fvec4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ fvec4 stream_load(const GLOBAL_AS float *p) {
    return __builtin_nontemporal_load(reinterpret_cast<const GLOBAL_AS fvec4 *>(p));
}

// float32 staging keeps X and its conjugate (every B operand a plain LDS
// read); float64 staging keeps X alone and flips the sign bit of the B value
// that needs it (an integer op beside a 16x16x4 f64 MFMA), so that two
// workgroups fit a CU's LDS at nbasis 64, nrhs 32.
template <typename T>
constexpr int site_apply_copies() {
    return sizeof(T) == 4 ? 2 : 1;
}

// LDS elements of T one workgroup needs (two buffers of the block, with its
// conjugate for float32, per group).
template <typename T>
__host__ __device__ constexpr size_t site_apply_lds_elems(int nb, int nr, int ps) {
    return (size_t)ps * 2 * site_apply_copies<T>() * nb * nr * 2;
}

// float4 loads per staging thread for one neighbour block: nb*nr*2*sizeof(T)/16
// of them over the >= 64*ceil(nb/16) threads of one point group; with
// nb <= 16*ceil(nb/16) and nr <= 8*NT that is at most NT*sizeof(T)/4.
template <typename T, int NT>
__host__ __device__ constexpr int site_apply_xv() {
    return (NT * (int)sizeof(T) + 3) / 4;
}

// Host-side check of the staging bound for a launch with group_threads threads
// per point group (every element of the block must have a staging lane).
template <typename T, int NT>
inline bool site_apply_staging_fits(int nb, int nr, int group_threads) {
    const int nvec = (int)((size_t)nb * nr * 2 * sizeof(T) / 16);
    return nr <= 8 * NT && (nvec + group_threads - 1) / group_threads <= site_apply_xv<T, NT>();
}

// NR_: nrhs at compile time (0 = runtime value up to 32); NT = 16-column tiles
//      of the 2*nrhs real output columns (compile time in both cases).
// NCH: 16-wide k' chunks per link block (= nbasis/8); 0 = runtime value up to 8.
// PD:  link prefetch depth in stencil points.
// PS:  point split -- the workgroup holds PS groups of row-tile waves; group pg
//      takes the stencil points p = pg, pg + PS, ... with its own staging
//      buffers, and the groups' sums are added in the epilogue.
template <typename T, int NR_, int NT, int NCH, int PD, int PS = 1>
__device__ __forceinline__ void site_apply_mfma(const Geom &g, const GLOBAL_AS float *__restrict__ links,
                                                const GLOBAL_AS T *__restrict__ x, GLOBAL_AS T *__restrict__ y,
                                                int nr_rt, const GLOBAL_AS T *__restrict__ sub, int s,
                                                unsigned char *smem_raw) {
    typedef typename std::conditional<sizeof(T) == 4, f32x4, f64x4>::type AccT;
    constexpr int MAXCH = NCH ? NCH : 8;
    constexpr int RING = PD + 1;
    constexpr int XV = site_apply_xv<T, NT>();
    const int nr = NR_ ? NR_ : nr_rt;
    const int nb = g.nb;
    const int nch = NCH ? NCH : (nb >> 3);
    const int nmt = (nb + 15) >> 4;
    // PS == 1: every thread of the workgroup stages (extra waves only help
    // staging). PS > 1: blockDim == 64 * nmt * PS, one group per point class.
    const int pg = PS == 1 ? 0 : (int)threadIdx.x / (64 * nmt);
    const int tid = PS == 1 ? (int)threadIdx.x : (int)threadIdx.x - pg * 64 * nmt;
    const int nthr = PS == 1 ? (int)blockDim.x : 64 * nmt;
    const int w = tid >> 6, t = tid & 63, il = t & 15, q = t >> 4;
    const bool wave_on = w < nmt;     // waves beyond the row tiles only help staging
    const int xblk = nb * nr * 2;     // T elements per neighbour block
    constexpr int CW = site_apply_copies<T>();
    // group buffers: [step parity][X | conj X] (float32) or [step parity][X] (float64)
    LDS_AS T *gbase = lds_ptr<T>(smem_raw) + pg * 2 * CW * xblk;

    // B operand of lane (il, q) at step st is X'[4st + q][16nt + il] with
    // h = q & 1 the Re/Im slot of X(j = 2st + q/2, r). Column part 0 (Yr)
    // reads (Re X, -Im X) = conj X at component h; part 1 (Yi) reads
    // (Im X, Re X) = X at component 1 - h. Per lane: one element offset per
    // tile into the pair [X | conj X]; the per-step offset is j * 2nr.
    int boff[NT];
    long long bflip[NT];  // float64: sign bit to flip in the B value (-Im X of conj X)
    {
        const int h = q & 1;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int n = 16 * nt + il;
            const int part = n / nr, r = n - part * nr;
            bflip[nt] = 0;
            if (part == 0) {
                boff[nt] = (CW == 2 ? xblk : 0) + 2 * r + h;
                if (CW == 1 && h == 1) bflip[nt] = (long long)1 << 63;
            } else if (part == 1) {
                boff[nt] = 2 * r + 1 - h;
            } else {
                boff[nt] = 0;  // padding column: any value, never stored
            }
            boff[nt] += (q >> 1) * 2 * nr;  // j = 2st + q/2
        }
    }

    int c[4];
    site_coords(g, s, c);

    // Loads are branch-free (all XV issued, surplus ones re-read the last
    // element): a load under a branch ends a basic block and the compiler's
    // wait-count insertion then waits for every outstanding load at the join.
    const int nvec = (xblk * (int)sizeof(T)) >> 4;
    const int xv = (nvec + nthr - 1) / nthr;  // staging float4 per thread in use, <= XV
    fvec4 xr[XV];
    auto load_x = [&](int p) {
        const int z = displaced(g, c, p, 1);
        const GLOBAL_AS fvec4 *src = reinterpret_cast<const GLOBAL_AS fvec4 *>(x + (size_t)z * xblk);
#pragma unroll
        for (int k = 0; k < XV; ++k) xr[k] = src[min(tid + k * nthr, nvec - 1)];
    };
    // store X (and, for float32, conj X: imaginary parts negated)
    auto store_x = [&](LDS_AS T *dst) {
        LDS_AS fvec4 *d4 = (LDS_AS fvec4 *)(dst);
        LDS_AS fvec4 *c4 = (LDS_AS fvec4 *)(dst + xblk);
#pragma unroll
        for (int k = 0; k < XV; ++k) {
            const int e = tid + k * nthr;
            if (k < xv && e < nvec) {
                d4[e] = xr[k];
                if (CW == 2) {  // float32: the conjugate beside it
                    fvec4 cj = xr[k];
                    cj.y = -cj.y;
                    cj.w = -cj.w;
                    c4[e] = cj;
                }
            }
        }
    };

    const size_t blk_floats = (size_t)nb * nb * 2;
    const GLOBAL_AS float *lsite = links + (size_t)s * g.np * blk_floats;
    // Lanes past the last row of a partial tile (and waves without a tile)
    // read a valid row of the block instead; their MFMA rows are never stored.
    const int w_ld = wave_on ? w : 0;
    const int rows_ld = min(16, nb - 16 * w_ld);
    const int lane_off = 16 * w_ld * 16 + (q * rows_ld + min(il, rows_ld - 1)) * 4;
    fvec4 ring[RING][MAXCH];
    auto load_a = [&](fvec4 *a, int p) {
        const GLOBAL_AS float *lb = lsite + (size_t)p * blk_floats + lane_off;
#pragma unroll
        for (int cc = 0; cc < MAXCH; ++cc) {
            if (NCH || cc < nch) a[cc] = stream_load(lb + cc * nb * 16);
        }
    };

    AccT acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = AccT{0, 0, 0, 0};

    // this group's points: p = pg + PS * i, i < npg; all groups run nsteps
    // steps (the barrier count must match), idle once their points run out
    const int np = g.np;
    const int npg = (np - pg + PS - 1) / PS;
    const int nsteps = (np + PS - 1) / PS;
    if (npg > 0) load_x(pg);
#pragma unroll
    for (int k = 0; k < PD; ++k)
        if (k < npg) load_a(ring[k], pg + PS * k);
    if (npg > 0) store_x(gbase);
    __syncthreads();

    // One pipeline step: stage the next neighbour block and prefetch the links
    // PD points ahead, consume the current ring slot, publish the staged block.
    auto step = [&](int i, fvec4(&cur)[MAXCH], fvec4(&nxt)[MAXCH], bool do_x, bool do_pref, bool mine) {
        // issue order matters: loads retire in order, and the staging store at
        // the end of this step waits for the neighbour block; issued first, it
        // does not drag the deep link prefetch with it
        if (do_x) load_x(pg + PS * (i + 1));
        if (do_pref) load_a(nxt, pg + PS * (i + PD));
        const LDS_AS T *xc = gbase + (i & 1) * CW * xblk;
        if (wave_on && mine) {
#pragma unroll
            for (int cc = 0; cc < MAXCH; ++cc) {
                if (NCH || cc < nch) {
                    const fvec4 a4 = cur[cc];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int jrow = 8 * cc + 2 * u;  // + q/2, folded into boff
                        const T av = (T)a4[u];
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt) {
                            T bv = xc[boff[nt] + jrow * 2 * nr];
                            if (CW == 1)
                                bv = __longlong_as_double(__double_as_longlong((double)bv) ^ bflip[nt]);
                            acc[nt] = mfma16x16x4(av, bv, acc[nt]);
                        }
                    }
                }
            }
        }
        if (do_x) store_x(gbase + ((i + 1) & 1) * CW * xblk);
        __syncthreads();
    };

    // Steady state: whole ring rounds whose loads are all in range, so the
    // body is branch-free (a branch would make the compiler's wait-count
    // insertion conservative and drain the prefetch at every join).
    int i0 = 0;
    for (; i0 + RING + PD <= npg; i0 += RING) {
#pragma unroll
        for (int k = 0; k < RING; ++k) step(i0 + k, ring[k], ring[(k + PD) % RING], true, true, true);
    }
    // Tail: the remaining steps (at most RING + PD, plus one for a group with
    // a point fewer), loads guarded.
#pragma unroll
    for (int k = 0; k < RING + PD + 1; ++k) {
        const int i = i0 + k;
        if (i < nsteps)
            step(i, ring[k % RING], ring[(k + PD) % RING], (i + 1) < npg, (i + PD) < npg, i < npg);
    }

    // epilogue: D tiles -> LDS [group][row][2*nr] -> sum over groups -> complex output
    LDS_AS T *out = gbase;
    const int two_nr = 2 * nr;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int n = 16 * nt + il;
        if (wave_on && n < two_nr) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // accumulator layout: lane group q holds rows 4q..4q+3 (f32) but
                // rows q, q+4, q+8, q+12 (f64) of the 16x16 tile, column il
                const int row = 16 * w + (sizeof(T) == 8 ? q + 4 * v : 4 * q + v);
                if (row < nb) out[row * two_nr + n] = acc[nt][v];
            }
        }
    }
    __syncthreads();
    GLOBAL_AS T *yo = y + (size_t)s * xblk;
    const GLOBAL_AS T *so = sub ? sub + (size_t)s * xblk : nullptr;
    const LDS_AS T *out0 = lds_ptr<T>(smem_raw);
    for (int e = threadIdx.x; e < nb * nr; e += blockDim.x) {
        const int i = e / nr, r = e - i * nr;
        T re = out0[i * two_nr + r], im = out0[i * two_nr + nr + r];
#pragma unroll
        for (int gq = 1; gq < PS; ++gq) {
            const LDS_AS T *og = out0 + gq * 2 * CW * xblk;
            re += og[i * two_nr + r];
            im += og[i * two_nr + nr + r];
        }
        if (so) {
            re = so[2 * e] - re;
            im = so[2 * e + 1] - im;
        }
        yo[2 * e] = re;
        yo[2 * e + 1] = im;
    }
    __syncthreads();  // LDS free for the next site
}

}  // namespace coarse
