// Block-CG linear algebra on MFMA for nrhs in {2, 4, 8, 16, 32}.
//
// Rows of the tall-skinny blocks (rows = V * nbasis, nrhs complex entries per
// row) are processed in 16-row tiles, one tile per wave at a time. Three
// per-tile primitives:
//
// * tile x small matrix, [16 x nrhs] . [nrhs x nrhs], as a 16 x (2 nrhs) x
//   (2 nrhs) real product in the 4M embedding: the row block streams from
//   HBM into the A operand in its complex64 memory order (lane (row, q) reads
//   the contiguous k' range [q*nrhs/2, (q+1)*nrhs/2)), the real embedding of
//   the small matrix is the B operand, kept in LDS.
// * "column values": lane (c, g) holds entries [4g+v][16k + c] (Re and Im)
//   of a tile -- the layout of the 16x16x4 accumulator, and of direct
//   coalesced loads of a tile.
// * tile Gram A^H B over 16 rows with f64 MFMA: for k' = 2(4g+v) + h the A
//   and B operands of lane (c, g) at step (v, h) are exactly that lane's own
//   column values, so a tile's Gram needs no data movement at all, and
//   products of complex64 values are exact in double.
//
// Kernels: the Gram D^H Z; E += D (N C) and T = Q - Z N with the Gram T^H T
// of the new T fused in; Q = T S^{-1} and D = Q + D S^H. Each workgroup owns
// a fixed contiguous row range and writes one partial Gram (summed later in a
// fixed order), so results are bitwise reproducible.
#include <type_traits>

#include "blas.hpp"
#include "small.hpp"

namespace coarse {

namespace {

template <int NR>
struct TileShape {
    static constexpr int NT = (2 * NR + 15) / 16;  // 16-column tiles of the 2*NR real output columns
    static constexpr int KS = NR / 2;              // 16x16x4 steps over K' = 2*NR
    static constexpr int CG = NR >= 16 ? NR / 16 : 1;  // 16-column groups of the complex columns
};

__device__ __forceinline__ float2 f2zero() { return make_float2(0.f, 0.f); }

// Real column k' (k' = 2c + h over the 2 NR floats of a row) that lane
// k-group q feeds at step s of a tile product. With KS % 4 == 0 the lane takes
// float4 chunk q of every 64-byte segment of the row (k' = 16 (s / 4) + 4 q +
// s % 4), so the four k-groups of a load instruction read one contiguous
// 64-byte piece of each of the 16 rows; otherwise the contiguous range
// [q KS, q KS + KS).
template <int NR>
__host__ __device__ __forceinline__ int tile_kp(int q, int s) {
    constexpr int KS = TileShape<NR>::KS;
    return KS % 4 == 0 ? 16 * (s >> 2) + 4 * q + (s & 3) : q * KS + s;
}

// Rows [row0, row0 + 16) of a [rows][NR] complex64 block, branch-free, in the
// A-operand layout: lane (il, q) gets floats tile_kp(q, s), s < KS, of row
// row0 + il. Rows at or past r1 re-read row r1 - 1 (valid
// memory, r0 < r1) and are zeroed after the load, so a wave can prefetch its
// next tile without a load under a branch (which would make the wait-count
// insertion drain every outstanding load at the join).
template <int NR>
__device__ __forceinline__ void load_arow_clamped(const float2 *__restrict__ base, long long row0, long long r1,
                                                  int t, float (&a)[TileShape<NR>::KS]) {
    constexpr int KS = TileShape<NR>::KS;
    const int il = t & 15, q = t >> 4;
    const long long row = row0 + il;
    const bool ok = row < r1;
    const float *rbase = reinterpret_cast<const float *>(base + (ok ? row : r1 - 1) * NR);
    const float *src = rbase + tile_kp<NR>(q, 0);
    if (KS % 4 == 0) {
#pragma unroll
        for (int k = 0; k < KS; k += 4) {
            const float4 v = *reinterpret_cast<const float4 *>(src + 4 * k);  // chunk q of segment k / 4
            a[k] = v.x;
            a[k + 1] = v.y;
            a[k + 2] = v.z;
            a[k + 3] = v.w;
        }
    } else if (KS == 2) {
        const float2 v = *reinterpret_cast<const float2 *>(src);
        a[0] = v.x;
        a[1] = v.y;
    } else {
#pragma unroll
        for (int k = 0; k < KS; ++k) a[k] = src[k];
    }
#pragma unroll
    for (int k = 0; k < KS; ++k) a[k] = ok ? a[k] : 0.f;
}

// Column values of a tile: lane (c, g) holds entry [4g+v][16k + c], k < CG.
template <int NR>
struct Cols {
    float2 x[TileShape<NR>::CG][4];
};

template <int NR>
__device__ __forceinline__ void load_cols(const float2 *__restrict__ base, long long row0, long long r1, int t,
                                          Cols<NR> &out) {
    const int c = t & 15, g = t >> 4;
#pragma unroll
    for (int k = 0; k < TileShape<NR>::CG; ++k) {
        const int col = 16 * k + c;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const long long row = row0 + 4 * g + v;
            out.x[k][v] = (col < NR && row < r1) ? base[row * NR + col] : f2zero();
        }
    }
}

template <int NR>
__device__ __forceinline__ void load_cols_clamped(const float2 *__restrict__ base, long long row0, long long r1, int t,
                                                  Cols<NR> &out) {
    const int c = t & 15, g = t >> 4;
#pragma unroll
    for (int k = 0; k < TileShape<NR>::CG; ++k) {
        const int col = 16 * k + c;
        const int cc = col < NR ? col : NR - 1;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const long long row = row0 + 4 * g + v;
            const bool ok = col < NR && row < r1;
            const float2 val = base[(row < r1 ? row : r1 - 1) * NR + cc];
            out.x[k][v] = ok ? val : f2zero();
        }
    }
}

template <int NR>
__device__ __forceinline__ void store_cols(float2 *__restrict__ base, long long row0, long long r1, int t,
                                           const Cols<NR> &in) {
    const int c = t & 15, g = t >> 4;
#pragma unroll
    for (int k = 0; k < TileShape<NR>::CG; ++k) {
        const int col = 16 * k + c;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const long long row = row0 + 4 * g + v;
            if (col < NR && row < r1) base[row * NR + col] = in.x[k][v];
        }
    }
}

// Real embedding of a complex64 nr x nr matrix W as the B operand of
// tile . W: Bl[(s*4 + q) * 16NT + n] = W'[q*KS + s][n], k' = 2c + h,
// column n: part 0 (Re of the result) r = n, part 1 (Im) r = n - NR.
template <int NR>
__device__ __forceinline__ void build_bop(const float2 *__restrict__ w, float *bl) {
    constexpr int NT = TileShape<NR>::NT, KS = TileShape<NR>::KS;
    for (int e = threadIdx.x; e < KS * 4 * 16 * NT; e += blockDim.x) {
        const int n = e % (16 * NT), sq = e / (16 * NT);
        const int s = sq >> 2, q = sq & 3;
        const int kp = tile_kp<NR>(q, s), cc = kp >> 1, h = kp & 1;
        const int part = n / NR, r = n - part * NR;
        float val = 0.f;
        if (part < 2) {
            const float2 v = w[cc * NR + r];
            if (part == 0)
                val = h ? -v.y : v.x;
            else
                val = h ? v.x : v.y;
        }
        bl[e] = val;
    }
}

// The same B operand from an np-strided complex128 matrix M in LDS (conj_t:
// from M^H), each entry rounded to complex64 as a stored copy would be.
template <int NR>
__device__ __forceinline__ void build_bop_lds(const double2 *M, int np, bool conj_t, float *bl) {
    constexpr int NT = TileShape<NR>::NT, KS = TileShape<NR>::KS;
    for (int e = threadIdx.x; e < KS * 4 * 16 * NT; e += blockDim.x) {
        const int n = e % (16 * NT), sq = e / (16 * NT);
        const int s = sq >> 2, q = sq & 3;
        const int kp = tile_kp<NR>(q, s), cc = kp >> 1, h = kp & 1;
        const int part = n / NR, r = n - part * NR;
        float val = 0.f;
        if (part < 2) {
            const double2 m = conj_t ? M[r * np + cc] : M[cc * np + r];
            const float2 v = make_float2((float)m.x, conj_t ? -(float)m.y : (float)m.y);
            if (part == 0)
                val = h ? -v.y : v.x;
            else
                val = h ? v.x : v.y;
        }
        bl[e] = val;
    }
}

// acc[nt] += A_tile . W' over K' = 2NR.
template <int NR>
__device__ __forceinline__ void tile_mm(const float (&a)[TileShape<NR>::KS], const float *bl, int t,
                                        f32x4 (&acc)[TileShape<NR>::NT]) {
    constexpr int NT = TileShape<NR>::NT, KS = TileShape<NR>::KS;
    const int il = t & 15, q = t >> 4;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[nt] = mfma16x16x4(a[s], bl[(s * 4 + q) * 16 * NT + 16 * nt + il], acc[nt]);
    }
}

// Accumulator (f32 16x16x4 layout, real columns) -> column values.
template <int NR>
__device__ __forceinline__ void acc_to_cols(const f32x4 (&acc)[TileShape<NR>::NT], int t, Cols<NR> &out) {
    constexpr int CG = TileShape<NR>::CG;
    if (NR >= 16) {
#pragma unroll
        for (int k = 0; k < CG; ++k)
#pragma unroll
            for (int v = 0; v < 4; ++v) out.x[k][v] = make_float2(acc[k][v], acc[k + CG][v]);
    } else {
        const int src = (t + NR) & 63;  // lane c + NR holds Im of column c (same lane group)
#pragma unroll
        for (int v = 0; v < 4; ++v) out.x[0][v] = make_float2(acc[0][v], __shfl(acc[0][v], src));
    }
}

// gacc[mt][nt'] += A^H B over one 16-row tile (f64 MFMA), from column values.
// Output G (nr x nr complex) is the real [Gr | Gi] (nr x 2nr): row a = 16mt + ...,
// column n < nr: Gr[a][n]; n >= nr: Gi[a][n - nr].
template <int NR>
__device__ __forceinline__ void tile_gram(const Cols<NR> &A, const Cols<NR> &B, int t,
                                          f64x4 (&gacc)[TileShape<NR>::CG][TileShape<NR>::NT]) {
    constexpr int CG = TileShape<NR>::CG, NT = TileShape<NR>::NT;
    const int c = t & 15;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        // B operand columns of this lane: for NR < 16 the Gi half of the single
        // tile reads column c - NR from lane t - NR.
        float2 bpart1[CG];
        if (NR < 16) {
            const int src = (t - NR) & 63;
            bpart1[0] = make_float2(__shfl(B.x[0][v].x, src), __shfl(B.x[0][v].y, src));
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            double aop[CG];
#pragma unroll
            for (int mt = 0; mt < CG; ++mt) {
                const float2 av = A.x[mt][v];
                aop[mt] = (16 * mt + c < NR) ? (double)(h ? av.y : av.x) : 0.0;
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                double bop;
                if (NR >= 16) {
                    const int part = nt / CG, k = nt % CG;
                    const float2 bv = B.x[k][v];
                    bop = part == 0 ? (double)(h ? bv.y : bv.x) : (double)(h ? -bv.x : bv.y);
                } else {
                    if (c < NR) {
                        const float2 bv = B.x[0][v];
                        bop = (double)(h ? bv.y : bv.x);
                    } else if (c < 2 * NR) {
                        const float2 bv = bpart1[0];
                        bop = (double)(h ? -bv.x : bv.y);
                    } else {
                        bop = 0.0;
                    }
                }
#pragma unroll
                for (int mt = 0; mt < CG; ++mt) gacc[mt][nt] = mfma16x16x4(aop[mt], bop, gacc[mt][nt]);
            }
        }
    }
}

// The NW waves' values of entry e (red[w * ne + e]) summed pairwise in a
// fixed tree, ((w0 + w1) + (w2 + w3)) + ...
template <int NW>
__device__ __forceinline__ double2 wave_tree_sum(const double2 *red, int ne, int e) {
    double2 v[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) v[w] = red[w * ne + e];
#pragma unroll
    for (int span = 1; span < NW; span *= 2)
#pragma unroll
        for (int w = 0; w + span < NW; w += 2 * span) v[w] = make_double2(v[w].x + v[w + span].x, v[w].y + v[w + span].y);
    return v[0];
}

// The NW waves' Gram accumulators -> one partial (nr x nr complex128), fixed order.
template <int NR, int NW = 4>
__device__ __forceinline__ void write_partial(const f64x4 (&gacc)[TileShape<NR>::CG][TileShape<NR>::NT],
                                              double2 *red, double2 *__restrict__ out) {
    constexpr int CG = TileShape<NR>::CG, NT = TileShape<NR>::NT;
    const int w = threadIdx.x >> 6, t = threadIdx.x & 63, c = t & 15, g = t >> 4;
    constexpr int NE = NR * NR;
    // f64 accumulator layout: lane (c, g) register v holds row g + 4v, column c
#pragma unroll
    for (int mt = 0; mt < CG; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int a = 16 * mt + g + 4 * v;
                const int n = 16 * nt + c;
                if (a < NR && n < 2 * NR) {
                    const int part = n / NR, b = n - part * NR;
                    double *slot = reinterpret_cast<double *>(&red[w * NE + a * NR + b]);
                    slot[part] = gacc[mt][nt][v];
                }
            }
    __syncthreads();
    for (int e = threadIdx.x; e < NE; e += blockDim.x) out[e] = wave_tree_sum<NW>(red, NE, e);
}

// ---------------------------------------------------------------------------
// 3M forms for nrhs >= 16 (three real products per complex multiply-add, 3/4
// of the 4M MFMA work):
//   tile x small matrix: Cr = T1 - T2, Ci = T3 - T1 - T2 with T1 = Ar Wr,
//   T2 = Ai Wi, T3 = (Ar + Ai)(Wr + Wi), K = the complex column index;
//   Gram A^H B: Gr = T1 + T2, Gi = T3 - T1 + T2 with T1 = Ar^T Br,
//   T2 = Ai^T Bi, T3 = (Ar - Ai)^T (Br + Bi), K = the row index (f64 MFMA;
//   T1 and T2 are sums of exact products of complex64 parts, T3's products
//   are of double sums, rounded once each).
// ---------------------------------------------------------------------------
template <int NR>
struct Tile3 {
    static constexpr int KS = NR / 4;    // k-steps over the NR complex columns
    static constexpr int NT = NR / 16;   // 16-column output tiles
    static constexpr int PLANE = KS * 4 * 16 * NT;  // floats of one B-operand plane
};

// Complex column k that k-group q feeds at step s: float4 chunk q of every
// 64-byte segment of a row, so the four k-groups of a load instruction read
// one contiguous 64-byte piece of each of the 16 rows.
__host__ __device__ __forceinline__ int tile3_k(int q, int s) { return 8 * (s >> 1) + 2 * q + (s & 1); }

// Rows [row0, row0 + 16) of a [rows][NR] complex64 block as the 3M A operand:
// lane (il, q) gets (Re, Im) of columns tile3_k(q, s), s < KS, of row row0 + il
// (branch-free as load_arow_clamped).
template <int NR>
__device__ __forceinline__ void load_arow3_clamped(const float2 *__restrict__ base, long long row0, long long r1,
                                                   int t, float2 (&a)[Tile3<NR>::KS]) {
    constexpr int KS = Tile3<NR>::KS;
    const int il = t & 15, q = t >> 4;
    const long long row = row0 + il;
    const bool ok = row < r1;
    const float2 *src = base + (ok ? row : r1 - 1) * NR + 2 * q;
#pragma unroll
    for (int m = 0; m < KS / 2; ++m) {
        const float4 v = *reinterpret_cast<const float4 *>(src + 8 * m);
        a[2 * m] = ok ? make_float2(v.x, v.y) : f2zero();
        a[2 * m + 1] = ok ? make_float2(v.z, v.w) : f2zero();
    }
}

// The three B-operand planes (Wr, Wi, Wr + Wi) of tile . W in LDS:
// plane[(s * 4 + q) * 16 NT + n] = W[tile3_k(q, s)][n], from a complex64 W or
// an np-strided complex128 M in LDS (conj_t: from M^H, rounded to complex64).
template <int NR>
__device__ __forceinline__ void build_bop3(const float2 *__restrict__ w, float *bl) {
    constexpr int NT = Tile3<NR>::NT, PLANE = Tile3<NR>::PLANE;
    for (int e = threadIdx.x; e < PLANE; e += blockDim.x) {
        const int n = e % (16 * NT), sq = e / (16 * NT);
        const float2 v = w[tile3_k(sq & 3, sq >> 2) * NR + n];
        bl[e] = v.x;
        bl[PLANE + e] = v.y;
        bl[2 * PLANE + e] = v.x + v.y;
    }
}

template <int NR>
__device__ __forceinline__ void build_bop3_lds(const double2 *M, int np, bool conj_t, float *bl) {
    constexpr int NT = Tile3<NR>::NT, PLANE = Tile3<NR>::PLANE;
    for (int e = threadIdx.x; e < PLANE; e += blockDim.x) {
        const int n = e % (16 * NT), sq = e / (16 * NT);
        const int k = tile3_k(sq & 3, sq >> 2);
        const double2 m = conj_t ? M[n * np + k] : M[k * np + n];
        const float vr = (float)m.x, vi = conj_t ? -(float)m.y : (float)m.y;
        bl[e] = vr;
        bl[PLANE + e] = vi;
        bl[2 * PLANE + e] = vr + vi;
    }
}

// C = A_tile . W as column values (lane (c, g): rows 4g + v of column 16k + c).
template <int NR>
__device__ __forceinline__ void tile_mm3(const float2 (&a)[Tile3<NR>::KS], const float *bl, int t, Cols<NR> &out) {
    constexpr int KS = Tile3<NR>::KS, NT = Tile3<NR>::NT, PLANE = Tile3<NR>::PLANE;
    const int il = t & 15, q = t >> 4;
    f32x4 t1[NT], t2[NT], t3[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) t1[nt] = t2[nt] = t3[nt] = f32x4{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const float ar = a[s].x, ai = a[s].y, as = ar + ai;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int o = (s * 4 + q) * 16 * NT + 16 * nt + il;
            t1[nt] = mfma16x16x4(ar, bl[o], t1[nt]);
            t2[nt] = mfma16x16x4(ai, bl[PLANE + o], t2[nt]);
            t3[nt] = mfma16x16x4(as, bl[2 * PLANE + o], t3[nt]);
        }
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            out.x[nt][v] = make_float2(t1[nt][v] - t2[nt][v], t3[nt][v] - t1[nt][v] - t2[nt][v]);
}

// Gram accumulators of the 3M form: T1, T2, T3 per (row tile, column tile).
template <int NR>
struct Gacc3 {
    f64x4 t[3][TileShape<NR>::CG][TileShape<NR>::CG];
};

template <int NR>
__device__ __forceinline__ void zero_gacc3(Gacc3<NR> &g) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int a = 0; a < TileShape<NR>::CG; ++a)
#pragma unroll
            for (int b = 0; b < TileShape<NR>::CG; ++b) g.t[i][a][b] = f64x4{0, 0, 0, 0};
}

// g += A^H B over one 16-row tile: at step v the operands of lane (c, g) are
// its own column values of row 4g + v (K = the row index).
template <int NR>
__device__ __forceinline__ void tile_gram3(const Cols<NR> &A, const Cols<NR> &B, Gacc3<NR> &g) {
    constexpr int CG = TileShape<NR>::CG;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        double ar[CG], ai[CG], ad[CG];
#pragma unroll
        for (int mt = 0; mt < CG; ++mt) {
            ar[mt] = (double)A.x[mt][v].x;
            ai[mt] = (double)A.x[mt][v].y;
            ad[mt] = ar[mt] - ai[mt];
        }
#pragma unroll
        for (int nt = 0; nt < CG; ++nt) {
            const double br = (double)B.x[nt][v].x, bi = (double)B.x[nt][v].y, bs = br + bi;
#pragma unroll
            for (int mt = 0; mt < CG; ++mt) {
                g.t[0][mt][nt] = mfma16x16x4(ar[mt], br, g.t[0][mt][nt]);
                g.t[1][mt][nt] = mfma16x16x4(ai[mt], bi, g.t[1][mt][nt]);
                g.t[2][mt][nt] = mfma16x16x4(ad[mt], bs, g.t[2][mt][nt]);
            }
        }
    }
}

// The NW waves' 3M Gram accumulators -> one partial (nr x nr complex128), fixed order.
template <int NR, int NW = 4>
__device__ __forceinline__ void write_partial3(const Gacc3<NR> &g, double2 *red, double2 *__restrict__ out) {
    constexpr int CG = TileShape<NR>::CG;
    const int w = threadIdx.x >> 6, t = threadIdx.x & 63, c = t & 15, gq = t >> 4;
    constexpr int NE = NR * NR;
    // f64 accumulator layout: lane (c, g) register v holds row g + 4v, column c
#pragma unroll
    for (int mt = 0; mt < CG; ++mt)
#pragma unroll
        for (int nt = 0; nt < CG; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int a = 16 * mt + gq + 4 * v, b = 16 * nt + c;
                const double t1 = g.t[0][mt][nt][v], t2 = g.t[1][mt][nt][v], t3 = g.t[2][mt][nt][v];
                red[w * NE + a * NR + b] = make_double2(t1 + t2, t3 - t1 + t2);
            }
    __syncthreads();
    for (int e = threadIdx.x; e < NE; e += blockDim.x) out[e] = wave_tree_sum<NW>(red, NE, e);
}

// Fixed row range of workgroup b (a multiple of 16 rows).
__device__ __forceinline__ void row_range(long long rows, long long &r0, long long &r1) {
    const long long tiles = (rows + 15) / 16;
    const long long per = (tiles + gridDim.x - 1) / gridDim.x;
    r0 = blockIdx.x * per * 16;
    r1 = r0 + per * 16;
    if (r1 > rows) r1 = rows;
    if (r0 > rows) r0 = rows;
}

template <int NR>
__device__ __forceinline__ void zero_gacc(f64x4 (&gacc)[TileShape<NR>::CG][TileShape<NR>::NT]) {
#pragma unroll
    for (int mt = 0; mt < TileShape<NR>::CG; ++mt)
#pragma unroll
        for (int nt = 0; nt < TileShape<NR>::NT; ++nt) gacc[mt][nt] = f64x4{0, 0, 0, 0};
}

// ---- one interface over the 4M (nrhs < 16) and 3M (nrhs >= 16) forms ----
template <int NR>
constexpr bool USE3M = NR >= 16;
// The 3M Gram needs 3 CG^2 accumulator tiles against 2 CG^2 for 4M; at nrhs
// 32 (CG = 2) the kernels that form it are held to two waves per SIMD (their
// grid's occupancy) by their launch bounds, which fits it without spilling.
template <int NR>
constexpr bool USE3M_GRAM = NR >= 16;

// A-operand registers of one row tile
template <int NR>
struct ARow {
    typename std::conditional<USE3M<NR>, float2[USE3M<NR> ? Tile3<NR>::KS : 1],
                              float[TileShape<NR>::KS]>::type v;
};

template <int NR>
__device__ __forceinline__ void load_arow_t(const float2 *__restrict__ base, long long row0, long long r1, int t,
                                            ARow<NR> &a) {
    if constexpr (USE3M<NR>)
        load_arow3_clamped<NR>(base, row0, r1, t, a.v);
    else
        load_arow_clamped<NR>(base, row0, r1, t, a.v);
}

// floats of the B operand(s) of one small matrix in LDS
template <int NR>
constexpr int bop_floats() {
    if constexpr (USE3M<NR>)
        return 3 * Tile3<NR>::PLANE;
    else
        return TileShape<NR>::KS * 4 * 16 * TileShape<NR>::NT;
}

template <int NR>
__device__ __forceinline__ void build_bop_t(const float2 *__restrict__ w, float *bl) {
    if constexpr (USE3M<NR>)
        build_bop3<NR>(w, bl);
    else
        build_bop<NR>(w, bl);
}

template <int NR>
__device__ __forceinline__ void build_bop_lds_t(const double2 *M, int np, bool conj_t, float *bl) {
    if constexpr (USE3M<NR>)
        build_bop3_lds<NR>(M, np, conj_t, bl);
    else
        build_bop_lds<NR>(M, np, conj_t, bl);
}

// out = A_tile . W as column values
template <int NR>
__device__ __forceinline__ void tile_mm_t(const ARow<NR> &a, const float *bl, int t, Cols<NR> &out) {
    if constexpr (USE3M<NR>) {
        tile_mm3<NR>(a.v, bl, t, out);
    } else {
        f32x4 acc[TileShape<NR>::NT];
#pragma unroll
        for (int nt = 0; nt < TileShape<NR>::NT; ++nt) acc[nt] = f32x4{0, 0, 0, 0};
        tile_mm<NR>(a.v, bl, t, acc);
        acc_to_cols<NR>(acc, t, out);
    }
}

template <int NR>
struct GramAcc {
    typename std::conditional<USE3M_GRAM<NR>, Gacc3<NR>, f64x4[TileShape<NR>::CG][TileShape<NR>::NT]>::type g;
};

template <int NR>
__device__ __forceinline__ void gram_zero(GramAcc<NR> &ga) {
    if constexpr (USE3M_GRAM<NR>)
        zero_gacc3<NR>(ga.g);
    else
        zero_gacc<NR>(ga.g);
}

template <int NR>
__device__ __forceinline__ void gram_tile(const Cols<NR> &A, const Cols<NR> &B, int t, GramAcc<NR> &ga) {
    if constexpr (USE3M_GRAM<NR>)
        tile_gram3<NR>(A, B, ga.g);
    else
        tile_gram<NR>(A, B, t, ga.g);
}

template <int NR, int NW = 4>
__device__ __forceinline__ void gram_write(const GramAcc<NR> &ga, double2 *red, double2 *__restrict__ out) {
    if constexpr (USE3M_GRAM<NR>)
        write_partial3<NR, NW>(ga.g, red, out);
    else
        write_partial<NR, NW>(ga.g, red, out);
}


}  // namespace

// G partial = A^H B over the workgroup's rows.
template <int NR>
__global__ __launch_bounds__(256, 2) void gram_mfma_kernel(const float2 *__restrict__ a, const float2 *__restrict__ b,
                                                        long long rows, double2 *__restrict__ partials,
                                                        const int *__restrict__ active) {
    __shared__ double2 red[4 * NR * NR];
    const int w = threadIdx.x >> 6, t = threadIdx.x & 63;
    long long r0, r1;
    row_range(rows, r0, r1);
    GramAcc<NR> gacc;
    gram_zero<NR>(gacc);
    long long row0 = r0 + 16 * w;
    // the first tile's loads (clamped into the valid rows, or the first row
    // of the blocks for a workgroup without rows) go out beside the active
    // flag's: a load under a branch would be waited for at the join
    const long long rf = row0 < r1 ? row0 : 0, rl = row0 < r1 ? r1 : 1;
    Cols<NR> A, B;
    load_cols_clamped<NR>(a, rf, rl, t, A);
    load_cols_clamped<NR>(b, rf, rl, t, B);
    const int flag = *(active != nullptr ? active : reinterpret_cast<const int *>(a));
    if (active != nullptr && flag == 0) return;  // uniform: before any barrier
    if (row0 < r1) {
        for (; row0 < r1; row0 += 64) {
            Cols<NR> An, Bn;  // the wave's next tile, in flight during this one
            load_cols_clamped<NR>(a, row0 + 64, r1, t, An);
            load_cols_clamped<NR>(b, row0 + 64, r1, t, Bn);
            gram_tile<NR>(A, B, t, gacc);
            A = An;
            B = Bn;
        }
    }
    gram_write<NR>(gacc, red, partials + (size_t)blockIdx.x * NR * NR);
}

// E += D W; T = Q - Z N (stored over Q); partial Gram T^H T of the new T. bw
// and bn hold the B operands of W and N; red (aliasing them) takes the four
// waves' Grams at the end.
// The wave's first tile of the xt sweep (nrhs <= 16: the sweep prefetches
// one tile ahead), loaded before the workgroup's prologue so that its latency
// overlaps the small dense step. Clamped loads, no branch: a wave without
// rows loads the block's first tile and never uses it.
template <int NR>
struct XtFirst {
    ARow<NR> ad, az;
    Cols<NR> E, Q;
};

template <int NR, int NW = 4>
__device__ __forceinline__ void xt_first(const float2 *__restrict__ e, const float2 *__restrict__ q,
                                         const float2 *__restrict__ d, const float2 *__restrict__ z, long long rows,
                                         XtFirst<NR> &f) {
    if (NR > 16) return;
    const int w = threadIdx.x >> 6, t = threadIdx.x & 63;
    long long r0, r1;
    row_range(rows, r0, r1);
    const long long row0 = r0 + 16 * w;
    const long long rf = row0 < r1 ? row0 : 0, rl = row0 < r1 ? r1 : 1;
    load_arow_t<NR>(d, rf, rl, t, f.ad);
    load_arow_t<NR>(z, rf, rl, t, f.az);
    load_cols_clamped<NR>(e, rf, rl, t, f.E);
    load_cols_clamped<NR>(q, rf, rl, t, f.Q);
}

template <int NR, int NW = 4>
__device__ __forceinline__ void xt_sweep(float2 *__restrict__ e, float2 *__restrict__ q, const float2 *__restrict__ d,
                                         const float2 *__restrict__ z, long long rows,
                                         double2 *__restrict__ partials, const float *bw, const float *bn,
                                         double2 *red, const XtFirst<NR> &first) {
    const int w = threadIdx.x >> 6, t = threadIdx.x & 63;
    long long r0, r1;
    row_range(rows, r0, r1);
    GramAcc<NR> gacc;
    gram_zero<NR>(gacc);
    // next-tile prefetch where the registers allow it (nrhs <= 16; at 32 the
    // doubled tile registers would halve the occupancy)
    constexpr bool PF = NR <= 16;
    ARow<NR> adn, azn;
    Cols<NR> En, Qn;
    long long row0 = r0 + 16 * w;
    if (PF) {
        adn = first.ad;
        azn = first.az;
        En = first.E;
        Qn = first.Q;
    }
    for (; row0 < r1; row0 += 16 * NW) {
        ARow<NR> ad, az;
        Cols<NR> E, Q;
        if (PF) {
            E = En;
            Q = Qn;
            ad = adn;
            az = azn;
            // the wave's next tile, in flight during this one
            load_arow_t<NR>(d, row0 + 16 * NW, r1, t, adn);
            load_arow_t<NR>(z, row0 + 16 * NW, r1, t, azn);
            load_cols_clamped<NR>(e, row0 + 16 * NW, r1, t, En);
            load_cols_clamped<NR>(q, row0 + 16 * NW, r1, t, Qn);
        } else {
            // nrhs 32: the two independent updates one after the other, so their
            // tiles are never live together (E += D W reads only D and E, T = Q - Z N
            // only Z and Q)
            load_arow_t<NR>(d, row0, r1, t, ad);
            load_cols_clamped<NR>(e, row0, r1, t, E);
            Cols<NR> P;
            tile_mm_t<NR>(ad, bw, t, P);
#pragma unroll
            for (int k = 0; k < TileShape<NR>::CG; ++k)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    E.x[k][v] = make_float2(E.x[k][v].x + P.x[k][v].x, E.x[k][v].y + P.x[k][v].y);
            store_cols<NR>(e, row0, r1, t, E);
            __builtin_amdgcn_sched_barrier(0);  // keep the second half's loads after the first half
            load_arow_t<NR>(z, row0, r1, t, az);
            load_cols_clamped<NR>(q, row0, r1, t, Q);
            tile_mm_t<NR>(az, bn, t, P);
#pragma unroll
            for (int k = 0; k < TileShape<NR>::CG; ++k)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    Q.x[k][v] = make_float2(Q.x[k][v].x - P.x[k][v].x, Q.x[k][v].y - P.x[k][v].y);
            store_cols<NR>(q, row0, r1, t, Q);
            gram_tile<NR>(Q, Q, t, gacc);
            continue;
        }
        Cols<NR> DW, ZN;
        tile_mm_t<NR>(ad, bw, t, DW);
        tile_mm_t<NR>(az, bn, t, ZN);
#pragma unroll
        for (int k = 0; k < TileShape<NR>::CG; ++k)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                E.x[k][v] = make_float2(E.x[k][v].x + DW.x[k][v].x, E.x[k][v].y + DW.x[k][v].y);
                Q.x[k][v] = make_float2(Q.x[k][v].x - ZN.x[k][v].x, Q.x[k][v].y - ZN.x[k][v].y);
            }
        store_cols<NR>(e, row0, r1, t, E);
        store_cols<NR>(q, row0, r1, t, Q);
        gram_tile<NR>(Q, Q, t, gacc);
    }
    __syncthreads();  // B operands no longer read: the buffer becomes the reduction area
    gram_write<NR, NW>(gacc, red, partials + (size_t)blockIdx.x * NR * NR);
}

template <int NR, int NW = 4>
struct XtShape {
    static constexpr int BL = bop_floats<NR>();
    // the two B operands during the sweep, then (aliased) the NW waves' Grams
    static constexpr int RAW = (2 * BL * 4) > (NW * NR * NR * 16) ? (2 * BL * 4) : (NW * NR * NR * 16);
};

template <int NR>
__global__ __launch_bounds__(256, 2) void update_xt_mfma_kernel(float2 *__restrict__ e, float2 *__restrict__ q,
                                                             const float2 *__restrict__ d,
                                                             const float2 *__restrict__ z,
                                                             const float2 *__restrict__ wm,
                                                             const float2 *__restrict__ nm, long long rows,
                                                             double2 *__restrict__ partials,
                                                             const int *__restrict__ active) {
    constexpr int BL = XtShape<NR>::BL;
    __shared__ __align__(16) unsigned char raw[XtShape<NR>::RAW];
    float *bw = reinterpret_cast<float *>(raw), *bn = bw + BL;
    XtFirst<NR> first;
    xt_first<NR>(e, q, d, z, rows, first);
    const int flag = *(active != nullptr ? active : reinterpret_cast<const int *>(d));
    if (active != nullptr && flag == 0) return;
    build_bop_t<NR>(wm, bw);
    build_bop_t<NR>(nm, bn);
    __syncthreads();
    xt_sweep<NR>(e, q, d, z, rows, partials, bw, bn, reinterpret_cast<double2 *>(raw), first);
}

// The block updates with the small step in their prologue run on
// STEP_BLOCKS workgroups of STEP_WAVES waves: one workgroup per CU, so the
// small step that every workgroup computes occupies one wave per SIMD (two
// 256-thread workgroups per CU made two of them share each SIMD's f64 issue:
// the 16 x 16 factorisation took 4.7 us against 3.3 us alone). The first
// 256 threads hold the matrix entries; the others wait at its barriers.
constexpr int STEP_WAVES = 8;
constexpr int STEP_BLOCKS = 256;

// The same update with the small step after the Gram D^H Z in the prologue:
// every workgroup factors the reduced Gram itself and forms N and W in LDS
// (the same instructions on the same data, so every workgroup holds the same
// matrices); workgroup 0 alone sets failure flags, and no workgroup reads what
// another one writes.
template <int NR>
__global__ __launch_bounds__(64 * STEP_WAVES) void step1_xt_mfma_kernel(SmallMats m, SolverState *state,
                                                                         float2 *__restrict__ e,
                                                                         float2 *__restrict__ q,
                                                                         const float2 *__restrict__ d,
                                                                         const float2 *__restrict__ z, long long rows,
                                                                         double2 *__restrict__ partials) {
    constexpr int BL = XtShape<NR, STEP_WAVES>::BL, NP = small_pad(NR, 4);
    __shared__ __align__(16) unsigned char raw[XtShape<NR, STEP_WAVES>::RAW];
    __shared__ double2 A[NP * NP], R[NP * NP], Cm[NP * NP];
    __shared__ double scratch[8];
    float *bw = reinterpret_cast<float *>(raw), *bn = bw + BL;
    const SmallCtx c = small_ctx<4>(NR);  // the first np^2 <= 256 threads hold an entry each
    XtFirst<NR> first;
    xt_first<NR, STEP_WAVES>(e, q, d, z, rows, first);  // in flight during the small step
    if (step1_body<4>(m, state, c, A, R, Cm, scratch, blockIdx.x == 0) != 1) return;
    build_bop_lds_t<NR>(R, NP, false, bw);  // W = N C
    build_bop_lds_t<NR>(A, NP, false, bn);  // N
    __syncthreads();
    xt_sweep<NR, STEP_WAVES>(e, q, d, z, rows, partials, bw, bn, reinterpret_cast<double2 *>(raw), first);
}

// Q = T S^{-1} (T held in Q); D = Q (init) or D = Q + D S^H, from the B
// operands bs (S^{-1}) and bh (S^H).
// The wave's first tile of the qd sweep, loaded before the prologue (as
// xt_first).
template <int NR>
struct QdFirst {
    ARow<NR> at, ad;
};

template <int NR, int NW = 4>
__device__ __forceinline__ void qd_first(const float2 *__restrict__ q, const float2 *__restrict__ d, long long rows,
                                         int init, QdFirst<NR> &f) {
    const int w = threadIdx.x >> 6, t = threadIdx.x & 63;
    long long r0, r1;
    row_range(rows, r0, r1);
    const long long row0 = r0 + 16 * w;
    const long long rf = row0 < r1 ? row0 : 0, rl = row0 < r1 ? r1 : 1;
    load_arow_t<NR>(q, rf, rl, t, f.at);
    if (!init) load_arow_t<NR>(d, rf, rl, t, f.ad);
}

template <int NR, int NW = 4>
__device__ __forceinline__ void qd_sweep(float2 *__restrict__ q, float2 *__restrict__ d, long long rows, int init,
                                         const float *bs, const float *bh, const QdFirst<NR> &first) {
    const int w = threadIdx.x >> 6, t = threadIdx.x & 63;
    long long r0, r1;
    row_range(rows, r0, r1);
    ARow<NR> atn = first.at, adn = first.ad;
    long long row0 = r0 + 16 * w;
    for (; row0 < r1; row0 += 16 * NW) {
        const ARow<NR> at = atn, ad = adn;
        // the wave's next tile, in flight during this one (init is uniform)
        load_arow_t<NR>(q, row0 + 16 * NW, r1, t, atn);
        if (!init) load_arow_t<NR>(d, row0 + 16 * NW, r1, t, adn);
        Cols<NR> Qn, Dn;
        tile_mm_t<NR>(at, bs, t, Qn);
        if (!init) {
            tile_mm_t<NR>(ad, bh, t, Dn);
#pragma unroll
            for (int k = 0; k < TileShape<NR>::CG; ++k)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    Dn.x[k][v] = make_float2(Qn.x[k][v].x + Dn.x[k][v].x, Qn.x[k][v].y + Dn.x[k][v].y);
        } else {
            Dn = Qn;
        }
        // every wave reads only its own rows, so in-place stores are safe
        store_cols<NR>(q, row0, r1, t, Qn);
        store_cols<NR>(d, row0, r1, t, Dn);
    }
}

template <int NR>
__global__ __launch_bounds__(256) void update_qd_mfma_kernel(float2 *__restrict__ q, float2 *__restrict__ d,
                                                             const float2 *__restrict__ sinv,
                                                             const float2 *__restrict__ sh, long long rows, int init,
                                                             const int *__restrict__ active) {
    constexpr int BL = XtShape<NR>::BL;
    __shared__ float bs[BL], bh[BL];
    QdFirst<NR> first;
    qd_first<NR>(q, d, rows, init, first);
    const int flag = *(active != nullptr ? active : reinterpret_cast<const int *>(q));
    if (active != nullptr && flag == 0) return;
    build_bop_t<NR>(sinv, bs);
    if (!init) build_bop_t<NR>(sh, bh);
    __syncthreads();
    qd_sweep<NR>(q, d, rows, init, bs, bh, first);
}

// The same update with the small step after the Gram T^H T in the prologue:
// every workgroup factors T^H T = S^H S itself; workgroup 0 alone updates C,
// the residual norms, the iteration count and the flags, which no workgroup of
// this launch reads. After the final iteration (converged or at the limit)
// the Q, D update still runs: each cycle starts them afresh, so it is unused.
template <int NR>
__global__ __launch_bounds__(64 * STEP_WAVES) void step2_qd_mfma_kernel(SmallMats m, SolverState *state,
                                                                         float2 *__restrict__ q,
                                                                         float2 *__restrict__ d, long long rows) {
    constexpr int BL = XtShape<NR>::BL, NP = small_pad(NR, 4);
    __shared__ float bs[BL], bh[BL];
    __shared__ double2 A[NP * NP], R[NP * NP], Cm[NP * NP];
    __shared__ double scratch[8];
    const SmallCtx c = small_ctx<4>(NR);
    QdFirst<NR> first;
    qd_first<NR, STEP_WAVES>(q, d, rows, 0, first);  // in flight during the small step
    if (step2_body<4>(m, state, c, A, R, Cm, scratch, blockIdx.x == 0) != 1) return;
    build_bop_lds_t<NR>(R, NP, true, bs);  // S^{-1} = (S^{-H})^H
    build_bop_lds_t<NR>(A, NP, true, bh);  // S^H
    __syncthreads();
    qd_sweep<NR, STEP_WAVES>(q, d, rows, 0, bs, bh, first);
}

bool blas_mfma_supported(int nr) { return nr == 2 || nr == 4 || nr == 8 || nr == 16 || nr == 32; }

#define BLAS_DISPATCH(NRV, CALL) \
    switch (NRV) {               \
        case 2: CALL(2); break;  \
        case 4: CALL(4); break;  \
        case 8: CALL(8); break;  \
        case 16: CALL(16); break; \
        default: CALL(32); break; \
    }

void gram_mfma(const float2 *a, const float2 *b, long long rows, int nr, double2 *partials, double2 *g,
               const int *active, hipStream_t st) {
#define L(N) hipLaunchKernelGGL(gram_mfma_kernel<N>, dim3(GRAM_BLOCKS), dim3(256), 0, st, a, b, rows, partials, active)
    BLAS_DISPATCH(nr, L)
#undef L
    gram_reduce(partials, nr, g, active, st);
}

void update_xt_gram_mfma(float2 *e, float2 *q, const float2 *d, const float2 *z, const float2 *w, const float2 *n,
                         long long rows, int nr, double2 *partials, double2 *g, const int *active, hipStream_t st) {
#define L(N)                                                                                                 \
    hipLaunchKernelGGL(update_xt_mfma_kernel<N>, dim3(GRAM_BLOCKS), dim3(256), 0, st, e, q, d, z, w, n, rows, \
                       partials, active)
    BLAS_DISPATCH(nr, L)
#undef L
    gram_reduce(partials, nr, g, active, st);
}

bool small_fused_supported(int nr) { return blas_mfma_supported(nr) && nr <= 16; }

void step1_update_xt_gram_mfma(SmallMats m, SolverState *state, float2 *e, float2 *q, const float2 *d,
                               const float2 *z, long long rows, int nr, hipStream_t st) {
#define L(N)                                                                                                   \
    hipLaunchKernelGGL(step1_xt_mfma_kernel<N>, dim3(STEP_BLOCKS), dim3(64 * STEP_WAVES), 0, st, m, state, e, q, d, \
                       z, rows, const_cast<double2 *>(m.partials))
    switch (nr) {
        case 2: L(2); break;
        case 4: L(4); break;
        case 8: L(8); break;
        default: L(16); break;
    }
#undef L
    gram_reduce_n(m.partials, STEP_BLOCKS, nr, m.G, &state->active, st);
}

void step2_update_qd_mfma(SmallMats m, SolverState *state, float2 *q, float2 *d, long long rows, int nr,
                          hipStream_t st) {
#define L(N) \
    hipLaunchKernelGGL(step2_qd_mfma_kernel<N>, dim3(STEP_BLOCKS), dim3(64 * STEP_WAVES), 0, st, m, state, q, d, rows)
    switch (nr) {
        case 2: L(2); break;
        case 4: L(4); break;
        case 8: L(8); break;
        default: L(16); break;
    }
#undef L
}

void update_qd_mfma(float2 *q, float2 *d, const float2 *sinv, const float2 *sh, long long rows, int nr, int init,
                    const int *active, hipStream_t st) {
#define L(N) \
    hipLaunchKernelGGL(update_qd_mfma_kernel<N>, dim3(GRAM_BLOCKS), dim3(256), 0, st, q, d, sinv, sh, rows, init, active)
    BLAS_DISPATCH(nr, L)
#undef L
}

}  // namespace coarse
