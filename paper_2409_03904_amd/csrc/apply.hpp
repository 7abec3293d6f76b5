// Launch interface of the coarse-operator apply kernels (used by the C ABI,
// the block solver and the batched launcher).
#pragma once
#include "common.hpp"

namespace coarse {

// Which kernel family an (nbasis, nrhs, link type, vector type) maps to.
enum ApplyPath { PATH_MFMA = 0, PATH_GENERIC = 1 };

// Forward apply y = M x (optionally y = sub - M x), asynchronous on `st`.
// `active`: device flag; the launch is a no-op when *active == 0 (NULL: always run).
// `variant` < 0 takes the tuned variant for the shape (default 0).
// `lowp_ws`: workspace of lowp_ws_bytes() bytes; with 16-bit links it selects
// the two-pass kernels (inputs converted once), NULL the one-pass kernel.
int32_t launch_apply(const Geom &g, const void *packed, int32_t link_dtype, const void *x, void *y,
                     int nrhs, int32_t vec_dtype, const void *sub, const int *active, hipStream_t st,
                     int force_generic = 0, int variant = -1, void *lowp_ws = nullptr);

// 3M-form apply (apply_3m.hip): complex64 links in the 3M layout, nbasis % 16 == 0.
// variant: 0 = one point of link prefetch, 1 = two.
void launch_apply_3m(const Geom &g, const float *links, const float *x, float *y, int nr, const float *sub,
                     const int *active, hipStream_t st, int variant);

// 3M-form apply y = M x with the Gram x^H y fused into the epilogue (the
// BlockCGrQ Gram D^H Z): nblk workgroups (apply_3m_gram_blocks; 0 when the
// shape has no fused form) each write one partial nr x nr complex128 Gram
// into partials[nblk][nr][nr], to be summed in order by gram_reduce_n.
int apply_3m_gram_blocks(const Geom &g, int nr);
void launch_apply_3m_gram(const Geom &g, const float *links, const float *x, float *y, int nr, double2 *partials,
                          int nblk, const int *active, hipStream_t st, int variant);

// The 3M-form apply with complex128 vectors and float64 accumulation (the
// outer residual y = sub - M x on 3M-layout links), nbasis % 16 == 0.
void launch_apply_3m_f64(const Geom &g, const float *links, const double *x, double *y, int nr, const double *sub,
                         const int *active, hipStream_t st);

// Adjoint y = M^H x in the 3M form on the same 3M-layout links (apply_3m.hip);
// variant: link prefetch depth 1 or 2 points.
void launch_adjoint_3m(const Geom &g, const float *links, const float *x, float *y, int nr, hipStream_t st,
                       int variant);

// One degree of a Chebyshev recurrence fused into the epilogue of the 3M
// apply: with z = M t at a site (t = the apply's input),
//   t_next = A z + B t + C t_prev,   y = D y + E t_next + F t,
// t_prev read only when C != 0 and y only when D != 0; t_next may be t_prev's
// buffer (each entry is read before the same lane writes it). t itself is
// read by other workgroups as neighbour data, so it is never written.
struct ChebEpi {
    const float *t_prev;
    float *t_next;
    float *y;
    float A, B, C, D, E, F;
};
void launch_apply_3m_cheb(const Geom &g, const float *links, const float *t, const ChebEpi &ce, int nr,
                          const int *active, hipStream_t st, int variant);

// Chebyshev polynomial P(M) x (chebyshev.hip): three block vectors of
// complex64 scratch (ta, tb, z; 256-byte aligned) and, for 16-bit links, the
// prepared-operand buffer of the two-pass apply. Every launch is a no-op once
// *active == 0 (active may be null).
struct ChebBuffers {
    void *ta, *tb, *z, *lowp;
};
int32_t chebyshev_poly(const Geom &d, const void *packed, int32_t link_dtype, const void *x, void *y, int nrhs,
                       double lo, double hi, int order, const ChebBuffers &b, const int *active, hipStream_t st);
int32_t check_chebyshev(double lo, double hi, int32_t order);

// Two-pass 16-bit apply (apply_lowp.hip): workspace bytes and launcher (kind 0 BF16, 1 FP16).
size_t lowp_ws_bytes(const Geom &g, int nr);
void launch_lowp_ws(const Geom &g, int kind, const uint16_t *q16, const float *self_c64, const float *scales,
                    const float *x, float *y, int nr, const float *sub, const int *active, void *ws,
                    hipStream_t st);

// Tuned variant (point split) of a shape; 0 when untuned.
int tuned_variant(int nb, int nr, int np, int link, int vec);

// Adjoint apply y = M^H x.
int32_t launch_apply_adjoint(const Geom &g, const void *packed, int32_t link_dtype, const void *x, void *y,
                             int nrhs, int32_t vec_dtype, hipStream_t st, int force_generic = 0);

// MFMA adjoint (complex64 links, nbasis % 8 == 0); false when it does not apply.
bool launch_adjoint_mfma(const Geom &g, const void *packed, int32_t link_dtype, const void *x, void *y, int nr,
                         int32_t vec_dtype, hipStream_t st);

// float32 / float64 MFMA apply launchers (apply_mfma_f32.hip, apply_mfma_f64.hip).
// variant: point split 1 << variant (clamped to what the shape allows).
// false (error text set) when the shape exceeds the kernel's staging bound.
bool launch_mfma_f32(const Geom &g, const float *links, const float *x, float *y, int nr, const float *sub,
                     const int *active, hipStream_t st, int variant);
bool launch_mfma_f64(const Geom &g, const float *links, const double *x, double *y, int nr, const double *sub,
                     const int *active, hipStream_t st);
int max_variant(int nb);

// True when the MFMA kernels cover this shape and type.
bool mfma_supported(int nb, int nrhs, int32_t link_dtype, int32_t vec_dtype);

}  // namespace coarse
