// Launch interface of the coarse-operator apply kernels (used by the C ABI,
// the block solver and the batched launcher).
#pragma once
#include "common.hpp"

namespace coarse {

// Which kernel family an (nbasis, nrhs, link type, vector type) maps to.
enum ApplyPath { PATH_MFMA = 0, PATH_GENERIC = 1 };

// Forward apply y = M x (optionally y = sub - M x), asynchronous on `st`.
// `active`: device flag; the launch is a no-op when *active == 0 (NULL: always run).
int32_t launch_apply(const Geom &g, const void *packed, int32_t link_dtype, const void *x, void *y,
                     int nrhs, int32_t vec_dtype, const void *sub, const int *active, hipStream_t st,
                     int force_generic = 0);

// Adjoint apply y = M^H x.
int32_t launch_apply_adjoint(const Geom &g, const void *packed, int32_t link_dtype, const void *x, void *y,
                             int nrhs, int32_t vec_dtype, hipStream_t st, int force_generic = 0);

// MFMA adjoint (complex64 links, nbasis % 8 == 0); false when it does not apply.
bool launch_adjoint_mfma(const Geom &g, const void *packed, int32_t link_dtype, const void *x, void *y, int nr,
                         int32_t vec_dtype, hipStream_t st);

// True when the MFMA kernels cover this shape and type.
bool mfma_supported(int nb, int nrhs, int32_t link_dtype, int32_t vec_dtype);

}  // namespace coarse
