// Block-CG linear algebra on the device: Gram reductions, the small double
// precision dense step, and the tall-skinny block-vector updates.
#pragma once
#include "common.hpp"

namespace coarse {

constexpr int GRAM_BLOCKS = 512;  // fixed split-K count: deterministic reduction order

// Device-resident solver state, read by the host every few iterations.
struct SolverState {
    int active;      // 1 while the inner iteration runs; kernels skip when 0
    int done;        // inner tolerance reached
    int breakdown;   // a Gram matrix was not positive definite
    int nonfinite;   // NaN/Inf met
    int iters;       // inner iterations completed in this cycle
    int max_inner;
    double tol;      // inner tolerance on max_j ||C e_j|| / norm0[j]
    double relres[32];
    double norm0[32];  // 1, or ||C_0 e_j|| for a stop test relative to the start
};

// Small matrices of the inner iteration (device buffers, all nr x nr, row-major).
struct SmallMats {
    const double2 *partials;  // split-K partial Gram matrices (summed into G in a fixed order)
    double2 *G;      // reduced Gram (complex128)
    double2 *C;      // C_k (complex128)
    float2 *W;       // N_k C_k       (complex64, for X += D W)
    float2 *N;       // N_k           (complex64, for T = Q - Z N)
    float2 *Sinv;    // S^{-1}        (complex64, for Q = T S^{-1}; also C_0^{-1})
    float2 *SH;      // S^H           (complex64, for D = Q + D S^H)
};

// partial[b] = sum over rows of block b of conj(A[row][a]) B[row][c]; then reduced.
// T2 = float2 (complex64) or double2 (complex128) inputs; double accumulation.
template <typename T2>
void gram(const T2 *a, const T2 *b, long long rows, int nr, double2 *partials, double2 *g, const int *active,
          hipStream_t st);
// Only the split-K partials (the small steps reduce them).
template <typename T2>
void gram_partials(const T2 *a, const T2 *b, long long rows, int nr, double2 *partials, const int *active,
                   hipStream_t st);

// Sum the GRAM_BLOCKS partials in a fixed order into g.
void gram_reduce(const double2 *partials, int nr, double2 *g, const int *active, hipStream_t st);
// The same over `count` partials (a multiple of 64).
void gram_reduce_n(const double2 *partials, int count, int nr, double2 *g, const int *active, hipStream_t st);

// MFMA versions for nrhs in {2, 4, 8, 16, 32} (complex64 blocks).
bool blas_mfma_supported(int nr);
void gram_mfma(const float2 *a, const float2 *b, long long rows, int nr, double2 *partials, double2 *g,
               const int *active, hipStream_t st);
// E += D W; T = Q - Z N (over Q); g = T^H T of the new T (partials fused, then reduced).
void update_xt_gram_mfma(float2 *e, float2 *q, const float2 *d, const float2 *z, const float2 *w, const float2 *n,
                         long long rows, int nr, double2 *partials, double2 *g, const int *active, hipStream_t st);
void update_qd_mfma(float2 *q, float2 *d, const float2 *sinv, const float2 *sh, long long rows, int nr, int init,
                    const int *active, hipStream_t st);
// nrhs in {2, 4, 8, 16}: the small steps run in the prologue of every
// workgroup of the block update that consumes them (no separate launch).
bool small_fused_supported(int nr);
// Step 1 on the reduced D^H Z (m.G), then E += D W; T = Q - Z N and the
// reduced Gram T^H T into m.G.
void step1_update_xt_gram_mfma(SmallMats m, SolverState *state, float2 *e, float2 *q, const float2 *d,
                               const float2 *z, long long rows, int nr, hipStream_t st);
// Step 2 on the reduced T^H T (m.G: C, residual norms, flags), then
// Q = T S^{-1}; D = Q + D S^H.
void step2_update_qd_mfma(SmallMats m, SolverState *state, float2 *q, float2 *d, long long rows, int nr,
                          hipStream_t st);

// Q = (complex64) R diag(1/rn) with rn = sqrt(diag of the residual Gram), E = 0.
void normalize_residual(const double2 *r, const double2 *gdiag, long long rows, int nr, float2 *q, float2 *e,
                        hipStream_t st);
// X += E diag(rn), rn = sqrt(diag(gres)).
void outer_update(double2 *x, const float2 *e, const double2 *gres, long long rows, int nr, hipStream_t st);

// Small dense steps (one workgroup, double precision) on the reduced m.G.
// relative: the stop test divides ||C e_j|| by its value at the start (else by 1).
void small_init(SmallMats m, SolverState *state, int nr, double tol, int max_inner, hipStream_t st,
                int relative = 0);
void small_step1(SmallMats m, SolverState *state, int nr, hipStream_t st);
void small_step2(SmallMats m, SolverState *state, int nr, hipStream_t st);

// Q = Q S^{-1} (in place); D = Q (init) or D = Q + D S^H.
void update_qd(float2 *q, float2 *d, const float2 *sinv, const float2 *sh, long long rows, int nr, int init,
               const int *active, hipStream_t st);
// E += D W; Q -= Z N (T in place of Q).
void update_xt(float2 *e, float2 *q, const float2 *d, const float2 *z, const float2 *w, const float2 *n,
               long long rows, int nr, const int *active, hipStream_t st);

// Preconditioned BlockCGrQ block updates (q, z: residual space; qp, zp: their
// images under the preconditioner):
// E += D W; q -= z N; qp -= zp N (t and T in place of q and qp).
void update_pxt(float2 *e, float2 *q, float2 *qp, const float2 *d, const float2 *z, const float2 *zp,
                const float2 *w, const float2 *n, long long rows, int nr, const int *active, hipStream_t st);
// q = q S^{-1}; qp = qp S^{-1}; D = qp (init) or D = qp + D S^H.
void update_pqd(float2 *q, float2 *qp, float2 *d, const float2 *sinv, const float2 *sh, long long rows, int nr,
                int init, const int *active, hipStream_t st);

}  // namespace coarse
