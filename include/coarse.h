/*
 * coarse.h - C ABI of the multi-RHS coarse-operator library for MI355X (gfx950).
 *
 * The library applies the multigrid coarse-grid operator of arXiv 2409.03904
 * to many right-hand sides at once and solves with it by block conjugate
 * gradients:
 *
 *   y(x) = sum_p A_p(x) . X(x + delta_p)                      (Sec. 2.6)
 *
 * on a periodic 4D coarse lattice, with nbasis x nbasis complex link matrices
 * A_p(x) and an nbasis x nrhs block of the multi-RHS vector per site (the
 * RHS index is the extra "fifth dimension" of Sec. 2). The block solver is
 * BlockCGrQ (Fig. 2, left) in single precision, wrapped in a double
 * precision defect-correction loop.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Site index: s = x0 + L0*(x1 + L1*(x2 + L2*x3)), x0 fastest, periodic.
 * - Public links: [V][npoint][nbasis][nbasis] complex64, row-major, element
 *   (i, j) of A_p(x) at ((s*npoint + p)*nbasis + i)*nbasis + j.
 * - Vectors: [V][nbasis][nrhs], rhs fastest; complex64 or complex128
 *   (interleaved re, im).
 * - offsets: host array [npoint][4] of int8 in {-1, 0, 1}, unique, npoint <= 81
 *   (the {-1,0,1}^4 stencil of Sec. 2.6). Offsets whose neighbours coincide on
 *   an extent-1 or extent-2 direction are summed, as in the plain definition.
 * - Every lattice pointer is a DEVICE pointer owned by the caller. The library
 *   never allocates or frees device memory; solver workspace is passed in.
 * - `stream` is a hipStream_t (NULL = the null stream). Apply, pack and
 *   gradient calls are asynchronous on it; the solver returns after completion.
 * - Validation happens on the host before any HIP call; on error nothing is
 *   launched and the return code says why (text in cg_last_error()).
 * - Inputs and outputs must not alias.
 * - Limits: 1 <= nbasis <= 64, 1 <= nrhs <= 32, every extent >= 1,
 *   V * nbasis * nrhs < 2^31.
 */
#ifndef COARSE_H
#define COARSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define CG_OK                    0  /* success */
#define CG_NOT_CONVERGED         1  /* solver limits hit; x holds the best iterate */
#define CG_INVALID_ARG          (-1) /* bad pointer, shape, offset list or aliasing */
#define CG_UNSUPPORTED          (-2) /* shape/dtype combination not built */
#define CG_HIP_ERROR            (-3) /* a HIP call failed; see cg_last_error() */
#define CG_BREAKDOWN            (-4) /* a block Gram matrix is not positive definite */
#define CG_NONFINITE            (-5) /* NaN/Inf met in the right-hand side or iteration */
#define CG_WORKSPACE_TOO_SMALL  (-6) /* ws_bytes below coarse_bcg_workspace_bytes() */

/* ---- element types ----------------------------------------------------- */
#define COARSE_C64   0  /* complex64 (float re, im) */
#define COARSE_C128  1  /* complex128 (double re, im); vectors only */
#define COARSE_BF16  2  /* links: bfloat16 pairs x one power-of-two float scale per (site, point) */
#define COARSE_FP16  3  /* links: IEEE half pairs x one power-of-two float scale per (site, point) */
#define COARSE_C64_3M 4 /* links: complex64 values in the layout of the 3M kernel (three real
                           products per complex multiply-add); nbasis % 16 == 0, complex64
                           vectors (coarse_apply / coarse_apply_ws / coarse_apply_adjoint,
                           inner links of the solver) and, in coarse_apply, complex128
                           vectors (the double 3M residual) */

/* Geometry of one coarse operator (read during the call only). */
typedef struct coarse_geom {
    int32_t dims[4];          /* L0..L3 */
    int32_t nbasis;           /* N_basis */
    int32_t npoint;           /* number of stencil points */
    const int8_t *offsets;    /* host [npoint][4] */
} coarse_geom;

/* Bytes of the packed link buffer for `link_dtype` (C64, BF16 or FP16).
 * BF16/FP16 need nbasis % 16 == 0; C64 accepts any nbasis <= 64. */
int32_t coarse_packed_bytes(const coarse_geom *g, int32_t link_dtype, size_t *out);

/* Repack public complex64 links into the kernel layout (Sec. 2.5: the
 * coefficients live inside the operator object in a compute-ready layout).
 * C64: same values, tile-ordered. BF16/FP16: every block except the self
 * point's is divided by 2^ceil(log2 max(|Re|,|Im|)) over the block, rounded to
 * nearest-even in the 16-bit type, the scale kept as a float; the self block
 * (displacement 0, if present) stays complex64. Mirror pairs
 * A_{-p}(x+delta_p) = A_p(x)^H get identical scales, so a Hermitian operator
 * stays exactly Hermitian. `packed` must hold coarse_packed_bytes() bytes;
 * `links_c64` may be reused once the stream has passed this call. */
int32_t coarse_pack_links(const coarse_geom *g, const void *links_c64, int32_t link_dtype,
                          void *packed, void *stream);

/* y = M x (Sec. 2.6, summed over the stencil). `packed`/`link_dtype` from
 * coarse_pack_links. vec_dtype C64: float32 MFMA, float32 accumulation.
 * vec_dtype C128 (C64 or C64_3M links): double accumulation of exact
 * products (with C64_3M links in the 3M form: three real products per complex
 * multiply-add, T1 = Ar Xr, T2 = Ai Xi, T3 = (Ar + Ai)(Xr + Xi) in double), the
 * residual path of defect correction. With BF16/FP16 links the input of
 * every non-self point is rounded to the 16-bit type (FP16 with one
 * power-of-two scale per (site, rhs column)), accumulation is float32. */
int32_t coarse_apply(const coarse_geom *g, const void *packed, int32_t link_dtype,
                     const void *x, void *y, int32_t nrhs, int32_t vec_dtype, void *stream);

/* Device workspace coarse_apply_ws needs: for BF16/FP16 links the 16-bit
 * input operands of every site (64 * ceil(nrhs / 16) bytes per row of
 * nbasis: one 16-bit copy of x, half its size when nrhs is a multiple of 16)
 * plus the FP16 column scales; 0 for C64. */
int32_t coarse_apply_workspace_bytes(const coarse_geom *g, int32_t link_dtype, int32_t nrhs, size_t *out);

/* Same result as coarse_apply. With BF16/FP16 links it converts the input to
 * 16-bit MFMA operands once (into `ws`, caller-owned device memory of at
 * least coarse_apply_workspace_bytes bytes, not aliasing x or y) and then
 * runs the stencil on them; the results are bit-identical to coarse_apply
 * with the same links. With C64 links `ws` is not used (may be NULL). Calls
 * sharing one workspace must be stream-ordered. */
int32_t coarse_apply_ws(const coarse_geom *g, const void *packed, int32_t link_dtype, const void *x, void *y,
                        int32_t nrhs, int32_t vec_dtype, void *ws, size_t ws_bytes, void *stream);

/* Workspace bytes of coarse_apply_gram: the split-K partial Grams (8 MiB at
 * most) plus, for BF16/FP16 links, the prepared operands of the two-pass
 * apply (coarse_apply_workspace_bytes). */
int32_t coarse_apply_gram_workspace_bytes(const coarse_geom *g, int32_t link_dtype, int32_t nrhs, size_t *out);

/* y = M x and gram = x^H y (Fig. 2: the operator application of a BlockCGrQ
 * iteration and the nrhs x nrhs matrix it inverts next; row-major
 * complex128, device memory), complex64 vectors. The Gram sums exact
 * products of complex64 values in double over fixed split-K partials summed
 * in a fixed order (Sec. 3.5's short-K products plus a sum), so repeated calls
 * agree bit for bit. With C64_3M links, nrhs in {2, 4, 8, 16} and a lattice
 * volume that splits into a multiple of 64 workgroups of one or more sites
 * (V a multiple of 64; several sites per workgroup beyond 2048 sites at
 * nbasis <= 32, 512 above), the Gram is accumulated in the apply's epilogue
 * (no second pass over x and y); otherwise the apply is followed by the Gram
 * kernel.
 * `ws`: caller-owned device memory of coarse_apply_gram_workspace_bytes,
 * aliasing none of x, y, gram; calls sharing it must be stream-ordered.
 * y is bit-identical to coarse_apply_ws with the same arguments. */
int32_t coarse_apply_gram(const coarse_geom *g, const void *packed, int32_t link_dtype, const void *x, void *y,
                          int32_t nrhs, void *gram, void *ws, size_t ws_bytes, void *stream);

/* Bytes of the device scratch array behind coarse_apply_noalloc (40 MiB: the
 * 16-bit operands of an 8^4 lattice at nbasis 64, nrhs 32 take 32.5 MiB). */
#define COARSE_APPLY_NOALLOC_SCRATCH_BYTES (40u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as coarse_apply_ws, bit for bit, without a caller workspace. With
 * BF16/FP16 links the prepared 16-bit input operands go to a device array
 * inside the library (COARSE_APPLY_NOALLOC_SCRATCH_BYTES bytes; each GPU the
 * library runs on holds its own copy until the process ends). The call
 * itself allocates nothing; its first call on a device looks the array's
 * address up (hipGetSymbolAddress) with that device current.
 *   - Shapes whose workspace (coarse_apply_workspace_bytes) exceeds the array
 *     return CG_WORKSPACE_TOO_SMALL before any HIP call.
 *   - `stream` must belong to the current device (CG_INVALID_ARG otherwise).
 *   - Every call on one GPU shares that GPU's array: calls that may overlap
 *     in time on one GPU (unordered streams, several host threads) race and
 *     give wrong results; stream-ordered calls are safe. Nothing in the array
 *     has to start at zero (each call writes the operands it reads).
 *   - C64 and C64_3M links use no scratch (same kernels as coarse_apply).
 * Other arguments as coarse_apply. */
int32_t coarse_apply_noalloc(const coarse_geom *g, const void *packed, int32_t link_dtype, const void *x, void *y,
                             int32_t nrhs, int32_t vec_dtype, void *stream);

/* y = M^H x: y(x) = sum_p A_p(x - delta_p)^H X(x - delta_p) (the transpose of the
 * gather above; each link is still read once). Same argument rules. With
 * C64_3M links it runs in the 3M form on MFMA (three real products per complex
 * multiply-add, the contraction over the link row), complex64 vectors only. */
int32_t coarse_apply_adjoint(const coarse_geom *g, const void *packed, int32_t link_dtype,
                             const void *x, void *y, int32_t nrhs, int32_t vec_dtype, void *stream);

/* Links of the adjoint operator, public layout in and out:
 *   links_adj[x][p] = links[x - delta_p][p]^H,
 * so that M^H is the stencil operator with these links at the displacements
 * -delta_p: packing links_adj (any link type, the 3M layout included) with a
 * geometry whose offsets are negated gives an operator whose forward apply
 * is M^H x (the transpose of the Sec. 2.6 gather as a gather). Both
 * [V][npoint][nbasis][nbasis] complex64, device, not overlapping;
 * asynchronous on `stream`. */
int32_t coarse_adjoint_links(const coarse_geom *g, const void *links, void *links_adj, void *stream);

/* Link gradient of a real loss through y = M x (PyTorch's conjugate convention):
 * dlinks[x][p] = alpha * gy(x) . x(x + delta_p)^H   (accumulate == 0), or
 * dlinks[x][p] += alpha * gy(x) . x(x + delta_p)^H  (accumulate != 0).
 * gy, x: [V][nbasis][nrhs] complex64; dlinks: public layout, complex64. */
int32_t coarse_link_grad(const coarse_geom *g, const void *gy, const void *x, void *dlinks,
                         float alpha, int32_t accumulate, int32_t nrhs, void *stream);

/* ---- block CG ---------------------------------------------------------- */

typedef struct cg_solve_params {
    double tol;            /* target: max_j ||b_j - M x_j|| / ||b_j|| (double precision) */
    double inner_tol;      /* inner BlockCGrQ stop: max_j ||C e_j|| (columns unit at start); a cycle
                              that starts from true relative residual r stops at
                              max(inner_tol, tol / (4 r)) instead (no further than the
                              outer target needs) */
    int32_t max_outer;     /* defect-correction cycles */
    int32_t max_inner;     /* inner iterations per cycle */
    int32_t check_every;   /* inner iterations between host checks (graph length), >= 1 */
    int32_t use_graph;     /* 1: replay the inner iterations as one captured hipGraph */
    int32_t outer_dtype;   /* link type of packed_outer: COARSE_C64 (0: a zeroed struct's value) or
                              COARSE_C64_3M (the double residual in the 3M form; nbasis % 16 == 0).
                              With packed_inner NULL the inner iterations use the same links. */
} cg_solve_params;

typedef struct cg_solve_stats {
    int32_t status;        /* same as the return value */
    int32_t cycles;        /* outer cycles run */
    int32_t iterations;    /* inner iterations, summed over cycles */
    int32_t nrhs;
    double relres_max;     /* final max_j true relative residual (double precision) */
    double relres[32];     /* per column */
    double seconds_total;
    double seconds_inner;  /* inner block CG (float32 / low precision) */
    double seconds_outer;  /* residual recomputation and corrections (double) */
} cg_solve_stats;

/* Workspace bytes for coarse_bcg_solve with these shapes. */
int32_t coarse_bcg_workspace_bytes(const coarse_geom *g, int32_t nrhs, const cg_solve_params *p,
                                   size_t *out);

/* Solve M X = B for Hermitian positive definite M.
 * Outer loop (double): R = B - M X with `packed_outer` (C64 or C64_3M links
 * as p->outer_dtype, double accumulation); per-column norms; stop when
 * max_j ||r_j||/||b_j|| <= tol; R^ = R diag(1/||r_j||) rounded to complex64;
 * inner BlockCGrQ (Fig. 2, left, with the iterate update D_k M_k C_k) on
 * M~ = `packed_inner` (C64, C64_3M, BF16 or FP16 as `inner_dtype`; NULL =
 * packed_outer, inner_dtype then ignored) from E = 0 to inner_tol;
 * X += E diag(||r_j||) in double. All Gram matrices are accumulated in double
 * and their Cholesky factorisations and inverses are computed in double on
 * the device. b, x: [V][nbasis][nrhs] complex128; x holds X_0 on entry (a
 * warm start; resuming a saved X is a restart from it) and the solution on
 * return. Returns CG_OK, CG_NOT_CONVERGED (x = last iterate), CG_BREAKDOWN
 * (rank-deficient block; x = last iterate), CG_NONFINITE, or an argument
 * error. `st` may be NULL. */
int32_t coarse_bcg_solve(const coarse_geom *g, const void *packed_outer, const void *packed_inner,
                         int32_t inner_dtype, const void *b, void *x, int32_t nrhs,
                         const cg_solve_params *p, cg_solve_stats *st, void *ws, size_t ws_bytes,
                         void *stream);

/* ---- preconditioned block CG (Fig. 2, right; Sec. 2.2 and 2.3) -------------- */

typedef struct cg_chebyshev_prec {
    double lo, hi;   /* interval of the Chebyshev interpolant of 1/x, 0 < lo < hi */
    int32_t order;   /* polynomial degree n, 0 .. 1000 (n applications of M~ per use) */
} cg_chebyshev_prec;

/* Workspace bytes for coarse_pbcg_solve: the coarse_bcg_solve workspace plus
 * five complex64 block vectors (preconditioned q and z, Chebyshev scratch). */
int32_t coarse_pbcg_workspace_bytes(const coarse_geom *g, int32_t nrhs, const cg_solve_params *p,
                                    const cg_chebyshev_prec *prec, size_t *out);

/* Solve M X = B as coarse_bcg_solve does (double defect correction outside,
 * same arguments, layouts, ownership and return codes), with the inner
 * iteration Preconditioned BlockCGrQ (Fig. 2, right, iterate update
 * D_k N_k C_k) and the stationary preconditioner M^{-1} = P(M~): the degree-n
 * Chebyshev interpolant of 1/x on [prec->lo, prec->hi] in the inner operator
 * (Sec. 2.3; the interpolant is positive on (0, hi], so P(M~) is Hermitian
 * positive definite when every eigenvalue of M~ is at most hi). Every inner
 * iteration applies M~ order + 1 times. The inner stop test is relative:
 * max_j ||C_k e_j|| / ||C_0 e_j|| <= inner_tol (or the last cycle's looser bound
 * described at cg_solve_params), ||C e_j|| being the P-norm
 * sqrt(r_j^H P r_j) of residual column j. Returns CG_INVALID_ARG for a NULL
 * prec or a bad interval or degree. */
int32_t coarse_pbcg_solve(const coarse_geom *g, const void *packed_outer, const void *packed_inner,
                          int32_t inner_dtype, const void *b, void *x, int32_t nrhs,
                          const cg_solve_params *p, const cg_chebyshev_prec *prec, cg_solve_stats *st,
                          void *ws, size_t ws_bytes, void *stream);

/* ---- multi-RHS deflation and the deflated Chebyshev coarse solve (Sec. 2.3) -- */

/* Workspace bytes for coarse_deflate with n_ev vectors (1 .. 4096) and nrhs
 * right-hand sides: split-K partial coefficient tiles and the two n_ev x nrhs
 * coefficient blocks. */
int32_t coarse_deflation_workspace_bytes(const coarse_geom *g, int32_t nev, int32_t nrhs, size_t *out);

/* Deflation of a block of right-hand sides on n_ev vectors |i> with values
 * lambda_i (Sec. 2.3; its multi-RHS BLAS form, Sec. 2.5):
 *   c = V^H x,   y = V diag(1/lambda) c = sum_i |i><i|x>/lambda_i,
 *   x_perp = x - V c   (only if x_perp is not NULL; x_perp may be x itself).
 * v: [V][nbasis][nev] complex64, one row (site, basis index) holding the n_ev
 * vectors' entries side by side; meant to be orthonormal (not checked).
 * lam: nev doubles, device memory; a vector whose lambda_i is not positive and
 * finite (such as a zero Ritz pair from coarse_block_lanczos past an exhausted
 * Krylov space) is left out of both y and x_perp, as if it were not in V.
 * x, y, x_perp: [V][nbasis][nrhs] complex64.
 * All device pointers, owned by the caller; y and the workspace must not
 * overlap any input. Asynchronous on `stream`; deterministic (fixed-order
 * split-K sums in double). CG_WORKSPACE_TOO_SMALL / CG_INVALID_ARG on bad
 * arguments, checked before any HIP call. */
int32_t coarse_deflate(const coarse_geom *g, const void *v, int32_t nev, const double *lam, const void *x,
                       void *y, void *x_perp, int32_t nrhs, void *ws, size_t ws_bytes, void *stream);

/* Workspace bytes for coarse_block_lanczos. */
int32_t coarse_block_lanczos_workspace_bytes(const coarse_geom *g, int32_t link_dtype, int32_t block,
                                             int32_t steps, int32_t nev, size_t *out);

/* Deflation vectors by block Lanczos with full reorthogonalisation on the
 * Hermitian operator in `packed` (any link type): from the start block x0
 * ([V][nbasis][block] complex64, full rank), `steps` block steps build an
 * orthonormal basis Q of K = steps * block columns (every new block
 * reorthogonalised twice against all earlier ones, then normalised by the
 * Cholesky factor of its Gram matrix); the K x K projected matrix Q^H M Q is
 * diagonalised on the host in double (coarse_hermitian_eigh) and the nev lowest Ritz pairs
 * returned: v_out [V][nbasis][nev] complex64 (the layout coarse_deflate
 * takes), lam_out[nev] and, if not NULL, res_out[nev] = ||M v - theta v|| from
 * the last block's factor (host arrays); *k_out (if not NULL) = the basis
 * size used (less than K when a new block is rank deficient: the Krylov space
 * is exhausted or numerically so; the residuals then come from the Gram matrix
 * of that last block, sqrt(z^H W^H W z) with z the last block of the Ritz
 * vector, and Ritz pairs past that size come back as zero values and zero
 * vectors, which coarse_deflate leaves out). Limits: block <= 32, K <= 512 and
 * <= V * nbasis, 1 <= nev <= K.
 * Synchronises `stream`. CG_BREAKDOWN for a rank-deficient start block. */
int32_t coarse_block_lanczos(const coarse_geom *g, const void *packed, int32_t link_dtype, const void *x0,
                             int32_t block, int32_t steps, int32_t nev, void *v_out, double *lam_out,
                             double *res_out, int32_t *k_out, void *ws, size_t ws_bytes, void *stream);

/* Host utility (no device work; the Rayleigh-Ritz step of coarse_block_lanczos):
 * eigenvalues ascending into w[n] and orthonormal eigenvectors into the columns
 * of z for the Hermitian n x n matrix a (both interleaved complex128,
 * row-major, host memory), by Householder reduction to a real tridiagonal
 * matrix and implicit QL. 1 <= n <= 4096; CG_INVALID_ARG otherwise. */
int32_t coarse_hermitian_eigh(int32_t n, const double *a, double *w, double *z);

/* Workspace bytes for coarse_deflated_chebyshev_apply. */
int32_t coarse_deflated_chebyshev_workspace_bytes(const coarse_geom *g, int32_t link_dtype, int32_t nev,
                                                  int32_t nrhs, size_t *out);

/* The two-part stationary coarse solve of Sec. 2.3:
 *   y = Defl(x) + P(M) x_perp,  x_perp = x - V V^H x,
 * P the degree-`order` Chebyshev interpolant of 1/x on [lo, hi] applied to
 * the operator in `packed` (any link type, as coarse_chebyshev_apply). With
 * V the lowest eigenvectors of M and lambda their eigenvalues this is
 * diag(1/lambda_1 .. 1/lambda_nev, P(lambda_nev+1) .. P(lambda_max)) in the
 * eigenbasis. Arguments as coarse_deflate and coarse_chebyshev_apply. */
int32_t coarse_deflated_chebyshev_apply(const coarse_geom *g, const void *packed, int32_t link_dtype,
                                        const void *v, int32_t nev, const double *lam, const void *x, void *y,
                                        int32_t nrhs, double lo, double hi, int32_t order, void *ws,
                                        size_t ws_bytes, void *stream);

/* ---- transfer between grids: block project and promote (Sec. 2.5) ---------- */

/* Block project, one product per coarse site x_c:
 *   C(x_c) = B(x_c)^H F(x_c)   (N_basis x N_rhs = (V_block x N_basis)^H (V_block x N_rhs)).
 * g: the coarse geometry (V sites, nbasis; offsets are not used but must be
 * valid). basis: [V][vblock][nbasis] complex64 (the fine degrees of freedom
 * of block x_c in a fixed order, each row holding the nbasis basis vectors'
 * entries); fine: [V][vblock][nrhs] complex64 in the same block order;
 * coarse_out: [V][nbasis][nrhs] complex64, the coarse vector layout. vblock
 * a multiple of 16 in [16, 65536], V <= 65535. Device pointers owned by the
 * caller, not aliasing; asynchronous on `stream`. CG_UNSUPPORTED /
 * CG_INVALID_ARG on bad shapes or pointers, checked before any HIP call. */
int32_t coarse_block_project(const coarse_geom *g, int32_t vblock, const void *basis, const void *fine,
                             void *coarse_out, int32_t nrhs, void *stream);

/* Block promote, one product per coarse site: F(x_c) = B(x_c) C(x_c).
 * Layouts and rules as coarse_block_project (coarse_in [V][nbasis][nrhs],
 * fine [V][vblock][nrhs]). */
int32_t coarse_block_promote(const coarse_geom *g, int32_t vblock, const void *basis, const void *coarse_in,
                             void *fine, int32_t nrhs, void *stream);

/* ---- several independent solves at once ------------------------------------ */

typedef struct coarse_solve_system {
    coarse_geom geom;
    int32_t nrhs;
    const void *packed_outer;  /* packed links defining M (link type p->outer_dtype) */
    const void *packed_inner;  /* inner links (C64, C64_3M, BF16, FP16); NULL = packed_outer */
    int32_t inner_dtype;
    const void *b;             /* [V][nbasis][nrhs] complex128 */
    void *x;                   /* [V][nbasis][nrhs] complex128, X_0 in, solution out */
} coarse_solve_system;

/* Workspace bytes for coarse_bcg_solve_batched: the systems' solver
 * workspaces back to back (256-byte aligned). */
int32_t coarse_bcg_batched_workspace_bytes(const coarse_solve_system *sys, int32_t nsys,
                                           const cg_solve_params *p, size_t *out);

/* coarse_bcg_solve for nsys (1..64) independent systems with common
 * parameters. Each system's residuals and inner start run on a stream of its
 * own; the inner BlockCGrQ iterations of all systems are captured into one
 * graph with one branch per system and replayed until every system's device
 * flag is down, so small systems run concurrently instead of one after the
 * other. st[k] receives system k's statistics (status per system). Returns
 * CG_OK when every system converged, else the first failing system's status
 * (argument errors are returned for the whole batch before any work). Distinct
 * systems must not share x. Returns after completion. */
int32_t coarse_bcg_solve_batched(const coarse_solve_system *sys, int32_t nsys, const cg_solve_params *p,
                                 cg_solve_stats *st, void *ws, size_t ws_bytes, void *stream);

/* ---- batches of independent systems (one persistent launch) ---------------- */

typedef struct coarse_system {
    coarse_geom geom;
    int32_t nrhs;
    const void *packed;    /* C64 packed links */
    const void *x;         /* [V][nbasis][nrhs] complex64 */
    void *y;               /* [V][nbasis][nrhs] complex64 */
} coarse_system;

/* Bytes of device workspace coarse_apply_batched needs for these systems: the
 * queue counter plus a copy of the system table (a few KB). */
int32_t coarse_batched_workspace_bytes(const coarse_system *sys, int32_t nsys, size_t *out);

/* y_i = M_i x_i for every system, in ONE persistent kernel launch over a
 * device work queue of (system, site) items, largest first. Systems may
 * differ in lattice, nbasis and nrhs. `ws` (caller-owned, device memory)
 * receives the queue counter and the system table, written by the launch on
 * the same stream; concurrent launches need separate workspaces. */
int32_t coarse_apply_batched(const coarse_system *sys, int32_t nsys, void *ws, size_t ws_bytes,
                             void *stream);

/* ---- tuning and reference paths --------------------------------------------
 * The complex64 (4M) apply has variants that split the stencil points of a
 * site over 1, 2 or 4 groups of waves inside one workgroup (the group sums are
 * added in the epilogue): more waves per workgroup at small nbasis; and one
 * without split that prefetches links one point ahead instead of two (fewer
 * registers, more waves per SIMD). The 3M
 * apply (COARSE_C64_3M) has two: link prefetch one or two points ahead.
 * Every variant computes the same operator; only the summation order or the
 * scheduling differs. */

/* Number of 4M variants for this nbasis (2 to 4), or a negative status. */
int32_t coarse_apply_variant_count(int32_t nbasis);

/* Time every variant on the caller's buffers (reps launches each; y is
 * overwritten), remember the fastest for this (nbasis, nrhs, npoint, link
 * dtype, vec dtype) in a process-wide table used by every later apply and
 * solve, and append it to the file named by the COARSE_TUNE_CACHE environment
 * variable when set (the table is loaded from that file on first use).
 * Synchronises the stream. */
int32_t coarse_tune_apply(const coarse_geom *g, const void *packed, int32_t link_dtype, const void *x, void *y,
                          int32_t nrhs, int32_t vec_dtype, int32_t reps, void *stream, int32_t *best_variant,
                          float *best_us);

/* Pin (variant >= 0, clamped to the count) or clear (variant < 0) a table entry. */
int32_t coarse_set_apply_variant(int32_t nbasis, int32_t nrhs, int32_t npoint, int32_t link_dtype,
                                 int32_t vec_dtype, int32_t variant);

/* Workgroups per compute unit of the persistent batched grid (1 to 16; 0
 * leaves it unchanged). Returns the value in effect. */
int32_t coarse_batched_set_occupancy(int32_t wg_per_cu);

/* The same operations as coarse_apply / coarse_apply_adjoint on the plain
 * vector-ALU kernels (one thread per output element, no MFMA): a second,
 * independent device implementation used to cross-check the MFMA kernels. */
int32_t coarse_apply_generic(const coarse_geom *g, const void *packed, int32_t link_dtype, const void *x, void *y,
                             int32_t nrhs, int32_t vec_dtype, void *stream);
int32_t coarse_apply_adjoint_generic(const coarse_geom *g, const void *packed, int32_t link_dtype, const void *x,
                                     void *y, int32_t nrhs, int32_t vec_dtype, void *stream);

/* ---- stationary Chebyshev polynomial of the operator -------------------
 * Sec. 2.3 replaces the data-dependent CG polynomial of the coarse solve by
 * the degree-n Chebyshev interpolant of 1/x on [lo, hi] (coefficients from
 * 1/x at the n + 1 Chebyshev points; the paper's coarse solve uses
 * [lo, hi, n] = [0.02, 40, 120]):
 *
 *   P(x) = sum_{k=0}^{n} c_k T_k(y(x)),  y(x) = (2x - (hi + lo)) / (hi - lo),
 *   c_k  = 2/(n+1) sum_j cos(k theta_j) / x_j  (c_0 halved),
 *   theta_j = pi (j + 1/2) / (n + 1),  x_j = (hi - lo)/2 cos(theta_j) + (hi + lo)/2.
 *
 * Limits: 0 < lo < hi, 0 <= order <= 1000. */

/* c[0..order] on the host (c: order + 1 doubles, caller-owned). */
int32_t coarse_chebyshev_coefficients(double lo, double hi, int32_t order, double *c);

/* Workspace bytes for coarse_chebyshev_apply (three complex64 block vectors,
 * plus the 16-bit apply's operand buffer for BF16/FP16 links). */
int32_t coarse_chebyshev_workspace_bytes(const coarse_geom *g, int32_t link_dtype, int32_t nrhs, size_t *out);

/* y = P(M) x for complex64 vectors x, y ([V][nbasis][nrhs]) and any link type
 * (C64, C64_3M, BF16, FP16), by the three-term recurrence T_0 = x,
 * T_1 = Y x, T_{k+1} = 2 Y T_k - T_{k-1} with Y = (2M - (hi + lo)) / (hi - lo):
 * `order` applies of M, each followed by one elementwise pass (recurrence and
 * accumulation fused). Float32 vectors: the recurrence is stable while the
 * spectrum of M lies in [lo, hi]; outside it T_k grows like cosh(k acosh|y|).
 * Asynchronous on `stream`. x, y and ws (ws_bytes >= the size above; not
 * needed for order 0) must not alias. */
int32_t coarse_chebyshev_apply(const coarse_geom *g, const void *packed, int32_t link_dtype, const void *x, void *y,
                               int32_t nrhs, double lo, double hi, int32_t order, void *ws, size_t ws_bytes,
                               void *stream);


/* ---- errors ---------------------------------------------------------------- */
const char *cg_status_string(int32_t status);
/* Text of the last error on the calling thread ("" if none). */
const char *cg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* COARSE_H */
