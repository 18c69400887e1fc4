/*
 * acr.h - accelerated cyclic reduction (ACR) on one MI355X (gfx950).
 *
 * Solves A u = f for the block-tridiagonal matrices of Eq. (originalMatrix)
 * of Chavez et al., "Accelerated Cyclic Reduction" (Parallel Computing 2017):
 * n_z plane blocks of size M = nx * ny coming from a 7-point stencil on an
 * nx x ny x nz grid.  The factorisation is the red/black block cyclic
 * reduction of Section 2.2 (Eq. elim, Algorithm 1) with every plane block held
 * as a weak-admissibility hierarchical (HODLR) matrix truncated at a relative
 * tolerance (Section 3.1); the solve is the forward reduction of the
 * right-hand side and the back-substitution of Eq. all_backSubs / Algorithm 2.
 *
 * Conventions for every entry point:
 *  - C linkage; no function throws; a failing call returns a status code and
 *    leaves its outputs unspecified (handles are never partially created).
 *  - Device pointers are HIP device addresses on the current device; sizes
 *    are element counts.  Matrices are column-major.
 *  - One handle may be used by one host thread at a time.  Calls are ordered
 *    on the stream passed in; acr_factor synchronises that stream before it
 *    returns, the solve calls do not (outputs are ready when the stream is).
 *    A call on a handle issued on another stream than the handle's previous
 *    call first makes its stream wait for the previous one (the handle's
 *    solve buffers are shared by its calls); acr_free synchronises every
 *    stream the handle was used on before it releases memory.
 */
#ifndef ACR_H
#define ACR_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct acr_factor_s* acr_handle_t;

typedef enum {
  ACR_SUCCESS = 0,
  ACR_ERROR_INVALID_VALUE = 1,  /* bad option, null pointer, non-zero out-of-grid stencil entry */
  ACR_ERROR_OUT_OF_MEMORY = 2,  /* device allocation (or the allocator callback) failed        */
  ACR_ERROR_HIP = 3,            /* a HIP runtime call failed                                   */
  ACR_ERROR_SINGULAR = 4,       /* zero / non-finite pivot in a leaf or capacitance inverse,  */
                                /* or non-finite stencil values                               */
  ACR_ERROR_RANK_CAPACITY = 5,  /* a truncated rank exceeded options.max_rank                  */
  ACR_ERROR_NOT_CONVERGED = 6,  /* acr_solve_refined reached maxit above tol                   */
  ACR_ERROR_NOT_SUPPORTED = 7
} acr_status_t;

typedef enum {
  ACR_PREC_FP64 = 0,           /* factors stored and applied in FP64                              */
  ACR_PREC_FP32 = 1,           /* factors in FP32 (QR / products FP32, Jacobi SVD sweeps FP64)   */
  ACR_PREC_FP32_BF16LEAF = 2,  /* as FP32, but the dense leaf x leaf products of the factorisation */
                               /* run on BF16 matrix-core inputs: each 32-wide K block of an       */
                               /* operand panel is scaled by a power of two (largest magnitude    */
                               /* into [0.5, 1)), rounded to nearest even, accumulated in FP32     */
  ACR_PREC_FP32_FP16LEAF = 3,  /* the same with FP16 inputs                                        */
  ACR_PREC_FP32_BF16 = 4,      /* as FP32, but every block product of the factorisation (leaves,  */
                               /* leaf x factor, factor x factor, the products of the inverse and */
                               /* of H x H) runs on BF16 matrix-core inputs, each 32-wide K block  */
                               /* of an operand panel scaled by a power of two (largest magnitude */
                               /* into [0.5, 1)), accumulated in FP32; the compression (Gram, QR, */
                               /* SVD, the rebuild of truncated factors) and the solves stay      */
                               /* FP32 / FP64                                                      */
  ACR_PREC_FP32_FP16 = 5       /* the same with FP16 inputs                                        */
} acr_precision_t;

typedef struct {
  int32_t nx, ny, nplanes;   /* grid; M = nx * ny unknowns per plane, N = M * nplanes          */
  double eps;                /* relative truncation tolerance per block, >= 0; 0 = exact      */
  int32_t leaf;              /* maximum points per leaf cluster of the planar bisection, >= 1 */
  int32_t max_rank;          /* cap on any truncated rank, 0 = none (exceeding it -> error)   */
  int32_t precision;         /* acr_precision_t                                                */
  double inner_eps_ratio;    /* intermediate blocks and accumulators inside one operation     */
                             /* (the SMW inverse, products, sums) are truncated at eps * ratio; */
                             /* 0 -> 1.  Ratio 1 truncates at every operation; ratios < 1       */
                             /* approach one truncation per stored block (indefinite operators  */
                             /* such as Helmholtz need about 0.01)                              */
  /* optional device allocator (e.g. a framework's caching allocator); both NULL -> hipMalloc */
  void* (*alloc)(size_t bytes, void* ctx, hipStream_t stream);
  void (*release)(void* ptr, void* ctx, hipStream_t stream);
  void* alloc_ctx;
  int32_t svd_fused_lds;     /* cores above 64 columns whose pivoted QR + Jacobi working set    */
                             /* needs at most this many bytes of LDS run both in one          */
                             /* workgroup; 0 = default (none), < 0 = never; capped at the     */
                             /* LDS budget.  Tuned by acr_autotune.                            */
  int32_t stencil_points;    /* layout of coef: 7 (0 -> 7) or 27, see acr_factor              */
  int32_t gemm_tiles;        /* matrix-core tiles of FP32 products whose output is at most 32 */
                             /* columns wide: 0 = 128 x 32 tiles, 1 = 64 x 64 tiles (as wider */
                             /* outputs).  Tuned by acr_autotune.                              */
} acr_options_t;

/* Fills defaults: eps 1e-6, leaf 64, FP64, no rank cap, no allocator, default SVD
 * dispatch. Grid fields 0. */
void acr_options_default(acr_options_t* opt);

/*
 * Factorisation (Algorithm 1 with the block-wise approximation of its first
 * step).  coef: DEVICE, FP64, layout coef[7][nplanes][ny][nx], slot order
 * {C, W(i-1), E(i+1), S(j-1), N(j+1), B(k-1), T(k+1)}:
 *   (A u)_r = C u_r + W u_{r-1} + E u_{r+1} + S u_{r-nx} + N u_{r+nx}
 *             + B u_{r-M} + T u_{r+M},   r = (k*ny + j)*nx + i.
 * D_k is the 5-point part of plane k, E_k = diag(B[k]), F_k = diag(T[k]).
 * With options.stencil_points = 27 (e.g. the trilinear finite elements of
 * Section 5.3) coef is coef[27][nplanes][ny][nx], slot
 * s = 9 (dz + 1) + 3 (dy + 1) + (dx + 1) coupling node (i, j, k) to
 * (i + dx, j + dy, k + dz); D_k, E_k and F_k are then the 9-point plane
 * operators of dz = 0, -1, +1, and E_k, F_k are approximated like D_k.
 * Entries reaching outside the grid must be 0.  coef is read during the call
 * only; the handle keeps its own FP64 copy for residuals.  On success *out is
 * a new handle owning all factor memory; on failure *out is NULL.
 */
acr_status_t acr_factor(const acr_options_t* opt, const double* coef, hipStream_t stream,
                        acr_handle_t* out);

/*
 * x = M^{-1} b, M the truncated factorisation (forward reduction of b by
 * Eq. elim, then Eq. all_backSubs).  b, x: DEVICE, FP64, N x nrhs column-major
 * with leading dimensions ldb, ldx >= N, natural ordering r as above; x may
 * alias b.  Stream-ordered; the launch sequence is captured in a HIP graph on
 * the first call for each nrhs and replayed afterwards.
 */
acr_status_t acr_solve(acr_handle_t h, int32_t nrhs, const double* b, int64_t ldb, double* x, int64_t ldx,
                       hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * x = M^{-1} b as acr_solve, with the same arguments, layouts and results, but
 * every buffer beyond b and x (the permuted and reduced right-hand sides, the
 * per-block inner products, the task arrays of the launches) lives in one
 * fixed device array of ACR_NOALLOC_SCRATCH_BYTES per GPU, which the library
 * holds from its first use on that GPU until the process ends.  The call
 * allocates no device memory and launches its kernels one by one on `stream`
 * (no graph).  The first call per (handle, nrhs) records the launch sequence
 * on the host; the task arrays are copied into the array, ordered on
 * `stream`, whenever the array was last used by another handle or nrhs.
 * Every handle on a GPU shares that GPU's array, which keeps the last call's
 * contents (nothing in it needs to start at zero): calls that overlap on one
 * GPU -- on different streams or host threads without ordering between them --
 * race and give wrong results.  b and x are owned by the caller; x may alias b.
 * Errors: ACR_ERROR_INVALID_VALUE as for acr_solve, and when the workspace of
 * this grid, precision and nrhs does not fit the array (the message of
 * acr_last_error_message names the limit); nothing is launched then.
 */
#define ACR_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
acr_status_t acr_solve_noalloc(acr_handle_t h, int32_t nrhs, const double* b, int64_t ldb, double* x,
                               int64_t ldx, hipStream_t stream);

/*
 * x = M^{-T} b with the same factors: the cyclic reduction of A^T, whose level
 * blocks are (D_j^T, F_{j-1}^T, E_{j+1}^T), applied with transposed blocks.
 * Exactly the transpose of the operator acr_solve applies (up to rounding).
 */
acr_status_t acr_solve_transpose(acr_handle_t h, int32_t nrhs, const double* b, int64_t ldb, double* x,
                                 int64_t ldx, hipStream_t stream);

/* Releases the handle and all its memory after synchronising every stream it was used on. NULL-safe. */
void acr_free(acr_handle_t h);

typedef struct {
  int32_t levels;            /* cyclic-reduction levels q                                  */
  int32_t depth;             /* HODLR depth L of every plane block                         */
  int32_t max_rank;          /* largest stored rank                                        */
  double avg_rank;           /* mean rank over stored off-diagonal blocks                  */
  double factor_bytes;       /* bytes of the stored factors (G, E, F of every level)       */
  double factor_seconds;     /* wall time of acr_factor                                    */
  double solve_bytes;        /* algorithmic bytes one acr_solve with nrhs = 1 moves         */
  double flops_gemm, flops_qr, flops_svd, flops_inverse;  /* launched work in acr_factor */
  int64_t launches;          /* kernel launches issued by acr_factor                       */
  int32_t level_max_rank[32];
  double level_avg_rank[32];
} acr_stats_t;

acr_status_t acr_get_stats(acr_handle_t h, acr_stats_t* st);

typedef struct {
  int32_t method;      /* 0: iterative refinement x += M^{-1} r; 1: right-preconditioned GMRES; */
                       /* 2: preconditioned (flexible) CG, for symmetric positive definite A   */
  int32_t restart;     /* GMRES restart length (default 30)                                  */
  int32_t maxit;       /* maximum preconditioner applications (default 200)                  */
  double tol;          /* stop when ||b - A x||_2 / ||b||_2 <= tol (FP64 residual)           */
  int32_t transpose;   /* 1: solve A^T x = b with M^{-T} as preconditioner                   */
} acr_refine_options_t;

typedef struct {
  int32_t iterations;  /* preconditioner applications                                        */
  int32_t converged;
  double relres;       /* final true FP64 relative residual                                  */
  double relres0;      /* relative residual of the first preconditioned solve               */
} acr_refine_result_t;

/*
 * FP64 refined solve of A x = b (or A^T x = b) for one right-hand side, the
 * factorisation used as preconditioner (Section 5: a low-accuracy factorisation
 * combined with an iteration).  b, x: DEVICE FP64 length N (x must not alias b).
 * The residual uses the handle's FP64 stencil.  history (host, optional) gets
 * up to history_len relative residual estimates.  Synchronises the stream.
 * Returns ACR_ERROR_NOT_CONVERGED (with x = last iterate) when maxit is hit.
 */
acr_status_t acr_solve_refined(acr_handle_t h, const acr_refine_options_t* ro, const double* b, double* x,
                               hipStream_t stream, acr_refine_result_t* res, double* history,
                               int32_t history_len);

/* r = b - A x (or b - A^T x) in FP64 with the handle's stencil; DEVICE vectors of length N. */
acr_status_t acr_residual(acr_handle_t h, const double* x, const double* b, double* r, int32_t transpose,
                          hipStream_t stream);

/*
 * Stencil of -div(kappa grad u) on the unit cube, vertex-centred, h = 1/(n+1)
 * per axis, face coefficient = harmonic mean of the two nodal kappa, boundary
 * faces weighted by the nodal kappa (the variable-coefficient model problem of
 * Section 2.2.1).  kappa: DEVICE FP64 [nz][ny][nx]; coef: DEVICE FP64, layout
 * as in acr_factor.  Stream-ordered.
 */
acr_status_t acr_assemble_diffusion(int32_t nx, int32_t ny, int32_t nz, const double* kappa, double* coef,
                                    hipStream_t stream);

/*
 * Gradient of a scalar L with respect to the nodal kappa of
 * acr_assemble_diffusion, given the state u (A u = f) and the adjoint lam
 * (A^T lam = dL/du): grad_c = -lam^T (dA/dkappa_c) u.  All DEVICE FP64 length
 * N.  Stream-ordered.
 */
acr_status_t acr_kappa_gradient(int32_t nx, int32_t ny, int32_t nz, const double* kappa, const double* u,
                                const double* lam, double* grad, hipStream_t stream);

const char* acr_status_string(acr_status_t s);

/*
 * Structure of a factorisation (integer set-up of the path): the planar
 * bisection cluster tree of a plane (Section 2.1.1: a box is split across its
 * longer side, x on ties, the first part keeping ceil(side/2) grid lines; every
 * box of a depth is split while any box of that depth holds more than leaf
 * points; points are numbered leaf by leaf, first part first, x fastest inside
 * a leaf), the permutation from cluster order to the natural in-plane index,
 * and the red/black level schedule of Section 2.2.2 (Eq. permuted_system,
 * Eq. next_step: the planes at even positions of a level are eliminated, the
 * others renumbered for the next level, until one plane is left).
 *
 * Sizes go to *info; every array argument may be NULL (then it is skipped),
 * otherwise it must hold the number of entries named here:
 *   perm[M]                 cluster position p -> natural index j*nx + i
 *   node_offset[nodes], node_size[nodes]
 *                           node (depth d, segment s) at index 2^d - 1 + s:
 *                           first cluster position and number of points
 *   level_size[levels]      planes alive at level i
 *   sched_plane[schedule_len], sched_elim[schedule_len]
 *                           the alive planes of every level in order, level
 *                           after level (original plane numbers), and 1 for
 *                           a plane eliminated at that level, 0 for a kept one
 * The usual pattern is one call with NULL arrays for the sizes, then a second.
 */
typedef struct {
  int32_t M;             /* points per plane, nx * ny                          */
  int32_t depth;         /* HODLR depth L: the leaves are the nodes of depth L */
  int32_t nodes;         /* 2^(L+1) - 1                                        */
  int32_t levels;        /* cyclic-reduction levels q                          */
  int32_t schedule_len;  /* sum over the levels of the planes alive            */
  int32_t last_plane;    /* the plane left after the last level                */
} acr_structure_t;

/* Host only, no device work: the structure acr_factor would build for these
 * sizes.  ACR_ERROR_INVALID_VALUE for non-positive sizes, a null info, or a
 * leaf size that would split a single point. */
acr_status_t acr_plan_structure(int32_t nx, int32_t ny, int32_t nplanes, int32_t leaf, acr_structure_t* info,
                                int32_t* perm, int32_t* node_offset, int32_t* node_size, int32_t* level_size,
                                int32_t* sched_plane, int32_t* sched_elim);

/* The structure a handle was factorised with: perm is read back from the
 * device copy the solves use (synchronous copy), the schedule from the levels
 * the factorisation stored (a plane counts as eliminated when its inverse was
 * stored at that level).  Arrays and errors as for acr_plan_structure. */
acr_status_t acr_get_structure(acr_handle_t h, acr_structure_t* info, int32_t* perm, int32_t* node_offset,
                               int32_t* node_size, int32_t* level_size, int32_t* sched_plane,
                               int32_t* sched_elim);

/*
 * Autotuner for the leaf size and the core-SVD dispatch (the tile-size knobs of
 * the factorisation).  It factorises a sample of the operator -- its first
 * sample_planes planes (0 -> 16, capped at nplanes), with the coupling out of
 * the last sample plane dropped -- for every candidate leaf size in
 * {32, 64, 128, opt->leaf} (those that fit the plane) and every SVD dispatch in
 * {never, 64 KiB, LDS budget} (as svd_fused_lds: -1, 65536, 159744), times
 * factorisation + 16 single-RHS solves
 * (the cost of a refined solve), and returns the fastest pair, trying them in
 * the order listed: a later pair replaces the current choice only when at
 * least 3% faster, so timing noise does not flip between equivalent ones.
 * At the chosen pair it then times gemm_tiles = 1 against 0 (the matrix-core
 * tile shape of narrow products) under the same 3% rule.
 * All other
 * options are taken from opt.  coef: DEVICE, as for acr_factor (read only).
 * cache_path (may be NULL): a text file of one result per line keyed by
 * (nx, ny, sample planes, eps, precision, max_rank, inner_eps_ratio); a
 * matching line is returned without measuring (from_cache = 1), a new result
 * is appended.  Synchronises `stream`; allocates and frees its own scratch.
 * Errors: ACR_ERROR_INVALID_VALUE for bad options or pointers; the status of
 * the last failure if no candidate factorises.
 */
typedef struct {
  int32_t leaf;            /* chosen leaf size                                   */
  int32_t svd_fused_lds;   /* chosen acr_options_t.svd_fused_lds                 */
  double seconds;          /* sample factorisation + 16 solves with that choice  */
  int32_t tried;           /* candidates measured (0 when read from the cache)   */
  int32_t from_cache;      /* 1 if the result came from cache_path                */
  int32_t gemm_tiles;      /* chosen acr_options_t.gemm_tiles                      */
} acr_tune_result_t;
acr_status_t acr_autotune(const acr_options_t* opt, const double* coef, int32_t sample_planes,
                          const char* cache_path, hipStream_t stream, acr_tune_result_t* out);

/*
 * Per-kernel-class timing (instrumentation).  acr_set_kernel_timing(level)
 * with level >= 1 clears the process-wide table and makes every later
 * factorisation launch record a pair of HIP events on its stream around each
 * kernel; the table accumulates, per kernel class, launches, event-measured
 * milliseconds and the algorithmic flops and bytes of those launches (counted
 * from the task shapes and, for the SVD kernels, from device counters).  At
 * level 1 solves still replay their graph and are not timed; at level 2 each
 * solve is replayed launch by launch with events (and synchronises its
 * stream).  acr_set_kernel_timing(0) stops recording and keeps the table.
 * acr_get_kernel_times copies up to cap entries and returns the number of
 * classes.  Host-side tables; not thread-safe with concurrent factorisations.
 */
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;
  double flops;
  double bytes;
} acr_kernel_time_t;
void acr_set_kernel_timing(int32_t level);
int32_t acr_get_kernel_times(acr_kernel_time_t* out, int32_t cap);

/*
 * Cached device memory.  With the default allocator (acr_options_t.alloc
 * NULL), device buffers that the library releases (a freed handle's arenas,
 * executor buffers) are kept per device and size and handed to later requests
 * of the same size instead of going back through hipFree / hipMalloc, which
 * synchronise the device.  acr_release_cached_memory() frees every cached
 * buffer (all devices) and returns the bytes released; an allocation that
 * fails does the same once before reporting ACR_ERROR_HIP.  Environment
 * ACR_NO_POOL=1 disables the cache.  Callers with their own allocator
 * callbacks are not affected.  Thread-safe.
 */
size_t acr_release_cached_memory(void);

/* Text of the last failure on the calling host thread ("" if none); valid until the next call. */
const char* acr_last_error_message(void);

#ifdef __cplusplus
}
#endif
#endif /* ACR_H */
