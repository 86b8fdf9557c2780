/*
 * nsrgs.h -- C ABI of the NS-RGS library for AMD MI355X (gfx950).
 *
 * NS-RGS (Peng, Han, Chen, Huang, "NS-RGS: Newton-Schulz Based Riemannian
 * Gradient Method for Orthogonal Group Synchronization") recovers
 * Z_1..Z_n in O(d) from the symmetric block measurement matrix
 *     A = Z Z^T + sigma W   (nd x nd, blocks A_ij = Z_i Z_j^T + sigma W_ij),
 * Sec. 2.2, eq. (def:measurements).  Algorithm 2 starts from the spectral
 * initialization X^0 = sgn(Y), Y the top-d eigenvectors of A, and then for
 * every block i in parallel (a Jacobi sweep over X^t):
 *     G_i = sum_{j != i} (X_i - A_ij X_j)            (Euclidean gradient)
 *     F_i = X_i - mu (G_i - X_i G_i^T X_i) / 2        (pseudo tangent step)
 *     X_i <- S^{Ts}(F_i),  S: S <- S (3I - S^T S)/2   (Algorithm 1)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every pointer argument named A/X/ws/out is a DEVICE pointer (HIP memory
 *   of the current device) owned by the caller.  The library never frees it.
 *   Pointers to nsrgs_matrix / nsrgs_info / option structs are HOST pointers.
 * - Stacked d x d blocks: an "n*d x d" array X is row-major, block i occupying
 *   rows [i*d, (i+1)*d).  X is double when A is NSRGS_A_F64, float otherwise.
 * - A is row-major with leading dimension ld (elements): element (r, c) at
 *   r*ld + c.  ld >= n*d and ld % 16 == 0; the buffer holds n*d full rows of
 *   ld elements (padding columns are never used as data); base pointers are
 *   16-byte aligned.  A must be symmetric; only the off-diagonal blocks enter
 *   the gradient, the diagonal blocks enter only the spectral initialization.
 * - Packed storage (ld == NSRGS_LD_PACKED): the upper block triangle of the
 *   symmetric A (Sec. 2.2: A_ji = A_ij^T) in about half the memory; see
 *   NSRGS_LD_PACKED below.  Read by sync_step_symmetric, by sync_solve with
 *   opts->symmetric = 1 and by sync_init_spectral (d <= 16, formats F64, F32,
 *   BF16, BF16_SPLIT); every other call refuses it with NSRGS_ERR_UNSUPPORTED.
 * - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue work
 *   on it and return without waiting unless stated otherwise.
 * - Return value: an nsrgs_status.  On error nothing has been enqueued and
 *   nsrgs_last_error() (per calling thread) describes the problem.  Device
 *   errors of earlier asynchronous work surface as NSRGS_ERR_DEVICE.
 * - Limits: 2 <= n, 1 <= d <= 16, n*d < 2^31.  sync_step, sync_step_polar,
 *   sync_step_gpm, sync_init_spectral, sync_solve, sync_read_info,
 *   sync_workspace_bytes and nsrgs_generate_measurement also take
 *   16 < d <= 32 with F64 or F32 storage (the matrix-core path; other formats
 *   are refused with NSRGS_ERR_UNSUPPORTED).
 * - The library never allocates device memory inside sync_step / sync_solve /
 *   sync_init_spectral: scratch space is the caller's workspace `ws` of
 *   sync_workspace_bytes() bytes, prepared once by sync_workspace_init().
 *   Two calls that run at the same time must not share a workspace.
 */
#ifndef NSRGS_H
#define NSRGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NSRGS_VERSION 100

typedef enum {
  NSRGS_OK = 0,
  NSRGS_ERR_INVALID_ARG = 1,   /* bad size, pointer, alignment, aliasing, format */
  NSRGS_ERR_UNSUPPORTED = 2,   /* valid request this build does not implement   */
  NSRGS_ERR_OUT_OF_MEMORY = 3, /* workspace too small / server memory exhausted  */
  NSRGS_ERR_DEVICE = 4,        /* a HIP runtime call failed                      */
  NSRGS_ERR_NOT_CONVERGED = 5, /* tolerance not met within the budget            */
  NSRGS_ERR_NONFINITE = 6      /* a NaN/Inf appeared in an iterate               */
} nsrgs_status;

/* Storage formats of A (precision forms).  The reduced formats are produced
 * from an FP32 matrix by nsrgs_convert(). */
typedef enum {
  NSRGS_A_F64 = 0,        /* double                                              */
  NSRGS_A_F32 = 1,        /* float                                               */
  NSRGS_A_BF16 = 2,       /* bfloat16 (uint16 codes), round-to-nearest-even of A */
  NSRGS_A_BF16_SPLIT = 3, /* hi = bf16(A) in `data`, lo = bf16(A - hi) in
                             `data_lo`; the value used is hi + lo               */
  NSRGS_A_FP8_E4M3 = 4    /* OCP e4m3 codes (uint8) and per-row float scales
                             s_r = max_c |A_rc| / 448; value = s_r * e4m3(code) */
} nsrgs_a_format;

/* Packed upper-block-triangle layout of a symmetric A, selected by
 * nsrgs_matrix.ld == NSRGS_LD_PACKED.  With ndp = n d rounded up to a multiple
 * of 64, row r of block row i = r / d keeps the columns [c0(i), ndp),
 * c0(i) = 64 floor(i d / 64): its part on and above the diagonal block,
 * widened to the left to a multiple of 64 (so every row starts on a 64-element
 * boundary: whole cache lines for the streaming loads, as in the full layout
 * with ld a multiple of 64).  Rows follow one another without gaps: element
 * (r, c), c0(i) <= c < ndp, is at
 *     off(r) + c - c0(i),   off(r) = d sum_{b < i} (ndp - c0(b)) + (r - i d)(ndp - c0(i)),
 * and the whole matrix takes nsrgs_packed_elems(n, d) elements, about
 * (n d)^2 / 2 + n d (d + 64) / 2.  Columns c >= n d are padding (the generator
 * writes zeros there); columns below the diagonal block that the widening
 * keeps hold A(r, c) when the generator writes them and are never used.
 * BF16_SPLIT keeps its low part in data_lo with the same layout. */
#define NSRGS_LD_PACKED (-1)
int64_t nsrgs_packed_elems(int n, int d);   /* 0 for n < 1, d < 1, d > 32 or n d >= 2^31 */

typedef struct {
  int32_t fmt;             /* nsrgs_a_format                                    */
  const void *data;        /* device; n*d rows of ld elements, or packed        */
  const void *data_lo;     /* device; BF16_SPLIT low part (same layout), else NULL */
  const float *row_scale;  /* device; FP8 per-row scales (n*d floats), else NULL */
  int64_t ld;              /* leading dimension in elements, or NSRGS_LD_PACKED */
} nsrgs_matrix;

/* Monitors of the last iteration, filled from device memory by the calls
 * that synchronize (sync_solve, sync_init_spectral, sync_read_info). */
typedef struct {
  int32_t iters;            /* iterations done (solve) / subspace iterations (init) */
  int32_t nonfinite;        /* 1 if a NaN/Inf was seen in the last iterate          */
  int32_t converged;        /* 1 if the tolerance was met                           */
  int32_t status;           /* nsrgs_status of the whole call                       */
  double rel_change;        /* ||X^{t+1}-X^t||_F / ||X^t||_F of the last step       */
  double max_orth_defect;   /* max_i ||I - F_i^T F_i||_F of the last step           */
  double init_residual;     /* init: ||A Y - Y T||_F / ||T||_F of the last iteration */
  double ritz[16];          /* init: top-d Ritz values (descending)                 */
  double ritz_next;         /* reserved (NaN)                                        */
  double objective;         /* F(X^t) of eq. (def:f) at the last evaluation, on the
                               matrix-core path with the objective stop rule (else NaN) */
  double objective_ratio;   /* R^{t-1} = (F(X^{t-1}) - F(X^t)) / F(X^t) (Sec. 4.1),
                               same conditions (NaN before two evaluations)        */
  double ritz_more[16];     /* init with d > 16: Ritz values 17 .. d               */
} nsrgs_info;

/* Retraction of sync_solve (Sec. 4.1 compares the three):
 *   NS_RGS: X_i <- Ts Newton-Schulz steps from F_i (Algorithms 1 and 2);
 *   POLAR : X_i <- sgn(F_i), the exact retraction (the sequence with a tilde
 *           in Sec. 3), F_i as in NS-RGS;
 *   GPM   : X_i <- sgn((A X)_i), the generalized power method, whole block
 *           row including the diagonal block.
 * sgn(M) = U V^T for M = U Sigma V^T (Sec. 2.1) is computed to FP64 accuracy. */
typedef enum { NSRGS_METHOD_NS_RGS = 0, NSRGS_METHOD_POLAR = 1, NSRGS_METHOD_GPM = 2 } nsrgs_method;

/* Stop rule of sync_solve when tol > 0:
 *   REL_CHANGE: after the first iteration with ||X^{t+1}-X^t||_F/||X^t||_F <= tol;
 *   OBJECTIVE : the paper's rule (Sec. 4.1), after the first iteration t with
 *               R^t = (F(X^t) - F(X^{t+1})) / F(X^{t+1}) < tol, returning X^{t+1}.
 *               F (eq. def:f) is evaluated in FP64 from per-block pieces of
 *               the product the step computes anyway, plus X^T X and, once per
 *               solve, sum_{i != j} ||A_ij||_F^2; the evaluation of F(X^{t+1})
 *               happens inside the next iteration, whose own output is then
 *               discarded.  With F32 storage the product's rounding (about
 *               1e-7 of its terms) limits how small a ratio can be resolved. */
typedef enum { NSRGS_STOP_REL_CHANGE = 0, NSRGS_STOP_OBJECTIVE = 1 } nsrgs_stop_rule;

/* Options of sync_solve beyond the arguments named in its signature.
 * Pass NULL for the defaults given in brackets. */
typedef struct {
  int32_t init;             /* 1: run sync_init_spectral into X first [1]           */
  int32_t init_iters;       /* max subspace iterations of the init [60]             */
  double init_tol;          /* init: relative residual tolerance [0: default]      */
  int32_t refine_iters;     /* precision form: final iterations on A_refine [0]     */
  const nsrgs_matrix *A_refine; /* matrix for those iterations (e.g. F32 or
                                   BF16_SPLIT copy of A), or NULL [NULL]          */
  int32_t check_every;      /* iterations enqueued between host checks [16]         */
  int32_t symmetric;        /* 1: every iteration is sync_step_symmetric's (A and
                               A_refine exactly symmetric, full or packed, formats
                               and d as there; ws of
                               sync_step_symmetric_workspace_bytes), and so is the
                               initialization's product W = A Y [0]                */
  int32_t method;           /* nsrgs_method [NS_RGS]; POLAR and GPM need F64 or F32 */
  int32_t stop_rule;        /* nsrgs_stop_rule [REL_CHANGE]; OBJECTIVE needs F64 or
                               F32 storage and no refinement                      */
} nsrgs_solve_opts;

/* ---- status and version ------------------------------------------------ */
const char *nsrgs_status_string(int status);
const char *nsrgs_last_error(void);
int nsrgs_version(void);

/* ---- workspace ----------------------------------------------------------
 * Bytes of device workspace needed by sync_step / sync_solve /
 * sync_init_spectral for one problem of size (n, d) in format fmt (0 on
 * invalid arguments).  sync_workspace_init clears its control words
 * (asynchronously, on `stream`); every later call leaves them cleared. */
size_t sync_workspace_bytes(int n, int d, int fmt);
int sync_workspace_init(void *ws, size_t ws_bytes, void *stream);

/* ---- sync_step: one iteration of Algorithm 2 (paper Sec. 2.2) -------------
 * X_out = NS-RGS update of X_in: for every block i,
 *   C_i = sum_{j != i} A_ij X_in_j, G_i = (n-1) X_in_i - C_i,
 *   F_i = X_in_i - mu (G_i - X_in_i G_i^T X_in_i)/2,
 *   X_out_i = ns_steps Newton-Schulz steps from F_i (Algorithm 1).
 * A is streamed from memory once; C, G and F stay on chip.
 * mu <= 0 selects mu = 1/n (Theorem 3.1).  ns_steps in [0, 64].
 * X_in and X_out are n*d x d device arrays that must not overlap.
 * For d > 16 (F64 / F32 storage) the product runs on the matrix cores
 * (v_mfma 16x16x4 tiles over column chunks, partial sums in the workspace)
 * and the per-block part in FP64; so does d >= 10 with F64 and d >= 13 with
 * F32 storage when ws holds sync_workspace_bytes(n, d, fmt) bytes, where the
 * streaming kernel's 2d FMAs per element of A make it the slower one.  (That
 * product covers whole rows and subtracts A_ii X_i afterwards, so there the
 * diagonal blocks must be finite; the streaming kernel never reads them.)
 * Monitors (rel_change, max_orth_defect, nonfinite) go to the workspace and
 * can be read with sync_read_info.  Asynchronous. */
int sync_step(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps,
              const void *X_in, void *X_out, void *ws, size_t ws_bytes,
              void *stream);

/* ---- the retractions the paper compares (Sec. 4.1) ------------------------
 * sync_step_polar: one step of Algorithm 2 with the exact retraction,
 *   X_out_i = sgn(F_i), F_i = X_in_i - mu (G_i - X_in_i G_i^T X_in_i)/2 as in
 *   sync_step (the sequence with a tilde in Sec. 3).
 * sync_step_gpm: one step of the generalized power method,
 *   X_out_i = sgn(sum_j A_ij X_in_j) over the whole block row (diagonal
 *   block included).
 * sgn(M) = U V^T (Sec. 2.1) is formed to FP64 accuracy by Newton-Schulz from
 * M scaled by the Gershgorin bound of M^T M, iterated to convergence (a
 * singular or non-finite M is reported as non-finite).  Both use the
 * matrix-core product (F64 or F32 storage, 1 <= d <= 32), allocate nothing,
 * take the sync_step workspace and are asynchronous; monitors as sync_step's
 * (for GPM, max_orth_defect is that of the output). */
int sync_step_polar(const nsrgs_matrix *A, int n, int d, double mu, const void *X_in, void *X_out,
                    void *ws, size_t ws_bytes, void *stream);
int sync_step_gpm(const nsrgs_matrix *A, int n, int d, const void *X_in, void *X_out, void *ws,
                  size_t ws_bytes, void *stream);

/* ---- sync_step_noalloc: sync_step without a caller workspace -------------
 * For callers that cannot allocate device memory or pass a workspace: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Computes exactly what sync_step computes (same kernels, same
 * launch shape, bitwise the same X_out), but its scratch -- the control block
 * and one 32-byte monitor record per panel -- is a fixed library-owned array
 * of NSRGS_NOALLOC_SCRATCH_BYTES bytes of device memory, one copy per GPU,
 * held until the process ends.  The call allocates nothing (no hipMalloc, no
 * hipFree, no allocating library routine); on its first use on a device it
 * looks up that device's copy of the array (hipGetSymbolAddress).
 * Limits: the sync_step checks, and at most (NSRGS_NOALLOC_SCRATCH_BYTES -
 * 4352) / 32 panels (panels = ceil(n d / (B d)), B the launch shape's blocks
 * per panel, so n <= 130000 for every shape); a larger problem is refused
 * with NSRGS_ERR_OUT_OF_MEMORY before any device work.
 * The monitors are not readable through sync_read_info (they live in the
 * library's array, not in a caller workspace).
 * Every call on one GPU shares that GPU's array and the array keeps the last
 * call's contents: calls on the same stream are ordered and safe, calls that
 * overlap on one GPU (different streams or threads without ordering) race.
 * Asynchronous, like sync_step. */
#define NSRGS_NOALLOC_SCRATCH_BYTES (4u << 20)
int sync_step_noalloc(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps,
                      const void *X_in, void *X_out, void *stream);

/* ---- sync_step_symmetric: sync_step reading half of A ---------------------
 * The measurement matrix is symmetric, A_ji = A_ij^T (Sec. 2.2), so every
 * product term of the step is available from the blocks above the block
 * diagonal.  This call reads only those blocks and uses each element twice,
 * for C_i += A_ij X_j and for C_j += A_ij^T X_i; the rest of the step is
 * sync_step's.  An iteration therefore streams about half of A.
 * The result equals sync_step's up to the order of the additions, provided
 * the stored A is exactly symmetric.  The generator's output and its BF16 and
 * hi+lo conversions are.
 * Values on and below the block diagonal are never used.  Cache lines
 * near the diagonal may still be loaded, so they must be readable memory;
 * their contents do not matter.  A may be packed (NSRGS_LD_PACKED), which
 * halves its footprint; the result is the same as from the full layout.
 * Formats F64, F32 (1 <= d <= 16), BF16 and BF16_SPLIT (1 <= d <= 12: above
 * that their tiles spill registers and run slower than sync_step, and the
 * call refuses them with NSRGS_ERR_UNSUPPORTED).  FP8_E4M3 is refused with
 * NSRGS_ERR_UNSUPPORTED: its per-row scales make the stored A_ij and A_ji
 * differ.
 * ws must hold sync_step_symmetric_workspace_bytes(n, d, fmt) bytes: the
 * sync_step workspace followed by the per-tile partial sums (sized for every
 * format with fmt's accumulation type, so one workspace serves F32, BF16 and
 * BF16_SPLIT matrices of the same n and d), about
 * (n d)^2 d (1/H + 1/CW) accumulator values, with strip height H of several
 * hundred rows (up to what 64 KiB of LDS holds) and chunk width CW = 256 V.  It is prepared by sync_workspace_init, and
 * sync_read_info reads the monitors as after sync_step.
 * The call returns 0 bytes for unsupported (n, d, fmt).  It is asynchronous. */
size_t sync_step_symmetric_workspace_bytes(int n, int d, int fmt);
int sync_step_symmetric(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps,
                        const void *X_in, void *X_out, void *ws, size_t ws_bytes,
                        void *stream);

/* ---- incomplete observations: block-sparse storage (Sec. 4.1) -------------
 * Each off-diagonal block pair (i, j) is observed with probability p; the
 * blocks that are not observed are zero.  Algorithm 2 is unchanged, with
 * mu = 1/(np).  Only the observed blocks are stored:
 *   row_ptr  n + 1 offsets: block row i holds blocks row_ptr[i] .. row_ptr[i+1]-1;
 *   col_idx  their block columns, ascending, in [0, n) and != i (a stored
 *            diagonal block, or an index outside [0, n), contributes nothing);
 *   values   the blocks of row i in groups of 64: group g = k / 64 holds
 *            w = min(64, m - 64 g) blocks (m = row_ptr[i+1] - row_ptr[i]),
 *            entry-major, so entry (a, b) of the k-th block is at
 *            values[row_ptr[i] d^2 + 64 g d^2 + (a d + b) w + k mod 64]
 *            (one entry of a group's blocks is contiguous, and so is the
 *            whole group).
 * All three are device arrays owned by the caller; fmt is NSRGS_A_F32 or
 * NSRGS_A_BF16 (element type of values).  1 <= d <= 32. */
typedef struct {
  int32_t fmt;
  int32_t reserved;
  const int64_t *row_ptr;
  const int32_t *col_idx;
  const void *values;
} nsrgs_bsr_matrix;

/* Block-sparse inputs on the device for the same model and seed as
 * nsrgs_generate_measurement (same observation mask, same element values).
 * nsrgs_bsr_count writes row_ptr (n + 1 int64 entries) from the mask, using
 * `counts` (n int64 entries of device scratch), and returns the number of
 * stored blocks in *nnzb (host).  It waits for the stream.  The caller then
 * allocates col_idx (nnzb int32) and values (nnzb d^2 elements) and calls
 * nsrgs_bsr_fill, which is asynchronous. */
int nsrgs_bsr_count(const double *Z, int n, int d, double p, uint64_t seed, int64_t *row_ptr,
                    void *counts, int64_t *nnzb, void *stream);
int nsrgs_bsr_fill(const double *Z, int n, int d, double sigma, double p, uint64_t seed,
                   const nsrgs_bsr_matrix *A, void *stream);

/* sync_step on block-sparse A: C_i = sum over stored j != i of A_ij X_j, then
 * the per-block step of sync_step.  X_in / X_out are FP32.  mu <= 0 selects
 * 1/n; for the incomplete observation model pass mu = 1/(np).  1 <= d <= 32.
 * For d <= 6, with ws of sync_step_bsr_workspace_bytes(n, d) bytes the step
 * runs sliced: block columns are cut into slices whose X fits 128 KiB of LDS,
 * each workgroup streams its block rows' blocks of one slice (their X_j read
 * from LDS), and an epilogue adds the slices' partial sums in slice order;
 * for d <= 8 with a smaller ws (at least the sync_step part of
 * sync_workspace_bytes) it runs one fused kernel, one wave per block row,
 * reading X_j through the caches.  Both give the same C_i up to the order of additions.  For d > 8
 * ws must hold sync_workspace_bytes(n, d, NSRGS_A_F32) bytes, and a
 * block-sparse product (chunks of blocks through LDS) is followed by the
 * matrix-core path's per-block epilogue.  Asynchronous. */
/* sync_workspace_bytes(n, d, NSRGS_A_F32) plus, for d <= 6, the sliced
 * product's slice bounds and partial sums after it; serves sync_step_bsr and
 * sync_solve_bsr. */
size_t sync_step_bsr_workspace_bytes(int n, int d);   /* 0 for unsupported (n, d) */
int sync_step_bsr(const nsrgs_bsr_matrix *A, int n, int d, double mu, int ns_steps,
                  const void *X_in, void *X_out, void *ws, size_t ws_bytes, void *stream);

/* Algorithm 2 end to end on block-sparse A (the incomplete observation model
 * of Sec. 4.1): spectral initialization (opts->init, default on) by the
 * subspace iteration of sync_init_spectral with the block-sparse product, then
 * at most max_iters iterations with the stop rule of opts->stop_rule (relative
 * change, or the paper's R^t; F counts the stored blocks, the others being
 * zero) when tol > 0.  opts->method NS_RGS or POLAR; GPM is refused
 * (NSRGS_ERR_UNSUPPORTED): it needs the diagonal blocks, which are not stored.
 * Symmetric steps and refinement are refused too.  The diagonal blocks count
 * as zero, which leaves the iteration unchanged (it never reads them) and
 * shifts the spectrum only by A_ii (= I in the paper's model, so the same
 * eigenvectors).  X: FP32 device n*d x d; ws of sync_workspace_bytes(n, d,
 * NSRGS_A_F32) bytes; 1 <= d <= 32.  With d <= 6 and ws of
 * sync_step_bsr_workspace_bytes(n, d) bytes every product (initialization and
 * iterations) runs on the sliced kernel of sync_step_bsr, its slice bounds
 * found once per call; NS-RGS iterations with the relative-change rule are
 * then sync_step_bsr's steps (its per-block epilogue, FP32), the others add
 * the slices' partial sums in slice order for the matrix-core path's FP64
 * per-block epilogue.  Otherwise, and for the first product of a solve with
 * the R^t rule (which also sums the squares of A), a chunked block-sparse
 * product that serves any d.  Waits for the stream and fills *info (the
 * objective fields only when the R^t rule or the matrix-core epilogue ran). */
int sync_solve_bsr(const nsrgs_bsr_matrix *A, int n, int d, double mu, int ns_steps, int max_iters,
                   double tol, void *X, void *ws, size_t ws_bytes, void *stream,
                   const nsrgs_solve_opts *opts, nsrgs_info *info);

/* Copy the monitors of the last step / init on this workspace to *info
 * (waits for `stream`). */
int sync_read_info(const void *ws, size_t ws_bytes, int n, int d, int fmt,
                   nsrgs_info *info, void *stream);

/* ---- sync_init_spectral: spectral initialization (Alg. 2) -----------------
 * Y = top-d (largest algebraic) eigenvectors of A by block subspace
 * iteration on d columns, Y_{k+1} = (A Y_k) R^{-1} with A Y_k = Q R by
 * Cholesky-QR (Grams reduced and factored in FP64), then X0_i = sgn(Y_i) for
 * every block (Newton-Schulz in FP64 from the Frobenius-scaled block, run to
 * convergence: the exact polar factor).  Stops after the first iteration
 * k >= 1 with ||A Y_k - Y_k T_k||_F <= tol ||T_k||_F, T_k = Y_k^T A Y_k
 * (tol <= 0: 1e-13 for F64 storage, 1e-5 otherwise), or after max_iters
 * iterations (<= 0: 60; returns NSRGS_ERR_NOT_CONVERGED, X0 still written).
 * info->ritz receives the eigenvalues of T_k (FP64 Jacobi), descending.
 * Subspace iteration finds the dominant (largest |lambda|) subspace, which is
 * the top-d one whenever lambda_d > |lambda_min| (true below the spectral
 * threshold of the measurement model).  X0 is an n*d x d device array.
 * A packed A (NSRGS_LD_PACKED) runs the product W = A Y on the symmetric
 * half-stream tiles plus the diagonal blocks; ws must then hold
 * sync_step_symmetric_workspace_bytes(n, d, fmt) bytes.
 * Waits for the stream and fills *info (nullable). */
int sync_init_spectral(const nsrgs_matrix *A, int n, int d, void *X0,
                       int max_iters, double tol, void *ws, size_t ws_bytes,
                       void *stream, nsrgs_info *info);

/* ---- sync_solve: Algorithm 2 end to end -----------------------------------
 * X (device, n*d x d) receives the result; with opts->init == 0 it must hold
 * X^0 on entry.  Runs at most max_iters iterations; tol > 0 stops after the
 * first iteration with ||X^{t+1}-X^t||_F / ||X^t||_F <= tol (tol <= 0 runs
 * exactly max_iters).  With opts->refine_iters = k > 0 and opts->A_refine
 * set, the last k of the max_iters iterations run on A_refine instead of A
 * (after an early stop on A, k more iterations run on A_refine).
 * Waits for the stream and fills *info (nullable).  Returns NSRGS_ERR_NONFINITE
 * if an iterate became non-finite. */
int sync_solve(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps,
               int max_iters, double tol, void *X, void *ws, size_t ws_bytes,
               void *stream, const nsrgs_solve_opts *opts, nsrgs_info *info);

/* ---- NS-RGS on the Stiefel manifold St(p, d)^n -----------------------------
 * The extension of the method to the Stiefel manifold that the paper names
 * as future work (Sec. 6), on St(p, d) = {S in R^{d x p} : S S^T = I_d}, the
 * manifold of the Burer-Monteiro relaxation recalled in Sec. 1 (d <= p).
 * The iterate S (device, n*d x p, row-major, block i rows [i d, (i+1) d)) is
 * double for F64 storage of A, float for F32.  One step of Algorithm 2 with
 * every d x d quantity widened to d x p:
 *     G_i = (n - 1) S_i - sum_{j != i} A_ij S_j
 *     P_i = G_i - sym(G_i S_i^T) S_i,   sym(M) = (M + M^T) / 2
 *     F_i = S_i - mu P_i,   S_i <- Ts steps of S <- (3 S - S S^T S) / 2
 * (mu <= 0: 1/n).  P_i is the orthogonal projection onto the tangent space
 * at S_i; the Newton-Schulz steps tend to the polar factor of F_i.  At p = d
 * and S_i in O(d) this is sync_step's iteration.  A (full layout, F64 or
 * F32) is streamed once per step on the matrix cores; the d x p block
 * arithmetic is FP64.  Limits: 2 <= n, 1 <= d <= p <= 32, n d p < 2^31.
 * ws holds sync_stiefel_workspace_bytes(n, d, p, fmt) bytes (0 when
 * unsupported), 256-byte aligned, prepared by sync_workspace_init; it is
 * also a valid sync_workspace_bytes(n, d, fmt) workspace, so sync_read_info
 * reads the monitors of the last step (relative change, max_i ||I - F_i
 * F_i^T||_F).  sync_step_stiefel is asynchronous.
 * sync_solve_stiefel runs at most max_iters steps from the start held in S
 * (for p > d a random point of St(p, d)^n: the relaxation of Sec. 1) and
 * writes the result to S; tol > 0 stops after the first step with
 * ||S^{t+1} - S^t||_F / ||S^t||_F <= tol.  It waits for the stream and fills
 * *info (nullable; init_residual, ritz and objective are not set).
 * sync_stiefel_round writes X (n*d x d) with X_i = sgn(S_i V), V the p x d
 * matrix of top-d eigenvectors of S^T S (FP64 Jacobi), the rounding of a
 * Stiefel point to O(d)^n; it waits for the stream and returns
 * NSRGS_ERR_NONFINITE if some S_i V is singular or not finite. */
size_t sync_stiefel_workspace_bytes(int n, int d, int p, int fmt);
int sync_step_stiefel(const nsrgs_matrix *A, int n, int d, int p, double mu, int ns_steps,
                      const void *S_in, void *S_out, void *ws, size_t ws_bytes, void *stream);
int sync_solve_stiefel(const nsrgs_matrix *A, int n, int d, int p, double mu, int ns_steps,
                       int max_iters, double tol, void *S, void *ws, size_t ws_bytes,
                       void *stream, nsrgs_info *info);
int sync_stiefel_round(const void *S, int n, int d, int p, int fmt, void *X, void *ws,
                       size_t ws_bytes, void *stream);

/* ---- batched solves: many problems per launch -----------------------------
 * Independent problems of uneven size (n, d) share every launch.  The unit of
 * work is one panel of B d rows of one problem (B fixed per d); the last panel
 * of each problem to finish an iteration updates that problem's iteration
 * count, monitors and stop state on the device.  Two schedules:
 *   grouped (default): one launch runs one iteration of Algorithm 2 for all
 *     still-active problems; the host enqueues the launches back to back and
 *     looks at the state only every opts->check_every launches, so a batch of
 *     512 problems costs max_iters launches, not 512 x max_iters;
 *   persistent (opts->persistent = 1): one launch runs the whole budget;
 *     workgroups take (iteration, unit) tickets in order from a device counter
 *     and wait on the device until the problem has finished the previous
 *     iteration, so a problem's next iteration overlaps the tail of others.
 * Each problem follows exactly the arithmetic of sync_step with the same
 * panel shape, in either schedule.  Every problem of a batch uses one storage
 * format: F64, F32 or BF16, and 1 <= d <= 16.  Problem memory (A, X) is the caller's; the
 * workspace holds the unit table, a second iterate buffer per problem and
 * per-panel monitors.  Waits for the stream. */
typedef struct {
  nsrgs_matrix A;          /* this problem's matrix                               */
  int32_t n, d;
  double mu;               /* <= 0: 1/n                                           */
  void *X;                 /* device n*d x d: X^0 on entry (unless opts->init),
                              the result on return                               */
  int32_t iters;           /* iteration budget (<= 0: max_iters of the call)      */
  double tol;              /* > 0: stop after the first iteration whose relative
                              change ||X^{t+1}-X^t||_F/||X^t||_F is <= tol        */
} nsrgs_problem;

typedef struct {
  int32_t iters, converged, nonfinite, status;
  double rel_change, max_orth_defect;
} nsrgs_problem_info;

typedef struct {
  int32_t waves;           /* waves per workgroup [0: tuned]                      */
  int32_t order;           /* unit order: 0 problem-major, largest first;
                              1 panels of all problems interleaved [0]            */
  int32_t init;            /* 1: spectral initialization of each problem first    */
  int32_t check_every;     /* launches between host looks at the state
                              [0: 8 if some tol > 0, else max_iters]              */
  int32_t persistent;      /* 1: one persistent launch for the whole budget
                              (workgroups take (iteration, unit) tickets in order
                              and wait only on earlier tickets); 0: one grouped
                              launch per iteration [0]                            */
  int32_t wait_polls;      /* persistent: polls per dependency wait before the
                              launch is abandoned with NSRGS_ERR_DEVICE
                              [0: about 2^21, a few seconds]                      */
  int32_t ticket_kb;       /* persistent: panels of a problem are merged into
                              tickets of at least this many KiB of A [0: 512]     */
} nsrgs_batch_opts;

/* Workspace bytes for a batch (with_init: include the initialization's). */
size_t sync_batch_workspace_bytes(const nsrgs_problem *probs, int count, int with_init);
int sync_solve_batched(const nsrgs_problem *probs, int count, int ns_steps, int max_iters,
                       void *ws, size_t ws_bytes, void *stream,
                       const nsrgs_batch_opts *opts /* nullable */,
                       nsrgs_problem_info *infos /* host, count entries, nullable */);

/* ---- serving: a request loop with continuous batching --------------------
 * A server owns a device memory pool (one allocation at creation), a
 * scheduler thread and ingest worker threads.  Requests describe a synthetic
 * measurement problem (n, d <= 16, sigma, seed, ground truth Z on the host);
 * they are admitted in arrival order when their footprint (A in the server's
 * storage format, two iterates, monitors, and transient ingest buffers) fits
 * the pool and a solve slot is free (a request that does not fit yet does
 * not block later, smaller ones).  On admission an ingest worker generates
 * A on the device (nsrgs_generate_measurement's element rule, in FP32 row
 * chunks converted to the storage format) and runs sync_init_spectral on the
 * worker's own stream.  The scheduler thread runs ticks of `iters_per_tick` grouped
 * launches over all ready requests (sync_solve_batched's kernel), each
 * request at its own iteration count, stopping a request at relative change
 * <= tol or after max_iters iterations; finished requests copy their result to
 * X_out, free their memory and post an nsrgs_result.  A request's result does
 * not depend on what else is being served.  All calls are thread-safe. */
typedef struct nsrgs_server nsrgs_server;

typedef struct {
  int32_t fmt;              /* NSRGS_A_BF16 or NSRGS_A_F32 (must be set when opts
                               is given; NULL opts: BF16)                         */
  int32_t max_active;       /* solve slots [0: 64]                                */
  int32_t iters_per_tick;   /* grouped launches per scheduler tick [0: 4]         */
  int32_t ns_steps;         /* Newton-Schulz steps [0: 3]                          */
  int32_t waves;            /* waves per workgroup [0: tuned]                      */
  int32_t ingest_workers;   /* threads (one stream each) preparing requests [0: 4] */
  uint64_t pool_bytes;      /* device memory for requests [0: half of free]       */
} nsrgs_server_opts;

typedef struct {
  int32_t n, d;
  double sigma;
  uint64_t seed;            /* generator seed of W                                 */
  const double *Z;          /* host n*d x d ground truth, copied at submit         */
  double tol;               /* relative-change stop [<= 0: 1e-6]                   */
  int32_t max_iters;        /* [<= 0: 300]                                         */
  float *X_out;             /* host n*d x d result buffer (nullable); must stay
                               valid until the request's result is posted         */
} nsrgs_request;

typedef struct {
  int64_t id;
  int32_t status, iters, converged, pad;
  double t_submit, t_admit, t_start, t_done;   /* seconds on the server clock */
  double rel_change;
} nsrgs_result;

typedef struct {
  int64_t submitted, completed, rejected;
  int32_t active, max_active_seen;
  double p50_latency_s, p99_latency_s, mean_latency_s;   /* submit -> result */
  double solves_per_s;     /* completed / (last result - first submit)        */
  uint64_t pool_bytes, pool_peak_bytes;
} nsrgs_server_stats;

int nsrgs_server_create(const nsrgs_server_opts *opts /* nullable */, nsrgs_server **out);
/* Queue a request; *id (nullable) receives its id.  A request larger than the
 * whole pool is accepted and immediately posted with NSRGS_ERR_OUT_OF_MEMORY. */
int nsrgs_server_submit(nsrgs_server *server, const nsrgs_request *req, int64_t *id);
/* Up to max posted results, oldest first; *count receives how many. */
int nsrgs_server_poll(nsrgs_server *server, nsrgs_result *results, int max, int *count);
/* Wait until nothing is queued, ingesting or iterating (timeout_s <= 0: no
 * limit; NSRGS_ERR_NOT_CONVERGED on timeout). */
int nsrgs_server_wait_idle(nsrgs_server *server, double timeout_s);
int nsrgs_server_get_stats(nsrgs_server *server, nsrgs_server_stats *stats);
double nsrgs_server_clock(const nsrgs_server *server);   /* seconds since creation */
/* Stop the threads; requests not finished are posted as NOT_CONVERGED and the
 * pool is freed. */
int nsrgs_server_destroy(nsrgs_server *server);

/* ---- tuning table ---------------------------------------------------------
 * Launch shapes measured by the autotuner.  kind 0: the single-problem step
 * (blocks_per_panel B: the workgroup's panel is B d rows; unroll U: 0 = one
 * 16-byte column vector per row per loop iteration with the next iteration's
 * loads issued before this one's arithmetic, U >= 1 = U vectors per row
 * loaded together; waves W splitting the columns, at most 4 with U = 0) for
 * storage format fmt,
 * block size d and n*d in [nd_min, nd_max]; an entry whose (B, U) is not
 * compiled for d is ignored.  kind 1: waves per workgroup of the
 * grouped batched launch for format fmt and batches whose largest d is <= d.
 * The first matching entry wins; entries replace the whole table (count 0
 * clears it).  Not thread-safe against concurrent launches. */
typedef struct {
  int32_t kind, fmt, d;
  int32_t nd_min, nd_max;
  int32_t blocks_per_panel, unroll, waves;
} nsrgs_tune_entry;
int nsrgs_set_tuning(const nsrgs_tune_entry *entries, int count);
int nsrgs_get_tuning(nsrgs_tune_entry *entries, int max_count);
/* The (blocks_per_panel, unroll) shapes of the step kernel compiled for block
 * size d (the choices a kind-0 tuning entry may name).  Writes up to max_count
 * pairs into the two caller-owned arrays (either may be NULL when max_count is
 * 0) and returns the number of shapes for d (0 for a d outside 1..16), or -1
 * (message in nsrgs_last_error) when max_count > 0 and an array is NULL. */
int nsrgs_step_variants(int d, int32_t *blocks_per_panel, int32_t *unroll, int max_count);

/* ---- autotuner ------------------------------------------------------------
 * Measure launch shapes on the caller's own problem (device memory and
 * workspace as for the call being tuned) and return them fastest first in
 * results[0 .. min(*count, max_results)); *count receives the number measured.
 * Nothing is installed: pass the winners to nsrgs_set_tuning (or the batch
 * options).  Both wait for the stream.
 *
 * nsrgs_autotune_step: every compiled (blocks_per_panel, unroll) shape of d
 *   and waves in {1, 2, 4, 8} (at most 4 for unroll = 0, the software-pipelined
 *   shapes, which launch with at most 4 waves per workgroup whatever the
 *   table or NSRGS_STEP_W asks); reps timed sync_step launches each (HIP events,
 *   after one untimed launch), T_s = 3, mu = 1/n.  X_out is overwritten.
 * nsrgs_autotune_batched: the grouped and persistent schedules, unit orders 0
 *   and 1, waves in {1, 2, 4}, persistent tickets of 128 / 512 / 2048 KiB;
 *   each candidate runs `iters` iterations of every problem (tolerances are
 *   ignored so every candidate does the same work), wall time per iteration.
 *   The problems' X are iterated on (overwritten); pass copies. */
typedef struct {
  int32_t blocks_per_panel, unroll, waves;   /* step shape (waves also batched) */
  int32_t persistent, order, ticket_kb;      /* batched schedule                */
  double ms;                                 /* time per iteration             */
} nsrgs_tune_result;
int nsrgs_autotune_step(const nsrgs_matrix *A, int n, int d, const void *X_in, void *X_out,
                        void *ws, size_t ws_bytes, void *stream, int reps,
                        nsrgs_tune_result *results, int max_results, int *count);
int nsrgs_autotune_batched(const nsrgs_problem *probs, int count, int ns_steps, int iters,
                           void *ws, size_t ws_bytes, void *stream,
                           nsrgs_tune_result *results, int max_results, int *n_results);

/* ---- inputs: measurement generator and format conversion ----------------
 * nsrgs_generate_measurement writes A = Z Z^T + sigma W in F64 or F32
 * (fmt), element (r, c) computed in double and rounded once, where
 * W(r, c) = W(c, r) = sqrt(-2 ln u1) cos(2 pi u2) with u1, u2 53-bit uniforms
 * from Philox4x32-10 (Salmon et al., SC'11) at counter
 * (max(r,c), min(r,c), 0, 0) and key (seed mod 2^32, seed >> 32).
 * zero_diag_blocks != 0 sets W_ii = 0 (paper's model, A_ii = I).  p < 1 keeps
 * an off-diagonal block pair with probability p (counter (j, i, 1, 0) for
 * blocks i < j, uniform from the first output word), else A_ij = A_ji = 0.
 * Z is an n*d x d double device array; 1 <= d <= 32.  ld == NSRGS_LD_PACKED
 * writes the packed layout (nsrgs_packed_elems(n, d) elements at A, padding
 * columns zero).  Asynchronous. */
int nsrgs_generate_measurement(const double *Z, int n, int d, double sigma,
                               uint64_t seed, int zero_diag_blocks, double p,
                               int fmt, void *A, int64_t ld, void *stream);

/* Convert an FP32 matrix (nd x nd, leading dimension ld) into `out` of format
 * out->fmt (BF16, BF16_SPLIT or FP8_E4M3, same ld); out's pointers name the
 * destination buffers (data, data_lo, row_scale).  Round to nearest even;
 * e4m3 saturates to +-448.  Asynchronous. */
int nsrgs_convert(const float *A32, int nd, int64_t ld, const nsrgs_matrix *out,
                  void *stream);

/* The same conversion for a packed FP32 matrix of n blocks of size d
 * (NSRGS_LD_PACKED layout, nsrgs_packed_elems(n, d) elements) into a packed
 * `out` (out->ld == NSRGS_LD_PACKED) of format BF16 or BF16_SPLIT.  FP8_E4M3
 * is refused with NSRGS_ERR_UNSUPPORTED: packed storage serves the symmetric
 * step, which does not read FP8.  Asynchronous. */
int nsrgs_convert_packed(const float *A32, int n, int d, const nsrgs_matrix *out,
                         void *stream);

#ifdef __cplusplus
}
#endif

#endif /* NSRGS_H */
