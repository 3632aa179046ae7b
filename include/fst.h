/*
 * fst.h — C ABI of the MI355X (gfx950) randomized functional sparse Tucker library.
 *
 * Method: Rai, Kolla, Cannada, Gorodetsky, "Randomized functional sparse Tucker tensor for
 * compression and fast visualization of scientific data" (arXiv 1907.05884).
 *
 *   model   u~(y) = sum_{j1,j2,j3} alpha_{j1 j2 j3} w1_{j1}(y1) w2_{j2}(y2) w3_{j3}(y3)   eq. (1)
 *   factors w^(k)_j(y) = sum_i C_k[i, j] phi_i(xi_k(y)),  few non-zero C_k[i, j]          eq. (2)
 *   basis   phi_i(t) = sqrt(2i+1) P_i(t), i = 0..p_k (orthonormal Legendre, Sec. 4.2)
 *   coords  xi_k = 2 (y_k - lo_k) / (hi_k - lo_k) - 1
 *   core    flattened in C order: j = (j1 r2 + j2) r3 + j3 (the paper only says "reshaped")
 *   refit   alpha^ = argmin ||v_S - A alpha||^2 over M uniformly sampled rows S, eq. (6) and
 *           Algorithm 2; A[q, j] = prod_k w^(k)_{j_k}(y^q_k); solved through the normal
 *           equations G = A^T A, h = A^T v_S with an FP64 Cholesky factorisation.
 *
 * Conventions for every call:
 *  - Return value: FST_OK (0) or a negative status; the message of the last failure on the
 *    calling thread is returned by fst_last_error().  No C++ exception crosses the ABI.
 *  - Points are structure-of-arrays: three arrays x, y, z of n coordinates plus n values.
 *    "device" arrays live in memory of the current HIP device (hipMalloc or torch tensors);
 *    "host" arrays are ordinary CPU memory.  Every pointer argument says which it is.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Calls marked
 *    "asynchronous" only enqueue work on it; the others synchronise it before returning.
 *  - The caller owns every buffer it passes.  The library owns fst_model objects (freed by
 *    fst_model_free) and the small device copy of a model that it uploads on first use.
 *  - Output is bitwise reproducible for identical inputs on the same device: reductions run
 *    in a fixed order and use no floating-point atomics.
 *  - Limits of this version: d = 3 (d = 3 or 4 through the d-way calls), 1 <= r_k <= 32,
 *    0 <= p_k <= 31, n < 2^31 points.
 */
#ifndef FST_H
#define FST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fst_status;
#define FST_OK             0
#define FST_E_INVAL       (-1)   /* bad argument: shape, range, NaN/Inf input, null pointer */
#define FST_E_NOMEM       (-2)   /* host or device allocation failed, or workspace too small */
#define FST_E_DEVICE      (-3)   /* a HIP runtime call or kernel launch failed */
#define FST_E_NOT_SPD     (-4)   /* Cholesky breakdown: the sampled Gram is not positive definite */
#define FST_E_UNSUPPORTED (-5)   /* outside the limits of this version */
#define FST_E_FORMAT      (-6)   /* malformed or truncated serialised model */

/* element type of points, values and evaluation arithmetic */
#define FST_F64 0
#define FST_F32 1

/* precision of the Gram contraction A^T A (the Cholesky and its solves are always FP64) */
#define FST_GRAM_F64  0   /* FP64 rows, FP64 MFMA */
#define FST_GRAM_F32  1   /* FP32 rows, FP32 MFMA, FP32 partial sums folded into FP64 */
#define FST_GRAM_BF16 2   /* BF16 rows, BF16 MFMA, FP32 accumulation folded into FP64 */
#define FST_GRAM_F16  3   /* FP16 rows (scaled), FP16 MFMA, FP32 accumulation folded into FP64 */
#define FST_GRAM_F16X2  4 /* FP16 rows split in two terms (hi + lo, scaled): four FP16 MFMA
                              products per entry pair, FP32 sums folded into FP64 */
#define FST_GRAM_BF16X3 5 /* BF16 rows split in three terms: six BF16 MFMA products per entry
                              pair, FP32 sums folded into FP64 */
#define FST_GRAM_BF16X2 6 /* BF16 rows split in two terms: four BF16 MFMA products per entry
                              pair, FP32 sums folded into FP64 */

/* random streams: state = seed * 256 + stream (SplitMix64) */
/* sparse solver of the singular-vector fits (Sec. 3, 4.2), both with leave-one-out selection */
#define FST_SOLVER_OMP  0   /* orthogonal matching pursuit */
#define FST_SOLVER_LARS 1   /* Lasso-modified least angle regression (the paper's solver) */

#define FST_STREAM_INTERP 1
#define FST_STREAM_LS     2

typedef struct fst_model fst_model;   /* opaque; library-owned */

/* Parameters of Algorithm 1 + Algorithm 2.  Set struct_size = sizeof(fst_fit_params). */
typedef struct {
  uint32_t struct_size;
  int32_t  dtype;            /* FST_F64 | FST_F32: type of the point/value arrays */
  double   lo[3], hi[3];     /* box mapped onto [-1,1]^3 */
  int32_t  grid[3];          /* I_k: equispaced interpolation grid incl. end points (Sec. 4.1) */
  int32_t  rank[3];          /* r_k: fixed Tucker ranks, r_k <= I_k and r_k <= r_l r_m */
  int32_t  degree[3];        /* p_k: Legendre degree per mode, p_k < I_k - 1 */
  double   interp_fraction;  /* share of the points interpolated onto the grid (paper: ~10%) */
  int32_t  idw_k;            /* neighbours of the inverse-distance interpolation (8) */
  double   idw_power;        /* distance power (2) */
  int64_t  n_samples;        /* M rows of Algorithm 2; r1 r2 r3 < M <= n */
  uint64_t seed;             /* method randomness (interpolation subset, sampled rows) */
  int32_t  gram_prec;        /* FST_GRAM_* */
  int32_t  refine_steps;     /* FP64-residual iterative-refinement steps after the solve */
  int32_t  n_threads;        /* host threads for the host steps; 0 = all hardware threads */
  double   eps;              /* > 0: ST-HOSVD ranks chosen from this compression precision
                                (Sec. 4.1, Table 1; fst_sthosvd_eps), with rank[] as caps;
                                0: the fixed ranks rank[] */
  int32_t  sparse_solver;    /* FST_SOLVER_OMP (default) or FST_SOLVER_LARS (Sec. 3, 4.2) */
  int32_t  wavelet_level;    /* s > 0: every singular vector is also fitted in the wavelet space
                                W_{s,q} and keeps the fit with the smaller leave-one-out error
                                (Sec. 4.2, Algorithm 1); 0: Legendre only */
  int32_t  wavelet_degree;   /* q of W_{s,q}: 0 <= q <= min(p_k, 7), (q + 1)(2^s - 1) <= 128 */
} fst_fit_params;

/* ------------------------------------------------------------------ library */

/* Message of the last failed call on this thread ("" if none).  Valid until the next call. */
const char* fst_last_error(void);
/* Version string of the library. */
const char* fst_version(void);
/* Fills defaults (idw_k 8, power 2, fraction 0.1, grid 32^3, ranks 8^3, degree 15, ...). */
void fst_fit_params_default(fst_fit_params* p);

/* ------------------------------------------------------------------ whole method */

/* Device workspace (bytes) that fst_fit / fst_refit_core need for n points. */
size_t fst_fit_workspace_bytes(const fst_fit_params* p, int64_t n);

/* Algorithm 1 then Algorithm 2 (Sec. 4-5).  x, y, z, v: device arrays of n elements of
 * p->dtype.  Host steps (subset draw, inverse-distance interpolation, ST-HOSVD, sparse
 * Legendre fit by OMP + leave-one-out) run on host threads; the refit (factor evaluation at
 * the sampled rows, Gram, Cholesky, solve, refinement) runs on the GPU.  ws: device
 * workspace of ws_bytes >= fst_fit_workspace_bytes(p, n), or NULL to let the library
 * allocate and free it.  Synchronises `stream`.  *out receives a new model. */
fst_status fst_fit(const fst_fit_params* p, int64_t n, const void* x, const void* y,
                   const void* z, const void* v, void* ws, size_t ws_bytes, void* stream,
                   fst_model** out);

/* Algorithm 1 only (Sec. 4): host arrays x, y, z, v (p->dtype, n elements).  The model's
 * core is the ST-HOSVD core of the interpolated grid tensor.  Host only, no GPU use. */
fst_status fst_compress_host(const fst_fit_params* p, int64_t n, const void* x, const void* y,
                             const void* z, const void* v, fst_model** out);

/* Algorithm 2 with its randomised mixing (steps 2-4): the design matrix W of all n points
 * and the values u are multiplied by random signs D (SplitMix64 stream 5 of `seed`: row i is
 * negated when the top bit of output i is set) and mixed by the normalised Walsh-Hadamard
 * transform F = H_N / sqrt(N) (Sylvester order; the real orthogonal stand-in for the FFT of
 * the paper), N the smallest power of two >= max(n, 4096), rows n .. N-1 zero; n_samples rows
 * of [0, N) are drawn uniformly without replacement (stream FST_STREAM_LS) and the core solves
 * the normal equations of those rows of F D W, F D u by an FP64 Cholesky factorisation.  Rows
 * and Gram are formed in the point dtype (FP32: FP32 MFMA with FP64 folding; FP64: FP64
 * MFMA); no refinement (the mixed rows are not regenerated in FP64).  x, y, z, v: device
 * arrays of n <= 2^23 points.  ws: device workspace >= fst_refit_core_mixed_workspace_bytes,
 * or NULL.  Synchronises `stream`; *out receives a new model (FST_E_NOT_SPD if the sampled
 * Gram is not positive definite). */
size_t fst_refit_core_mixed_workspace_bytes(const fst_model* m, int32_t dtype, int64_t n,
                                            int64_t n_samples);
fst_status fst_refit_core_mixed(const fst_model* m, int32_t dtype, int64_t n, const void* x,
                                const void* y, const void* z, const void* v, int64_t n_samples,
                                uint64_t seed, void* ws, size_t ws_bytes, void* stream,
                                fst_model** out);

/* The S sampled rows of the mixed problem of Algorithm 2 (steps 2-4: sign flips D, the
 * normalised Walsh-Hadamard transform over N = max(4096, 2^ceil(log2 n)) rows, S rows drawn
 * uniformly without replacement with stream FST_STREAM_LS of `seed`) for diagnostics such as
 * leverage scores (Sec. 5, Sec. 6 Fig. 4): At (device, dtype, R x Sp with Sp = S rounded up to
 * 64; row j holds design column j of the sampled mixed rows, zero past S) and b (device,
 * dtype, Sp; may be NULL): the mixed values.  S = N keeps every mixed row.  Same inputs and
 * workspace as fst_refit_core_mixed (fst_refit_core_mixed_workspace_bytes).  Asynchronous. */
fst_status fst_mixed_rows(const fst_model* m, int32_t dtype, int64_t n, const void* x,
                          const void* y, const void* z, const void* v, int64_t n_samples,
                          uint64_t seed, void* At, void* b, void* ws, size_t ws_bytes,
                          void* stream);

/* Leverage scores of rows (Sec. 5: the squared row norms of the left singular vectors of a
 * full-column-rank design, equal to l_q = a_q^T (A^T A)^-1 a_q): out[q] = ||y||^2 with L y = a_q
 * for the rows q < mrows of At (device FP64, R x Sp, row j = design column j), L from
 * fst_cholesky of A^T A (device FP64 R x R; columns it skipped count zero).  1 <= R <= 8192,
 * mrows <= Sp.  out: device FP64 mrows.  Asynchronous. */
fst_status fst_leverage(int64_t R, int64_t Sp, int64_t mrows, const double* At,
                        const double* L, double* out, void* stream);

/* Device workspace (bytes) of fst_refit_core for a model, point dtype, M and refinement. */
size_t fst_refit_workspace_bytes(const fst_model* m, int32_t dtype, int64_t n_samples,
                                 int32_t refine_steps);

/* Algorithm 2 (Sec. 5) for a given model's factor functions: re-estimates the core from
 * M = n_samples uniformly sampled rows (stream FST_STREAM_LS of `seed`).  x, y, z, v:
 * device arrays of `dtype`.  ws: device workspace >= fst_refit_workspace_bytes(...), or
 * NULL to let the library allocate it: then it also allocates the room of the dense Gram
 * route (fst_gram_dense_workspace_bytes or fst_gram_split_workspace_bytes beyond the
 * minimum) when the device has that much free memory plus 2 GiB.  The split precisions
 * (FST_GRAM_F16X2, BF16X3, BF16X2) need that room; without it the FP32 Gram is formed.  Writes the new
 * core into *out (a new model with m's factors).  Synchronises `stream`. */
fst_status fst_refit_core(const fst_model* m, int32_t dtype, int64_t n, const void* x,
                          const void* y, const void* z, const void* v, int64_t n_samples,
                          uint64_t seed, int32_t gram_prec, int32_t refine_steps, void* ws,
                          size_t ws_bytes, void* stream, fst_model** out);

/* Reconstruction at points of interest (eq. (1), Sec. 6): out[i] = u~(x[i], y[i], z[i]).
 * x, y, z, out: device arrays of n elements of `dtype`.  Asynchronous on `stream`. */
fst_status fst_eval(const fst_model* m, int32_t dtype, int64_t n, const void* x,
                    const void* y, const void* z, void* out, void* stream);

/* Preview on a tensor grid (Sec. 6, fast visualisation): out[(i1 n2 + i2) n3 + i3] =
 * f(gx[i1], gy[i2], gz[i3]) with f the model of eq. (1), formed as the mode products
 * alpha x_1 U1 x_2 U2 x_3 U3 of the core with the factor functions (eq. (2)) evaluated once
 * per grid line, at 2 r1 flop per grid point instead of 2 R.  A 2-D slice is a grid with one
 * count equal to 1.  gx, gy, gz: device coordinate arrays of `dtype` (FST_F32 or FST_F64) of
 * lengths n1, n2, n3 >= 1 (any order, any spacing); out: device array of `dtype` with
 * n1 n2 n3 entries, C order (i3 fastest), owned by the caller.  Intermediates and output
 * are computed in `dtype`.  ws: device workspace >= fst_eval_grid_workspace_bytes (NULL: the
 * library allocates and synchronises `stream` before freeing it); otherwise asynchronous.
 * FST_E_INVAL for a count below 1 or above 2^31 - 1; FST_E_UNSUPPORTED for more than
 * 65535 x 32 grid lines along one axis. */
size_t fst_eval_grid_workspace_bytes(const fst_model* m, int32_t dtype, int64_t n1, int64_t n2,
                                     int64_t n3);
fst_status fst_eval_grid(const fst_model* m, int32_t dtype, const void* gx, int64_t n1,
                         const void* gy, int64_t n2, const void* gz, int64_t n3, void* out,
                         void* ws, size_t ws_bytes, void* stream);

/* Data error of the reconstruction (the scattered analogue of the precision of Sec. 4.1):
 * sums_out (host double[2]) receives sum_i (v_i - f(x_i))^2 and sum_i v_i^2, accumulated in
 * FP64 in a fixed order, so ||v - f|| / ||v|| = sqrt(sums_out[0] / sums_out[1]).  v: device
 * values of the points' dtype.  ws: device workspace >= fst_eval_error_workspace_bytes
 * (NULL: the library allocates).  Synchronises `stream`. */
size_t fst_eval_error_workspace_bytes(int32_t dtype, int64_t n);
fst_status fst_eval_error(const fst_model* m, int32_t dtype, int64_t n, const void* x,
                          const void* y, const void* z, const void* v, void* ws,
                          size_t ws_bytes, void* stream, double* sums_out);

/* ------------------------------------------------------------------ per-step GPU calls */

/* Rows of Algorithm 2 step 1 at sampled points, eq. (2): for q < m and i = idx[q] (or i = q
 * if idx is NULL), U[(o_k + j) * m + q] = w^(k)_j(point i), o_1 = 0, o_2 = r1, o_3 = r1 + r2
 * (feature-major, points contiguous), and vs[q] = v[i] (vs, v may be NULL).  x, y, z, v, idx,
 * U, vs: device arrays; idx int32.  Asynchronous. */
fst_status fst_factor_eval(const fst_model* m, int32_t dtype, int64_t n, const void* x,
                           const void* y, const void* z, const void* v, const int32_t* idx,
                           int64_t mrows, void* U, void* vs, void* stream);

/* Normal equations of the sampled problem (Algorithm 2 step 5, eq. (6)):
 * G = A^T A (lower triangle incl. diagonal written; strictly upper part untouched) and
 * h = A^T vs, with A[q, j] = U1[q, j1] U2[q, j2] U3[q, j3] formed on the fly from U as
 * written by fst_factor_eval (stored only by the dense route below, in the workspace).  U, vs: device, `dtype` (FST_F64 needs
 * gram_prec FST_GRAM_F64; FST_F32 takes F32, BF16, F16 or a split precision).  G: device FP64 R x R
 * row-major, h: device FP64 R; either may be NULL to skip that product (not both).  ws: device workspace >= fst_gram_workspace_bytes.
 * Asynchronous. */
size_t fst_gram_workspace_bytes(const fst_model* m, int64_t mrows);
/* Workspace that lets fst_gram form G by its dense route: with FST_GRAM_F32 or FST_GRAM_F64 and
 * a workspace above fst_gram_workspace_bytes that holds at least 4096 rows of A^T (R x rows
 * of the row dtype), the design rows are written transposed into it, as many rows at a time
 * as fit (all of them with this size: R x M x 4 bytes for FP32, 11 GB at R = 13,824,
 * M = 200,000), and G is formed from them by a dense MFMA Gram (FP32 partial sums folded into
 * FP64 every 64 rows, as in the other route).  With FST_GRAM_BF16 or FST_GRAM_F16 and room for
 * all rows in 16 bits (R x (M rounded up to 128) x 2 bytes beyond the partials; this size
 * holds them) the rows are written in BF16 or scaled FP16 and G formed by a dense 16-bit MFMA
 * Gram, equal bit for bit to the other route's.  Otherwise G is formed from U directly.
 * fst_refit_core and fst_fit take the same route when their workspace exceeds
 * fst_refit_workspace_bytes (fst_fit_workspace_bytes) by this much. */
size_t fst_gram_dense_workspace_bytes(const fst_model* m, int32_t dtype, int64_t mrows);
/* Workspace for fst_gram with a split precision (FST_GRAM_F16X2, FST_GRAM_BF16X3,
 * FST_GRAM_BF16X2; FP32 factor values): beyond the A^T v partials, the design rows in 2 or 3
 * planes of 16-bit terms, each R x (M rounded up to 64) x 2 bytes (11.1 GB for two terms,
 * 16.6 GB for three at R = 13,824, M = 200,000).  Entry e of A (formed in FP32) is split as
 * t0 = rnd(e), t1 = rnd(e - t0), t2 = rnd(e - t0 - t1) (FP16: e scaled by a power of two that
 * keeps it below 2^15).
 * G = sum of t_a^T t_b over all a, b for two terms (4 products: the exact Gram of the
 * two-term representation, 22 significant bits for FP16, 16 for BF16) and over a + b <= 2
 * for three BF16 terms (6 products, 24 bits); on 16-bit MFMA with FP32 sums folded into FP64
 * every 512 rows.  fst_gram fails with FST_E_NOMEM when a split precision gets less
 * workspace; fst_refit_core and fst_fit form the FP32 Gram instead (reported by
 * fst_model_fit_info).  Returns 0 for a non-split precision or bad arguments. */
size_t fst_gram_split_workspace_bytes(const fst_model* m, int32_t gram_prec, int64_t mrows);
fst_status fst_gram(const fst_model* m, int32_t dtype, int64_t mrows, const void* U,
                    const void* vs, int32_t gram_prec, double* G, double* h, void* ws,
                    size_t ws_bytes, void* stream);

/* The two steps of the dense route as separate calls, for callers that keep the design rows.
 * fst_design_rows: the design matrix of Algorithm 2 step 5 (eq. (6)) written transposed,
 * At[j * Sp + q] = A[q, j] for design column j (C order of the core, j = ((j1 r2 + j2) r3 + j3)
 * [r4 + j4]) and row q < mrows, zero for mrows <= q < Sp, and b[q] = vs[q] (zero past mrows;
 * b and vs may be NULL).  A 3-way or 4-way model; U in the layout fst_factor_eval writes
 * for mrows rows (for a 4-way model mode 4 follows at o_4 = r1 + r2 + r3).  Sp: a multiple
 * of 64, >= mrows >= 1.  U, vs, At, b: device, `dtype` (FST_F32 or FST_F64); At holds R x Sp
 * entries.
 * fst_gram_rows: G = At At^T (lower triangle incl. diagonal, FP64; strictly upper part
 * untouched) by dense MFMA tiles of 128 x 128 (FP32 products accumulated in FP32 over 64
 * rows, then folded into FP64; FP64 products in FP64), and h = At b in FP64 with a fixed order; G or
 * h may be NULL to skip that product.  accumulate != 0 adds to G and h (the sum over chunks of
 * rows), 0 overwrites them.  Sp: a positive multiple of 64, R x Sp < 2^40.
 * Both asynchronous; FST_E_INVAL for a bad size or a missing array. */
fst_status fst_design_rows(const fst_model* m, int32_t dtype, int64_t mrows, const void* U,
                           const void* vs, int64_t Sp, void* At, void* b, void* stream);
fst_status fst_gram_rows(int32_t dtype, int64_t R, int64_t Sp, const void* At, const void* b,
                         double* G, double* h, int32_t accumulate, void* stream);

/* In-place FP64 Cholesky G + shift diag(G) = L L^T of a device R x R row-major matrix
 * (lower triangle read, L written there; the strictly upper triangle of each 64 x 64
 * diagonal block receives the transposed strictly lower triangle of that block's inverse,
 * used by fst_cholesky_solve; the rest of the strictly upper triangle is untouched).
 * shift in [0, 1): relative diagonal shift, 0 for none (the fits use none).
 * Synchronises `stream`; returns FST_E_NOT_SPD if a pivot is not above R * 2^-52 times its
 * diagonal entry before the factorisation (numerically rank-deficient system), with its
 * index in *info (1-based; 0 on success; info may be NULL).
 * ws: device workspace >= fst_cholesky_workspace_bytes(R). */
size_t fst_cholesky_workspace_bytes(int64_t R);
fst_status fst_cholesky(int64_t R, double* G, double shift, int64_t* info, void* ws,
                        size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): fst_cholesky with its scratch (breakdown
 * flags and the original diagonal, 256 + 8 R bytes) in a file-scope device array of the
 * library instead of a caller workspace.  Same arguments, results and errors as
 * fst_cholesky; no hipMalloc, hipFree or other allocating call.  Limit:
 * R <= FST_CHOLESKY_NOALLOC_MAX_R (larger R: FST_E_INVAL, nothing launched); the array takes
 * 256 + 8 * 65,536 bytes (512.25 KiB) on every GPU the library runs on, until the process
 * ends.  All calls on one GPU share that GPU's array, which keeps the last call's contents
 * (the flags are cleared by a kernel at the start of every call): calls that overlap on one
 * GPU (several streams or host threads) race and must be serialised by the caller. */
#define FST_CHOLESKY_NOALLOC_MAX_R 65536
fst_status fst_cholesky_noalloc(int64_t R, double* G, double shift, int64_t* info, void* stream);

/* Algorithm 2 step 5 from given normal equations: the FP64 Cholesky of G, the solve for the
 * core, and refine_steps FP64-residual refinement steps on the sampled rows, with the
 * precision ladder of fst_model_fit_info (a Gram that breaks down or stalls above 1e-8 is
 * formed again from FP32 rows, then FP64 rows, then with dependent columns skipped; a split
 * Gram is first factored again with dependent columns skipped).  The calls fst_refit_core
 * makes after its Gram, for callers that form the Gram themselves.
 * x, y, z, v: device points and values (dtype, n); idx: device int32 mrows sampled row
 * indices in [0, n) (as fst_sample_indices draws them; not checked on the device); U, vs: their factor values and values as
 * fst_factor_eval writes them (read when the ladder forms the Gram again); gram_prec: the
 * precision G was formed at.  G: device FP64 R x R, on entry the lower triangle of A^T A,
 * on return the Cholesky factor (fst_cholesky layout) of the Gram actually used; h: device
 * FP64 R, A^T v on entry (formed again from FP64 rows when the ladder reaches them); alpha:
 * device FP64 R, the core (C order).  gram_prec_used, dropped, steps_kept, rel_residual: as
 * fst_model_fit_info; any may be NULL.  ws >= fst_solve_core_workspace_bytes(m, mrows,
 * gram_prec) (FST_E_NOMEM below).  r1 r2 r3 < mrows <= n; 0 <= refine_steps <= 100.
 * Synchronises `stream`. */
size_t fst_solve_core_workspace_bytes(const fst_model* m, int64_t mrows, int32_t gram_prec);
fst_status fst_solve_core(const fst_model* m, int32_t dtype, int64_t n, const void* x,
                          const void* y, const void* z, const void* v, const int32_t* idx,
                          int64_t mrows, const void* U, const void* vs, int32_t gram_prec,
                          int32_t refine_steps, double* G, double* h, double* alpha,
                          int32_t* gram_prec_used, int64_t* dropped, int32_t* steps_kept,
                          double* rel_residual, void* ws, size_t ws_bytes, void* stream);

/* Solves L L^T x = b with L from fst_cholesky (device FP64, including its stored
 * diagonal-block inverses); b and x may alias.
 * Asynchronous. */
fst_status fst_cholesky_solve(int64_t R, const double* L, const double* b, double* x,
                              void* stream);

/* FP64 normal-equations residual r = A^T (v_S - A alpha) at the sampled rows idx (device
 * int32, mrows), with rows regenerated in FP64 from the points (x, y, z, v: device, dtype).
 * alpha: device FP64 R; r: device FP64 R.  ws >= fst_residual_workspace_bytes.
 * Asynchronous. */
size_t fst_residual_workspace_bytes(const fst_model* m, int64_t mrows);
fst_status fst_residual(const fst_model* m, int32_t dtype, int64_t n, const void* x,
                        const void* y, const void* z, const void* v, const int32_t* idx,
                        int64_t mrows, const double* alpha, double* r, void* ws,
                        size_t ws_bytes, void* stream);

/* One step of iterative refinement of the sampled least-squares core: r = A^T (v_S - A alpha)
 * with FP64 rows (as fst_residual), delta = (L L^T)^-1 r with L from fst_cholesky (device
 * FP64 R x R), alpha += delta.  alpha: device FP64 R, updated in place; r_out (may be NULL):
 * device FP64 R receiving delta.  ws >= fst_refine_workspace_bytes.  Asynchronous. */
size_t fst_refine_workspace_bytes(const fst_model* m, int64_t mrows);
fst_status fst_refine_step(const fst_model* m, int32_t dtype, int64_t n, const void* x,
                           const void* y, const void* z, const void* v, const int32_t* idx,
                           int64_t mrows, const double* L, double* alpha, double* r_out,
                           void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ host steps */

/* M distinct indices of [0, n), sorted ascending, from a partial Fisher-Yates shuffle driven
 * by SplitMix64 with state seed * 256 + stream.  out: host int64[m].  0 <= m <= n < 2^32. */
fst_status fst_sample_indices(uint64_t seed, int32_t stream, int64_t n, int64_t m,
                              int64_t* out);

/* Inverse-distance interpolation onto the equispaced grid of Sec. 4.1: for every node
 * (C order, last mode fastest) the k nearest points in reference coordinates, weights d^-power;
 * a node that coincides with a point takes its value.  xi: host FP64 (K, 3) row-major
 * reference coordinates; v: host FP64 K; out: host FP64 I1*I2*I3.  n_threads 0 = all. */
fst_status fst_idw_grid(const double* xi, const double* v, int64_t K, const int32_t grid[3],
                        int32_t k, double power, int32_t n_threads, double* out);

/* ST-HOSVD at fixed ranks (Sec. 4.1): modes in the order 1, 2, 3; each factor's columns are
 * the leading left singular vectors of the current unfolding, signed so that the entry of
 * largest magnitude is positive.  T: host FP64 I1 x I2 x I3 (C order); core: host FP64
 * r1 r2 r3 (C order); W[k]: host FP64 I_k x r_k row-major; sigma[k] (may be NULL): host
 * FP64 I_k singular values of the unfolding seen at step k (zero-padded). */
fst_status fst_sthosvd(const double* T, const int32_t dims[3], const int32_t rank[3],
                       int32_t n_threads, double* core, double* const W[3],
                       double* const sigma[3]);

/* ST-HOSVD with ranks chosen from a compression precision eps (Sec. 4.1, Table 1): in mode
 * order 1, 2, 3, r_k is the smallest r with sum_{i > r} sigma_i^2 <= eps^2 ||T||_F^2 / 3 over
 * the singular values of the current (already truncated) unfolding, which guarantees
 * ||T - T~||_F <= eps ||T||_F; r_k is capped at max_rank[k] (the guarantee then need not
 * hold).  0 < eps < 1.  rank_out: host int32[3], the chosen ranks; core: host FP64 of at least
 * max_rank[0] max_rank[1] max_rank[2] entries, receives r1 r2 r3 (C order); W[k]: host FP64 of
 * at least I_k max_rank[k] entries, receives I_k x r_k row-major; sigma as fst_sthosvd. */
fst_status fst_sthosvd_eps(const double* T, const int32_t dims[3], double eps,
                           const int32_t max_rank[3], int32_t n_threads, int32_t rank_out[3],
                           double* core, double* const W[3], double* const sigma[3]);

/* Sparse Legendre fit of the columns of W (Sec. 4.2): orthogonal matching pursuit with
 * normalised correlations, support size chosen by the smallest leave-one-out (PRESS) error.
 * W: host FP64 I x r row-major, sampled at the equispaced nodes; C: host FP64 (p+1) x r
 * row-major (zeros off the support). */
fst_status fst_sparse_fit(const double* W, int32_t I, int32_t r, int32_t p, double* C);

/* The same fit with the Lasso-modified LARS path (Efron et al.) on the unit-norm columns of
 * the basis matrix instead of OMP: every active set of the path (after each entry or exit) is
 * refitted by least squares and scored by its leave-one-out error, and the first set with the
 * smallest error is kept (entry ties to the lowest index; a column that has just left is not
 * re-admitted in the next step; at most min(p + 1, I - 2) active columns). */
fst_status fst_sparse_fit_lars(const double* W, int32_t I, int32_t r, int32_t p, double* C);

/* ------------------------------------------------------------------ wavelet space (Sec. 4.2)
 * W_{s,q}: the piecewise polynomials of degree <= q on the 2^s dyadic cells of [-1, 1], with
 * Alpert's multiwavelet basis (orthonormal under dt/2): the global Legendre functions
 * phi_0..phi_q and, for each level l < s and cell c < 2^l, the functions
 * psi_{l,c,m}(t) = 2^(l/2) psi_m(2^l (t + 1) - 2c - 1), m = 0..q.  The mother wavelets psi_m are
 * polynomials of degree <= q on each half of [-1, 1]; psi_m is the unit function orthogonal to
 * phi_0..phi_{q+m} and to psi_{m+1}..psi_q, signed so that its largest coefficient on the right
 * half, in the basis sqrt(2) phi_n(2x - 1), is positive.  A point's cell at level l is
 * floor((t + 1) 2^(l-1)) clamped to [0, 2^l - 1].  A mode holding both spaces (q <= p) has the
 * basis phi_0..phi_p followed by the (q + 1)(2^s - 1) detail functions psi_{l,c,m} in the order
 * (l, c, m); its coefficient matrices have that many rows. */

/* The per-column choice of Algorithm 1: each column of W (host FP64 I x r row-major, sampled at
 * the I equispaced nodes) is fitted in P_p and in W_{s,q} with the given solver (leave-one-out
 * selection) and keeps the fit with the smaller leave-one-out error (P_p on ties).
 * C: host FP64 (p + 1 + (q + 1)(2^s - 1)) x r row-major. */
fst_status fst_sparse_fit_choice(const double* W, int32_t I, int32_t r, int32_t p, int32_t s,
                                 int32_t q, int32_t solver, double* C);

/* ------------------------------------------------------------------ model */

/* Builds a model from its parts.  lo, hi: host double[3]; rank, degree: host int32[3];
 * core: host FP64 r1 r2 r3 (C order); coefs[k]: host FP64 (p_k + 1) x r_k row-major. */
fst_status fst_model_from_parts(const double lo[3], const double hi[3], const int32_t rank[3],
                                const int32_t degree[3], const double* core,
                                const double* const coefs[3], fst_model** out);
void fst_model_free(fst_model* m);
/* A model whose modes may hold a wavelet space: as fst_model_from_parts_d, with wlevel[k] = s_k
 * (0: Legendre only) and wdegree[k] = q_k per mode (host int32[d]); coefs[k] has
 * p_k + 1 + (q_k + 1)(2^s_k - 1) rows. */
fst_status fst_model_from_parts_wavelet(int32_t d, const double* lo, const double* hi,
                                        const int32_t* rank, const int32_t* degree,
                                        const int32_t* wlevel, const int32_t* wdegree,
                                        const double* core, const double* const* coefs,
                                        fst_model** out);
/* wlevel, wdegree: host int32[d] receiving s_k, q_k (0, 0 for Legendre-only modes) */
fst_status fst_model_wavelets(const fst_model* m, int32_t* wlevel, int32_t* wdegree);
/* lo, hi (double[3]), rank, degree (int32[3]), nnz: non-zero coefficients; any may be NULL */
fst_status fst_model_info(const fst_model* m, double* lo, double* hi, int32_t* rank,
                          int32_t* degree, int64_t* nnz);
/* core_out: host FP64 r1 r2 r3 */
fst_status fst_model_core(const fst_model* m, double* core_out);
/* C_out: host FP64 (p_k + 1 + detail functions) x r_k row-major, zeros off the support */
fst_status fst_model_coefs(const fst_model* m, int32_t k, double* C_out);
/* Factor k in the compressed-column form the sparse fit produces (Sec. 3: the coefficients
 * of each factor function on its selected basis functions, eq. (2)): column j (factor
 * function j of mode k) holds rowidx[colptr[j] .. colptr[j+1]) (basis function indices,
 * ascending: Legendre degree i for i <= p_k, then the wavelet functions) with values vals[..]
 * (host FP64).  colptr: host int32[r_k + 1]; rowidx: host int32[nnz]; vals: host
 * double[nnz]; *nnz: number of non-zeros.  Any output may be NULL (call with only nnz to size
 * the arrays).  Explicit zeros of the dense form are not stored. */
fst_status fst_model_factor(const fst_model* m, int32_t k, int32_t* colptr, int32_t* rowidx,
                            double* vals, int64_t* nnz);
/* How the core of a model from fst_fit, fst_refit_core or fst_fit_batched was solved.
 * Precision ladder: a Gram whose Cholesky breaks down, or whose refinement makes the FP64
 * normal-equation residual grow, or whose refinement ends with ||A^T (v - A alpha)|| / ||A^T v||
 * above 1e-8, is formed again from FP32 rows (from BF16/FP16 rows), then from FP64 rows (G
 * and h; split 16-bit rows go there directly); the FP64 step skips numerically dependent
 * columns instead of failing.  Refinement undoes a step that does not reduce the residual
 * and stops there; after refine_steps steps a residual above 1e-8 gets further steps while
 * each one at least halves it, up to 4 x refine_steps in all.
 * gram_prec_used: the Gram precision the core was solved with (-1 for other models);
 * dropped: core entries fixed at zero because their design columns are numerically
 * dependent on earlier ones (the fitted field is unaffected); refine_steps: refinement steps
 * kept; rel_residual: final ||A^T (v - A alpha)|| / ||A^T v|| in FP64 (NaN without
 * refinement).  Any pointer may be NULL. */
fst_status fst_model_fit_info(const fst_model* m, int32_t* gram_prec_used, int64_t* dropped,
                              int32_t* refine_steps, double* rel_residual);
/* Storage in the paper's convention (Sec. 2): 8 bytes per stored value, core entries plus
 * non-zero coefficients, locations not counted. */
int64_t fst_model_paper_bytes(const fst_model* m);
/* Versioned little-endian serialisation.  buf == NULL queries the size into *nbytes; else
 * *nbytes is the capacity on input and the bytes written on output. */
fst_status fst_model_save(const fst_model* m, void* buf, size_t* nbytes);
fst_status fst_model_load(const void* buf, size_t nbytes, fst_model** out);

/* ------------------------------------------------------------------ d-way models (d = 3 or 4) */
/* Sec. 2 states the functional Tucker format for any number of modes d; Sec. 6 applies it to
 * data in three space dimensions plus time.  These calls take models with d = 3 or d = 4;
 * every call above that takes x, y, z (and fst_model_info) takes 3-way models only and
 * returns FST_E_INVAL for a 4-way one.  fst_model_core, fst_model_coefs (k < d),
 * fst_model_fit_info, fst_model_paper_bytes, fst_model_save / fst_model_load and
 * fst_model_free take both.  The core is in C order, j = ((j1 r2 + j2) r3 + j3) r4 + j4. */

/* lo, hi: host double[d]; rank, degree: host int32[d]; core: host FP64 r1 .. rd (C order);
 * coefs[k]: host FP64 (p_k + 1) x r_k row-major.  FST_E_UNSUPPORTED for d other than 3, 4. */
fst_status fst_model_from_parts_d(int32_t d, const double* lo, const double* hi, const int32_t* rank,
                                  const int32_t* degree, const double* core,
                                  const double* const* coefs, fst_model** out);
/* d: modes; lo, hi (double[d]), rank, degree (int32[d]), nnz; any may be NULL (pass arrays of
 * 4 entries when d is not known yet) */
fst_status fst_model_info_d(const fst_model* m, int32_t* d, double* lo, double* hi, int32_t* rank,
                            int32_t* degree, int64_t* nnz);

/* Reconstruction at points of interest, eq. (1) with d factors: out[i] = u~(c_1[i], .., c_d[i]).
 * coords: host array of d device coordinate arrays of n elements of `dtype`; out: device array
 * of n elements of `dtype`.  Asynchronous on `stream`.  (d = 3 runs the kernel of fst_eval.) */
fst_status fst_eval_d(const fst_model* m, int32_t dtype, int64_t n, const void* const* coords,
                      void* out, void* stream);

/* Algorithm 2 (Sec. 5) for a d-way model: M = n_samples rows drawn uniformly without
 * replacement (stream FST_STREAM_LS of `seed`, sorted), the factor functions of the d modes
 * evaluated at them (eq. (2)), the design rows A[q, j] = prod_k w^(k)_{j_k}(point q) of eq. (6)
 * formed in chunks of 16384 rows (device workspace, A^T layout) and contracted into
 * G = A^T A and h = A^T v on MFMA in the point dtype (FP32 rows: FP32 MFMA with FP64
 * accumulation across chunks; FP64 rows: FP64 MFMA), then solved by the FP64 Cholesky
 * factorisation (no refinement, no precision ladder: FST_E_NOT_SPD if the sampled Gram is
 * not numerically positive definite).  coords: host array of d device coordinate arrays;
 * v: device values; all of n elements of `dtype`.  R < n_samples <= n, r_k <= p_k + 1.
 * ws: device workspace >= fst_refit_core_d_workspace_bytes (G alone is R^2 FP64), or NULL to
 * let the library allocate it.  Synchronises `stream`; *out receives a new model with m's
 * factors. */
size_t fst_refit_core_d_workspace_bytes(const fst_model* m, int32_t dtype, int64_t n_samples);
fst_status fst_refit_core_d(const fst_model* m, int32_t dtype, int64_t n, const void* const* coords,
                            const void* v, int64_t n_samples, uint64_t seed, void* ws,
                            size_t ws_bytes, void* stream, fst_model** out);

/* Parameters of Algorithm 1 + Algorithm 2 for d = 3 or 4 modes (entries k >= d unused); the
 * fields mean what they mean in fst_fit_params.  Set struct_size = sizeof(fst_fit_params_d). */
typedef struct {
  uint32_t struct_size;
  int32_t  dtype;            /* FST_F64 | FST_F32: type of the coordinate and value arrays */
  int32_t  d;                /* 3 or 4 */
  double   lo[4], hi[4];     /* box mapped onto [-1,1]^d */
  int32_t  grid[4];          /* I_k of the interpolation grid (Sec. 4.1), I_1 .. I_d <= 2^28 nodes */
  int32_t  rank[4];          /* r_k (caps when eps > 0), r_k <= I_k, r_k <= prod of the others */
  int32_t  degree[4];        /* p_k, r_k <= p_k + 1 */
  double   interp_fraction;
  int32_t  idw_k;
  double   idw_power;
  int64_t  n_samples;        /* M rows of Algorithm 2; r1 .. rd < M <= n */
  uint64_t seed;
  int32_t  n_threads;
  double   eps;              /* > 0: ranks from this precision (Sec. 4.1), threshold eps^2 ||T||^2 / d */
  int32_t  sparse_solver;    /* FST_SOLVER_OMP or FST_SOLVER_LARS */
  int32_t  wavelet_level;    /* as in fst_fit_params */
  int32_t  wavelet_degree;
} fst_fit_params_d;

/* Fills defaults for d modes (grid 16, ranks 4, degree 15, fraction 0.1, idw 8 / 2.0, ...). */
void fst_fit_params_d_default(fst_fit_params_d* p, int32_t d);
/* Device workspace (bytes) of fst_fit_d for n points (the refit at the rank caps). */
size_t fst_fit_d_workspace_bytes(const fst_fit_params_d* p, int64_t n);
/* Algorithm 1 then Algorithm 2 for a d-way dataset (Sec. 4-5): the interpolation subset
 * (stream 1) is gathered from the device, interpolated onto the d-dimensional grid by inverse
 * distances, decomposed by ST-HOSVD (modes in order 1 .. d) and fitted by sparse Legendre
 * expansions on host threads; the core is then refitted on the GPU as in fst_refit_core_d.
 * coords: host array of d device coordinate arrays; v: device values; n elements of
 * p->dtype each.  ws >= fst_fit_d_workspace_bytes, or NULL.  Synchronises `stream`. */
fst_status fst_fit_d(const fst_fit_params_d* p, int64_t n, const void* const* coords, const void* v,
                     void* ws, size_t ws_bytes, void* stream, fst_model** out);
/* Algorithm 1 only, on host arrays (coords: host array of d host arrays, v: host values). */
fst_status fst_compress_host_d(const fst_fit_params_d* p, int64_t n, const void* const* coords,
                               const void* v, fst_model** out);

/* ------------------------------------------------------------------ batched form */
/* Many field variables on one shared point set (device arrays x, y, z of n points, dtype
 * base->dtype), with per-variable ranks (V x 3) and degrees (V x 3), both host int32.  All
 * variables share the interpolation subset of base->seed; variable v draws its least-squares
 * rows from stream FST_STREAM_LS of seed base->seed + v.  Host steps run on host threads;
 * the Gram matrices of all variables are formed in one persistent launch; each variable is
 * then solved in FP64 (with at most base->refine_steps refinement steps), climbing the
 * precision ladder of fst_model_fit_info where needed; gram_prec_used (may be NULL): host
 * int32[V] receiving the Gram precision each variable was solved with.  values: host
 * array of V device pointers.  out: host array receiving V new models.  timings (may be NULL): host
 * double[5] = host steps, row generation, batched Gram, A^T v, solves with refinement
 * (seconds, each phase synchronised).  Allocates its
 * device buffers (sum over variables of R_v^2 * 8 bytes for the Gram matrices) for the
 * duration of the call.  Synchronises `stream`. */
fst_status fst_fit_batched(const fst_fit_params* base, int32_t V, const int32_t* ranks,
                           const int32_t* degrees, int64_t n, const void* x, const void* y,
                           const void* z, const void* const* values, void* stream,
                           fst_model** out, int32_t* gram_prec_used, double* timings);
/* Reconstruction of V models at the same points: outs host array of V device arrays.
 * Asynchronous. */
fst_status fst_eval_batched(const fst_model* const* models, int32_t V, int32_t dtype, int64_t n,
                            const void* x, const void* y, const void* z, void* const* outs,
                            void* stream);
/* The same batched reconstruction captured once into a HIP graph, replayed by
 * fst_graph_launch on any stream.  The models and every array passed must stay alive and at
 * the same addresses until fst_graph_free. */
typedef struct fst_graph fst_graph;
fst_status fst_eval_graph_create(const fst_model* const* models, int32_t V, int32_t dtype, int64_t n,
                                 const void* x, const void* y, const void* z, void* const* outs,
                                 fst_graph** out);
fst_status fst_graph_launch(const fst_graph* g, void* stream);
void fst_graph_free(fst_graph* g);

/* ------------------------------------------------------------------ learned residual corrector */
/* A small network g(xi) = W3 s(W2 s(W1 xi + b1) + b2) + b3, s(z) = z / (1 + e^-z), layers
 * 3 -> 64 -> 64 -> 1 on the reference coordinates xi of the model's box, trained by Adam on the
 * mean squared error against the model's residual divided by its standard deviation; the
 * corrected reconstruction is u~(x) + sd * g(xi(x)).  Not part of the paper: an optional
 * addition judged against the plain model (which is also the fallback).  BF16 weights and
 * activations on MFMA for the 64 x 64 layer with FP32 accumulation, FP32 master weights.
 * Flat parameter order (4481 values): W1 (64 x 3) | b1 (64) | W2 (64 x 64, [out][in]) | b2 (64)
 * | W3 (64) | b3 (1).  Initial weights: Xavier-uniform from SplitMix64 (state seed*256 + 4),
 * zero biases; minibatch rows: SplitMix64 output number step*batch + i of state seed*256 + 3,
 * bounded to [0, n) (with replacement). */
typedef struct fst_corrector fst_corrector;   /* opaque; library-owned */
typedef struct {
  uint32_t struct_size;      /* sizeof(fst_train_params) */
  int32_t  steps;            /* Adam steps (2000) */
  int32_t  batch;            /* minibatch size (8192) */
  double   lr, beta1, beta2, eps;   /* 1e-3, 0.9, 0.999, 1e-8 */
  uint64_t seed;
  const float* init_params;  /* host float[4481] initial parameters, or NULL (Xavier-uniform) */
} fst_train_params;

void fst_train_params_default(fst_train_params* tp);
/* device workspace of fst_corrector_train for n training points */
size_t fst_corrector_workspace_bytes(const fst_train_params* tp, int64_t n);
/* Trains a corrector on the residual of model m at the n training points (device arrays x, y,
 * z, v of dtype).  Synchronises `stream`. */
fst_status fst_corrector_train(const fst_model* m, int32_t dtype, int64_t n, const void* x, const void* y,
                               const void* z, const void* v, const fst_train_params* tp, void* ws,
                               size_t ws_bytes, void* stream, fst_corrector** out);
/* Builds a corrector from host FP32 parameters (4481) and output scale; lo, hi: box. */
fst_status fst_corrector_from_params(const double lo[3], const double hi[3], const float* params,
                                     float out_scale, fst_corrector** out);
/* params_out: host float[4481] (stored values, BF16-rounded after training); either may be NULL */
fst_status fst_corrector_params(const fst_corrector* c, float* params_out, float* out_scale);
/* training loss every 50 steps: *count in = capacity of out, out = entries available */
fst_status fst_corrector_losses(const fst_corrector* c, float* out, int32_t* count);
void fst_corrector_free(fst_corrector* c);
/* stored size: BF16 weights (2 bytes each) plus the FP32 output scale */
int64_t fst_corrector_stored_bytes(const fst_corrector* c);
/* out[i] += sd * g(xi(x[i], y[i], z[i])) for device arrays of dtype.  Asynchronous. */
fst_status fst_corrector_apply(const fst_corrector* c, int32_t dtype, int64_t n, const void* x, const void* y,
                               const void* z, void* out, void* stream);
/* fst_eval followed by fst_corrector_apply (c may be NULL: plain reconstruction). */
fst_status fst_eval_corrected(const fst_model* m, const fst_corrector* c, int32_t dtype, int64_t n,
                              const void* x, const void* y, const void* z, void* out, void* stream);
/* Gradient of mean((g(xi_b) - target_b)^2) over the batch rows idx (device int32[batch]) at the
 * corrector's stored parameters: grad_out device float[4482] (4481 gradients, then the sum of
 * squared errors).  target: device float[n].  Synchronises `stream`. */
size_t fst_mlp_grad_workspace_bytes(int32_t batch);
fst_status fst_mlp_grad(const fst_corrector* c, int32_t dtype, int64_t n, const void* x, const void* y,
                        const void* z, const float* target, const int32_t* idx, int32_t batch,
                        float* grad_out, void* ws, size_t ws_bytes, void* stream);
/* The same gradient with the 64 x 64 layer in FP32 from the FP32 master weights, activations
 * not rounded to BF16: the reference mode of the training kernel (the BF16 MFMA layer is the
 * one fst_corrector_train uses).  Same arguments, workspace and errors as fst_mlp_grad. */
fst_status fst_mlp_grad_fp32(const fst_corrector* c, int32_t dtype, int64_t n, const void* x,
                             const void* y, const void* z, const float* target, const int32_t* idx,
                             int32_t batch, float* grad_out, void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* FST_H */
