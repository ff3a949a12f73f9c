/*
 * qgt_block.h -- C ABI of the block-layer QGT stochastic-reconfiguration library
 * for AMD Instinct MI355X (gfx950).
 *
 * The operation (paper, Sec. 2 "Natural Gradient Descent for NQS and Block-Layer
 * QGT", Eq. 2 and Eq. 3):
 *
 *   given the per-sample log-derivative Jacobian O (n_s x n_p, complex), whose
 *   columns are split into contiguous layer blocks b = 0..B-1, and the local
 *   energies E_loc (n_s, complex),
 *
 *     dE      = E_loc - mean(E_loc)
 *     mu      = column means of O,            dO = O - mu
 *     F_b     = dO_b^H dE / n_s                        (force of block b)
 *     S_b     = dO_b^H dO_b / n_s                      (block QGT, Eq. 3)
 *     delta_b = (S_b + lambda I)^{-1} F_b              (independent shifted solve)
 *     delta   = (delta_0, ..., delta_{B-1})            (concatenation)
 *
 *   Where n_s < n_b the same delta_b is obtained in sample space:
 *     (dO_b dO_b^H / n_s + lambda I) z_b = dE,  delta_b = dO_b^H z_b / n_s.
 *
 *   The library returns delta = S~^{-1} F; the optimiser's step
 *   theta <- theta - eta * delta (Sec. 2) is left to the caller.
 *
 * Numerics.  The column means, the force, the diagonal shift, the Cholesky
 * factorisation, the triangular solves and the refinement are FP64.  The Gram
 * contraction dO_b^H dO_b (or dO_b dO_b^H) may run in FP32 or in BF16 with FP32
 * accumulation; the centred operand is formed in FP64 and rounded to
 * nearest-even once.  A plan may ask (qgt_plan_options.factor) for blocks with
 * a BF16 Gram to be stored in complex64 and factored in FP32 instead (the
 * Gram's own rounding dwarfs that of the factorisation); the triangular solves
 * then still accumulate in FP64.  The Cholesky factor L of the shifted Gram serves as the
 * preconditioner M = L L^H of a conjugate-gradient iteration in FP64 on the
 * exact shifted operator, applied matrix-free from O; the iteration removes the
 * Gram's rounding error.  A Cholesky pivot below lambda (impossible in exact
 * arithmetic, since every pivot of S_b + lambda I is >= lambda) is raised to
 * lambda.
 *
 * Layouts.  All complex data are interleaved (re, im).
 *   O      : row-major n_s x n_p, leading dimension ldo >= n_p elements,
 *            complex64 (QGT_C64) or complex128 (QGT_C128).  Block b is the
 *            column range [off_b, off_b + n_b), off_b = sum_{c<b} n_c.
 *   E_loc  : n_s complex128.
 *   delta  : n_p complex128, same indexing as the columns of O.
 *   All device pointers must be 16-byte aligned.
 *
 * Ownership.  The caller owns O, E_loc, delta and the workspace (device memory,
 * for instance PyTorch tensors).  O and E_loc must stay valid and unmodified
 * until qgt_block_solve has completed on the stream: the refinement and the
 * sample-space back-projection read O again.  The plan owns a small device
 * buffer of metadata allocated by qgt_block_plan and freed by qgt_plan_destroy.
 * qgt_block_form and qgt_block_solve allocate nothing, synchronise nothing and
 * only enqueue kernels on the given stream, so they may be captured in a HIP
 * graph.  Calls on one plan must not overlap.
 *
 * Errors.  Argument errors are returned synchronously (non-positive or
 * non-finite lambda, block sizes that are not positive, n_s < 2, ldo < n_p,
 * null pointers, a workspace that is too small).  Numerical failures (a NaN or
 * infinite pivot from non-finite input: QGT_ERR_NOT_POSITIVE_DEFINITE; an
 * iteration that has not met refine_rtol: QGT_ERR_NOT_CONVERGED) are recorded
 * per block on the device and read with qgt_plan_status after the stream has
 * been synchronised.  No C++
 * exception crosses this interface.  qgt_last_error returns a thread-local
 * message describing the last failure.
 */
#ifndef QGT_BLOCK_H
#define QGT_BLOCK_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QGT_OK = 0,
  QGT_ERR_INVALID_ARGUMENT = 1,
  QGT_ERR_UNSUPPORTED = 2,
  QGT_ERR_WORKSPACE_TOO_SMALL = 3,
  QGT_ERR_HIP = 4,
  QGT_ERR_NOT_POSITIVE_DEFINITE = 5,
  QGT_ERR_NOT_CONVERGED = 6,
  QGT_ERR_NON_FINITE = 7,
  QGT_ERR_INTERNAL = 8
} qgt_status;

/* Element type of O (interleaved complex). */
typedef enum { QGT_C64 = 0, QGT_C128 = 1 } qgt_dtype;

/* Precision of the Gram contraction.  AUTO: FP64 for complex128 input; for
 * complex64 input BF16 on sample-space blocks with n_b >= 2 n_s, FP32 on the
 * other sample-space blocks, FP64 on parameter-space blocks whose Gram costs at
 * most 1e11 flops (4 n_s n_b^2) and FP32 on the larger parameter-space
 * blocks. */
typedef enum { QGT_GRAM_FP64 = 0, QGT_GRAM_FP32 = 1, QGT_GRAM_BF16 = 2, QGT_GRAM_AUTO = 3 } qgt_precision;

/* Per-block solve form.  AUTO: sample space iff n_s < n_b (parameter space at
 * equality). */
typedef enum { QGT_FORM_AUTO = 0, QGT_FORM_PARAM = 1, QGT_FORM_SAMPLE = 2 } qgt_form;

/* One SR problem: n_samples rows of O, the layer partition of its columns
 * (Sec. 2, the layer groups theta_l) and the uniform diagonal shift lambda. */
typedef struct {
  int64_t n_samples;
  int32_t n_blocks;
  const int64_t* block_sizes; /* host array of n_blocks positive sizes */
  double lambda;              /* > 0 */
} qgt_problem;

/* Precision of the stored shifted Gram and of its Cholesky factorisation.
 * FP64: every block (the default).  FP32_FOR_BF16: blocks whose Gram runs in
 * BF16 are stored in complex64 and factored in FP32; the others stay FP64. */
typedef enum { QGT_FACTOR_FP64 = 0, QGT_FACTOR_FP32_FOR_BF16 = 1 } qgt_factor;

/* Tile shapes and schedules of one block (0 in a field: the planner's
 * default).  Any choice gives the same result up to the order of the
 * floating-point sums; block indexing, forms and precisions do not change.
 *   gram_tile  : BF16 Gram output tiles, 1 = 128x128, 2 = 256x128 (only when
 *                the padded matrix order is a multiple of 256 and >= 1024;
 *                the default), 3 = 128x128 with two workgroups per CU and no
 *                split.  FP32 and FP64 Grams always use 128x128.
 *   gram_items : with 128x128 tiles, the block's Gram is split along the
 *                contraction until it has about this many work items (at
 *                least 16 LDS stages per split); default 256.
 *   chol_chunk : panels per trailing-update task of the persistent Cholesky
 *                (1..16); default 4.
 *   gram_patch : height of the patches of 128-row tile rows in which the
 *                Gram tiles are ordered (1..16, default 4; the patches are 8
 *                tile columns wide), so that the tiles an XCD runs at a time
 *                share operand panels in its L2. */
typedef struct {
  int32_t gram_tile;
  int32_t gram_items;
  int32_t chol_chunk;
  int32_t gram_patch;
} qgt_block_tuning;

/* How the Cholesky factorisations of a solve are launched.  HOST_STEPS: the
 * host issues the tile steps of all blocks together (one launch per POTRF,
 * TRSM and trailing-update step, the bulk of each pair's update on a second
 * stream).  PERSISTENT: one launch over the DAG of tile tasks of all blocks
 * (dependency counters in the workspace).  AUTO: the mode the autotuner
 * measured faster for the plan's set of blocks (a plan entry of the tuning
 * cache named by QGT_TUNE_CACHE), else PERSISTENT. */
typedef enum { QGT_CHOL_AUTO = 0, QGT_CHOL_HOST_STEPS = 1, QGT_CHOL_PERSISTENT = 2 } qgt_cholesky;

/* Optional plan settings; pass NULL for defaults (a zero-filled struct gives
 * the defaults too). */
typedef struct {
  const int32_t* forms; /* host, one qgt_form per block over all problems in order, or NULL */
  int32_t timing;       /* non-zero: record HIP events around the Gram launches */
  int32_t factor;       /* qgt_factor */
  /* host, one qgt_block_tuning per block over all problems in order, or NULL:
   * then, when the environment variable QGT_TUNE_CACHE names a tuning cache
   * written by qgt_autotune, each block takes the entry of its shape class
   * tuned inside the plan's set of blocks, else the entry of its shape class
   * (fields it lacks, and blocks whose class has no entry, take the
   * defaults). */
  const qgt_block_tuning* tuning;
  int32_t cholesky;     /* qgt_cholesky */
  int32_t pad;
} qgt_plan_options;

typedef struct qgt_plan_s* qgt_plan;

/* Plan a batch of n_probs independent problems solved together in the same
 * launches (one SR step of several independent optimisations).  Validates the
 * arguments, fixes per block the form and the Gram precision, builds the tile
 * work lists, uploads them to a device buffer owned by the plan (on the current
 * device) and returns the workspace size the caller must provide.
 *   max_refine : number of preconditioned-CG iterations after the first
 *                solve x = M^{-1} rhs (0..16); each costs one application of
 *                the shifted operator (two passes over O) and one pair of
 *                triangular solves.
 *   refine_rtol: >= 0.  When positive and max_refine >= 1, a block whose
 *                estimated relative error exceeds refine_rtol after the last
 *                iteration is marked QGT_ERR_NOT_CONVERGED.  The estimate is
 *                the size of the last preconditioned correction relative to
 *                the corrected solution, ||M^{-1} r|| / ||x + M^{-1} r|| (the
 *                error left once the correction is added is smaller still
 *                when the iteration contracts).  The same test
 *                runs after every iteration: a block that meets it stops
 *                there (its later operator passes, triangular solves and CG
 *                updates are skipped; its last correction is still added), so
 *                max_refine is an upper bound.  0: no test, every block runs
 *                max_refine iterations.
 * Returns QGT_OK, QGT_ERR_INVALID_ARGUMENT, QGT_ERR_UNSUPPORTED or QGT_ERR_HIP. */
qgt_status qgt_block_plan(const qgt_problem* probs, int32_t n_probs, qgt_dtype o_dtype,
                          qgt_precision gram, int32_t max_refine, double refine_rtol,
                          qgt_plan* out, size_t* workspace_bytes);

/* As qgt_block_plan, with options (per-block form override, kernel timing). */
qgt_status qgt_block_plan_ex(const qgt_problem* probs, int32_t n_probs, qgt_dtype o_dtype,
                             qgt_precision gram, int32_t max_refine, double refine_rtol,
                             const qgt_plan_options* opts, qgt_plan* out, size_t* workspace_bytes);

/* Host-only planning: the workspace size qgt_block_plan_ex would return, with
 * the same argument validation.  Makes no HIP call. */
qgt_status qgt_block_workspace_query(const qgt_problem* probs, int32_t n_probs, qgt_dtype o_dtype,
                                     qgt_precision gram, int32_t max_refine,
                                     const qgt_plan_options* opts, size_t* workspace_bytes);

/* Form step (paper Sec. 2: Eq. 1 for the centred energy, Eq. 2 for the
 * centred log-derivatives and the force, Eq. 3 for the blocks, and the uniform
 * shift S_l + lambda I_l stated after it): centring, mean, force, packed
 * operand and the shifted block Grams (S_b + lambda I, or the sample-space
 * matrix).  O[p], ldo[p], e_loc[p] are the device pointer, leading dimension
 * and device local energies of problem p.  The workspace (device, >=
 * workspace_bytes) is bound to the plan until the next form call. */
qgt_status qgt_block_form(qgt_plan plan, const void* const* O, const int64_t* ldo,
                          const void* const* e_loc, void* workspace, size_t workspace_bytes,
                          hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture that must not call hipMalloc, tight serving loops, harnesses that
 * forbid allocation): qgt_block_form with the workspace taken from a static
 * array of the library instead of the caller, so that neither this call nor
 * the qgt_block_solve that follows allocates anything.  The array holds 64 MiB
 * (QGT_STATIC_WORKSPACE_BYTES) per device; it is set up on the first call on a
 * device and kept until the process ends.  The plan (made beforehand with
 * qgt_block_plan on the current device) must need at most that much
 * workspace, else QGT_ERR_WORKSPACE_TOO_SMALL is returned and nothing is
 * launched.  Every call on one device shares that device's array and finds in
 * it whatever the previous call left; the kernels initialise everything they
 * read.  Calls that overlap on one device (the form of one plan and the solve
 * of another, on different streams or threads, before the first has completed)
 * race on the array and give wrong results: serialise them.  The workspace stays
 * bound to the plan until its next form call, as with qgt_block_form.  Other
 * arguments and errors as for qgt_block_form. */
#define QGT_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
qgt_status qgt_block_form_static(qgt_plan plan, const void* const* O, const int64_t* ldo,
                                 const void* const* e_loc, hipStream_t stream);

/* Solve step (paper Sec. 2: each shifted block inverted independently,
 * delta_l = S~_l^{-1} F_l, and the block updates concatenated in parameter
 * order): the Cholesky factorisation of every block of every problem as one
 * persistent launch over a DAG of 64x64 tile tasks (FP64; FP32 for BF16 Grams
 * when the plan asks for it), triangular solves, at most max_refine FP64
 * preconditioned-CG iterations, sample-space back-projection, and the scatter
 * of delta_b into delta[p] (device, n_p complex128 per problem). */
qgt_status qgt_block_solve(qgt_plan plan, void* const* delta, hipStream_t stream);

/* Full-QGT SR with FP64 Gram and solve (paper Eq. 2, S delta = F with the
 * whole QGT, shifted by lambda): the same kernels with one block spanning all
 * n_p parameters (parameter space if n_p <= n_s, else sample space).  p must
 * have n_blocks == 1 or block_sizes summing to n_p (the blocks are merged).
 * The workspace must hold qgt_full_workspace_bytes bytes.  The plan of each
 * (n_s, n_p, lambda, dtype) is made on the first call of that shape (metadata
 * upload, synchronous: not capture-safe) and kept in a cache; later calls of
 * the shape only enqueue kernels (capture-safe).  Concurrent calls are safe:
 * calls sharing a cached plan enqueue one at a time (each still needs its own
 * workspace).  qgt_full_release frees the cached plans (it synchronises the
 * device; no full solve may be in flight). */
size_t qgt_full_workspace_bytes(const qgt_problem* p, qgt_dtype o_dtype);
qgt_status qgt_full_solve(const qgt_problem* p, qgt_dtype o_dtype, const void* O, int64_t ldo,
                          const void* e_loc, void* delta, void* workspace, size_t ws_bytes,
                          hipStream_t stream);
void qgt_full_release(void);

/* Autotuner (host, synchronous; allocates device memory for its trials, so
 * it belongs to set-up, not to a capture).  On the current device it builds
 * synthetic inputs of exactly these problems and times (HIP events, `reps`
 * runs after a warm-up) the whole set under candidate tunings, by coordinate
 * descent over the shape classes of its blocks (arch, Gram precision, form,
 * padded matrix order, contraction length rounded up to a power of two, FP64
 * factor) that carry at least 2% of the set's Gram work (the others keep
 * the defaults), largest Gram work first: for each class the Gram's tile shape,
 * split and patch order on the form step, then one tile kind for all BF16
 * classes at once, then for each class the Cholesky chunk on form + solve
 * with the persistent factorisation.  A candidate
 * (timed as the fastest of its runs) replaces the best so far only when it
 * is faster by more than 1%, the default coming first, so every class is
 * tuned inside the launches it shares with the others.  Finally form + solve
 * of the tuned set is timed with both Cholesky launch modes, and the plan's
 * class (the sorted shape classes of all its blocks) gets the faster one
 * (HOST_STEPS only if faster by more than 1%).  Each tuned class is stored
 * twice: as the class's entry, and as its entry inside the plan's class (the
 * planner prefers the latter, so a set tuned in its own right keeps its
 * choices when another set sharing a class is tuned later).  The entries
 * (with the measured times) are merged into the JSON cache at cache_path
 * (created if absent; other entries are kept) and written back atomically.
 * With the environment variable QGT_TUNE_LOG set (non-empty), each decision
 * is printed to stderr as it is taken.  Returns the number of classes tuned in
 * *n_classes.  Errors: QGT_ERR_INVALID_ARGUMENT, QGT_ERR_HIP, or
 * QGT_ERR_INTERNAL when the cache file cannot be read or written. */
qgt_status qgt_autotune(const qgt_problem* probs, int32_t n_probs, qgt_dtype o_dtype, qgt_precision gram,
                        const char* cache_path, int32_t reps, int32_t* n_classes);

/* The tuning global block g of a plan runs with (defaults filled in), and
 * where it came from: *source = 0 defaults, 1 the caller's options, 2 the
 * tuning cache's entry for the block's shape class, 3 the cache's entry for
 * that class inside the plan's set of blocks.  Host only. */
qgt_status qgt_plan_block_tuning(qgt_plan plan, int32_t g, qgt_block_tuning* tuning, int32_t* source);

/* How the plan's Cholesky factorisations launch: *mode = QGT_CHOL_HOST_STEPS
 * or QGT_CHOL_PERSISTENT (AUTO resolved), *source = 0 the default, 1 the
 * caller's options, 2 the tuning cache.  Host only. */
qgt_status qgt_plan_cholesky(qgt_plan plan, int32_t* mode, int32_t* source);

/* Host only, no HIP call: the launch mode and source qgt_plan_cholesky would
 * report for a plan of these problems (for tests of the cache). */
qgt_status qgt_cholesky_query(const qgt_problem* probs, int32_t n_probs, qgt_dtype o_dtype, qgt_precision gram,
                              const qgt_plan_options* opts, int32_t* mode, int32_t* source);

/* Host only, no HIP call: the tuning a plan of these problems would give
 * global block g, as qgt_plan_block_tuning reports it (for tests of the cache
 * and of the lookup). */
qgt_status qgt_block_tuning_query(const qgt_problem* probs, int32_t n_probs, qgt_dtype o_dtype,
                                  qgt_precision gram, const qgt_plan_options* opts, int32_t g,
                                  qgt_block_tuning* tuning, int32_t* source);

/* Paper Sec. 3, Eq. 4 (a) and (b), on the device: after qgt_block_solve,
 * with A the inverse of problem `problem`'s shifted block-layer QGT (the
 * block-diagonal matrix of the inverses (S_b + lambda I)^{-1} = L_b^{-H}
 * L_b^{-1}, from the Cholesky factors the solve left in the workspace) and B a
 * reference inverse (device, n_p x n_p complex128, row-major, leading
 * dimension ldb >= n_p, for instance the inverse of the shifted exact QGT),
 * writes five FP64 sums to sums (device):
 *   sums[0] = Re Tr[A^H B], sums[1] = ||A||_F^2, sums[2] = ||B||_F^2,
 *   sums[3] = sum_b ||A_b - B_bb||_F^2, sums[4] = sum_b ||B_bb||_F^2,
 * from which F(A, B) = sums[0] / sqrt(sums[1] sums[2]) and eps_F(A, B) =
 * sqrt(sums[3] + sums[2] - sums[4]) / sqrt(sums[2]).  Every block of the
 * problem must be in parameter form and of order <= 2048
 * (QGT_ERR_UNSUPPORTED otherwise).  scratch (device, 256-byte aligned) must
 * hold qgt_block_inverse_scratch_bytes bytes (0 when unsupported).  Enqueues
 * on the stream, allocates nothing; fixed-order sums. */
size_t qgt_block_inverse_scratch_bytes(qgt_plan plan, int32_t problem);
qgt_status qgt_block_inverse_diagnostics(qgt_plan plan, int32_t problem, const void* B, int64_t ldb,
                                         void* scratch, size_t scratch_bytes, double* sums,
                                         hipStream_t stream);

/* Per-block numerical status, host array of one int32 per block over all
 * problems (QGT_OK, QGT_ERR_NOT_POSITIVE_DEFINITE, QGT_ERR_NOT_CONVERGED, or
 * QGT_ERR_INTERNAL when a bounded device-side wait of the persistent
 * Cholesky or of the triangular solves gave up).  Call
 * after synchronising the stream of the last solve.  Returns the worst status. */
qgt_status qgt_plan_status(qgt_plan plan, int32_t* per_block_status);

/* Plan introspection (host): total blocks over all problems, and for global
 * block g its problem, column offset, size, chosen form (1 param, 2 sample) and
 * Gram precision (qgt_precision). */
int32_t qgt_plan_num_blocks(qgt_plan plan);
qgt_status qgt_plan_block_info(qgt_plan plan, int32_t g, int32_t* problem, int64_t* offset,
                               int64_t* size, int32_t* form, int32_t* precision);

/* Number of Cholesky pivots of each block that were raised to lambda in the
 * last solve (host array of one int32 per block over all problems; call after
 * synchronising the stream of that solve).  Every pivot of S_b + lambda I is
 * >= lambda in exact arithmetic; a smaller computed pivot comes from the
 * rounding of a low-precision Gram (or of an FP32 factorisation).  The factor is
 * then that of a nearby positive definite matrix and still serves as the
 * preconditioner, but a count well above zero means a degraded preconditioner:
 * more CG iterations, or a larger error where the iteration count is fixed. */
qgt_status qgt_plan_pivot_floors(qgt_plan plan, int32_t* per_block_floors);

/* Factor precision of global block g: *factor_fp32 = 1 when the block is
 * stored and factored in complex FP32 (QGT_FACTOR_FP32_FOR_BF16 on a BF16
 * Gram), 0 for complex FP64. */
qgt_status qgt_plan_block_factor(qgt_plan plan, int32_t g, int32_t* factor_fp32);

/* Device addresses of intermediate results inside the bound workspace, for
 * tests: which = 0 mean mu (n_p c128), 1 force F (n_p c128), 2 centred energy
 * (n_s c128), 3 shifted Gram of block g (m x m, row-major, complex64 when the
 * block is factored in FP32 and complex128 otherwise, leading dimension written to *ld; only
 * the lower triangle is defined; a FP32 or BF16
 * sample-space Gram also holds the rank-one term (t_g / n_s^2) 1 1^T that keeps
 * its null vector 1 away from the rounding level; after qgt_block_solve it
 * holds the Cholesky factor), 4 packed Gram operand of
 * block g (planar Re then Im, K_pad x m_pad elements each of the Gram
 * precision, the contraction index in groups of G = 16 / sizeof(element):
 * element (k, m) at ((k / G) * m_pad + m) * G + k % G; parameter form k =
 * sample, m = column of the block, sample form k = column, m = sample and the
 * imaginary plane negated; K_pad = K rounded up to a multiple of 4 G, m_pad = m
 * rounded up to a multiple of 128 and written to *ld; padding is zero), 5
 * trace of the block QGT t_g = sum_{k in g} S_kk (one double), 6 the error
 * estimate of block g's CG iteration (one double, after the solve; see
 * refine_rtol), 7 the number of CG iterations block g ran in the last solve
 * (one int32; below max_refine when it met refine_rtol early).
 * index is the problem (0..2) or the global block (3..7). */
qgt_status qgt_plan_debug_ptr(qgt_plan plan, int32_t which, int32_t index, void** ptr, int64_t* ld);

/* Timing of the Gram kernel of one precision (QGT_GRAM_FP64, _FP32 or _BF16)
 * when the plan was made with timing on: the sum of the durations (ms, HIP
 * events recorded on the launch stream around that kernel's launch) and the
 * number of launches since the last reset, and the algorithmic flops of one
 * launch (4 n_s n_b^2 per parameter-space block, 4 n_s^2 n_b per sample-space
 * block, over the blocks of that precision).  Synchronises on the recorded
 * events.  reset != 0 clears the totals after reading them. */
qgt_status qgt_plan_gram_timing(qgt_plan plan, int32_t precision, double* total_ms, int64_t* launches,
                                double* flops_per_launch, int32_t reset);

void qgt_plan_destroy(qgt_plan plan);
const char* qgt_status_string(qgt_status s);
const char* qgt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* QGT_BLOCK_H */
