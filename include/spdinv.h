/*
 * spdinv -- explicit inverse of symmetric positive definite matrices on
 * MI355X (gfx950), as the three-stage tile algorithm of Agullo, Bouwmeester,
 * Dongarra, Kurzak, Langou and Rosenberg, "Towards an Efficient Tile Matrix
 * Inversion of Symmetric Positive Definite Matrices on Multicore
 * Architectures":
 *
 *   step 1  A = L L^T          (tile Cholesky: POTRF, SYRK, GEMM, TRSM)
 *   step 2  X = L^{-1}         (tile triangular inverse: TRTRI, TRMM, GEMM)
 *   step 3  A^{-1} = X^T X     (tile product: LAUUM, TRMM, GEMM, SYRK)
 *
 * (Section 2, Algorithm 1), with the anti-dependences removed by array
 * renaming, the step-2 GEMM chain reversed (loop order UDU) and the three
 * steps pipelined through one dependency-tracked DAG (Section 3, Table 1).
 * Every task runs on the GPU inside one persistent scheduler kernel.
 *
 * Conventions common to every entry point
 * ---------------------------------------
 * - Matrices are column-major with a leading dimension ld >= max(1, n).
 *   Pointers documented as "device" must be device memory of the current HIP
 *   device; "host" pointers are ordinary host memory.
 * - Only the lower triangle (row >= column) of an input SPD matrix is read;
 *   on success the lower triangle holds the lower triangle of A^{-1}.  The
 *   strictly upper triangle is neither read nor written unless
 *   spdinv_opts.fill_upper is set (then it receives the mirror image).
 * - The caller owns every buffer.  The library never frees caller memory and
 *   performs no allocation on the call path, except that the first call for
 *   a given tile count and variant uploads that plan into a library-owned
 *   device arena that lives until spdinv_release_plans() or process exit.
 * - Work is enqueued on `stream` and the call returns without waiting, unless
 *   a host report is requested.
 * - Return value: 0 = enqueued; -i = the i-th argument is invalid (checked on
 *   the host, nothing enqueued); SPDINV_ERR_WORKSPACE = work_bytes too small;
 *   SPDINV_ERR_HIP = a HIP runtime call failed; SPDINV_ERR_TIMEOUT = the
 *   device scheduler gave up waiting (reported only when a host report was
 *   requested).
 * - Numerical failure is reported asynchronously through `d_info` (device
 *   int, may be NULL), with the LAPACK xPOTRF meaning: k > 0 when the leading
 *   minor of order k is not positive definite (the contents of A are then
 *   unspecified).  n = 0 returns 0 at once.
 */
#ifndef SPDINV_H
#define SPDINV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* hipStream_t without the HIP headers */
typedef struct ihipStream_t* spdinv_stream_t;

enum {
  SPDINV_ERR_WORKSPACE = 1,
  SPDINV_ERR_HIP = 2,
  SPDINV_ERR_TIMEOUT = 3,
  SPDINV_ERR_UNSUPPORTED = 4
};

typedef enum {
  SPDINV_FP64 = 0,       /* every tile task in binary64 */
  SPDINV_FP32 = 1,       /* FP32 storage (float matrices): tile products on FP32 matrix
                            cores with FP32 accumulation, diagonal tiles factored and
                            inverted in binary64 and rounded to FP32; no refinement */
  SPDINV_MIXED_FP32 = 2, /* tile products on FP32 matrix cores (FP32 accumulation),
                            diagonal tiles in binary64, then Newton-Schulz refinement
                            X <- X + X (I - A X) with binary64 residuals */
  SPDINV_MIXED_BF16 = 3  /* as MIXED_FP32 with bfloat16 operands (rounded to nearest
                            even from the FP32 tiles) on v_mfma_f32_16x16x16_bf16,
                            FP32 accumulation; default max_refine 8 */
} spdinv_mode;

typedef struct {
  int nb;          /* tile order; 0 = library choice.  Supported: 128        */
  int pipelined;   /* 1 = one DAG over the three steps (default); 0 = barriers
                      between steps (Section 3, "Pipelining")                 */
  int renamed;     /* 1 = out-of-place variant with copies B = L and C = L^{-1}
                      (default, Section 3 "Array renaming"); 0 = in place     */
  int loop_order;  /* 0 = UDU (default), 1 = UUU (Section 3, "Loop reversal") */
  int trtri_first; /* 0 = LAPACK 3.2.1 order in step 2 (default); 1 = TRTRI(j)
                      at the head of iteration j                              */
  int workers;     /* 0 = every resident workgroup; > 0 caps the persistent
                      grid (1 = program order on one worker)                  */
  int fill_upper;  /* 1 = also write the strictly upper triangle (mirror)     */
  int trace;       /* 1 = record per-task timestamps (see spdinv_trace_*)    */
  int max_refine;  /* mixed modes: most refinement steps (0 = library default:
                      6 for MIXED_FP32, 8 for MIXED_BF16)                     */
  double refine_tol; /* mixed modes: stop once ||I - A X||_F / ||A||_F <= refine_tol
                        (0 = library default, 1e-13)                            */
  int chain;       /* FP64, FP32, mixed and batched forms: most consecutive products of one output
                      tile's update chain that run as one device task, the tile
                      staying in registers between them (0 = library default,
                      8; 1 = one device task per task of the paper's stream;
                      at most 16).  Same products in the same order: results
                      are bit-identical for every value.  The last product
                      before a chain's closing task always runs alone.  */
  int per_cu;      /* FP64, FP32 and mixed forms: persistent workgroups per
                      compute unit (0 = library choice: 2 when the matrix has
                      at least 96 tiles per side, where the DAG keeps enough
                      tasks ready, else 1; or 1 or 2).  Results do not
                      depend on it.                                          */
  int no_split;    /* FP64 form: 0 (default) = with more than one worker, run
                      the products on chains of dependent tasks as row-part
                      tasks, run side by side (four quarters below 96 tiles
                      per side, two halves from there): TRSM(j+1, j)
                      and the last SYRK into tile (j+1, j+1), between POTRF(j)
                      and POTRF(j+1), and in the solve each multiplication by
                      D_i or D_i^T with the last update before it; 1 = as
                      whole tasks.  Results do not depend on it.             */
  int parts;       /* FP64 form, with the split on: row parts per split product
                      (0 = library choice as above; 2 = halves; 4 = quarters).
                      Results do not depend on it.                           */
  int rename_tiles; /* FP64 inverse with renamed = 1: memory-constrained
                      partial renaming (Section 3, "Array renaming").  0 =
                      full renaming (copies B of L and C of L^{-1} for every
                      lower tile, 2T tiles); k > 0 = at most k copy tiles:
                      whole tile rows of B and C are renamed, chosen greedily
                      by the critical path of the task DAG they shorten
                      (bottom C rows first where no single row shortens it),
                      the other rows are read in place with the paper's
                      anti-dependences, and the workspace shrinks
                      accordingly.  Results do not depend on it.  Ignored by
                      spd_cholesky and the solves; rejected (-8) by the FP32
                      and mixed modes.                                       */
  int tree_levels; /* FP64 plans with step 2: tree reduction of the step-2
                      update chains A_ij += sum_k X_ik L_kj (associativity,
                      the paper's conclusion).  0 = the sequential chains
                      (default); L = 1 or 2: each chain is cut into 2^L
                      consecutive segments accumulated side by side (into
                      A_ij and into 2^L - 1 partial-sum tiles per lower
                      tile, after the pool's other regions) and added in a
                      fixed binary tree, so results are bit-identical across
                      schedules but differ in rounding from L = 0.  Ignored by
                      the batched form; rejected (-8) by the FP32 and mixed
                      modes.                                                  */
  int batch_group; /* batched form: schedule.  -1 = one workgroup per matrix
                      (largest first), running its tasks in order on the
                      workgroup's own pool; -2 = one DAG over the batch,
                      dispatched in the order of a list-scheduling
                      simulation on 512 workers (or `workers`): the largest
                      matrices first, each matrix's longest remaining path
                      first, matrices that run one after another sharing
                      pool slots; g > 0 = one DAG, the matrices' task lists
                      interleaved position by position in groups of g
                      matrices, each with its own pool; 0 (default) = the
                      library's choice: -1 when the batch has at least two
                      matrices per worker, else -2.  Results do not depend
                      on it.                                                 */
  int correction64; /* mixed modes: 0 (default) = the correction X R of each
                      refinement step that another residual follows runs on
                      the FP32 matrix cores (X and R rounded to FP32, FP32
                      accumulation, added to X in binary64), the last step's
                      in binary64; a low-precision step that fails to square
                      the residual (within a factor 100) switches the
                      remaining steps to binary64.  1 = every correction in
                      binary64.                                               */
} spdinv_opts;

typedef struct {
  int info;            /* as d_info */
  int status;          /* 0, or SPDINV_ERR_TIMEOUT */
  int nb;              /* tile order used */
  int tiles;           /* t = ceil(n / nb) */
  long long tasks;     /* tasks executed */
  int critical_path;   /* critical path of the executed DAG, in tasks */
  int workers;         /* persistent workgroups launched */
  int refine_iters;    /* mixed modes: refinement steps taken                    */
  int fell_back;       /* mixed modes: the result comes from the FP64 path because
                          1: the low-precision start failed (the FP32
                          factorization broke down, its residual
                          ||I - A X0||_F was estimated above 2 from random
                          probes, or measured >= 1), or
                          2: the library's default step limit ran out before
                          the stop rule was met; 0 otherwise                  */
  double resid_fro_rel; /* mixed modes: ||I - A X||_F / ||A||_F of the returned X
                           as the stop rule saw it: measured, or (predicted = 1)
                           the prediction ||R_k||_F^2 plus a binary64 rounding
                           floor of 4 u ||A||_F ||X||_F, divided by ||A||_F   */
  double resid0_fro_rel; /* mixed modes: the same, measured, for the start X0   */
  double resid_last_rel; /* mixed modes: the last residual actually formed      */
  int converged;       /* mixed modes: 1 when the stop rule was met           */
  int predicted;       /* mixed modes: 1 when the loop stopped on the prediction
                          (the residual of the returned X was not formed)     */
  int low_corrections; /* mixed modes: refinement steps whose correction ran on
                          the FP32 matrix cores                               */
  double resid0_probe_rel; /* mixed modes: ||I - A X0||_F / ||A||_F estimated from
                          128 random sign probes V (||R0 V||_F^2 / 128
                          estimates ||R0||_F^2) before the full residual is
                          formed; -1 when not taken                           */
} spdinv_report;

/* Fills `opts` with the defaults. */
void spdinv_default_opts(spdinv_opts* opts);

/* Bytes of device workspace that spd_inverse needs for order n.  The
   workspace holds the three tile copies (A, B, C), the inverted diagonal
   tiles and the scheduler state. */
size_t spd_inverse_workspace_bytes(int n, spdinv_mode mode, const spdinv_opts* opts);
/* (for the mixed modes this also holds the FP32 tile pool and four square
   binary64 matrices of ceil(n/128)*128: A, X, the next X and the residual) */

/*
 * A <- A^{-1} for one SPD matrix (Algorithm 1 with the variants of Section 3).
 * A holds doubles, except in mode SPDINV_FP32, where it holds floats.
 * mode SPDINV_FP64 runs every task in binary64.  mode SPDINV_FP32 (renamed
 * plan only) runs the same DAG on FP32 tiles: products on FP32 matrix cores,
 * diagonal tiles in binary64 rounded to FP32; the result is the FP32 inverse
 * without refinement.  mode SPDINV_MIXED_FP32
 * (renamed plan only) runs the same DAG with FP32 tiles to get X0, then
 * refines by Newton-Schulz: R = I - A X in binary64, stop when
 * ||R||_F / ||A||_F <= refine_tol, else X <- X + X R (lower tiles, mirrored);
 * since I - A (X + X R) = R^2, the loop also stops, without forming the
 * next residual, once (||R||_F^2 + 4 u ||A||_F ||X||_F) / ||A||_F meets the
 * rule (u = 2^-53).  That last correction is formed in binary64, the earlier
 * ones on the FP32 matrix cores (see opts->correction64).  It synchronizes
 * the stream once per step.  It falls back to the FP64 path when the FP32
 * factorization breaks down, when ||R_0||_F estimated from 128 random sign
 * probes (two thin products, before the full residual) exceeds 2, when
 * ||R_0||_F >= 1, or when the default step limit runs out first (with an
 * explicit max_refine or refine_tol it returns the refined X instead, with
 * report->converged = 0).
 *   n        order (>= 0)
 *   A        device, column-major, lda >= max(1,n); lower triangle read and
 *            overwritten with the lower triangle of A^{-1}
 *   work     device workspace of at least spd_inverse_workspace_bytes bytes
 *            (any contents on entry; clobbered)
 *   stream   HIP stream (NULL = default stream)
 *   opts     host, may be NULL (defaults)
 *   d_info   device int or NULL; receives INFO (0 on success)
 *   report   host or NULL; when given, the call waits for the stream and
 *            fills it (INFO is then also returned through report->info)
 */
int spd_inverse(int n, void* A, int lda, spdinv_mode mode, void* work, size_t work_bytes,
                spdinv_stream_t stream, const spdinv_opts* opts, int* d_info,
                spdinv_report* report);

/* ---- the steps on their own ------------------------------------------------ */
/*
 * Cholesky factor only: A = L L^T by step 1 of Algorithm 1 (tile POTRF,
 * SYRK, GEMM, TRSM; Section 2), on the same scheduler.  The lower triangle of
 * A (column-major, lda >= max(1,n)) is read and overwritten with L; the
 * strictly upper triangle is neither read nor written (opts->fill_upper is
 * ignored).  Workspace: spd_inverse_workspace_bytes(n, SPDINV_FP64, opts)
 * bytes.  d_info, report, stream and opts as for spd_inverse (FP64 only;
 * the steps on their own run the renamed plan, so renamed = 0 and
 * rename_tiles > 0 are rejected as invalid options):
 * INFO = k > 0 when the leading minor of order k is not positive definite
 * (the contents of A are then unspecified).  Returns 0, -i for an invalid
 * i-th argument, SPDINV_ERR_WORKSPACE or SPDINV_ERR_HIP.
 */
int spd_cholesky(int n, double* A, int lda, void* work, size_t work_bytes,
                 spdinv_stream_t stream, const spdinv_opts* opts, int* d_info,
                 spdinv_report* report);

/*
 * Inverse from a given Cholesky factor: (L L^T)^{-1} by steps 2 and 3 of
 * Algorithm 1 (TRTRI: tile TRTRI, TRMM, GEMM, TRSM; LAUUM: tile LAUUM, TRMM,
 * SYRK, GEMM).  A prologue kernel first makes what step 1 would leave for
 * step 2 (the inverted diagonal tiles and the transposed copies of L's
 * tiles).  The lower triangle of L (column-major, ldl >= max(1,n)) holds the
 * factor on entry (its strictly upper triangle is not read) and the lower
 * triangle of the inverse on exit; the strictly upper triangle receives the
 * mirror only with opts->fill_upper.  INFO = k > 0 when L_kk = 0 (the
 * contents are then unspecified).  Workspace, stream, opts, d_info, report
 * and return codes as for spd_cholesky.
 */
int spd_inverse_from_factor(int n, double* L, int ldl, void* work, size_t work_bytes,
                            spdinv_stream_t stream, const spdinv_opts* opts, int* d_info,
                            spdinv_report* report);

/*
 * Solve A X = B for an SPD A: the Cholesky factor by step 1 of Algorithm 1,
 * then the forward substitution L Y = B and the backward substitution
 * L^T X = Y over 128 x 128 tiles of B, all in one DAG on the scheduler (the
 * substitutions multiply by the inverted diagonal tiles that step 1 makes,
 * as its TRSMs do).  As LAPACK's xPOSV: the lower triangle of A is replaced
 * by L (the strictly upper triangle is neither read nor written) and B
 * (column-major n x nrhs, ldb >= max(1,n)) by X.  Workspace:
 * spd_solve_workspace_bytes(n, nrhs, opts).  opts as for spd_cholesky (the
 * renamed plan: renamed = 0 and rename_tiles > 0 are invalid).  d_info:
 * INFO = k > 0 when the leading minor of order k is not positive definite
 * (A and B are then unspecified).  Returns 0, -i for an invalid i-th argument,
 * SPDINV_ERR_WORKSPACE or SPDINV_ERR_HIP.  nrhs <= 8192.
 */
size_t spd_solve_workspace_bytes(int n, int nrhs, const spdinv_opts* opts);
int spd_solve(int n, int nrhs, double* A, int lda, double* B, int ldb, void* work,
              size_t work_bytes, spdinv_stream_t stream, const spdinv_opts* opts, int* d_info,
              spdinv_report* report);

/*
 * Solve with a given Cholesky factor (as LAPACK's xPOTRS): the lower triangle
 * of L (column-major, ldl) holds the factor and is only read; B (n x nrhs,
 * ldb) is replaced by X with L L^T X = B.  The prologue of
 * spd_inverse_from_factor makes the inverted diagonal tiles and the
 * transposed copies of L's tiles.  INFO = k > 0 when L_kk = 0.  Workspace,
 * return codes and the other arguments as for spd_solve.
 */
int spd_solve_from_factor(int n, int nrhs, const double* L, int ldl, double* B, int ldb,
                          void* work, size_t work_bytes, spdinv_stream_t stream,
                          const spdinv_opts* opts, int* d_info, spdinv_report* report);

/* ---- batched form ---------------------------------------------------------- */
/* Bytes of device workspace that batched_spd_inverse needs for these orders
   on the current device (0 when batch <= 0 or an order is invalid). */
size_t batched_spd_inverse_workspace_bytes(int batch, const int* h_n, spdinv_mode mode,
                                           const spdinv_opts* opts);

/*
 * A_i <- A_i^{-1} for `batch` independent SPD matrices of uneven orders, as
 * one dependency-tracked DAG in one persistent launch (after a reset kernel).
 * Every matrix with n > 128 runs the tile plan of Section 3 for its tile
 * count (renamed, UDU, pipelined) between a copy-in task (its lower triangle
 * to its own tiles) and a copy-out task; a matrix with n <= 128 is one task
 * that inverts it in LDS in binary64.  The host merges the task lists into
 * one dispatch order by simulating the launch (opts->batch_group), so the
 * persistent workers run the tasks of many matrices side by side.
 *   batch   number of matrices (0 <= batch < 2^19)
 *   h_n     host int[batch], orders 0 <= n_i <= 2048 (the tile count of each
 *           matrix selects its task list; sizes the workspace)
 *   d_n     device int[batch], the same orders
 *   d_A     device array of batch device pointers to column-major matrices of
 *           doubles (SPDINV_FP64) or floats (SPDINV_FP32); the lower triangle
 *           of each is read and overwritten
 *   d_lda   device int[batch], leading dimensions (>= max(1, n_i))
 *   mode    SPDINV_FP64 or SPDINV_FP32 (FP32 tiles and matrix cores,
 *           binary64 diagonal tiles and small matrices, rounded to FP32)
 *   work    device workspace of batched_spd_inverse_workspace_bytes bytes:
 *           the tile pools (3T + 2t tiles for a matrix of tile count t >= 2,
 *           T = t(t+1)/2) - one per workgroup with batch_group = -1 (each
 *           workgroup's matrices use it in turn), slots shared by matrices
 *           that the dispatch order runs one after another with -2, one per
 *           matrix with g > 0 - and the per-task counters (2.6 GB in FP64
 *           for 8192 orders uniform on 16..512 with the library's choice)
 *   opts    host or NULL: renamed, loop_order, trtri_first and chain select
 *           the tile plan (FP32: renamed only); batch_group the
 *           interleaving; fill_upper mirrors each result; workers caps the
 *           grid
 *   d_info  device int[batch] or NULL: INFO of each matrix (0, k > 0 as for
 *           spd_inverse, or -1 when its d_n/d_lda/d_A entry is invalid on the
 *           device or its order is not of the tile count given in h_n)
 * Returns 0, -i for an invalid i-th argument, SPDINV_ERR_WORKSPACE or
 * SPDINV_ERR_HIP.  The launch is asynchronous.  The first call for a new set
 * of tile counts (per matrix) builds and uploads its task lists into a
 * library-owned device arena; a later call with the same tile counts
 * allocates nothing and can be captured in a HIP graph.  The matrices must
 * not overlap.
 */
int batched_spd_inverse(int batch, const int* h_n, const int* d_n, void* const* d_A,
                        const int* d_lda, spdinv_mode mode, void* work, size_t work_bytes,
                        spdinv_stream_t stream, const spdinv_opts* opts, int* d_info);

/* ---- backward ------------------------------------------------------------- */
/* Bytes of device workspace that spd_inverse_backward needs for order n
   (three square tile-major matrices of ceil(n/128)*128). */
size_t spd_inverse_backward_workspace_bytes(int n);

/*
 * Adjoint of the inverse.  For the loss L = sum(G o A^{-1}) of a symmetric A
 * (A parametrized as a symmetric matrix), the gradient is
 *     gradA = -sym(A^{-1} G A^{-1}) = -X S X,   X = A^{-1},  S = (G + G^T)/2,
 * formed as W = X S followed by the lower tiles of -W X, mirrored.  It is the
 * derivative of the map of Section 2 (A -> A^{-1}), which the paper does not
 * treat; the operation count is about 3 n^3.
 *   n       order (>= 0)
 *   X       device, column-major, ldx >= max(1,n): the inverse, of which only
 *           the lower triangle is used (the output of spd_inverse)
 *   G       device, column-major, ldg >= max(1,n): the full upstream
 *           gradient dL/dA^{-1} (not necessarily symmetric)
 *   gradA   device, column-major, ldga >= max(1,n): receives the full
 *           symmetric gradient (both triangles); must not overlap X or G
 *   work    device workspace of spd_inverse_backward_workspace_bytes(n)
 *   stream  HIP stream; the call is asynchronous
 * Returns 0, -i for an invalid i-th argument (nothing enqueued),
 * SPDINV_ERR_WORKSPACE or SPDINV_ERR_HIP.  n = 0 returns 0 at once.
 */
int spd_inverse_backward(int n, const double* X, int ldx, const double* G, int ldg, double* gradA,
                         int ldga, void* work, size_t work_bytes, spdinv_stream_t stream);

/* ---- allocation-free entry point -------------------------------------------- */
/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP64
 * inverse of spd_inverse, same plan and kernels and therefore the same bits,
 * with the workspace and the plan's device tables in a scratch array that the
 * library holds in device memory: SPDINV_NOALLOC_SCRATCH_BYTES (57 MiB) on
 * each GPU the library runs on, from the first call on that GPU until the
 * process ends.  The call performs no hipMalloc, hipFree or other device
 * allocation; it copies the plan's tables (host memory kept by the library)
 * into the scratch with hipMemcpyAsync on `stream` when the previous call on
 * this GPU used another plan.
 *   n        order, 0 <= n <= SPDINV_NOALLOC_MAX_N; a larger n returns -1
 *            (nothing is enqueued)
 *   A, lda   as for spd_inverse (device, column-major, lower triangle read
 *            and overwritten; lda >= max(1,n))
 *   stream   HIP stream; the call is asynchronous (it never waits)
 *   opts     host or NULL, as for spd_inverse (FP64 variants, chain, per_cu,
 *            no_split, parts, fill_upper, workers, rename_tiles); trace
 *            and tree_levels (whose partial sums need more than the
 *            scratch array holds) are rejected (-5)
 *   d_info   device int or NULL: INFO as for spd_inverse
 * Returns 0, -i for an invalid i-th argument, or SPDINV_ERR_HIP.
 * Every call on one GPU uses that GPU's single scratch array, whose contents
 * persist between calls (each call first resets what must start at zero):
 * calls that may overlap on one GPU (other streams, other host threads)
 * race and give unspecified results.  Serialize them on one stream.
 */
#define SPDINV_NOALLOC_MAX_N 2048
#define SPDINV_NOALLOC_SCRATCH_BYTES ((size_t)59768832)
int spd_inverse_noalloc(int n, double* A, int lda, spdinv_stream_t stream,
                        const spdinv_opts* opts, int* d_info);

/*
 * The same adjoint for `batch` matrices of uneven orders in one persistent
 * launch (after a fill kernel that clears its counters): grad_i =
 * -X_i sym(G_i) X_i.  The tile tasks of every matrix (packing of X_i from
 * its lower triangle and of sym(G_i), the tiles of W_i = X_i S_i, the lower
 * tiles of -W_i X_i, the output tiles) run in phase order on persistent
 * workgroups, each waiting for the tiles it reads through per-matrix
 * counters.
 *   batch    number of matrices (0 <= batch < 2^19)
 *   h_n      host int[batch], orders 0 <= n_i <= 2048
 *   d_n      device int[batch], the same orders (an order or leading
 *            dimension on the device that does not fit leaves that
 *            matrix's output unwritten)
 *   d_X      device array of device pointers: X_i = A_i^{-1}, column-major,
 *            lower triangle used;  d_ldx device int[batch]
 *   d_G      device array of device pointers: G_i, full; d_ldg device int[batch]
 *   d_gradA  device array of device pointers: the full symmetric gradients
 *            (must not overlap X_i or G_i);  d_ldga device int[batch]
 *   work     device workspace of batched_spd_inverse_backward_workspace_bytes
 *            bytes: 4 t_i^2 tiles of 128 x 128 doubles per matrix
 *            (t_i = ceil(n_i/128)) and the counters
 * Returns 0, -i for an invalid i-th argument, SPDINV_ERR_WORKSPACE or
 * SPDINV_ERR_HIP.  The first call for a set of tile counts uploads its task
 * list into a library-owned device arena; later calls with the same tile
 * counts allocate nothing and can be captured in a HIP graph.
 */
size_t batched_spd_inverse_backward_workspace_bytes(int batch, const int* h_n);
int batched_spd_inverse_backward(int batch, const int* h_n, const int* d_n,
                                 const double* const* d_X, const int* d_ldx,
                                 const double* const* d_G, const int* d_ldg,
                                 double* const* d_gradA, const int* d_ldga, void* work,
                                 size_t work_bytes, spdinv_stream_t stream);

/* ---- autotuner ------------------------------------------------------------ */
typedef struct {
  int nb;            /* tile order (128: the tile kernels of this library)        */
  int per_cu;        /* FP64 form: workgroups per CU chosen                       */
  int chain;         /* products per device task chosen                           */
  int parts;         /* FP64 form: row parts of split products (0 = whole)        */
  int batch_group;   /* batched form: schedule chosen (as spdinv_opts.batch_group) */
  double ms;         /* median time of the chosen candidate                       */
  double ms_default; /* median time of the built-in choice                        */
  int candidates;    /* candidates timed                                          */
} spdinv_tuning;

/*
 * Autotuner of the FP64 single-matrix form for order n (1 <= n <= 65536):
 * times schedules on a synthetic SPD matrix of order n (generated on the
 * device; the task DAG does not depend on the values), `reps` timed calls
 * each (median, HIP events on `stream`, after one untimed call), by
 * coordinate descent from the built-in choice over workgroups per CU {1, 2},
 * products per device task {6, 8, 12} and row parts of the split products
 * {whole, halves, quarters}.  The fastest becomes the library's choice for
 * every matrix of the same tile count, for the fields that callers leave at
 * 0 in spdinv_opts.  Allocates and frees its own device buffers (two n x n
 * matrices and the workspace) and synchronizes the stream.  Returns 0, -1
 * for an invalid n, or SPDINV_ERR_HIP.
 */
int spdinv_autotune(int n, int reps, spdinv_stream_t stream, spdinv_tuning* out);

/*
 * Autotuner of the batched form for a batch of these orders (as for
 * batched_spd_inverse) in mode SPDINV_FP64 or SPDINV_FP32: times the
 * schedules batch_group = -1, -2 and 512, each with chains of 1, 4 and 8
 * products, on synthetic SPD matrices of the same orders; the fastest
 * becomes the library's choice for batches with the same number of
 * matrices of each tile count.  Allocates and frees its own device buffers
 * and synchronizes the stream.  Returns 0, -i for an invalid i-th argument,
 * or SPDINV_ERR_HIP.
 */
int spdinv_autotune_batched(int batch, const int* h_n, spdinv_mode mode, int reps,
                            spdinv_stream_t stream, spdinv_tuning* out);

/* Forgets every tuned choice (the built-in choices apply again). */
int spdinv_tuning_clear(void);
/* Writes the tuned choices to a text file / adds those of a file written by
   spdinv_tuning_save.  Return 0, or a negative value when the file cannot
   be written or read or is malformed (nothing is added then). */
int spdinv_tuning_save(const char* path);
int spdinv_tuning_load(const char* path);

/* Frees every cached plan (device arena and host tables).  The host tables of
   spd_inverse_noalloc's plans are kept, since an upload from them may still
   be pending on a stream. */
void spdinv_release_plans(void);

/* ---- planner introspection (host only; no GPU needed) -------------------- */

typedef struct {
  long long tasks;
  long long edges;
  long long count[16];   /* tasks per kind, indexed by the SPDINV_TASK_* ids */
  int cp_step[3];        /* critical path of each step's own DAG (Table 1)   */
  int cp_unpipelined;    /* sum of the three                                  */
  int cp_plan;           /* critical path of the DAG the plan executes        */
} spdinv_plan_stats;

enum {
  SPDINV_TASK_NOP = 0, SPDINV_TASK_SYRK1 = 1, SPDINV_TASK_POTRF = 2, SPDINV_TASK_GEMM1 = 3,
  SPDINV_TASK_TRSM1 = 4, SPDINV_TASK_TRTRI = 5, SPDINV_TASK_TRMM2L = 6, SPDINV_TASK_GEMM2 = 7,
  SPDINV_TASK_TRSM2R = 8, SPDINV_TASK_TRMM3 = 9, SPDINV_TASK_LAUUM = 10, SPDINV_TASK_GEMM3 = 11,
  SPDINV_TASK_SYRK3 = 12, SPDINV_TASK_GEMMS = 13, SPDINV_TASK_TRSMS = 14,
  SPDINV_TASK_TADD = 15
};

/* Builds (without caching) the plan for t tiles per side and returns its
   statistics.  Returns 0, or -1 for t < 1 or t > 1024. */
int spdinv_plan_stats_get(int t, const spdinv_opts* opts, spdinv_plan_stats* out);

/*
 * Exports a plan for inspection: per task (program order) 8 int32 fields
 *   kind, out, a, b, copy, aux, succ_begin, succ_end
 * (tile indices into the pool layout: A tiles [0,T), B [T,2T), C [2T,3T),
 * inverted diagonal tiles [3T, 3T+t), T = t(t+1)/2, lower tile (i,j) at
 * i(i+1)/2+j; in the inverse's plan only the renamed rows of B and C are
 * stored, row after row, and the inverted diagonal tiles follow them: at T
 * in place, after the chosen rows with opts->rename_tiles), the successor
 * array, the step of each task, its packed paper
 * indices (i<<20 | j<<10 | k) and the device dispatch order.  With
 * opts->chain != 1 a product task may carry further links: bits 20-23 of
 * kind count them, aux indexes the first in `links` (int32 pairs: operand
 * tiles a, b).  With workers > 1 and opts->no_split == 0, bit 24 of kind
 * marks a row-part task: part p (bits 25-26) of the output tile's rows and
 * of its renaming copy, rows 64p..64p+63 of two halves, or rows
 * 32p..32p+31 of four quarters with bit 27; the parts of a product are
 * adjacent in program order and have the same predecessors and successors.
 * Pass NULL buffers to query the sizes (ntasks, nsucc, nlinks).  `workers`
 * sizes the list-scheduling simulation that produces the order.
 */
int spdinv_plan_export(int t, const spdinv_opts* opts, int workers, int32_t* tasks8,
                       int32_t* succ, int32_t* step, int32_t* idx, int32_t* order,
                       long long* ntasks, long long* nsucc, int32_t* links,
                       long long* nlinks);
/* The same for a plan of some steps of Algorithm 1: steps = 7 (the SPD
   inverse, as spdinv_plan_export), 1 (the plan of spd_cholesky), 6 (the
   plan of spd_inverse_from_factor), 9 (spd_solve: step 1, then the forward
   and backward substitutions) or 8 (spd_solve_from_factor), with rhs_tiles
   = ceil(nrhs/128) tile columns of right-hand sides (1..64) for 9 and 8 and
   0 otherwise.  Right-hand-side tile (i, c) is pool tile 3T + 2t + i + t c.
   Returns -2 for another combination. */
int spdinv_plan_export_steps(int steps, int rhs_tiles, int t, const spdinv_opts* opts,
                             int workers, int32_t* tasks8, int32_t* succ, int32_t* step,
                             int32_t* idx, int32_t* order, long long* ntasks, long long* nsucc,
                             int32_t* links, long long* nlinks);

/*
 * The batched form's task list for one matrix of t tiles per side (1 <= t <=
 * 16; t = 1 is the single small-matrix task): per position (the device id)
 * the 8 int32 fields of spdinv_plan_export, with the kinds 16 (copy-in:
 * lower triangle to the matrix's tiles), 17 (copy-out, writes INFO) and 18
 * (a matrix of order <= 128 inverted in LDS) besides the plan's; successors
 * are positions; links as for spdinv_plan_export.  Position 0 is the copy-in
 * task and the last position the copy-out task.  NULL buffers query the
 * sizes.  Returns 0, or a negative value for an invalid t, mode or opts.
 */
int spdinv_batch_template_export(int t, spdinv_mode mode, const spdinv_opts* opts,
                                 int32_t* tasks8, int32_t* succ, int32_t* links, long long* ntask,
                                 long long* nsucc, long long* nlinks);
/*
 * The batched form's dispatch order for the orders h_n (as batched_spd_inverse
 * builds it for a launch of `workers` workgroups): per ticket
 * (matrix << 12) | template position, and per matrix 4 int32 (its template
 * tile count, first counter index, first pool tile, 0).  NULL buffers query
 * the size.  Returns the number of tickets, or a negative value for invalid
 * arguments.
 */
long long spdinv_batch_plan_export(int batch, const int* h_n, spdinv_mode mode,
                                   const spdinv_opts* opts, int workers, int32_t* disp,
                                   int32_t* mat4);

/* ---- per-task trace (opts.trace = 1) -------------------------------------- */
/* Copies the per-task trace that the last spd_inverse call with
   opts->trace = 1 left in its workspace `work` (device) into `host`: 4 int64
   per task in plan order (worker, claim, start, end), the times in ticks of
   the device's constant 100 MHz real-time counter; start is the moment the
   task's dependencies were satisfied.  n and opts must be those of that call.
   Synchronous.  Returns the number of tasks copied (at most max_tasks) or a
   negative value on error. */
long long spdinv_trace_copy(const void* work, int n, const spdinv_opts* opts, int64_t* host,
                            long long max_tasks);

/* ---- kernel timing --------------------------------------------------------- */
/* enable != 0: from now on every spd_inverse call records a pair of HIP events
   on its stream immediately around the launch of the scheduler kernel (the
   kernel that executes every tile task).  enable = 0 stops recording.  Both
   discard what was recorded so far.  Returns 0. */
int spdinv_kernel_timer(int enable);
/* Waits for the recorded events, returns the summed scheduler-kernel time in
   milliseconds over the launches recorded since the last read (their count
   in *launches if non-NULL) and discards them.  Negative on a HIP error. */
double spdinv_kernel_timer_read(long long* launches);

/* Library version string. */
const char* spdinv_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPDINV_H */
