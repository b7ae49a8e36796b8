// Internal interface between the C-ABI layer (api.cpp) and the HIP kernels
// (device.hip).  Not part of the public header.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.hpp"

namespace spdinv {

constexpr int NB = 128;          // tile order
constexpr int NTHREADS = 256;    // threads per worker workgroup (4 wave64)

// Scheduler control block in the caller's workspace (int32 words).
enum Ctrl : int {
  CTRL_TICKET = 0,   // next dispatch ticket
  CTRL_INFO = 1,     // LAPACK-style INFO (0 = ok); min over failing pivots
  CTRL_ABORT = 2,    // set when a worker's dependency wait timed out
  CTRL_FAILED = 3,   // set once a diagonal factorization broke down
  CTRL_DONE = 4,     // tasks completed
  CTRL_WORDS = 16
};

// Task arrays on the device are in dispatch order: task id = ticket.
struct SchedArgs {
  const DevTask* tasks;
  const int32_t* succ;
  int32_t* indeg;      // mutable in-degree counters (reset before each run)
  int32_t* ctrl;       // Ctrl words
  double* pool;        // tile pool
  const int32_t* links;  // further links of chained products (or nullptr)
  int coherent_only;   // 1: ignore the planner's L2-cacheable read marks
  int last_valid;      // rows/columns of the last tile block inside the matrix
                       // (NB when n is a multiple of NB)
  long long* trace;    // 4 per task, or nullptr
  int ntask;
  int tiles_T;         // lower tiles per copy, T = t(t+1)/2 (pool layout)
  int tiles;           // tiles per side, t
  int info_base;       // offset added to the global pivot index in INFO
  long long spin_limit;  // longest dependency wait, in 100 MHz clock ticks
  int d_base;          // first inverted diagonal tile: D_j at d_base + j, D_j^T
                       // at d_base + tiles + j (3T unless renaming is partial)
};

// Batched form: the largest tile count per matrix (n <= 2048).
constexpr int MAX_BATCH_T = 16;

// Resets the in-degree counters and the control block (a fill kernel, so
// that the sequence stays capturable in a graph).
hipError_t launch_reset(const int32_t* indeg0, int32_t* indeg, int ntask, int32_t* ctrl,
                        hipStream_t s);

// ---- batched form as one DAG over the batch (bsched_loop.hpp) ----
// Task kinds that only the batched templates use (after the plan's kinds).
enum BatchKind : int32_t {
  K_BCOPYIN = 16,   // the matrix's lower triangle -> its A tiles (identity padding);
                    // checks its order and leading dimension first
  K_BCOPYOUT = 17,  // A tiles -> lower triangle of the matrix; writes its INFO
  K_BSMALL = 18     // a matrix of order <= NB inverted in LDS; writes its INFO
};
// Bit of BSchedArgs::mat[m].x: the copy-in task of matrix m waits for the
// copy-out task of the previous occupant of its pool slot.
constexpr int BM_PREV = 1 << 8;
constexpr int BM_T = 0xff;
// Dispatch entry: (matrix << BT_SHIFT) | template position.
constexpr int BT_SHIFT = 12;
constexpr int BT_MASK = (1 << BT_SHIFT) - 1;
constexpr int MAX_BATCH = (1 << (31 - BT_SHIFT)) - 1;

struct BSchedArgs {
  const int32_t* disp;                      // ticket -> matrix and template position
  const int4* mat;                          // per matrix: x = template tile count (1 for
                                            // n <= NB) | BM_PREV if the matrix's pool
                                            // slot had an earlier occupant; y = first
                                            // counter; z = first pool tile; w = counter
                                            // of the copy-in task of the slot's next
                                            // occupant, or -1
  const DevTask* tmpl[MAX_BATCH_T + 1];     // per tile count: template tasks
  const int32_t* tsucc[MAX_BATCH_T + 1];    // their successors (template positions)
  const int32_t* tlinks[MAX_BATCH_T + 1];   // their chained-product links
  const int32_t* tindeg0[MAX_BATCH_T + 1];  // their initial in-degrees
  int32_t* indeg;                           // counters, per (matrix, template task)
  int32_t* ctrl;                            // CTRL_WORDS: ticket, abort, done
  int32_t* mctrl;                           // CTRL_WORDS per matrix: INFO, FAILED
  void* pool;                               // tiles of every matrix (FP64 or FP32)
  const int* n;                             // device: orders
  void* const* A;                           // device: matrix pointers
  const int* lda;                           // device: leading dimensions
  int* info;                                // device INFO per matrix (or nullptr)
  int ntotal;                               // tickets
  int fill_upper;
  long long spin_limit;
  // One workgroup per matrix (seq = 1): a ticket is a matrix (disp holds
  // (m << BT_SHIFT) entries, largest matrices first), whose template tasks
  // the workgroup runs in template order on its own pool of wg_pool_tiles
  // tiles (reused by its next matrix); no counters.
  int seq;
  long long wg_pool_tiles;
  int tntask[MAX_BATCH_T + 1];              // tasks of each template
  int tdbase[MAX_BATCH_T + 1];              // first inverted diagonal tile of each
                                            // template's pool
};

// Resets the counters of a batch (from each template's initial in-degrees),
// the per-matrix INFO/FAILED words and the control words.
hipError_t launch_breset(const BSchedArgs& b, int batch, hipStream_t s);
// The FP64 batched scheduler (two workgroups per CU).
hipError_t launch_bsched(const BSchedArgs& b, int grid, hipStream_t s);
int bsched_blocks_per_cu();

// Column-major lower triangle of A -> A tiles of the pool, identity padding
// beyond n (the padded matrix is block diagonal with an identity block, whose
// inverse holds A^{-1} in its leading block).
hipError_t launch_copy_in(const double* A, int lda, int n, int t, double* pool, hipStream_t s);

// A tiles of the pool -> lower triangle of A (and its mirror if fill_upper).
hipError_t launch_copy_out(const double* pool, int t, double* A, int lda, int n, int fill_upper,
                           hipStream_t s);

// Copies ctrl[CTRL_INFO] to a device int (may be nullptr: no-op).
hipError_t launch_info_out(const int32_t* ctrl, int* d_info, hipStream_t s);

// Inverse from a given factor: the transposed copies B_ij = L_ij^T and the
// inverted diagonal tiles D_j, D_j^T that step 2 reads, from the factor's
// tiles in the pool (after copy-in).  Sets INFO on a zero diagonal entry.
hipError_t launch_factor_prologue(double* pool, int t, int32_t* ctrl, hipStream_t s);

// Right-hand sides of the solve: column-major B (n x nrhs, ldb) into the
// transposed tiles R (t x ceil(nrhs/128) tiles, tile i + t c holds R_ic^T,
// zero outside B) and back.
hipError_t launch_rhs_in(const double* B, int ldb, int n, int nrhs, int t, double* R,
                         hipStream_t s);
hipError_t launch_rhs_out(const double* R, int t, int n, int nrhs, double* B, int ldb,
                          hipStream_t s);

// Synthetic SPD matrices for timing runs (the autotuner): mats[m] (device
// pointers, column-major, ld = orders[m]) <- a_ij = 1/(1+|i-j|), a_ii = n.
hipError_t launch_fill_spd(void* const* mats, const int* orders, int count, bool fp32,
                           hipStream_t s);

// Writes 0 to a device int (nullptr: no-op), as a kernel so that the call
// can be captured in a graph.
hipError_t launch_info_zero(int* d_info, hipStream_t s);

// Device scratch of the allocation-free entry point: a file-scope device
// array, one per GPU, holding a plan's device tables (the first
// NOALLOC_PLAN_BYTES) and the workspace of an inversion of order up to
// NOALLOC_MAX_N (the pool of pool_tiles(16) = 440 tiles, then the in-degree
// counters and the control words).
constexpr int NOALLOC_MAX_N = 2048;
constexpr size_t NOALLOC_PLAN_BYTES = size_t(1) << 20;
constexpr size_t NOALLOC_WORK_BYTES = size_t(440) * NB * NB * sizeof(double) + (size_t(1) << 20);
constexpr size_t NOALLOC_SCRATCH_BYTES = NOALLOC_PLAN_BYTES + NOALLOC_WORK_BYTES;
// Device address of the current device's scratch (looked up once per device
// with that device current) and its size.
hipError_t noalloc_scratch(void** ptr, size_t* bytes);

// Persistent scheduler over the plan's tasks.
// per_cu: 1 keeps every workgroup alone on its CU, 2 lets two share one.
hipError_t launch_sched(const SchedArgs& a, int grid, int per_cu, hipStream_t s);

// Persistent workgroups per CU that fit for the scheduler kernel.
int sched_blocks_per_cu();

}  // namespace spdinv
