// Host-side planner for the tile SPD inverse.
//
// The paper (Section 2, Algorithm 1; Section 3) describes the inversion as a
// sequential stream of tile tasks that a dynamic scheduler unfolds into a DAG
// using read-after-write, write-after-read and write-after-write hazards.  The
// planner does exactly that on the host: it emits the task stream of the
// chosen variant in program order, each task with the tiles it reads and
// writes (named as in the paper: A_ij, the renaming copies B_ij and C_ij),
// derives every hazard edge, and computes critical paths and a priority order
// for the device scheduler.
//
// Variants (Section 3):
//   renamed     -- array renaming: the out-of-place variant where step 2 reads
//                  the copy B of L and step 3 reads the copy C of L^{-1}, so
//                  that the anti-dependences disappear.  Copies are fused into
//                  the task that produces the final tile (weight 0).
//   loop_order  -- loop reversal: UDU (the step-2 GEMM chain runs k downward)
//                  or UUU (all chains upward).
//   pipelined   -- one DAG over the three steps, or barriers between them.
//   trtri_first -- the step-2 reading with TRTRI(j) at the head of iteration j
//                  and the right multiplication by the inverted diagonal tile;
//                  the default is the LAPACK 3.2.1 order (right solve with the
//                  factor's diagonal tile, TRTRI(j) after column j).
//   chain       -- device task granularity (not a variant of the paper): up to
//                  `chain` consecutive products of one output tile's update
//                  chain run as one device task that keeps the tile in
//                  registers between them.  The products, their order and
//                  their operands are unchanged, so results are bit-identical
//                  to chain = 1 (one device task per task of the paper's
//                  stream); the statistics always describe the paper's DAG.
#pragma once
#include <cstdint>
#include <vector>

namespace spdinv {

// Task kinds.  The device executes each kind as one tile operation; see
// tile_tasks.hpp (run_task) for the arithmetic of each.
enum Kind : int32_t {
  K_NOP = 0,     // barrier between steps (no work, weight 0)
  K_SYRK1 = 1,   // A_jj -= A_jk A_jk^T
  K_POTRF = 2,   // A_jj <- chol(A_jj); also D_j <- inverse of the factor tile
  K_GEMM1 = 3,   // A_ij -= A_ik A_jk^T
  K_TRSM1 = 4,   // A_ij <- A_ij L_jj^{-T}
  K_TRTRI = 5,   // A_jj <- L_jj^{-1}
  K_TRMM2L = 6,  // A_ij <- X_ii A_ij
  K_GEMM2 = 7,   // A_ij += X_ik L_kj
  K_TRSM2R = 8,  // A_ij <- -A_ij L_jj^{-1}
  K_TRMM3 = 9,   // A_ij <- X_ii^T A_ij
  K_LAUUM = 10,  // A_ii <- A_ii^T A_ii
  K_GEMM3 = 11,  // A_ij += X_ki^T X_kj
  K_SYRK3 = 12,  // A_ii += X_ki^T X_ki
  K_GEMMS = 13,  // solve: R_ic -= L_ik R_kc (forward) or L_ki^T R_kc (backward)
  K_TRSMS = 14,  // solve: R_ic <- L_ii^{-1} R_ic = D_i R_ic (or D_i^T R_ic)
  K_TADD = 15,   // tree reduction of a step-2 update chain: A_ij += Z (a partial sum)
  K_COUNT = 16
};

struct PlanOptions {
  int t = 1;            // tiles per side
  int renamed = 1;
  int loop_order = 0;   // 0 = UDU, 1 = UUU
  int pipelined = 1;
  int trtri_first = 0;
  int chain = 1;        // most products per device task (1 <= chain <= MAX_CHAIN)
  // 1: the last product of an update chain (the one before the tile's
  // closing task) may join the chain too.  In a parallel DAG it runs alone,
  // as it waits for the most recently finished operand; a plan that one
  // workgroup runs in order (the batched form's per-matrix templates) has
  // every operand ready.
  int chain_tails = 0;
  // Steps of Algorithm 1 in the plan: bit 0 step 1 (Cholesky), bit 1 step 2
  // (inverse of the factor), bit 2 step 3 (the product L^-T L^-1).  7 = the
  // SPD inverse, 1 = the Cholesky factor only, 6 = the inverse from a given
  // factor (the caller provides what step 1 leaves for step 2: the
  // transposed copies B = L^T and the diagonal inverses D_j, D_j^T).
  // Bit 3: the solve A X = R with the factor (forward substitution with L,
  // then backward with L^T) over rhs_tiles tile columns of right-hand sides:
  // 9 = factor and solve, 8 = solve with a given factor (the same prologue
  // as 6).
  int steps = 7;
  int rhs_tiles = 0;
  // Split the products of the chains of dependent tasks into split (2 or 4)
  // row-part tasks (K_PART), 0 = none: TRSM(j+1, j) and the last SYRK into
  // tile (j+1, j+1), between POTRF(j) and POTRF(j+1), and in the solve each
  // multiplication by D_i or D_i^T with the last update before it.
  int split = 0;
  // Tree reduction of the step-2 update chains (associativity; the
  // conclusion's proposal): 0 = the paper's sequential chains; L = 1 or 2:
  // each chain A_ij += sum_k X_ik L_kj is cut into 2^L consecutive segments
  // (in the chain's order), accumulated side by side -- the first into A_ij,
  // the others into partial-sum tiles Z -- and the partial sums are added in
  // a fixed binary tree (K_TADD), so the result does not depend on the
  // schedule.  The 2^L - 1 partial-sum tiles of each lower tile follow the
  // pool's other regions.
  int tree_levels = 0;
  // Partial renaming (renamed = 1): per tile row i, ren_b[i] / ren_c[i] say
  // whether the tiles of row i have the renaming copy B (of L) / C (of
  // L^{-1}); rows without it are read in place, with the paper's
  // anti-dependences.  Empty = every row (full renaming).
  std::vector<char> ren_b, ren_c;
};
constexpr int MAX_CHAIN = 16;

// Copy tiles of the renaming rows: row i has i + 1 lower tiles.
int renamed_tiles(const PlanOptions& opt);

// Unit-weight critical path of the DAG of the options' steps (no chains, no
// row parts): the cost the renaming choice below minimizes.
int plan_critical_path(const PlanOptions& opt);

// Memory-constrained partial renaming: chooses the rows of B and C to rename
// under a budget of copy tiles (greedy: each round adds the row whose copy
// shortens the critical path most per tile; when no single row shortens it
// -- or beyond 16 tiles per side, where the candidates are not evaluated --
// the bottom C rows first, then the bottom B rows) and sets opt->ren_b /
// ren_c.  A budget of 2T or more is full renaming.
void choose_renaming(PlanOptions* opt, long long budget_tiles);

// Operation flags of a tile product, C (+)= +-op(A) op(B) (bits 8-15 of
// DevTask::kind).
enum ProductFlags : int32_t {
  F_TA = 1,       // op(A) = A^T
  F_TB = 2,       // op(B) = B^T
  F_MA = 4,       // A is lower triangular (entries above the diagonal ignored)
  F_MB = 8,       // B is lower triangular
  F_LOWER = 16,   // only output blocks on or below the diagonal are stored
  F_NEG = 32,     // C gets -op(A) op(B)
  F_ACC = 64,     // accumulate into C (else overwrite)
  F_COPYT = 128   // the copy destination receives the transposed result
};
// Bit 16 of DevTask::kind on a POTRF task: no task reads the factor tile
// (in place or as its renaming copy) -- the device uses the explicit inverse
// D_j instead -- so only D_j and D_j^T are stored.  The task keeps every
// hazard edge of the paper's DAG.
constexpr int32_t K_POTRF_FACTOR_DEAD = 1 << 16;
// Bit 29 of DevTask::kind on a POTRF task: no task reads D_j^T (the
// factor alone, whose TRSMs read D_j), so it is not stored.
constexpr int32_t K_POTRF_INVT_DEAD = 1 << 29;
// Bits 17/18 of DevTask::kind on a tile product: operand a / b may be read
// through the L2 cache (default cache policy) instead of the device-coherent
// policy.  The planner grants it only for tiles that are written exactly once
// in the plan and not accessed before that write (the renaming copies and the
// inverted diagonal tiles): their only version is read after it is written
// (RAW), so no L2 line of such a tile can hold anything else within a
// launch, and lines left by an earlier launch are invalidated at the kernel
// boundary.  (Device-coherent loads can leave lines in the reading XCD's L2,
// so a tile read in an earlier version is never read through the cache.)
constexpr int32_t K_NC_A = 1 << 17;
constexpr int32_t K_NC_B = 1 << 18;
// Bit 19 of DevTask::kind on a column-form product (op(A) = A, op(B) = B^T):
// the stored columns of its operands, i.e. its reduction index, are the last
// tile block.  When the order n is not a multiple of NB, that block is
// padded, and the device skips the k-panels past the valid extent: their
// products are exact zeros (padded rows of off-diagonal tiles are zero), or
// they only feed the padded diagonal block of the last diagonal tile, which
// no later task reads and copy-out does not write.  On a link entry the same
// mark is LINK_KLAST.
constexpr int32_t K_KLAST = 1 << 19;
constexpr int32_t LINK_KLAST = 1 << 30;
// Bits 20-23 of DevTask::kind on a tile product: number of further links of
// a chained task.  Link p (p = 1..count) multiplies the operand tiles
// links[2 (aux + p - 1)] and links[2 (aux + p - 1) + 1] (the same op and sign
// as the first link, always accumulating; the tile index of operand a may
// carry LINK_KLAST).  A chained task reads every operand device-coherent: it
// carries no K_NC_A / K_NC_B marks.
constexpr int K_LINKS_SHIFT = 20;
constexpr int32_t K_LINKS_MASK = 0xf << K_LINKS_SHIFT;
inline int task_links(int32_t k) { return (k & K_LINKS_MASK) >> K_LINKS_SHIFT; }
// Bit 24 of DevTask::kind on a single column-form product: a row-part task,
// which forms and stores only part idx (bits 25-26) of the output tile's
// rows (and their part of the renaming copy): rows 64 idx .. 64 idx + 63 of
// two halves, or with bit 27 rows 32 idx .. 32 idx + 31 of four quarters.
// The planner splits a product on a chain of dependent tasks (see
// PlanOptions::split) into its parts, so that several workgroups share it:
// every part takes the product's predecessors and every successor waits for
// all of them (the parts write disjoint rows; an in-place product reads only
// its own rows of the output tile).
constexpr int32_t K_PART = 1 << 24;
constexpr int K_PART_SHIFT = 25;
constexpr int32_t K_PARTS4 = 1 << 27;
// Bit 28: the task is near-critical (its slack in the dispatch cost model
// is under half a single product): its waves run at a raised issue
// priority, ahead of a co-resident workgroup's.  Scheduling only; results
// do not depend on it.
constexpr int32_t K_URGENT = 1 << 28;
inline int32_t task_kind(int32_t k) { return k & 0xff; }
inline int32_t task_flags(int32_t k) { return (k >> 8) & 0xff; }

// Device task descriptor (32 bytes).  Tile fields index the tile pool:
//   [0, T)          A tiles, T = t(t+1)/2, lower tile (i,j) at i(i+1)/2 + j
//   [T, 2T)         B tiles: the renaming copy of L, stored transposed
//                   (B_ij holds L_ij^T)
//   [2T, 3T)        C tiles: the renaming copy of L^{-1}, stored transposed
//   [3T, 3T+t)      D_j, inverse of the j-th diagonal factor tile (zeros above
//                   the diagonal)
//   [3T+t, 3T+2t)   D_j^T
// In the inverse's plan (steps 7) only the renamed rows of B and C are
// stored, row after row, and D, D^T follow them (Plan::d_base): the layout
// above with full renaming, D at T in place, in between with partial
// renaming.  The partial plans keep the layout above.
// Storing the copies transposed lets every product of the renamed plan read
// both operands along contiguous columns (op(A) = A, op(B) = B^T).
struct DevTask {
  int32_t kind;  // task kind (bits 0-7) | product flags (bits 8-15)
  int32_t out;   // tile updated in place
  int32_t a;     // first operand tile (or -1)
  int32_t b;     // second operand tile (or -1)
  int32_t copy;  // renaming destination that receives the same result (or -1)
  int32_t aux;   // POTRF: D_j (D_j^T follows t tiles later); chained
                 // product: index of its first further link; else -1
  int32_t succ_begin;
  int32_t succ_end;
};

struct PlanStats {
  int64_t ntasks;
  int64_t nedges;
  int64_t count[K_COUNT];
  int cp_step[3];        // critical path of each step's DAG alone (tasks)
  int cp_unpipelined;    // sum of the step critical paths
  int cp_pipelined;      // critical path of the single DAG over all steps
  int cp_plan;           // critical path of the DAG this plan executes
};

struct Plan {
  PlanOptions opt;
  int T = 0;                       // lower tiles per copy
  int d_base = 0;                  // first inverted diagonal tile (D_j at d_base + j,
                                   // D_j^T at d_base + t + j); 3T with full renaming
  int64_t pool_tiles = 0;          // tiles of the pool this plan addresses
  std::vector<DevTask> tasks;      // program order
  std::vector<int32_t> step;       // step (1..3, 0 for barriers) per task
  std::vector<int32_t> idx;        // packed (i,j,k) paper indices, 10 bits each
  std::vector<int32_t> succ;       // CSR successor lists (by task)
  std::vector<int32_t> indeg;      // initial in-degree per task
  std::vector<int32_t> order;      // device dispatch order (topological)
  std::vector<int32_t> links;      // further links of chained tasks (pairs)
  PlanStats stats{};               // of the paper's DAG (before chaining)
};

// Builds the plan.  `workers` and `cost` drive the list-scheduling simulation
// that orders the dispatch list (cost[kind] = estimated duration of a task of
// that kind, any unit; cost[K_COUNT] = duration of each further link of a
// chained product; cost[K_COUNT + 1] = a row half's fraction of its
// product's duration (a quarter: 0.75 of that); null = unit durations, a
// part 1/split).
void build_plan(const PlanOptions& opt, int workers, const double* cost, Plan* out);

// Tile pool size in tiles for t tiles per side (and s tile columns of
// right-hand sides, after the other regions: R_ic at 3T + 2t + i + t c).
inline int64_t pool_tiles(int t, int s);
inline int64_t pool_tiles(int t) {
  int64_t T = (int64_t)t * (t + 1) / 2;
  return 3 * T + 2 * (int64_t)t;
}
inline int64_t pool_tiles(int t, int s) { return pool_tiles(t) + (int64_t)t * s; }

}  // namespace spdinv
