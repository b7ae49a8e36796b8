// C-ABI of the spdinv library: argument checking, plan cache, workspace
// layout and the launch sequence of one inversion.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <queue>
#include <tuple>
#include <vector>

#include "dense.hpp"
#include "device.hpp"
#include "mixed.hpp"
#include "plan.hpp"
#include "spdinv.h"

using namespace spdinv;

namespace {

// Relative durations of the task kinds, used only to order the dispatch list
// (list-scheduling simulation); a single 128^3 tile product task is the unit.
// Measured per-task times at n = 8192 on MI355X: product 25.5 us, POTRF
// (factor + inverse of the factor tile) 63 us, TRTRI copy 8.5 us, each further
// link of a chained product 19.5 us (the next-to-last entry); a row half of
// a split product, as a fraction of the whole product (the last entry).
const double kCost[K_COUNT + 2] = {
    0.0,    // NOP
    1.0,    // SYRK1
    2.47,   // POTRF
    1.0,    // GEMM1
    0.96,   // TRSM1
    0.33,   // TRTRI (copy)
    1.0,    // TRMM2L
    1.0,    // GEMM2
    0.96,   // TRSM2R
    1.0,    // TRMM3
    1.0,    // LAUUM
    1.0,    // GEMM3
    1.0,    // SYRK3
    1.2,    // GEMMS (solve update; general product, untransposed operand)
    1.2,    // TRSMS (solve: multiplication by D_i or D_i^T)
    0.15,   // TADD (a partial sum of a tree-reduced chain added to its tile)
    0.76,   // each further link of a chained product
    0.6,    // a row half of a split product (fraction of the product)
};

// Products per device task of the FP64 scheduler when opts.chain is 0.
constexpr int kDefaultChain = 8;

struct Key {
  int device, t, renamed, loop_order, pipelined, trtri_first, workers, chain, steps, rhs, split;
  long long rename;  // copy-tile budget of a partial renaming, 0 = full
  int tree;          // tree-reduction levels of the step-2 chains
  bool operator<(const Key& o) const {
    return std::tie(device, t, renamed, loop_order, pipelined, trtri_first, workers, chain, steps,
                    rhs, split, rename, tree) <
           std::tie(o.device, o.t, o.renamed, o.loop_order, o.pipelined, o.trtri_first, o.workers,
                    o.chain, o.steps, o.rhs, o.split, o.rename, o.tree);
  }
};

// The device tables of a plan as one host image (tasks in dispatch order,
// CSR successors by dispatch position, initial in-degrees, chain links), at
// 256-byte aligned offsets, ready to be copied to device memory as a whole.
struct PlanImage {
  std::vector<char> bytes;
  size_t o_tasks = 0, o_succ = 0, o_indeg = 0, o_links = 0;
  bool has_links = false;
};

struct DevPlan {
  Plan host;
  PlanImage image;
  void* arena = nullptr;
  DevTask* d_tasks = nullptr;  // dispatch order
  int32_t* d_succ = nullptr;
  int32_t* d_indeg0 = nullptr;
  int32_t* d_links = nullptr;  // further links of chained tasks (or null)
};

std::mutex g_mu;
std::map<Key, std::unique_ptr<DevPlan>> g_plans;
std::map<int, int> g_grid;  // device -> compute units

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

spdinv_opts defaults() {
  spdinv_opts o;
  std::memset(&o, 0, sizeof(o));
  o.nb = 0;
  o.pipelined = 1;
  o.renamed = 1;
  o.loop_order = 0;
  o.trtri_first = 0;
  o.workers = 0;
  o.fill_upper = 0;
  o.trace = 0;
  o.max_refine = 0;
  o.refine_tol = 0.0;
  o.chain = 0;
  o.per_cu = 0;
  o.no_split = 0;
  o.parts = 0;
  o.batch_group = 0;
  o.rename_tiles = 0;
  o.tree_levels = 0;
  o.correction64 = 0;
  return o;
}

int chain_for(const spdinv_opts& o) { return o.chain > 0 ? o.chain : kDefaultChain; }

int tiles_for(int n) { return (n + NB - 1) / NB; }

// Device tasks of a plan at most, for t tiles per side and s tile columns of
// right-hand sides: the paper's tasks of the three steps, two barriers, the
// solve's (t (t+1) s <= 2 t^2 s), the further row parts of split products
// (at most 3 each, for at most 2t products of step 1 and 4ts of the solve),
// and with a tree reduction of `tree` levels at most 2^tree - 1 tile
// additions per off-diagonal tile.
long long task_count(int t, int s = 0, int tree = 0) {
  const long long tt = t, ss = s;
  return 3 * (tt * (tt - 1) * (tt - 2) / 6) + 6 * (tt * (tt - 1) / 2) + 3 * tt + 2 +
         2 * tt * tt * ss + 3 * (2 * tt + 4 * tt * ss) +
         (tree > 0 ? ((1LL << tree) - 1) * (tt * (tt - 1) / 2) : 0);
}

// Tree-reduction levels of the step-2 chains for these options: plans that
// contain step 2 (the inverse and the inverse from a factor).
int tree_for(const spdinv_opts& o, int steps) { return (steps & 2) ? o.tree_levels : 0; }

// Copy-tile budget of a partial renaming for these options (0 = full
// renaming): only the inverse (steps 7) of a renamed plan whose budget is
// below the 2T tiles of full renaming.
long long rename_budget(int t, const spdinv_opts& o, int steps) {
  if (!o.renamed || o.rename_tiles <= 0 || steps != 7) return 0;
  return (long long)o.rename_tiles >= (long long)t * (t + 1) ? 0 : o.rename_tiles;
}

// The renamed rows chosen under a budget (cached per variant).
struct RenRows {
  std::vector<char> b, c;
  int copy_tiles = 0;
};
std::mutex g_ren_mu;
std::map<std::tuple<int, int, int, int, long long>, RenRows> g_ren;

const RenRows& renaming_rows(int t, const spdinv_opts& o, long long budget) {
  std::lock_guard<std::mutex> lk(g_ren_mu);
  const auto k = std::make_tuple(t, o.loop_order, o.trtri_first ? 1 : 0, o.pipelined ? 1 : 0,
                                 budget);
  auto it = g_ren.find(k);
  if (it != g_ren.end()) return it->second;
  PlanOptions po;
  po.t = t;
  po.renamed = 1;
  po.loop_order = o.loop_order;
  po.pipelined = o.pipelined ? 1 : 0;
  po.trtri_first = o.trtri_first ? 1 : 0;
  choose_renaming(&po, budget);
  RenRows r;
  r.b = po.ren_b;
  r.c = po.ren_c;
  r.copy_tiles = renamed_tiles(po);
  return g_ren.emplace(k, std::move(r)).first->second;
}

// Tiles of the pool of a plan: A, the stored copy rows, D and D^T, and the
// right-hand sides.
long long pool_tiles_for(int t, const spdinv_opts& o, int steps, int s) {
  const long long T = (long long)t * (t + 1) / 2;
  const int tree = tree_for(o, steps);
  const long long z = tree ? T * ((1LL << tree) - 1) : 0;  // partial sums, after the rest
  if (steps != 7) return pool_tiles(t, s) + z;  // the standard layout of the partial plans
  if (!o.renamed) return T + 2LL * t + z;       // in place: no copies
  const long long budget = rename_budget(t, o, steps);
  if (!budget) return pool_tiles(t, s) + z;
  return T + renaming_rows(t, o, budget).copy_tiles + 2LL * t + (long long)t * s + z;
}

struct Layout {
  size_t pool, indeg, ctrl, trace, total;
};

Layout layout(int n, const spdinv_opts& o, int nrhs = 0, int steps = 7) {
  Layout L;
  const int t = tiles_for(n);
  const int s = (nrhs + NB - 1) / NB;
  const long long nt = task_count(t, s, tree_for(o, steps));
  L.pool = 0;
  L.indeg = align_up((size_t)pool_tiles_for(t, o, steps, s) * NB * NB * sizeof(double), 256);
  L.ctrl = L.indeg + align_up((size_t)nt * sizeof(int32_t), 256);
  L.trace = L.ctrl + align_up(CTRL_WORDS * sizeof(int32_t), 256);
  L.total = L.trace + (o.trace ? align_up((size_t)nt * 4 * sizeof(long long), 256) : 0);
  return L;
}

int check_opts(const spdinv_opts& o) {
  if (o.nb != 0 && o.nb != NB) return 1;
  if (o.loop_order < 0 || o.loop_order > 1) return 1;
  if (o.workers < 0) return 1;
  if (o.chain < 0 || o.chain > MAX_CHAIN) return 1;
  if (o.per_cu < 0 || o.per_cu > 2) return 1;
  if (o.no_split < 0 || o.no_split > 1) return 1;
  if (o.parts != 0 && o.parts != 2 && o.parts != 4) return 1;
  if (o.batch_group < -2) return 1;
  if (o.rename_tiles < 0) return 1;
  if (o.tree_levels < 0 || o.tree_levels > 2) return 1;
  if (o.correction64 < 0 || o.correction64 > 1) return 1;
  return 0;
}


// Persistent workgroups per CU for an order of t tiles.  The scheduler's
// kernel fits two on a CU, which pays only where the DAG keeps twice as many
// tasks ready.  Measured against one per CU: 30% slower at 64 tiles per
// side (workers wait for dependencies while the busy ones share CUs), 5%
// slower at 80, 11% faster at 96, 14% at 112, 4-8% at 128.
constexpr int kWideTiles = 96;

// Row-part split of the products on chains of dependent tasks: only with
// several workers (the parts then run side by side) and unless the caller
// turned it off.
// Four row parts per product below kWideTiles tiles per side, two from there
// (measured at n = 8192: quarters made the Cholesky factor 6 % and the solve
// 7 % faster than halves, the inverse the same; at n = 16384, with two
// workgroups per CU, the inverse was 3 % slower with quarters).
int split_for(const spdinv_opts& o, int t, int workers) {
  if (o.no_split || workers <= 1) return 0;
  if (o.parts) return o.parts;
  return t < kWideTiles ? 4 : 2;
}

int per_cu_for(int t, const spdinv_opts& o) {
  static int capacity = 0;  // workgroups per CU that fit (same for every device here)
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!capacity) capacity = sched_blocks_per_cu();
  }
  const int want = o.per_cu ? o.per_cu : (t >= kWideTiles ? 2 : 1);
  return want < capacity ? want : capacity;
}

int grid_for(int device, int t, const spdinv_opts& o) {
  int cus;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_grid.find(device);
    if (it != g_grid.end()) {
      cus = it->second;
    } else {
      cus = 0;
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
          cus <= 0)
        cus = 1;
      g_grid[device] = cus;
    }
  }
  int g = cus * per_cu_for(t, o);
  if (o.workers > 0 && o.workers < g) g = o.workers;
  return g;
}

// ---- tuning tables (filled by spdinv_autotune*, read by the entry points) ---
// FP64 single-matrix form, per tile count: the schedule that the autotuner
// measured fastest.  Entry points apply it to every field the caller left at
// 0 (library choice).
struct TunedFp64 {
  int per_cu, chain, split;  // split: 0 = whole products, 2 = halves, 4 = quarters
};
std::map<int, TunedFp64> g_tuned64;

// Batched form, per (precision, count of matrices of each tile count).
struct TunedBatch {
  int group, chain;
};
typedef std::pair<int, std::vector<int>> TBKey;
std::map<TBKey, TunedBatch> g_tuned_batch;

// o with the library-choice fields of the FP64 form at t tiles per side
// resolved from the tuning table (fields without an entry keep 0, the
// built-in choice).
spdinv_opts tuned_fp64(const spdinv_opts& o, int t) {
  spdinv_opts r = o;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_tuned64.find(t);
  if (it == g_tuned64.end()) return r;
  if (r.per_cu == 0) r.per_cu = it->second.per_cu;
  if (r.chain == 0) r.chain = it->second.chain;
  if (r.parts == 0 && !r.no_split) {
    if (it->second.split == 0) r.no_split = 1;
    else r.parts = it->second.split;
  }
  return r;
}

TBKey batch_key(bool fp32, const int* h_n, int batch) {
  std::vector<int> counts(MAX_BATCH_T + 1, 0);
  for (int i = 0; i < batch; ++i) {
    const int n = h_n[i];
    const int t = n <= NB ? 1 : (n + NB - 1) / NB;
    if (t >= 1 && t <= MAX_BATCH_T) ++counts[t];
  }
  return TBKey(fp32 ? 1 : 0, counts);
}

// The batched form's options with batch_group and chain resolved from the
// tuning table when the caller left them at 0.
spdinv_opts tuned_batch(const spdinv_opts& o, bool fp32, const int* h_n, int batch) {
  spdinv_opts r = o;
  if (r.batch_group != 0 && r.chain != 0) return r;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_tuned_batch.find(batch_key(fp32, h_n, batch));
  if (it == g_tuned_batch.end()) return r;
  if (r.batch_group == 0) r.batch_group = it->second.group;
  if (r.chain == 0) r.chain = it->second.chain;
  return r;
}

// Device-table image of a built plan: the task list permuted into dispatch
// order (a task's id on the device is its dispatch ticket), successors
// renumbered to dispatch positions.
void make_image(const Plan& p, PlanImage* im) {
  const size_t nt = p.tasks.size();
  std::vector<int32_t> pos(nt);
  for (size_t k = 0; k < nt; ++k) pos[p.order[k]] = (int32_t)k;
  std::vector<DevTask> dtask(nt);
  std::vector<int32_t> dsucc;
  dsucc.reserve(p.succ.size());
  std::vector<int32_t> dindeg(nt);
  for (size_t k = 0; k < nt; ++k) {
    const int v = p.order[k];
    DevTask d = p.tasks[v];
    const int b = (int)dsucc.size();
    for (int e = d.succ_begin; e < d.succ_end; ++e) dsucc.push_back(pos[p.succ[e]]);
    d.succ_begin = b;
    d.succ_end = (int)dsucc.size();
    dtask[k] = d;
    dindeg[k] = p.indeg[v];
  }
  im->o_tasks = 0;
  im->o_succ = align_up(im->o_tasks + nt * sizeof(DevTask), 256);
  im->o_indeg = align_up(im->o_succ + dsucc.size() * sizeof(int32_t) + 4, 256);
  im->o_links = align_up(im->o_indeg + nt * sizeof(int32_t), 256);
  const size_t bytes = align_up(im->o_links + p.links.size() * sizeof(int32_t) + 4, 256);
  im->bytes.assign(bytes, 0);
  char* h = im->bytes.data();
  std::memcpy(h + im->o_tasks, dtask.data(), nt * sizeof(DevTask));
  if (!dsucc.empty()) std::memcpy(h + im->o_succ, dsucc.data(), dsucc.size() * sizeof(int32_t));
  std::memcpy(h + im->o_indeg, dindeg.data(), nt * sizeof(int32_t));
  if (!p.links.empty())
    std::memcpy(h + im->o_links, p.links.data(), p.links.size() * sizeof(int32_t));
  im->has_links = !p.links.empty();
}

// Points the device-table pointers of dp into `base`, where its image lives.
void bind_tables(DevPlan* dp, char* base) {
  dp->d_tasks = (DevTask*)(base + dp->image.o_tasks);
  dp->d_succ = (int32_t*)(base + dp->image.o_succ);
  dp->d_indeg0 = (int32_t*)(base + dp->image.o_indeg);
  dp->d_links = dp->image.has_links ? (int32_t*)(base + dp->image.o_links) : nullptr;
}

Key plan_key(int device, int t, const spdinv_opts& o, int workers, int chain, int steps,
             int rhs_tiles, bool allow_split) {
  return Key{device, t, o.renamed ? 1 : 0, o.loop_order, o.pipelined ? 1 : 0,
             o.trtri_first ? 1 : 0, workers, chain, steps, rhs_tiles,
             allow_split ? split_for(o, t, workers) : 0, rename_budget(t, o, steps),
             tree_for(o, steps)};
}

std::unique_ptr<DevPlan> build_dev_plan(const Key& k) {
  std::unique_ptr<DevPlan> dp(new DevPlan);
  PlanOptions po;
  po.t = k.t;
  po.renamed = k.renamed;
  po.loop_order = k.loop_order;
  po.pipelined = k.pipelined;
  po.trtri_first = k.trtri_first;
  po.chain = k.chain;
  po.steps = k.steps;
  po.rhs_tiles = k.rhs;
  po.split = k.split;
  po.tree_levels = k.tree;
  if (k.rename) {
    spdinv_opts o = defaults();
    o.loop_order = k.loop_order;
    o.trtri_first = k.trtri_first;
    o.pipelined = k.pipelined;
    const RenRows& r = renaming_rows(k.t, o, k.rename);
    po.ren_b = r.b;
    po.ren_c = r.c;
  }
  build_plan(po, k.workers, kCost, &dp->host);
  make_image(dp->host, &dp->image);
  return dp;
}

// The plan for t tiles per side, built once per (device, variant, workers,
// chain, split) and kept with its device copy in a library-owned arena.
// chain: most products per device task (1 for executors that run the
// paper's tasks one by one).  allow_split: the executor runs row-half tasks
// (the FP64 scheduler).
DevPlan* get_plan(int device, int t, const spdinv_opts& o, int workers, int chain,
                  hipError_t* err, int steps = 7, int rhs_tiles = 0, bool allow_split = false) {
  const Key k = plan_key(device, t, o, workers, chain, steps, rhs_tiles, allow_split);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_plans.find(k);
  if (it != g_plans.end()) return it->second.get();
  std::unique_ptr<DevPlan> dp = build_dev_plan(k);
  const size_t bytes = dp->image.bytes.size();
  void* arena = nullptr;
  *err = hipMalloc(&arena, bytes);
  if (*err != hipSuccess) return nullptr;
  *err = hipMemcpy(arena, dp->image.bytes.data(), bytes, hipMemcpyHostToDevice);
  if (*err != hipSuccess) {
    (void)hipFree(arena);
    return nullptr;
  }
  dp->arena = arena;
  bind_tables(dp.get(), (char*)arena);
  DevPlan* raw = dp.get();
  g_plans[k] = std::move(dp);
  return raw;
}

// Optional timing of the scheduler kernel: a pair of HIP events recorded on
// the caller's stream around each scheduler launch.
struct KernelTimer {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  size_t used = 0;
};
KernelTimer g_timer;

bool timer_pair(hipEvent_t* a, hipEvent_t* b) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_timer.on) return false;
  if (g_timer.used == g_timer.ev.size()) {
    hipEvent_t x, y;
    if (hipEventCreate(&x) != hipSuccess) return false;
    if (hipEventCreate(&y) != hipSuccess) return false;
    g_timer.ev.push_back({x, y});
  }
  *a = g_timer.ev[g_timer.used].first;
  *b = g_timer.ev[g_timer.used].second;
  g_timer.used++;
  return true;
}

long long spin_limit() {
  const char* e = std::getenv("SPDINV_SPIN_LIMIT");
  if (e && *e) {
    long long v = std::atoll(e);
    if (v > 0) return v;
  }
  return 2000000000LL;  // 20 s
}

// The FP64 path: copy-in, the persistent scheduler over the plan (the steps
// of Algorithm 1 selected by `steps`), copy-out.  For the inverse from a
// given factor (steps 2 and 3) a prologue kernel first makes what step 1
// would leave for step 2.
// `given`: the plan with its device tables already in place (the
// allocation-free entry point); null = the cached plan in its arena.
int run_fp64(int n, double* A, int lda, void* work, size_t work_bytes, hipStream_t stream,
             const spdinv_opts& o_in, int* d_info, spdinv_report* report, int steps = 7,
             int nrhs = 0, double* Bm = nullptr, int ldb = 1, DevPlan* given = nullptr) {
  const spdinv_opts o = tuned_fp64(o_in, tiles_for(n));
  const Layout L = layout(n, o, nrhs, steps);
  const int s = (nrhs + NB - 1) / NB;
  if (work_bytes < L.total) return SPDINV_ERR_WORKSPACE;

  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return SPDINV_ERR_HIP;
  const int t = tiles_for(n);
  const int grid = grid_for(device, t, o);
  hipError_t err = hipSuccess;
  DevPlan* dp = given ? given : get_plan(device, t, o, grid, chain_for(o), &err, steps, s, true);
  if (!dp) return SPDINV_ERR_HIP;
  const int ntask = (int)dp->host.tasks.size();
  // the in-degree counters fill the region sized for the bound
  if ((size_t)ntask * sizeof(int32_t) > L.ctrl - L.indeg) return SPDINV_ERR_WORKSPACE;

  char* w = (char*)work;
  double* pool = (double*)(w + L.pool);
  int32_t* indeg = (int32_t*)(w + L.indeg);
  int32_t* ctrl = (int32_t*)(w + L.ctrl);
  long long* trace = o.trace ? (long long*)(w + L.trace) : nullptr;

  if (launch_reset(dp->d_indeg0, indeg, ntask, ctrl, stream) != hipSuccess) return SPDINV_ERR_HIP;
  if (launch_copy_in(A, lda, n, t, pool, stream) != hipSuccess) return SPDINV_ERR_HIP;
  if ((steps == 6 || steps == 8) && launch_factor_prologue(pool, t, ctrl, stream) != hipSuccess)
    return SPDINV_ERR_HIP;
  double* rhs = pool + (size_t)(dp->host.d_base + 2 * t) * NB * NB;  // R tiles, after D and D^T
  if (s && launch_rhs_in(Bm, ldb, n, nrhs, t, rhs, stream) != hipSuccess) return SPDINV_ERR_HIP;
  SchedArgs a;
  a.tasks = dp->d_tasks;
  a.succ = dp->d_succ;
  a.indeg = indeg;
  a.ctrl = ctrl;
  a.pool = pool;
  a.links = dp->d_links;
  a.coherent_only = 0;
  a.last_valid = n - (t - 1) * NB;
  a.trace = trace;
  a.ntask = ntask;
  a.tiles_T = t * (t + 1) / 2;
  a.tiles = t;
  a.info_base = 0;
  a.spin_limit = spin_limit();
  a.d_base = dp->host.d_base;
  hipEvent_t ev0, ev1;
  const bool timed = !given && timer_pair(&ev0, &ev1);
  if (timed && hipEventRecord(ev0, stream) != hipSuccess) return SPDINV_ERR_HIP;
  if (launch_sched(a, grid, per_cu_for(t, o), stream) != hipSuccess) return SPDINV_ERR_HIP;
  if (timed && hipEventRecord(ev1, stream) != hipSuccess) return SPDINV_ERR_HIP;
  // the factor leaves the strictly upper triangle untouched; a given factor
  // (the solve with it) is not written back
  if (steps != 8 &&
      launch_copy_out(pool, t, A, lda, n, (steps & 1) && !(steps & 2) ? 0 : o.fill_upper,
                      stream) != hipSuccess)
    return SPDINV_ERR_HIP;
  if (s && launch_rhs_out(rhs, t, n, nrhs, Bm, ldb, stream) != hipSuccess) return SPDINV_ERR_HIP;
  if (launch_info_out(ctrl, d_info, stream) != hipSuccess) return SPDINV_ERR_HIP;

  if (report) {
    if (hipStreamSynchronize(stream) != hipSuccess) return SPDINV_ERR_HIP;
    int32_t c[CTRL_WORDS];
    if (hipMemcpy(c, ctrl, sizeof(c), hipMemcpyDeviceToHost) != hipSuccess) return SPDINV_ERR_HIP;
    report->info = (c[CTRL_INFO] == INT_MAX) ? 0 : c[CTRL_INFO];
    report->status = c[CTRL_ABORT] ? SPDINV_ERR_TIMEOUT : 0;
    report->nb = NB;
    report->tiles = t;
    report->tasks = c[CTRL_DONE];
    report->critical_path = dp->host.stats.cp_plan;
    report->workers = grid;
    if (c[CTRL_ABORT]) return SPDINV_ERR_TIMEOUT;
  }
  return 0;
}

}  // extern "C"

namespace {

// ---- batched backward --------------------------------------------------------
// Per matrix of t = ceil(n/NB) tiles: 4 t^2 workspace tiles and 1 + t + t^2
// counters; tasks in phase order (all packs, all W tiles, all lower gradient
// tiles, all output tiles), the matrices of each phase largest first.
struct BBackComp {
  void* arena = nullptr;
  const int2* d_task = nullptr;
  const int4* d_mat = nullptr;
  int ntask = 0;
  long long tiles = 0, ncnt = 0;
};
std::map<std::pair<int, std::vector<int8_t>>, std::unique_ptr<BBackComp>> g_bbcomp;

void bback_sizes(int batch, const int* h_n, long long* tiles, long long* ncnt) {
  *tiles = 0;
  *ncnt = 0;
  for (int i = 0; i < batch; ++i) {
    const long long t = tiles_for(h_n[i]);
    *tiles += 4 * t * t;
    *ncnt += t ? 1 + t + t * t : 0;
  }
}

size_t bback_bytes(long long tiles, long long ncnt) {
  return 256 + align_up((size_t)ncnt * sizeof(int32_t), 256) + (size_t)tiles * NB * NB * sizeof(double);
}

BBackComp* get_bbcomp(int device, int batch, const int* h_n, hipError_t* err) {
  std::vector<int8_t> tv(batch);
  for (int i = 0; i < batch; ++i) tv[i] = (int8_t)tiles_for(h_n[i]);
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(device, tv);
  auto it = g_bbcomp.find(key);
  if (it != g_bbcomp.end()) return it->second.get();
  std::vector<int> order;
  for (int t = MAX_BATCH_T; t >= 1; --t)
    for (int i = 0; i < batch; ++i)
      if (tv[i] == t) order.push_back(i);
  std::vector<int4> mat(batch, make_int4(0, 0, 0, 0));
  long long tb = 0, cb = 0;
  for (int m : order) {
    const int t = tv[m];
    mat[m] = make_int4(t, (int)tb, (int)cb, 0);
    tb += 4LL * t * t;
    cb += 1 + t + t * t;
  }
  if (tb > INT_MAX || cb > INT_MAX) {
    *err = hipErrorInvalidValue;
    return nullptr;
  }
  std::vector<int2> task;
  for (int phase = 0; phase < 4; ++phase)
    for (int m : order) {
      const int t = tv[m];
      for (int j = 0; j < t; ++j)
        for (int i = 0; i < t; ++i)
          if (phase != 2 || i >= j) task.push_back(make_int2(m, (phase << BB_PHASE_SHIFT) | (i << 8) | j));
    }
  std::unique_ptr<BBackComp> bc(new BBackComp);
  const size_t o_mat = align_up(task.size() * sizeof(int2), 256);
  const size_t bytes = align_up(o_mat + (size_t)batch * sizeof(int4), 256);
  std::vector<char> img(bytes, 0);
  if (!task.empty()) std::memcpy(img.data(), task.data(), task.size() * sizeof(int2));
  std::memcpy(img.data() + o_mat, mat.data(), (size_t)batch * sizeof(int4));
  void* arena = nullptr;
  *err = hipMalloc(&arena, bytes);
  if (*err != hipSuccess) return nullptr;
  *err = hipMemcpy(arena, img.data(), bytes, hipMemcpyHostToDevice);
  if (*err != hipSuccess) {
    (void)hipFree(arena);
    return nullptr;
  }
  bc->arena = arena;
  bc->d_task = (const int2*)arena;
  bc->d_mat = (const int4*)((char*)arena + o_mat);
  bc->ntask = (int)task.size();
  bc->tiles = tb;
  bc->ncnt = cb;
  BBackComp* raw = bc.get();
  g_bbcomp[key] = std::move(bc);
  return raw;
}

// ---- batched form: one DAG over the batch ---------------------------------
// Task template of one matrix of t tiles per side: the plan of Algorithm 1
// in dispatch order, preceded by its copy-in task (an edge to every task
// without predecessors) and followed by its copy-out task (an edge from every
// task without successors); for t = 1 a single small-matrix task.  Positions
// in the template are the device ids; successors are positions.  The host
// part (image, durations, bottom levels) is built once per variant; its
// device copy once per device.
struct BTemplate {
  int ntask = 0;
  int d_base = 0;  // first inverted diagonal tile of the plan's pool
  PlanImage image;
  std::vector<double> cost;     // estimated duration per position (product units)
  std::vector<double> bottom;   // longest cost path from each position to the end
  std::vector<int32_t> succ;    // successors (positions), CSR by the tasks' fields
  std::vector<DevTask> tasks;   // host copy of the tasks
  std::vector<int32_t> indeg0;  // initial in-degrees
  std::vector<int32_t> links;   // chained-product links
};

struct BTemplateDev {
  const BTemplate* h = nullptr;
  void* arena = nullptr;
  const DevTask* d_tasks = nullptr;
  const int32_t* d_succ = nullptr;
  const int32_t* d_indeg0 = nullptr;
  const int32_t* d_links = nullptr;
};

void make_btemplate(const Plan* p, BTemplate* bt) {
  std::vector<DevTask> tasks;
  std::vector<std::vector<int32_t>> succ;
  std::vector<int32_t> indeg;
  auto special = [](int32_t kind) { return DevTask{kind, -1, -1, -1, -1, -1, 0, 0}; };
  if (!p) {
    tasks.push_back(special(K_BSMALL));
    succ.resize(1);
    indeg.assign(1, 0);
  } else {
    const int nt = (int)p->tasks.size(), N = nt + 2;
    std::vector<int32_t> pos(nt);
    for (int k = 0; k < nt; ++k) pos[p->order[k]] = k + 1;
    tasks.assign(N, special(K_NOP));
    succ.resize(N);
    indeg.assign(N, 0);
    tasks[0] = special(K_BCOPYIN);
    tasks[N - 1] = special(K_BCOPYOUT);
    for (int k = 0; k < nt; ++k) {
      const int v = p->order[k];
      const DevTask& d = p->tasks[v];
      tasks[k + 1] = d;
      for (int e = d.succ_begin; e < d.succ_end; ++e) succ[k + 1].push_back(pos[p->succ[e]]);
      indeg[k + 1] = p->indeg[v];
      if (p->indeg[v] == 0) {
        succ[0].push_back(k + 1);
        ++indeg[k + 1];
      }
      if (d.succ_begin == d.succ_end) {
        succ[k + 1].push_back(N - 1);
        ++indeg[N - 1];
      }
    }
    bt->links = p->links;
  }
  const int N = (int)tasks.size();
  bt->succ.clear();
  for (int k = 0; k < N; ++k) {
    tasks[k].succ_begin = (int32_t)bt->succ.size();
    bt->succ.insert(bt->succ.end(), succ[k].begin(), succ[k].end());
    tasks[k].succ_end = (int32_t)bt->succ.size();
  }
  bt->tasks = tasks;
  bt->indeg0 = indeg;
  bt->ntask = N;
  PlanImage* im = &bt->image;
  const size_t nl = bt->links.size();
  im->o_tasks = 0;
  im->o_succ = align_up(N * sizeof(DevTask), 256);
  im->o_indeg = align_up(im->o_succ + bt->succ.size() * sizeof(int32_t) + 4, 256);
  im->o_links = align_up(im->o_indeg + N * sizeof(int32_t), 256);
  im->bytes.assign(align_up(im->o_links + nl * sizeof(int32_t) + 4, 256), 0);
  char* h = im->bytes.data();
  std::memcpy(h + im->o_tasks, tasks.data(), N * sizeof(DevTask));
  if (!bt->succ.empty())
    std::memcpy(h + im->o_succ, bt->succ.data(), bt->succ.size() * sizeof(int32_t));
  std::memcpy(h + im->o_indeg, indeg.data(), N * sizeof(int32_t));
  if (nl) std::memcpy(h + im->o_links, bt->links.data(), nl * sizeof(int32_t));
  im->has_links = nl > 0;
}

// Estimated durations of the template tasks (the planner's cost units: a
// single 128^3 product is 1) and their bottom levels.  A copy task moves the
// matrix's lower tiles (about 0.12 per tile); the small-matrix task costs
// about what the diagonal-tile task costs.
void btemplate_costs(BTemplate* bt, int t) {
  const int N = bt->ntask;
  bt->cost.assign(N, 0.0);
  const double tiles = t * (t + 1) / 2.0;
  for (int k = 0; k < N; ++k) {
    const int32_t kind = bt->tasks[k].kind;
    const int kd = kind & 0xff;
    double c;
    if (kd == K_BCOPYIN || kd == K_BCOPYOUT) c = 0.12 * tiles;
    else if (kd == K_BSMALL) c = 2.5;
    else if (kd < K_COUNT) c = kCost[kd] + kCost[K_COUNT] * task_links(kind);
    else c = 1.0;
    bt->cost[k] = c;
  }
  bt->bottom.assign(N, 0.0);
  for (int k = N - 1; k >= 0; --k) {  // positions are topological
    double b = 0.0;
    for (int e = bt->tasks[k].succ_begin; e < bt->tasks[k].succ_end; ++e)
      b = std::max(b, bt->bottom[bt->succ[e]]);
    bt->bottom[k] = b + bt->cost[k];
  }
}

int btemplate_chain(const spdinv_opts& o, bool /*fp32*/) { return chain_for(o); }

// Device tasks of the template of t at most (without building it).
long long btemplate_bound(int t) { return t <= 1 ? 1 : task_count(t) + 2; }

// Template key: template tile count, FP32, chain, renamed, loop order,
// TRTRI(j) placement.
typedef std::tuple<int, int, int, int, int, int> BTKey;
std::map<BTKey, std::unique_ptr<BTemplate>> g_btmpl;
std::map<std::pair<int, BTKey>, std::unique_ptr<BTemplateDev>> g_btmpl_dev;

// Host template (built once per variant).  Called with g_mu held.
const BTemplate* btemplate_host(int t, bool fp32, const spdinv_opts& o) {
  const BTKey k{t, fp32 ? 1 : 0, btemplate_chain(o, fp32), o.renamed ? 1 : 0, o.loop_order,
                o.trtri_first ? 1 : 0};
  auto it = g_btmpl.find(k);
  if (it != g_btmpl.end()) return it->second.get();
  std::unique_ptr<BTemplate> bt(new BTemplate);
  if (t <= 1) {
    make_btemplate(nullptr, bt.get());
  } else {
    PlanOptions po;
    po.t = t;
    po.renamed = o.renamed ? 1 : 0;
    po.loop_order = o.loop_order;
    po.pipelined = 1;
    po.trtri_first = o.trtri_first ? 1 : 0;
    po.chain = btemplate_chain(o, fp32);
    po.chain_tails = 1;  // one workgroup runs a matrix's tasks in order: every operand is ready
    Plan p;
    // one worker: the list-scheduling order is a priority order of the
    // matrix's tasks, and chains form wherever the contraction rules allow
    // (the other matrices of the batch keep the workers busy)
    build_plan(po, 1, kCost, &p);
    make_btemplate(&p, bt.get());
    bt->d_base = p.d_base;
  }
  btemplate_costs(bt.get(), t);
  const BTemplate* raw = bt.get();
  g_btmpl[k] = std::move(bt);
  return raw;
}

BTemplateDev* get_btemplate(int device, int t, bool fp32, const spdinv_opts& o, hipError_t* err) {
  std::lock_guard<std::mutex> lk(g_mu);
  const BTemplate* h = btemplate_host(t, fp32, o);
  const BTKey k{t, fp32 ? 1 : 0, btemplate_chain(o, fp32), o.renamed ? 1 : 0, o.loop_order,
                o.trtri_first ? 1 : 0};
  auto it = g_btmpl_dev.find({device, k});
  if (it != g_btmpl_dev.end()) return it->second.get();
  if (h->ntask > BT_MASK + 1) {
    *err = hipErrorInvalidValue;
    return nullptr;
  }
  std::unique_ptr<BTemplateDev> bd(new BTemplateDev);
  bd->h = h;
  void* arena = nullptr;
  *err = hipMalloc(&arena, h->image.bytes.size());
  if (*err != hipSuccess) return nullptr;
  *err = hipMemcpy(arena, h->image.bytes.data(), h->image.bytes.size(), hipMemcpyHostToDevice);
  if (*err != hipSuccess) {
    (void)hipFree(arena);
    return nullptr;
  }
  char* base = (char*)arena;
  bd->arena = arena;
  bd->d_tasks = (const DevTask*)(base + h->image.o_tasks);
  bd->d_succ = (const int32_t*)(base + h->image.o_succ);
  bd->d_indeg0 = (const int32_t*)(base + h->image.o_indeg);
  bd->d_links = h->image.has_links ? (const int32_t*)(base + h->image.o_links) : nullptr;
  BTemplateDev* raw = bd.get();
  g_btmpl_dev[{device, k}] = std::move(bd);
  return raw;
}

int tiles_of_order(int n) { return n <= NB ? 1 : (n + NB - 1) / NB; }

// Dispatch order by a list-scheduling simulation of the whole batch on
// `workers` workers with the templates' estimated durations: whenever a
// worker is free it starts the ready task of the earliest matrix in `order`
// (the longest matrices first), the task with the longest path to its
// matrix's end first.  The order of the simulated starts is topological.
// Pool slots: a matrix of t >= 2 tiles takes a free slot of its tile count
// when its copy-in task starts and frees it when its copy-out task ends;
// slot[m] receives the slot, prev[m] the slot's previous occupant (or -1),
// nslots[t] the slots of each tile count.
void batch_list_schedule(const std::vector<int>& order, const std::vector<int8_t>& tv,
                         const BTemplate* const* tmpl, const std::vector<int4>& mat, int workers,
                         std::vector<int32_t>* disp, std::vector<int>* slot,
                         std::vector<int>* prev, std::vector<int>* nslots) {
  const int batch = (int)tv.size();
  std::vector<int> rank(batch);
  for (int r = 0; r < (int)order.size(); ++r) rank[order[r]] = r;
  long long total = 0;
  for (int m = 0; m < batch; ++m) total += tmpl[tv[m]]->ntask;
  std::vector<int32_t> left((size_t)total);
  for (int m = 0; m < batch; ++m) {
    const BTemplate* bt = tmpl[tv[m]];
    std::copy(bt->indeg0.begin(), bt->indeg0.end(), left.begin() + mat[m].y);
  }
  struct Ready {
    int rank;
    double bottom;
    int m, pos;
    bool operator<(const Ready& o) const {  // priority_queue: top is the largest
      if (rank != o.rank) return rank > o.rank;
      if (bottom != o.bottom) return bottom < o.bottom;
      return pos > o.pos;
    }
  };
  struct Done {
    double time;
    int m, pos;
    bool operator<(const Done& o) const { return time > o.time; }
  };
  std::priority_queue<Ready> ready;
  std::priority_queue<Done> running;
  for (int m = 0; m < batch; ++m) ready.push(Ready{rank[m], tmpl[tv[m]]->bottom[0], m, 0});
  slot->assign(batch, -1);
  prev->assign(batch, -1);
  nslots->assign(MAX_BATCH_T + 1, 0);
  std::vector<std::vector<int>> free_slots(MAX_BATCH_T + 1);
  std::vector<std::vector<int>> last(MAX_BATCH_T + 1);  // last occupant of each slot
  int free_workers = std::max(1, workers);
  double now = 0.0;
  while (!ready.empty() || !running.empty()) {
    while (free_workers > 0 && !ready.empty()) {
      const Ready r = ready.top();
      ready.pop();
      const int t = tv[r.m];
      if (r.pos == 0 && t >= 2) {  // copy-in: take a pool slot
        int sl;
        if (!free_slots[t].empty()) {
          sl = free_slots[t].back();
          free_slots[t].pop_back();
        } else {
          sl = (*nslots)[t]++;
          last[t].push_back(-1);
        }
        (*slot)[r.m] = sl;
        (*prev)[r.m] = last[t][sl];
        last[t][sl] = r.m;
      }
      disp->push_back((r.m << BT_SHIFT) | r.pos);
      running.push(Done{now + tmpl[t]->cost[r.pos], r.m, r.pos});
      --free_workers;
    }
    const Done d = running.top();
    running.pop();
    now = d.time;
    ++free_workers;
    const BTemplate* bt = tmpl[tv[d.m]];
    if (tv[d.m] >= 2 && d.pos == bt->ntask - 1) free_slots[tv[d.m]].push_back((*slot)[d.m]);
    const DevTask& task = bt->tasks[d.pos];
    for (int e = task.succ_begin; e < task.succ_end; ++e) {
      const int q = bt->succ[e];
      if (--left[(size_t)mat[d.m].y + q] == 0) ready.push(Ready{rank[d.m], bt->bottom[q], d.m, q});
    }
  }
}

// Composition of a batch (host): per matrix its template, first counter and
// first pool tile; the dispatch list.  The matrices are ranked by decreasing
// tile count (the longest first, stable).  group > 0: the templates are
// interleaved position by position in groups of `group` matrices; group < 0:
// one ticket per matrix, run whole by one of `workers` workgroups; else the
// list-scheduling order on `workers` workers.  Returns 0 or -1 when the
// counters or pool tiles overflow int32.
struct BCompHost {
  std::vector<int32_t> disp;
  std::vector<int4> mat;
  long long ncnt = 0;
  long long pool_tiles = 0;
  long long wg_pool_tiles = 0;  // one workgroup per matrix: pool tiles per workgroup
};

int build_bcomp(const std::vector<int8_t>& tv, const BTemplate* const* tmpl, int group,
                int workers, BCompHost* out) {
  const int batch = (int)tv.size();
  std::vector<int> order;
  order.reserve(batch);
  for (int t = MAX_BATCH_T; t >= 1; --t)
    for (int i = 0; i < batch; ++i)
      if (tv[i] == t) order.push_back(i);
  out->mat.assign(batch, make_int4(0, 0, 0, -1));
  long long cnt = 0, ptile = 0;
  for (int m : order) {
    const int t = tv[m];
    out->mat[m] = make_int4(t, (int)cnt, (int)ptile, -1);
    cnt += tmpl[t]->ntask;
    if (t >= 2) ptile += pool_tiles(t);
    if (cnt > INT_MAX || ptile > INT_MAX) return -1;
  }
  out->ncnt = cnt;
  out->pool_tiles = ptile;
  out->disp.clear();
  out->disp.reserve((size_t)cnt);
  if (group == -1) {  // one workgroup per matrix: a ticket per matrix, pools per workgroup
    int tmax = 1;
    for (int m : order) {
      out->disp.push_back(m << BT_SHIFT);
      tmax = std::max(tmax, (int)tv[m]);
    }
    out->ncnt = 0;
    out->pool_tiles = tmax >= 2 ? (long long)workers * pool_tiles(tmax) : 0;
    out->wg_pool_tiles = tmax >= 2 ? pool_tiles(tmax) : 0;
    return 0;
  }
  if (group > 0) {  // every matrix keeps its own pool
    for (size_t g0 = 0; g0 < order.size(); g0 += group) {
      const size_t g1 = std::min(order.size(), g0 + (size_t)group);
      int longest = 0;
      for (size_t q = g0; q < g1; ++q) longest = std::max(longest, tmpl[tv[order[q]]]->ntask);
      for (int pos = 0; pos < longest; ++pos)
        for (size_t q = g0; q < g1; ++q)
          if (pos < tmpl[tv[order[q]]]->ntask) out->disp.push_back((order[q] << BT_SHIFT) | pos);
    }
    return 0;
  }
  std::vector<int> slot, prev, nslots;
  batch_list_schedule(order, tv, tmpl, out->mat, workers, &out->disp, &slot, &prev, &nslots);
  // pool: the slots of each tile count, largest tile count first
  std::vector<long long> slot_base(MAX_BATCH_T + 1, 0);
  ptile = 0;
  for (int t = MAX_BATCH_T; t >= 2; --t) {
    slot_base[t] = ptile;
    ptile += (long long)nslots[t] * pool_tiles(t);
  }
  if (ptile > INT_MAX) return -1;
  out->pool_tiles = ptile;
  for (int m = 0; m < batch; ++m) {
    const int t = tv[m];
    if (t < 2) continue;
    out->mat[m].z = (int)(slot_base[t] + (long long)slot[m] * pool_tiles(t));
    if (prev[m] >= 0) {
      out->mat[m].x |= BM_PREV;
      out->mat[prev[m]].w = out->mat[m].y;  // copy-in of m is position 0
    }
  }
  return 0;
}

// Host compositions, cached per (precision, template variant, dispatch rule
// with its worker count, tile counts of the batch).
typedef std::tuple<int, int, int, int, int, int, std::vector<int8_t>> BHKey;
std::map<BHKey, std::unique_ptr<BCompHost>> g_bcomp_host;

// The batched schedule the library picks when opts.batch_group is 0: one
// workgroup per matrix when the batch has at least two matrices per worker
// (every worker then runs whole matrices, no dependency waits), else the
// list-scheduled DAG (a few large matrices spread over every worker).
// Measured on 8192 orders uniform on 16..512 (FP64): one workgroup per
// matrix 20.7 ms, the list-scheduled DAG 26.3 ms, groups of 512 23.5 ms.
int batch_schedule(int batch, const spdinv_opts& o, int workers) {
  if (o.batch_group != 0) return o.batch_group;
  return batch >= 2 * workers ? -1 : -2;
}

// Called with g_mu held.  Returns null when the composition overflows.
const BCompHost* bcomp_host(const std::vector<int8_t>& tv, bool fp32, const spdinv_opts& o,
                            int workers) {
  const int group = batch_schedule((int)tv.size(), o, workers);
  const BHKey k{fp32 ? 1 : 0, btemplate_chain(o, fp32),
                group > 0 ? group : (group == -1 ? -(1 << 30) - workers : -workers),
                o.renamed ? 1 : 0, o.loop_order, o.trtri_first ? 1 : 0, tv};
  auto it = g_bcomp_host.find(k);
  if (it != g_bcomp_host.end()) return it->second.get();
  const BTemplate* tmpl[MAX_BATCH_T + 1] = {};
  for (size_t i = 0; i < tv.size(); ++i)
    if (!tmpl[tv[i]]) tmpl[tv[i]] = btemplate_host(tv[i], fp32, o);
  std::unique_ptr<BCompHost> hc(new BCompHost);
  if (build_bcomp(tv, tmpl, group, workers, hc.get())) return nullptr;
  const BCompHost* raw = hc.get();
  g_bcomp_host[k] = std::move(hc);
  return raw;
}

// Device copy of a composition, cached per (device, precision, template
// variant, dispatch rule, tile counts of the batch).
struct BComp {
  void* arena = nullptr;
  const int32_t* d_disp = nullptr;
  const int4* d_mat = nullptr;
  int ntotal = 0;
  long long ncnt = 0;
  long long pool_tiles = 0;
  long long wg_pool_tiles = 0;
};
typedef std::tuple<int, int, int, int, int, int, int, std::vector<int8_t>> BCKey;
std::map<BCKey, std::unique_ptr<BComp>> g_bcomp;

struct BLayout {
  size_t ctrl, mctrl, indeg, pool, total;
};

BLayout blayout(int batch, long long ncnt, long long pool_tiles_total, bool fp32) {
  BLayout L;
  L.ctrl = 0;
  L.mctrl = 256;
  L.indeg = L.mctrl + align_up((size_t)batch * CTRL_WORDS * sizeof(int32_t), 256);
  L.pool = L.indeg + align_up((size_t)ncnt * sizeof(int32_t), 256);
  L.total = L.pool + (size_t)pool_tiles_total * NB * NB * (fp32 ? sizeof(float) : sizeof(double));
  return L;
}

// Upper bound of the counters and the pool tiles of a batch, from its orders;
// -2 when an order is out of range.
int batch_bounds(int batch, const int* h_n, long long* ncnt, long long* ptiles) {
  *ncnt = 0;
  *ptiles = 0;
  for (int i = 0; i < batch; ++i) {
    if (h_n[i] < 0 || h_n[i] > MAX_BATCH_T * NB) return -2;
    const int t = tiles_of_order(h_n[i]);
    *ncnt += btemplate_bound(t);
    if (t >= 2) *ptiles += pool_tiles(t);
  }
  return 0;
}

int batched_grid(int device, const spdinv_opts& o, bool fp32) {
  static std::map<std::pair<int, int>, int> grids;
  int g;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = grids.find({device, fp32 ? 1 : 0});
    if (it != grids.end()) {
      g = it->second;
    } else {
      int cus = 0;
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
          cus <= 0)
        cus = 1;
      g = cus * (fp32 ? bsched32_blocks_per_cu() : bsched_blocks_per_cu());
      grids[{device, fp32 ? 1 : 0}] = g;
    }
  }
  if (o.workers > 0 && o.workers < g) g = o.workers;
  return g;
}

// Workers of the list-scheduling simulation: the caller's cap, else 512 (two
// workgroups on each of the MI355X's 256 CUs).  A fixed count keeps the
// dispatch order and the pool size (its slots) independent of the device;
// any topological order is correct.
constexpr int kBatchSimWorkers = 512;
int batch_sim_workers(const spdinv_opts& o) { return o.workers > 0 ? o.workers : kBatchSimWorkers; }

BComp* get_bcomp(int device, int batch, const int* h_n, bool fp32, const spdinv_opts& o,
                 int workers, hipError_t* err) {
  const int group = batch_schedule(batch, o, workers);
  std::vector<int8_t> tv(batch);
  for (int i = 0; i < batch; ++i) tv[i] = (int8_t)tiles_of_order(h_n[i]);
  BCKey k{device, fp32 ? 1 : 0, btemplate_chain(o, fp32),
          group > 0 ? group : (group == -1 ? -(1 << 30) - workers : -workers),
          o.renamed ? 1 : 0, o.loop_order, o.trtri_first ? 1 : 0, tv};
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_bcomp.find(k);
  if (it != g_bcomp.end()) return it->second.get();
  const BCompHost* hp = bcomp_host(tv, fp32, o, workers);
  if (!hp) {
    *err = hipErrorInvalidValue;
    return nullptr;
  }
  const BCompHost& hc = *hp;
  std::unique_ptr<BComp> bc(new BComp);
  const size_t o_mat = align_up(hc.disp.size() * sizeof(int32_t), 256);
  const size_t bytes = align_up(o_mat + (size_t)batch * sizeof(int4), 256);
  std::vector<char> img(bytes, 0);
  std::memcpy(img.data(), hc.disp.data(), hc.disp.size() * sizeof(int32_t));
  std::memcpy(img.data() + o_mat, hc.mat.data(), (size_t)batch * sizeof(int4));
  void* arena = nullptr;
  *err = hipMalloc(&arena, bytes);
  if (*err != hipSuccess) return nullptr;
  *err = hipMemcpy(arena, img.data(), bytes, hipMemcpyHostToDevice);
  if (*err != hipSuccess) {
    (void)hipFree(arena);
    return nullptr;
  }
  bc->arena = arena;
  bc->d_disp = (const int32_t*)arena;
  bc->d_mat = (const int4*)((char*)arena + o_mat);
  bc->ntotal = (int)hc.disp.size();
  bc->ncnt = hc.ncnt;
  bc->pool_tiles = hc.pool_tiles;
  bc->wg_pool_tiles = hc.wg_pool_tiles;
  BComp* raw = bc.get();
  g_bcomp[k] = std::move(bc);
  return raw;
}

}  // namespace

extern "C" {

size_t batched_spd_inverse_workspace_bytes(int batch, const int* h_n, spdinv_mode mode,
                                           const spdinv_opts* opts) {
  if (batch <= 0 || batch > MAX_BATCH || !h_n) return 0;
  if (mode != SPDINV_FP64 && mode != SPDINV_FP32) return 0;
  const bool fp32 = mode == SPDINV_FP32;
  const spdinv_opts o = tuned_batch(opts ? *opts : defaults(), fp32, h_n, batch);
  if (check_opts(o)) return 0;
  long long ncnt, ptiles;
  if (batch_bounds(batch, h_n, &ncnt, &ptiles)) return 0;
  const int workers = batch_sim_workers(o);
  std::vector<int8_t> tv(batch);
  for (int i = 0; i < batch; ++i) tv[i] = (int8_t)tiles_of_order(h_n[i]);
  std::lock_guard<std::mutex> lk(g_mu);
  const BCompHost* hc = bcomp_host(tv, fp32, o, workers);
  if (!hc) return 0;
  return blayout(batch, hc->ncnt, hc->pool_tiles, fp32).total;
}

int batched_spd_inverse(int batch, const int* h_n, const int* d_n, void* const* d_A,
                        const int* d_lda, spdinv_mode mode, void* work, size_t work_bytes,
                        spdinv_stream_t stream_, const spdinv_opts* opts, int* d_info) {
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  if (batch < 0 || batch > MAX_BATCH) return -1;
  if (batch == 0) return 0;
  if (!h_n) return -2;
  if (!d_n) return -3;
  if (!d_A) return -4;
  if (!d_lda) return -5;
  if (mode != SPDINV_FP64 && mode != SPDINV_FP32) return -6;
  const bool fp32 = mode == SPDINV_FP32;
  const spdinv_opts o = tuned_batch(opts ? *opts : defaults(), fp32, h_n, batch);
  if (check_opts(o) || (fp32 && !o.renamed)) return -10;
  long long ncnt_bound, ptiles;
  if (batch_bounds(batch, h_n, &ncnt_bound, &ptiles)) return -2;
  if (!work) return -7;
  if (work_bytes < batched_spd_inverse_workspace_bytes(batch, h_n, mode, &o))
    return SPDINV_ERR_WORKSPACE;
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return SPDINV_ERR_HIP;

  BSchedArgs b;
  std::memset(&b, 0, sizeof(b));
  BTemplateDev* tmpl[MAX_BATCH_T + 1] = {};
  for (int i = 0; i < batch; ++i) {
    const int t = tiles_of_order(h_n[i]);
    if (tmpl[t]) continue;
    hipError_t err = hipSuccess;
    tmpl[t] = get_btemplate(device, t, fp32, o, &err);
    if (!tmpl[t]) return SPDINV_ERR_HIP;
    b.tmpl[t] = tmpl[t]->d_tasks;
    b.tsucc[t] = tmpl[t]->d_succ;
    b.tlinks[t] = tmpl[t]->d_links;
    b.tindeg0[t] = tmpl[t]->d_indeg0;
    b.tdbase[t] = tmpl[t]->h->d_base;
  }
  hipError_t err = hipSuccess;
  const int grid = batched_grid(device, o, fp32);
  BComp* bc = get_bcomp(device, batch, h_n, fp32, o, batch_sim_workers(o), &err);
  if (!bc) return SPDINV_ERR_HIP;
  const BLayout L = blayout(batch, bc->ncnt, bc->pool_tiles, fp32);
  char* w = (char*)work;
  b.disp = bc->d_disp;
  b.mat = bc->d_mat;
  b.indeg = (int32_t*)(w + L.indeg);
  b.ctrl = (int32_t*)(w + L.ctrl);
  b.mctrl = (int32_t*)(w + L.mctrl);
  b.pool = (void*)(w + L.pool);
  b.n = d_n;
  b.A = d_A;
  b.lda = d_lda;
  b.info = d_info;
  b.ntotal = bc->ntotal;
  b.fill_upper = o.fill_upper ? 1 : 0;
  b.spin_limit = spin_limit();
  b.seq = batch_schedule(batch, o, batch_sim_workers(o)) == -1 ? 1 : 0;
  b.wg_pool_tiles = bc->wg_pool_tiles;
  for (int t = 1; t <= MAX_BATCH_T; ++t) b.tntask[t] = tmpl[t] ? tmpl[t]->h->ntask : 0;
  if (launch_breset(b, batch, stream) != hipSuccess) return SPDINV_ERR_HIP;
  // one workgroup per matrix: at most as many workgroups as per-workgroup pools
  const int g2 = b.seq ? std::min(grid, batch_sim_workers(o)) : grid;
  if ((fp32 ? launch_bsched32(b, g2, stream) : launch_bsched(b, g2, stream)) != hipSuccess)
    return SPDINV_ERR_HIP;
  return 0;
}

size_t batched_spd_inverse_backward_workspace_bytes(int batch, const int* h_n) {
  if (batch <= 0 || batch > MAX_BATCH || !h_n) return 0;
  for (int i = 0; i < batch; ++i)
    if (h_n[i] < 0 || h_n[i] > MAX_BATCH_T * NB) return 0;
  long long tiles, ncnt;
  bback_sizes(batch, h_n, &tiles, &ncnt);
  return bback_bytes(tiles, ncnt);
}

int batched_spd_inverse_backward(int batch, const int* h_n, const int* d_n,
                                 const double* const* d_X, const int* d_ldx,
                                 const double* const* d_G, const int* d_ldg,
                                 double* const* d_gradA, const int* d_ldga, void* work,
                                 size_t work_bytes, spdinv_stream_t stream_) {
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  if (batch < 0 || batch > MAX_BATCH) return -1;
  if (batch == 0) return 0;
  if (!h_n) return -2;
  for (int i = 0; i < batch; ++i)
    if (h_n[i] < 0 || h_n[i] > MAX_BATCH_T * NB) return -2;
  if (!d_n) return -3;
  if (!d_X) return -4;
  if (!d_ldx) return -5;
  if (!d_G) return -6;
  if (!d_ldg) return -7;
  if (!d_gradA) return -8;
  if (!d_ldga) return -9;
  if (!work) return -10;
  long long tiles, ncnt;
  bback_sizes(batch, h_n, &tiles, &ncnt);
  if (work_bytes < bback_bytes(tiles, ncnt)) return SPDINV_ERR_WORKSPACE;
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return SPDINV_ERR_HIP;
  hipError_t err = hipSuccess;
  BBackComp* bc = get_bbcomp(device, batch, h_n, &err);
  if (!bc) return SPDINV_ERR_HIP;
  if (bc->ntask == 0) return 0;  // every order is 0
  static std::map<int, int> grids;
  int grid;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = grids.find(device);
    if (it == grids.end()) {
      int cus = 0;
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
          cus <= 0)
        cus = 1;
      it = grids.emplace(device, cus * bback_blocks_per_cu()).first;
    }
    grid = it->second;
  }
  char* w = (char*)work;
  BBackArgs b;
  std::memset(&b, 0, sizeof(b));
  b.task = bc->d_task;
  b.ntask = bc->ntask;
  b.mat = bc->d_mat;
  b.n = d_n;
  b.X = d_X;
  b.ldx = d_ldx;
  b.G = d_G;
  b.ldg = d_ldg;
  b.gradA = d_gradA;
  b.ldga = d_ldga;
  b.ctrl = (int32_t*)w;
  b.cnt = (int32_t*)(w + 256);
  b.tiles = (double*)(w + 256 + align_up((size_t)bc->ncnt * sizeof(int32_t), 256));
  b.spin_limit = spin_limit();
  if (launch_bback(b, (int)bc->ncnt, grid, stream) != hipSuccess) return SPDINV_ERR_HIP;
  return 0;
}

size_t spd_inverse_backward_workspace_bytes(int n) {
  if (n <= 0) return 0;
  const size_t t = (size_t)tiles_for(n);
  return 3 * t * t * (size_t)NB * NB * sizeof(double);
}

int spd_inverse_backward(int n, const double* X, int ldx, const double* G, int ldg, double* gradA,
                         int ldga, void* work, size_t work_bytes, spdinv_stream_t stream_) {
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  const int ldmin = n > 1 ? n : 1;
  if (n < 0) return -1;
  if (n > 0 && !X) return -2;
  if (ldx < ldmin) return -3;
  if (n > 0 && !G) return -4;
  if (ldg < ldmin) return -5;
  if (n > 0 && !gradA) return -6;
  if (ldga < ldmin) return -7;
  if (n == 0) return 0;
  if (!work) return -8;
  if (work_bytes < spd_inverse_backward_workspace_bytes(n)) return SPDINV_ERR_WORKSPACE;
  const int t = tiles_for(n);
  const size_t sq = (size_t)t * t * NB * NB;
  double* Xf = (double*)work;  // X, full symmetric
  double* S = Xf + sq;         // sym(G), later the lower tiles of the gradient
  double* W = S + sq;          // X sym(G)
  if (launch_pack(X, ldx, n, t, PACK_SYM_LOWER, Xf, stream) != hipSuccess) return SPDINV_ERR_HIP;
  if (launch_pack(G, ldg, n, t, PACK_SYM_AVG, S, stream) != hipSuccess) return SPDINV_ERR_HIP;
  // W = X S: W(i, j) = sum_k X(i, k) S(k, j) = sum_k X(i, k) S(j, k)^T (S symmetric)
  if (launch_gemm_nt(Xf, S, W, t, 0, 0, stream) != hipSuccess) return SPDINV_ERR_HIP;
  // grad = -W X on the lower tiles: sum_k W(i, k) X(j, k)^T (X symmetric)
  if (launch_gemm_nt(W, Xf, S, t, 1, 1, stream) != hipSuccess) return SPDINV_ERR_HIP;
  if (launch_unpack_sym(S, t, n, gradA, ldga, stream) != hipSuccess) return SPDINV_ERR_HIP;
  return 0;
}

// Mixed-precision form.  Workspace: the FP32 tile pool and the scheduler
// state, then four square tile-major binary64 matrices (A, X, the next X, the
// residual), the norm scratch and the FP32 copy of the residual for the
// low-precision correction (the FP32 copy of X takes the pool's place, dead
// once X0 is widened).  The FP64 fallback reuses the workspace from offset 0
// (everything in it is dead by then; A itself is untouched until the final
// copy-out).
struct MixedLayout {
  size_t indeg, ctrl, asq, x, x2, r, partial, r32, probe, total;
};

MixedLayout mixed_layout(int n, const spdinv_opts& o) {
  MixedLayout M;
  const int t = tiles_for(n);
  const long long nt = task_count(t);
  const size_t sq = (size_t)t * t * NB * NB * sizeof(double);
  M.indeg = align_up(pool_bytes32(t), 256);
  M.ctrl = M.indeg + align_up((size_t)nt * sizeof(int32_t), 256);
  M.asq = M.ctrl + align_up(CTRL_WORDS * sizeof(int32_t), 256);
  M.x = M.asq + sq;
  M.x2 = M.x + sq;
  M.r = M.x2 + sq;
  M.partial = M.r + sq;
  M.r32 = M.partial + align_up(((size_t)t * t + 8) * sizeof(double), 256);
  M.probe = M.r32 + align_up(sq / 2, 256);  // 3 tile columns: V^T, (A V)^T, (R V)^T
  M.total = M.probe + align_up((size_t)3 * t * NB * NB * sizeof(double), 256);
  spdinv_opts o64 = o;
  o64.trace = 0;
  M.total = std::max(M.total, layout(n, o64).total);
  return M;
}

// Workgroups per CU of the FP32 scheduler: as for the FP64 one (two from
// kWideTiles tiles per side, where the DAG keeps enough tasks ready: with
// chained tasks, 46.3 against 50.1 ms at n = 16384 and 12.5 against 9.6 ms
// at n = 8192), or the caller's per_cu, within what fits.
int per_cu32_for(int t, const spdinv_opts& o) {
  static int capacity = 0;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!capacity) capacity = sched32_blocks_per_cu();
  }
  const int want = o.per_cu ? o.per_cu : (t >= kWideTiles ? 2 : 1);
  return want < capacity ? want : capacity;
}

int grid32_for(int device, int t, const spdinv_opts& o) {
  static std::map<int, int> cus_of;
  int cus;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = cus_of.find(device);
    if (it != cus_of.end()) {
      cus = it->second;
    } else {
      cus = 0;
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
          cus <= 0)
        cus = 1;
      cus_of[device] = cus;
    }
  }
  int g = cus * per_cu32_for(t, o);
  if (o.workers > 0 && o.workers < g) g = o.workers;
  return g;
}

// The FP32 form (SPDINV_FP32): FP32 tiles of the caller's FP32 matrix, the
// renamed plan on the FP32 scheduler, copy-out; no refinement.
struct Fp32Layout {
  size_t indeg, ctrl, total;
};

Fp32Layout fp32_layout(int n) {
  Fp32Layout F;
  const int t = tiles_for(n);
  F.indeg = align_up(pool_bytes32(t), 256);
  F.ctrl = F.indeg + align_up((size_t)task_count(t) * sizeof(int32_t), 256);
  F.total = F.ctrl + align_up(CTRL_WORDS * sizeof(int32_t), 256);
  return F;
}

int run_fp32(int n, float* A, int lda, void* work, size_t work_bytes, hipStream_t stream,
             const spdinv_opts& o, int* d_info, spdinv_report* report) {
  const Fp32Layout F = fp32_layout(n);
  if (work_bytes < F.total) return SPDINV_ERR_WORKSPACE;
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return SPDINV_ERR_HIP;
  const int t = tiles_for(n);
  const int grid = grid32_for(device, t, o);
  hipError_t err = hipSuccess;
  DevPlan* dp = get_plan(device, t, o, grid, chain_for(o), &err);
  if (!dp) return SPDINV_ERR_HIP;
  const int ntask = (int)dp->host.tasks.size();
  char* w = (char*)work;
  float* pool = (float*)w;
  int32_t* indeg = (int32_t*)(w + F.indeg);
  int32_t* ctrl = (int32_t*)(w + F.ctrl);
  if (launch_reset(dp->d_indeg0, indeg, ntask, ctrl, stream) != hipSuccess) return SPDINV_ERR_HIP;
  if (launch_copy_in32f(A, lda, n, t, pool, stream) != hipSuccess) return SPDINV_ERR_HIP;
  SchedArgs a;
  std::memset(&a, 0, sizeof(a));
  a.tasks = dp->d_tasks;
  a.succ = dp->d_succ;
  a.indeg = indeg;
  a.ctrl = ctrl;
  a.pool = reinterpret_cast<double*>(pool);
  a.links = dp->d_links;
  a.last_valid = NB;
  a.ntask = ntask;
  a.tiles_T = t * (t + 1) / 2;
  a.tiles = t;
  a.spin_limit = spin_limit();
  a.d_base = 3 * a.tiles_T;
  if (launch_sched32(a, grid, per_cu32_for(t, o), false, stream) != hipSuccess)
    return SPDINV_ERR_HIP;
  if (launch_copy_out32f(pool, t, A, lda, n, o.fill_upper, stream) != hipSuccess)
    return SPDINV_ERR_HIP;
  if (launch_info_out(ctrl, d_info, stream) != hipSuccess) return SPDINV_ERR_HIP;
  if (report) {
    if (hipStreamSynchronize(stream) != hipSuccess) return SPDINV_ERR_HIP;
    int32_t c[CTRL_WORDS];
    if (hipMemcpy(c, ctrl, sizeof(c), hipMemcpyDeviceToHost) != hipSuccess) return SPDINV_ERR_HIP;
    report->info = (c[CTRL_INFO] == INT_MAX) ? 0 : c[CTRL_INFO];
    report->status = c[CTRL_ABORT] ? SPDINV_ERR_TIMEOUT : 0;
    report->nb = NB;
    report->tiles = t;
    report->tasks = c[CTRL_DONE];
    report->critical_path = dp->host.stats.cp_plan;
    report->workers = grid;
    if (c[CTRL_ABORT]) return SPDINV_ERR_TIMEOUT;
  }
  return 0;
}

int run_mixed(int n, double* A, int lda, void* work, size_t work_bytes, hipStream_t stream,
              const spdinv_opts& o, bool bf16, int* d_info, spdinv_report* report) {
  const MixedLayout M = mixed_layout(n, o);
  if (work_bytes < M.total) return SPDINV_ERR_WORKSPACE;
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return SPDINV_ERR_HIP;
  const int t = tiles_for(n);
  const int grid = grid32_for(device, t, o);
  hipError_t err = hipSuccess;
  DevPlan* dp = get_plan(device, t, o, grid, chain_for(o), &err);
  if (!dp) return SPDINV_ERR_HIP;
  const int ntask = (int)dp->host.tasks.size();
  int max_refine = o.max_refine > 0 ? o.max_refine : (bf16 ? 8 : 6);
  if (o.max_refine <= 0) {  // test hook: a smaller library default, set from the host
    const char* e = std::getenv("SPDINV_DEFAULT_MAX_REFINE");
    if (e && *e && std::atoi(e) >= 0) max_refine = std::atoi(e);
  }
  const double tol = o.refine_tol > 0.0 ? o.refine_tol : 1e-13;

  char* w = (char*)work;
  float* pool = (float*)w;
  int32_t* indeg = (int32_t*)(w + M.indeg);
  int32_t* ctrl = (int32_t*)(w + M.ctrl);
  if (launch_reset(dp->d_indeg0, indeg, ntask, ctrl, stream) != hipSuccess) return SPDINV_ERR_HIP;
  if (launch_copy_in32(A, lda, n, t, pool, stream) != hipSuccess) return SPDINV_ERR_HIP;
  SchedArgs a;
  a.tasks = dp->d_tasks;
  a.succ = dp->d_succ;
  a.indeg = indeg;
  a.ctrl = ctrl;
  a.pool = reinterpret_cast<double*>(pool);
  a.links = dp->d_links;
  a.coherent_only = 0;
  a.last_valid = NB;
  a.trace = nullptr;
  a.ntask = ntask;
  a.tiles_T = t * (t + 1) / 2;
  a.tiles = t;
  a.info_base = 0;
  a.spin_limit = spin_limit();
  a.d_base = 3 * a.tiles_T;
  if (launch_sched32(a, grid, per_cu32_for(t, o), bf16, stream) != hipSuccess)
    return SPDINV_ERR_HIP;
  int32_t c[CTRL_WORDS];
  if (hipMemcpyAsync(c, ctrl, sizeof(c), hipMemcpyDeviceToHost, stream) != hipSuccess)
    return SPDINV_ERR_HIP;
  if (hipStreamSynchronize(stream) != hipSuccess) return SPDINV_ERR_HIP;
  if (c[CTRL_ABORT]) return SPDINV_ERR_TIMEOUT;

  bool fallback = c[CTRL_FAILED] != 0;
  int fell_back = fallback ? 1 : 0;
  int iters = 0, converged = 0, predicted = 0, low_steps = 0;
  double r0 = -1.0, rl = -1.0, rpred = -1.0, r0_probe = -1.0;
  double* X = nullptr;
  if (!fallback) {
    double* Asq = (double*)(w + M.asq);
    X = (double*)(w + M.x);
    double* X2 = (double*)(w + M.x2);
    double* R = (double*)(w + M.r);
    double* partial = (double*)(w + M.partial);
    double* dnorm = partial + (size_t)t * t;  // [0] ||A||^2, [1] ||R||^2, [2] ||X0||^2,
                                              // [3] ||R0 V||^2 of the probes
    const int sq_tiles = t * t;
    if (launch_pack(A, lda, n, t, PACK_SYM_LOWER, Asq, stream) != hipSuccess) return SPDINV_ERR_HIP;
    if (launch_sumsq(Asq, sq_tiles, partial, dnorm, stream) != hipSuccess) return SPDINV_ERR_HIP;
    if (launch_x0_to_sym64(pool, t, n, X, stream) != hipSuccess) return SPDINV_ERR_HIP;
    if (launch_sumsq(X, sq_tiles, partial, dnorm + 2, stream) != hipSuccess) return SPDINV_ERR_HIP;
    // Newton-Schulz needs ||R_0|| < 1.  Estimate ||R_0||_F from NB random
    // sign probes first, E ||R_0 V||_F^2 = NB ||R_0||_F^2 (relative spread
    // at most sqrt(2 / NB) = 0.125): a start estimated above 2 falls back
    // at once, without the 2 n^3 of the full residual
    {
      double* Vt = (double*)(w + M.probe);
      double* Yt = Vt + (size_t)t * NB * NB;
      double* RVt = Yt + (size_t)t * NB * NB;
      if (launch_fill_probe(Vt, t, n, stream) != hipSuccess ||
          launch_gemm_thin(Vt, Asq, Yt, t, 0, stream) != hipSuccess ||      // (A V)^T
          launch_gemm_thin(Yt, X, RVt, t, 1, stream, Vt) != hipSuccess ||   // (V - X0 A V)^T
          launch_sumsq(RVt, t, partial, dnorm + 3, stream) != hipSuccess)
        return SPDINV_ERR_HIP;
      double h[4];
      if (hipMemcpyAsync(h, dnorm, sizeof(h), hipMemcpyDeviceToHost, stream) != hipSuccess)
        return SPDINV_ERR_HIP;
      if (hipStreamSynchronize(stream) != hipSuccess) return SPDINV_ERR_HIP;
      const double est = std::sqrt(h[3] / NB);
      r0_probe = est / std::sqrt(h[0]);
      if (!(est <= 2.0)) {  // NaN included
        fallback = true;
        fell_back = 1;
        r0 = r0_probe;
      }
    }
    float* X32 = (float*)w;  // the FP32 pool is dead once X0 is widened
    float* R32 = (float*)(w + M.r32);
    const size_t sq_elems = (size_t)sq_tiles * NB * NB;
    // the correction X R runs on the FP32 matrix cores while another
    // residual follows it, as long as the steps it made stay quadratic
    bool low_ok = !o.correction64;
    bool last_low = false;
    double prev_rnorm = 0.0;
    double anorm = 0.0, floor_abs = 0.0;
    for (int k = 0; !fallback; ++k) {
      // R^T = I - X A (A and X symmetric); ||R^T||_F = ||R||_F
      if (launch_gemm_nt(X, Asq, R, t, 0, 1, stream, nullptr, n) != hipSuccess) return SPDINV_ERR_HIP;
      if (launch_sumsq(R, sq_tiles, partial, dnorm + 1, stream) != hipSuccess) return SPDINV_ERR_HIP;
      double h[3];
      if (hipMemcpyAsync(h, dnorm, sizeof(h), hipMemcpyDeviceToHost, stream) != hipSuccess)
        return SPDINV_ERR_HIP;
      if (hipStreamSynchronize(stream) != hipSuccess) return SPDINV_ERR_HIP;
      const double rnorm = std::sqrt(h[1]);
      if (k == 0) {
        anorm = std::sqrt(h[0]);
        // binary64 rounding floor of a residual, u ||A||_F ||X||_F up to a
        // small factor (the typical size of the rounding of I - A X and of
        // the stored X + X R)
        floor_abs = 4.0 * 0x1p-53 * anorm * std::sqrt(h[2]);
        r0 = rnorm / anorm;
        if (!(rnorm < 1.0)) {  // Newton-Schulz needs ||R_0|| < 1 (NaN included)
          fallback = true;
          fell_back = 1;
          break;
        }
      }
      const double rel = rnorm / anorm;
      rl = rel;
      if (rel <= tol) {  // the measured residual of X meets the stop rule
        converged = 1;
        rpred = rel;
        break;
      }
      if (k >= max_refine) break;
      // a low-precision step that did not square the residual (to within a
      // factor: its rounding, about u_32 ||X|| ||R|| times kappa, has caught
      // up with ||R||^2) leaves the remaining corrections to binary64
      if (last_low && rnorm > 0.01 * prev_rnorm) low_ok = false;
      prev_rnorm = rnorm;
      // I - A X' = R^2 exactly for X' = X + X R, so ||I - A X'||_F <=
      // ||R||_F^2 up to the rounding floor: when that prediction meets the
      // stop rule, the step is the last (in binary64) and the residual of X'
      // is not formed; otherwise another residual follows and the step's
      // correction may run in FP32
      const double pred = (rnorm * rnorm + floor_abs) / anorm;
      const bool low = low_ok && pred > tol;
      // X' = X + X R on the lower tiles, X R = sum_k X(i, k) (R^T)(j, k)^T; then mirror
      if (low) {
        if (launch_round32(X, X32, sq_elems, stream) != hipSuccess) return SPDINV_ERR_HIP;
        if (launch_round32(R, R32, sq_elems, stream) != hipSuccess) return SPDINV_ERR_HIP;
        if (launch_gemm_nt32_lower(X32, R32, X, X2, t, stream) != hipSuccess)
          return SPDINV_ERR_HIP;
        ++low_steps;
      } else if (launch_gemm_nt(X, R, X2, t, 1, 0, stream, X, 0) != hipSuccess) {
        return SPDINV_ERR_HIP;
      }
      if (launch_mirror_lower(X2, t, stream) != hipSuccess) return SPDINV_ERR_HIP;
      std::swap(X, X2);
      ++iters;
      last_low = low;
      if (!low && pred <= tol) {
        converged = 1;
        predicted = 1;
        rpred = pred;
        break;
      }
    }
    // the library's own step limit ran out before the stop rule was met:
    // the FP64 path gives the result (a caller-chosen limit or tolerance
    // keeps the refined X and reports converged = 0)
    if (!fallback && !converged && o.max_refine <= 0 && !(o.refine_tol > 0.0)) {
      fallback = true;
      fell_back = 2;
    }
  }
  if (fallback) {
    spdinv_opts o64 = o;
    o64.trace = 0;
    const int rc = run_fp64(n, A, lda, work, work_bytes, stream, o64, d_info, report);
    if (report) {
      report->fell_back = fell_back;
      report->resid0_fro_rel = r0;
      report->resid_fro_rel = -1.0;
      report->resid_last_rel = rl;
      report->refine_iters = iters;
      report->converged = 0;
      report->predicted = 0;
      report->low_corrections = low_steps;
      report->resid0_probe_rel = r0_probe;
    }
    return rc;
  }
  if (launch_unpack_sym(X, t, n, A, lda, stream, o.fill_upper ? 0 : 1) != hipSuccess)
    return SPDINV_ERR_HIP;
  if (launch_info_out(ctrl, d_info, stream) != hipSuccess) return SPDINV_ERR_HIP;
  if (report) {
    if (hipStreamSynchronize(stream) != hipSuccess) return SPDINV_ERR_HIP;
    report->info = 0;
    report->status = 0;
    report->nb = NB;
    report->tiles = t;
    report->tasks = ntask;
    report->critical_path = dp->host.stats.cp_plan;
    report->workers = grid;
    report->refine_iters = iters;
    report->fell_back = 0;
    report->resid_fro_rel = rpred >= 0.0 ? rpred : rl;
    report->resid0_fro_rel = r0;
    report->resid_last_rel = rl;
    report->converged = converged;
    report->predicted = predicted;
    report->low_corrections = low_steps;
    report->resid0_probe_rel = r0_probe;
  }
  return 0;
}

}  // namespace

extern "C" {

void spdinv_default_opts(spdinv_opts* opts) {
  if (opts) *opts = defaults();
}

size_t spd_inverse_workspace_bytes(int n, spdinv_mode mode, const spdinv_opts* opts) {
  if (n <= 0) return 0;
  const spdinv_opts o = opts ? *opts : defaults();
  if (mode == SPDINV_MIXED_FP32 || mode == SPDINV_MIXED_BF16) return mixed_layout(n, o).total;
  if (mode == SPDINV_FP32) return fp32_layout(n).total;
  return layout(n, o).total;
}

int spd_inverse(int n, void* A_, int lda, spdinv_mode mode, void* work, size_t work_bytes,
                spdinv_stream_t stream_, const spdinv_opts* opts, int* d_info,
                spdinv_report* report) {
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  double* A = static_cast<double*>(A_);
  if (n < 0) return -1;
  if (n > 0 && !A) return -2;
  if (lda < (n > 1 ? n : 1)) return -3;
  if (mode != SPDINV_FP64 && mode != SPDINV_FP32 && mode != SPDINV_MIXED_FP32 &&
      mode != SPDINV_MIXED_BF16)
    return -4;
  const spdinv_opts o = opts ? *opts : defaults();
  if (check_opts(o)) return -8;
  const bool mixed = mode == SPDINV_MIXED_FP32 || mode == SPDINV_MIXED_BF16;
  if ((mixed || mode == SPDINV_FP32) &&
      (!o.renamed || o.trace || o.rename_tiles || o.tree_levels))
    return -8;
  if (report) std::memset(report, 0, sizeof(*report));
  if (n == 0) {
    if (d_info) {
      int zero = 0;
      if (hipMemcpyAsync(d_info, &zero, sizeof(int), hipMemcpyHostToDevice, stream) != hipSuccess)
        return SPDINV_ERR_HIP;
      if (hipStreamSynchronize(stream) != hipSuccess) return SPDINV_ERR_HIP;
    }
    return 0;
  }
  if (!work) return -5;
  if (mode == SPDINV_FP32)
    return run_fp32(n, static_cast<float*>(A_), lda, work, work_bytes, stream, o, d_info, report);
  if (mixed)
    return run_mixed(n, A, lda, work, work_bytes, stream, o, mode == SPDINV_MIXED_BF16, d_info,
                     report);
  return run_fp64(n, A, lda, work, work_bytes, stream, o, d_info, report);
}

// Shared argument checks of the FP64 entry points over one matrix.
static int fp64_entry(int n, double* A, int lda, void* work, size_t work_bytes,
                      spdinv_stream_t stream_, const spdinv_opts* opts, int* d_info,
                      spdinv_report* report, int steps) {
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  if (n < 0) return -1;
  if (n > 0 && !A) return -2;
  if (lda < (n > 1 ? n : 1)) return -3;
  const spdinv_opts o = opts ? *opts : defaults();
  // the steps on their own run the renamed plan in the standard layout
  if (check_opts(o) || !o.renamed || o.rename_tiles) return -7;
  if (report) std::memset(report, 0, sizeof(*report));
  if (n == 0) {
    if (d_info) {
      int zero = 0;
      if (hipMemcpyAsync(d_info, &zero, sizeof(int), hipMemcpyHostToDevice, stream) != hipSuccess)
        return SPDINV_ERR_HIP;
      if (hipStreamSynchronize(stream) != hipSuccess) return SPDINV_ERR_HIP;
    }
    return 0;
  }
  if (!work) return -4;
  return run_fp64(n, A, lda, work, work_bytes, stream, o, d_info, report, steps);
}

int spd_cholesky(int n, double* A, int lda, void* work, size_t work_bytes,
                 spdinv_stream_t stream, const spdinv_opts* opts, int* d_info,
                 spdinv_report* report) {
  return fp64_entry(n, A, lda, work, work_bytes, stream, opts, d_info, report, 1);
}

int spd_inverse_from_factor(int n, double* L, int ldl, void* work, size_t work_bytes,
                            spdinv_stream_t stream, const spdinv_opts* opts, int* d_info,
                            spdinv_report* report) {
  return fp64_entry(n, L, ldl, work, work_bytes, stream, opts, d_info, report, 6);
}

size_t spd_solve_workspace_bytes(int n, int nrhs, const spdinv_opts* opts) {
  if (n < 0 || nrhs < 0) return 0;
  const spdinv_opts o = opts ? *opts : defaults();
  return layout(n, o, nrhs).total;
}

// The solve entry points: the factor (steps 1, with_factor = 0) or a given
// one (with_factor = 1), then the forward and backward substitutions.
static int solve_entry(int n, int nrhs, double* A, int lda, double* Bm, int ldb, void* work,
                       size_t work_bytes, spdinv_stream_t stream_, const spdinv_opts* opts,
                       int* d_info, spdinv_report* report, bool with_factor) {
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  if (n < 0) return -1;
  if (nrhs < 0 || nrhs > 64 * NB) return -2;
  if (n > 0 && !A) return -3;
  if (lda < (n > 1 ? n : 1)) return -4;
  if (n > 0 && nrhs > 0 && !Bm) return -5;
  if (ldb < (n > 1 ? n : 1)) return -6;
  const spdinv_opts o = opts ? *opts : defaults();
  if (check_opts(o) || !o.renamed || o.rename_tiles) return -10;
  if (report) std::memset(report, 0, sizeof(*report));
  if (n == 0) {
    if (d_info) {
      int zero = 0;
      if (hipMemcpyAsync(d_info, &zero, sizeof(int), hipMemcpyHostToDevice, stream) != hipSuccess)
        return SPDINV_ERR_HIP;
      if (hipStreamSynchronize(stream) != hipSuccess) return SPDINV_ERR_HIP;
    }
    return 0;
  }
  if (!work) return -7;
  const int steps = (with_factor ? 0 : 1) | (nrhs > 0 ? 8 : 0);
  if (steps == 0) {  // a given factor and no right-hand side: nothing to do
    if (d_info) {
      int zero = 0;
      if (hipMemcpyAsync(d_info, &zero, sizeof(int), hipMemcpyHostToDevice, stream) != hipSuccess)
        return SPDINV_ERR_HIP;
      if (hipStreamSynchronize(stream) != hipSuccess) return SPDINV_ERR_HIP;
    }
    return 0;
  }
  return run_fp64(n, A, lda, work, work_bytes, stream, o, d_info, report, steps, nrhs, Bm, ldb);
}

int spd_solve(int n, int nrhs, double* A, int lda, double* B, int ldb, void* work,
              size_t work_bytes, spdinv_stream_t stream, const spdinv_opts* opts, int* d_info,
              spdinv_report* report) {
  return solve_entry(n, nrhs, A, lda, B, ldb, work, work_bytes, stream, opts, d_info, report,
                     false);
}

int spd_solve_from_factor(int n, int nrhs, const double* L, int ldl, double* B, int ldb,
                          void* work, size_t work_bytes, spdinv_stream_t stream,
                          const spdinv_opts* opts, int* d_info, spdinv_report* report) {
  return solve_entry(n, nrhs, const_cast<double*>(L), ldl, B, ldb, work, work_bytes, stream, opts,
                     d_info, report, true);
}

// ---- allocation-free entry point -------------------------------------------
// Plans whose device tables live in the device scratch, and per device the
// plan whose tables the scratch currently holds (uploaded again only when a
// call needs another one).
static_assert(NOALLOC_SCRATCH_BYTES == SPDINV_NOALLOC_SCRATCH_BYTES, "scratch size in the header");
static_assert(NOALLOC_MAX_N == SPDINV_NOALLOC_MAX_N, "largest order in the header");
static_assert(NOALLOC_MAX_N <= MAX_BATCH_T * NB, "the pool is sized for 16 tiles per side");
static std::map<Key, std::unique_ptr<DevPlan>> g_static_plans;
static std::map<int, Key> g_static_loaded;

int spd_inverse_noalloc(int n, double* A, int lda, spdinv_stream_t stream_,
                        const spdinv_opts* opts, int* d_info) {
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  if (n < 0 || n > SPDINV_NOALLOC_MAX_N) return -1;
  if (n > 0 && !A) return -2;
  if (lda < (n > 1 ? n : 1)) return -3;
  const spdinv_opts o0 = opts ? *opts : defaults();
  if (check_opts(o0) || o0.trace || o0.tree_levels) return -5;
  if (n == 0) return launch_info_zero(d_info, stream) == hipSuccess ? 0 : SPDINV_ERR_HIP;
  const spdinv_opts o = tuned_fp64(o0, tiles_for(n));
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return SPDINV_ERR_HIP;
  char* scratch = nullptr;
  size_t scratch_bytes = 0;
  if (noalloc_scratch((void**)&scratch, &scratch_bytes) != hipSuccess) return SPDINV_ERR_HIP;
  char* tables = scratch;
  char* work = scratch + NOALLOC_PLAN_BYTES;
  const size_t work_bytes = scratch_bytes - NOALLOC_PLAN_BYTES;
  const Layout L = layout(n, o);
  if (L.total > work_bytes) return SPDINV_ERR_WORKSPACE;  // not reached for n <= the maximum
  const int t = tiles_for(n);
  const int grid = grid_for(device, t, o);
  const Key k = plan_key(device, t, o, grid, chain_for(o), 7, 0, true);
  DevPlan* dp = nullptr;
  bool upload = false;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_static_plans.find(k);
    if (it == g_static_plans.end()) {
      std::unique_ptr<DevPlan> p = build_dev_plan(k);
      if (p->image.bytes.size() > NOALLOC_PLAN_BYTES) return SPDINV_ERR_WORKSPACE;
      bind_tables(p.get(), tables);
      it = g_static_plans.emplace(k, std::move(p)).first;
    }
    dp = it->second.get();
    auto ld = g_static_loaded.find(device);
    upload = ld == g_static_loaded.end() || ld->second < k || k < ld->second;
    if (upload) g_static_loaded[device] = k;
  }
  // the image stays in the host cache for the life of the process, so the
  // copy may complete after this call returns
  if (upload && hipMemcpyAsync(tables, dp->image.bytes.data(), dp->image.bytes.size(),
                               hipMemcpyHostToDevice, stream) != hipSuccess) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_static_loaded.erase(device);
    return SPDINV_ERR_HIP;
  }
  return run_fp64(n, A, lda, work, work_bytes, stream, o, d_info, nullptr, 7, 0, nullptr, 1, dp);
}

// ---- autotuner ---------------------------------------------------------------
}  // extern "C"

namespace {

// Median over reps of one timed call (HIP events on `stream`); prep runs
// before each call, untimed.  Returns a negative value on an error.
template <class Prep, class Call>
double time_median(hipStream_t stream, int reps, Prep prep, Call call) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1.0;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1.0;
  }
  std::vector<double> ms;
  bool ok = true;
  for (int r = 0; r < reps && ok; ++r) {
    ok = prep() == hipSuccess && hipEventRecord(e0, stream) == hipSuccess && call() == 0 &&
         hipEventRecord(e1, stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    float v = 0.0f;
    ok = ok && hipEventElapsedTime(&v, e0, e1) == hipSuccess;
    ms.push_back(v);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!ok) return -1.0;
  std::sort(ms.begin(), ms.end());
  return ms[ms.size() / 2];
}

// Device buffers of a tuning run, freed on every exit.
struct DevBufs {
  std::vector<void*> p;
  void* get(size_t bytes, hipError_t* e) {
    void* q = nullptr;
    *e = hipMalloc(&q, bytes ? bytes : 1);
    if (*e == hipSuccess) p.push_back(q);
    return *e == hipSuccess ? q : nullptr;
  }
  ~DevBufs() {
    for (void* q : p) (void)hipFree(q);
  }
};

}  // namespace

extern "C" {

int spdinv_autotune(int n, int reps, spdinv_stream_t stream_, spdinv_tuning* out) {
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  if (n < 1 || n > 65536) return -1;
  if (reps < 1) reps = 3;
  const int t = tiles_for(n);
  // the built-in choice, then coordinate descent over one knob at a time
  TunedFp64 best{t >= kWideTiles ? 2 : 1, kDefaultChain, t < kWideTiles ? 4 : 2};
  const int per_cu_c[] = {1, 2}, chain_c[] = {6, 8, 12}, split_c[] = {0, 2, 4};
  size_t wmax = 0;
  for (int pc : per_cu_c)
    for (int sp : split_c) {
      spdinv_opts o = defaults();
      o.per_cu = pc;
      o.parts = sp;
      o.no_split = sp == 0;
      wmax = std::max(wmax, layout(n, o).total);
    }
  DevBufs bufs;
  hipError_t e = hipSuccess;
  double* A0 = (double*)bufs.get((size_t)n * n * sizeof(double), &e);
  double* A = (double*)bufs.get((size_t)n * n * sizeof(double), &e);
  void* work = bufs.get(wmax, &e);
  void** ptr = (void**)bufs.get(sizeof(void*), &e);
  int* ord = (int*)bufs.get(sizeof(int), &e);
  if (e != hipSuccess) return SPDINV_ERR_HIP;
  if (hipMemcpyAsync(ptr, &A0, sizeof(void*), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(ord, &n, sizeof(int), hipMemcpyHostToDevice, stream) != hipSuccess ||
      launch_fill_spd(ptr, ord, 1, false, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return SPDINV_ERR_HIP;
  int count = 0;
  auto measure = [&](const TunedFp64& c) -> double {
    spdinv_opts o = defaults();
    o.per_cu = c.per_cu;
    o.chain = c.chain;
    o.parts = c.split;
    o.no_split = c.split == 0;
    auto prep = [&]() {
      return hipMemcpyAsync(A, A0, (size_t)n * n * sizeof(double), hipMemcpyDeviceToDevice, stream);
    };
    auto call = [&]() {
      return spd_inverse(n, A, n, SPDINV_FP64, work, wmax, (spdinv_stream_t)stream, &o, nullptr,
                         nullptr);
    };
    if (time_median(stream, 1, prep, call) < 0.0) return -1.0;  // plan and warm-up
    ++count;
    return time_median(stream, reps, prep, call);
  };
  const double ms_default = measure(best);
  if (ms_default < 0.0) return SPDINV_ERR_HIP;
  double ms_best = ms_default;
  for (int dim = 0; dim < 3; ++dim) {
    const int* cand = dim == 0 ? per_cu_c : dim == 1 ? chain_c : split_c;
    const int nc = dim == 0 ? 2 : 3;
    TunedFp64 base = best;
    for (int q = 0; q < nc; ++q) {
      TunedFp64 c = base;
      (dim == 0 ? c.per_cu : dim == 1 ? c.chain : c.split) = cand[q];
      if (c.per_cu == base.per_cu && c.chain == base.chain && c.split == base.split) continue;
      const double ms = measure(c);
      if (ms < 0.0) return SPDINV_ERR_HIP;
      if (ms < ms_best) {
        ms_best = ms;
        best = c;
      }
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_tuned64[t] = best;
  }
  if (out) {
    std::memset(out, 0, sizeof(*out));
    out->nb = NB;
    out->per_cu = best.per_cu;
    out->chain = best.chain;
    out->parts = best.split;
    out->ms = ms_best;
    out->ms_default = ms_default;
    out->candidates = count;
  }
  return 0;
}

int spdinv_autotune_batched(int batch, const int* h_n, spdinv_mode mode, int reps,
                            spdinv_stream_t stream_, spdinv_tuning* out) {
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  if (batch < 1 || batch > MAX_BATCH) return -1;
  if (!h_n) return -2;
  for (int i = 0; i < batch; ++i)
    if (h_n[i] < 0 || h_n[i] > MAX_BATCH_T * NB) return -2;
  if (mode != SPDINV_FP64 && mode != SPDINV_FP32) return -3;
  if (reps < 1) reps = 3;
  const bool fp32 = mode == SPDINV_FP32;
  const size_t es = fp32 ? sizeof(float) : sizeof(double);
  // candidates: one workgroup per matrix, the list-scheduled DAG, groups of
  // 512; chains of 1, 4 and 8 products
  std::vector<TunedBatch> cand;
  for (int g : {-1, -2, 512})
    for (int c : {1, 4, 8}) cand.push_back(TunedBatch{g, c});
  std::vector<size_t> off(batch + 1, 0);
  for (int i = 0; i < batch; ++i) off[i + 1] = off[i] + (size_t)h_n[i] * h_n[i] * es;
  size_t wmax = 0;
  for (const TunedBatch& c : cand) {
    spdinv_opts o = defaults();
    o.batch_group = c.group;
    o.chain = c.chain;
    wmax = std::max(wmax, batched_spd_inverse_workspace_bytes(batch, h_n, mode, &o));
  }
  DevBufs bufs;
  hipError_t e = hipSuccess;
  char* A0 = (char*)bufs.get(off[batch], &e);
  char* A = (char*)bufs.get(off[batch], &e);
  void** p0 = (void**)bufs.get(batch * sizeof(void*), &e);
  void** p = (void**)bufs.get(batch * sizeof(void*), &e);
  int* dn = (int*)bufs.get(batch * sizeof(int), &e);
  void* work = bufs.get(wmax, &e);
  if (e != hipSuccess) return SPDINV_ERR_HIP;
  std::vector<void*> hp0(batch), hp(batch);
  for (int i = 0; i < batch; ++i) {
    hp0[i] = A0 + off[i];
    hp[i] = A + off[i];
  }
  if (hipMemcpy(p0, hp0.data(), batch * sizeof(void*), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p, hp.data(), batch * sizeof(void*), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dn, h_n, batch * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      launch_fill_spd(p0, dn, batch, fp32, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return SPDINV_ERR_HIP;
  TunedBatch best{0, 0};
  double ms_best = -1.0, ms_default = -1.0;
  int count = 0;
  for (const TunedBatch& c : cand) {
    spdinv_opts o = defaults();
    o.batch_group = c.group;
    o.chain = c.chain;
    auto prep = [&]() { return hipMemcpyAsync(A, A0, off[batch], hipMemcpyDeviceToDevice, stream); };
    auto call = [&]() {
      return batched_spd_inverse(batch, h_n, dn, p, dn, mode, work, wmax,
                                 (spdinv_stream_t)stream, &o, nullptr);
    };
    if (time_median(stream, 1, prep, call) < 0.0) return SPDINV_ERR_HIP;
    ++count;
    const double ms = time_median(stream, reps, prep, call);
    if (ms < 0.0) return SPDINV_ERR_HIP;
    // the built-in choice: the schedule picked by batch size, chain 8
    const int builtin = batch >= 2 * kBatchSimWorkers ? -1 : -2;
    if (c.group == builtin && (fp32 || c.chain == kDefaultChain)) ms_default = ms;
    if (ms_best < 0.0 || ms < ms_best) {
      ms_best = ms;
      best = c;
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_tuned_batch[batch_key(fp32, h_n, batch)] = best;
  }
  if (out) {
    std::memset(out, 0, sizeof(*out));
    out->nb = NB;
    out->chain = best.chain;
    out->batch_group = best.group;
    out->ms = ms_best;
    out->ms_default = ms_default;
    out->candidates = count;
  }
  return 0;
}

int spdinv_tuning_clear(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_tuned64.clear();
  g_tuned_batch.clear();
  return 0;
}

int spdinv_tuning_save(const char* path) {
  if (!path) return -1;
  FILE* f = std::fopen(path, "w");
  if (!f) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  std::fprintf(f, "spdinv-tuning 1\n");
  for (const auto& kv : g_tuned64)
    std::fprintf(f, "fp64 %d %d %d %d\n", kv.first, kv.second.per_cu, kv.second.chain,
                 kv.second.split);
  for (const auto& kv : g_tuned_batch) {
    std::fprintf(f, "batch %d %d %d", kv.first.first, kv.second.group, kv.second.chain);
    for (int c : kv.first.second) std::fprintf(f, " %d", c);
    std::fprintf(f, "\n");
  }
  const int rc = std::fclose(f) == 0 ? 0 : -1;
  return rc;
}

int spdinv_tuning_load(const char* path) {
  if (!path) return -1;
  FILE* f = std::fopen(path, "r");
  if (!f) return -1;
  char tag[32];
  int ver = 0;
  if (std::fscanf(f, "%31s %d", tag, &ver) != 2 || std::strcmp(tag, "spdinv-tuning") != 0 ||
      ver != 1) {
    std::fclose(f);
    return -2;
  }
  std::map<int, TunedFp64> t64;
  std::map<TBKey, TunedBatch> tb;
  int rc = 0;
  while (std::fscanf(f, "%31s", tag) == 1) {
    if (std::strcmp(tag, "fp64") == 0) {
      int t, pc, ch, sp;
      if (std::fscanf(f, "%d %d %d %d", &t, &pc, &ch, &sp) != 4 || t < 1 || pc < 1 || pc > 2 ||
          ch < 1 || ch > MAX_CHAIN || (sp != 0 && sp != 2 && sp != 4)) {
        rc = -2;
        break;
      }
      t64[t] = TunedFp64{pc, ch, sp};
    } else if (std::strcmp(tag, "batch") == 0) {
      int fp, g, ch;
      if (std::fscanf(f, "%d %d %d", &fp, &g, &ch) != 3 || g < -2 || ch < 1 || ch > MAX_CHAIN) {
        rc = -2;
        break;
      }
      std::vector<int> counts(MAX_BATCH_T + 1, 0);
      for (int k = 0; k <= MAX_BATCH_T && rc == 0; ++k)
        if (std::fscanf(f, "%d", &counts[k]) != 1) rc = -2;
      if (rc) break;
      tb[TBKey(fp ? 1 : 0, counts)] = TunedBatch{g, ch};
    } else {
      rc = -2;
      break;
    }
  }
  std::fclose(f);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(g_mu);
  for (const auto& kv : t64) g_tuned64[kv.first] = kv.second;
  for (const auto& kv : tb) g_tuned_batch[kv.first] = kv.second;
  return 0;
}

void spdinv_release_plans(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_plans)
    if (kv.second->arena) (void)hipFree(kv.second->arena);
  g_plans.clear();
}

static PlanOptions plan_options(int t, const spdinv_opts* opts, int steps = 7) {
  const spdinv_opts o = opts ? *opts : defaults();
  PlanOptions po;
  po.t = t;
  po.renamed = o.renamed ? 1 : 0;
  po.loop_order = o.loop_order;
  po.pipelined = o.pipelined ? 1 : 0;
  po.trtri_first = o.trtri_first ? 1 : 0;
  po.chain = std::min(std::max(chain_for(o), 1), MAX_CHAIN);
  po.tree_levels = tree_for(o, steps);
  const long long budget = rename_budget(t, o, steps);
  if (budget) {
    const RenRows& r = renaming_rows(t, o, budget);
    po.ren_b = r.b;
    po.ren_c = r.c;
  }
  return po;
}

int spdinv_plan_stats_get(int t, const spdinv_opts* opts, spdinv_plan_stats* out) {
  if (t < 1 || t > 1024 || !out) return -1;
  Plan p;
  build_plan(plan_options(t, opts), 1, nullptr, &p);
  std::memset(out, 0, sizeof(*out));
  out->tasks = p.stats.ntasks;
  out->edges = p.stats.nedges;
  for (int k = 0; k < K_COUNT; ++k) out->count[k] = p.stats.count[k];
  for (int s = 0; s < 3; ++s) out->cp_step[s] = p.stats.cp_step[s];
  out->cp_unpipelined = p.stats.cp_unpipelined;
  out->cp_plan = p.stats.cp_plan;
  return 0;
}

int spdinv_plan_export(int t, const spdinv_opts* opts, int workers, int32_t* tasks8, int32_t* succ,
                       int32_t* step, int32_t* idx, int32_t* order, long long* ntasks,
                       long long* nsucc, int32_t* links, long long* nlinks) {
  return spdinv_plan_export_steps(7, 0, t, opts, workers, tasks8, succ, step, idx, order, ntasks,
                                  nsucc, links, nlinks);
}

int spdinv_plan_export_steps(int steps, int rhs_tiles, int t, const spdinv_opts* opts, int workers,
                             int32_t* tasks8, int32_t* succ, int32_t* step, int32_t* idx,
                             int32_t* order, long long* ntasks, long long* nsucc, int32_t* links,
                             long long* nlinks) {
  if (t < 1 || t > 1024) return -1;
  if (steps != 7 && steps != 1 && steps != 6 && steps != 9 && steps != 8) return -2;
  if ((steps & 8) ? (rhs_tiles < 1 || rhs_tiles > 64) : rhs_tiles != 0) return -2;
  Plan p;
  PlanOptions po = plan_options(t, opts, steps);
  po.steps = steps;
  po.rhs_tiles = rhs_tiles;
  po.split = split_for(opts ? *opts : defaults(), t, workers);
  build_plan(po, workers > 0 ? workers : 1, kCost, &p);
  if (ntasks) *ntasks = (long long)p.tasks.size();
  if (nsucc) *nsucc = (long long)p.succ.size();
  if (tasks8) std::memcpy(tasks8, p.tasks.data(), p.tasks.size() * sizeof(DevTask));
  if (succ && !p.succ.empty()) std::memcpy(succ, p.succ.data(), p.succ.size() * sizeof(int32_t));
  if (step) std::memcpy(step, p.step.data(), p.step.size() * sizeof(int32_t));
  if (idx) std::memcpy(idx, p.idx.data(), p.idx.size() * sizeof(int32_t));
  if (order) std::memcpy(order, p.order.data(), p.order.size() * sizeof(int32_t));
  if (nlinks) *nlinks = (long long)p.links.size();
  if (links && !p.links.empty())
    std::memcpy(links, p.links.data(), p.links.size() * sizeof(int32_t));
  return 0;
}

int spdinv_batch_template_export(int t, spdinv_mode mode, const spdinv_opts* opts,
                                 int32_t* tasks8, int32_t* succ, int32_t* links, long long* ntask,
                                 long long* nsucc, long long* nlinks) {
  if (t < 1 || t > MAX_BATCH_T) return -1;
  if (mode != SPDINV_FP64 && mode != SPDINV_FP32) return -2;
  const spdinv_opts o = opts ? *opts : defaults();
  if (check_opts(o)) return -3;
  std::lock_guard<std::mutex> lk(g_mu);
  const BTemplate* bt = btemplate_host(t, mode == SPDINV_FP32, o);
  if (ntask) *ntask = bt->ntask;
  if (nsucc) *nsucc = (long long)bt->succ.size();
  if (nlinks) *nlinks = (long long)bt->links.size() / 2;
  if (tasks8) std::memcpy(tasks8, bt->tasks.data(), bt->tasks.size() * sizeof(DevTask));
  if (succ && !bt->succ.empty())
    std::memcpy(succ, bt->succ.data(), bt->succ.size() * sizeof(int32_t));
  if (links && !bt->links.empty())
    std::memcpy(links, bt->links.data(), bt->links.size() * sizeof(int32_t));
  return 0;
}

long long spdinv_batch_plan_export(int batch, const int* h_n, spdinv_mode mode,
                                   const spdinv_opts* opts, int workers, int32_t* disp,
                                   int32_t* mat4) {
  if (batch < 1 || batch > MAX_BATCH || !h_n) return -1;
  if (mode != SPDINV_FP64 && mode != SPDINV_FP32) return -2;
  for (int i = 0; i < batch; ++i)
    if (h_n[i] < 0 || h_n[i] > MAX_BATCH_T * NB) return -1;
  const spdinv_opts o = tuned_batch(opts ? *opts : defaults(), mode == SPDINV_FP32, h_n, batch);
  if (check_opts(o)) return -3;
  std::vector<int8_t> tv(batch);
  for (int i = 0; i < batch; ++i) {
    if (h_n[i] < 0 || h_n[i] > MAX_BATCH_T * NB) return -1;
    tv[i] = (int8_t)tiles_of_order(h_n[i]);
  }
  BCompHost hc;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    const BTemplate* tmpl[MAX_BATCH_T + 1] = {};
    for (int i = 0; i < batch; ++i)
      if (!tmpl[tv[i]]) tmpl[tv[i]] = btemplate_host(tv[i], mode == SPDINV_FP32, o);
    const int w = workers > 0 ? workers : 1;
    if (build_bcomp(tv, tmpl, batch_schedule(batch, o, w), w, &hc)) return -4;
  }
  if (disp) std::memcpy(disp, hc.disp.data(), hc.disp.size() * sizeof(int32_t));
  if (mat4) std::memcpy(mat4, hc.mat.data(), hc.mat.size() * sizeof(int4));
  return (long long)hc.disp.size();
}

long long spdinv_trace_copy(const void* work, int n, const spdinv_opts* opts, int64_t* host,
                            long long max_tasks) {
  if (!work || !host || n <= 0 || !opts || !opts->trace) return -1;
  const spdinv_opts o = tuned_fp64(*opts, tiles_for(n));
  const Layout L = layout(n, o);
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return -2;
  hipError_t err = hipSuccess;
  DevPlan* dp = get_plan(device, tiles_for(n), o, grid_for(device, tiles_for(n), o),
                        chain_for(o), &err, 7, 0, true);
  if (!dp) return -2;
  const Plan& p = dp->host;
  const long long nt = (long long)p.tasks.size();
  // the device records by dispatch position; the host order is program order
  std::vector<long long> dev((size_t)nt * 4);
  if (hipMemcpy(dev.data(), (const char*)work + L.trace, (size_t)nt * 4 * sizeof(long long),
                hipMemcpyDeviceToHost) != hipSuccess)
    return -2;
  const long long m = nt < max_tasks ? nt : max_tasks;
  for (long long k = 0; k < nt; ++k) {
    const long long v = p.order[k];
    if (v < m)
      for (int f = 0; f < 4; ++f) host[4 * v + f] = dev[4 * k + f];
  }
  return m;
}

int spdinv_kernel_timer(int enable) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_timer.on = enable != 0;
  g_timer.used = 0;
  return 0;
}

double spdinv_kernel_timer_read(long long* launches) {
  std::lock_guard<std::mutex> lk(g_mu);
  double total = 0.0;
  for (size_t k = 0; k < g_timer.used; ++k) {
    float ms = 0.0f;
    if (hipEventSynchronize(g_timer.ev[k].second) != hipSuccess) return -1.0;
    if (hipEventElapsedTime(&ms, g_timer.ev[k].first, g_timer.ev[k].second) != hipSuccess) return -1.0;
    total += ms;
  }
  if (launches) *launches = (long long)g_timer.used;
  g_timer.used = 0;
  return total;
}

const char* spdinv_version(void) { return "spdinv 0.1 (gfx950, FP64 tile inverse)"; }

}  // extern "C"
