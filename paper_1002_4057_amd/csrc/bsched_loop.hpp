// The persistent worker loop of the batched form: one dependency-tracked DAG
// over every matrix of a batch, run by the same kind of persistent workers
// as the single-matrix scheduler (sched_loop.hpp).
//
// Each matrix of tile count t runs the task template of t: the plan of
// Algorithm 1 (renamed, UDU, pipelined) for one matrix in a topological
// order, with a copy-in task first (column-major lower triangle -> the
// matrix's own tile pool) and a copy-out task last; a matrix of at most NB
// rows is a single task that inverts it in LDS.  The host interleaves the
// templates of the matrices into one dispatch list (ticket -> matrix m,
// template position k); every template is topological and matrices share no
// tiles, so the list is topological and the loop is deadlock-free for any
// number of resident workgroups, as in sched_loop.  In-degree counters are
// per (matrix, task); a matrix whose factorization broke down skips its
// remaining tasks but still runs its copy-out task, which reports its INFO.
// Matrices that run one after another may share a pool slot: the copy-out
// task of the earlier one releases the copy-in task of the later one (an
// edge the host's dispatch order respects).
#pragma once
#include "device.hpp"
#include "mfma_tile.hpp"

namespace spdinv {
namespace {

using tile::now_ticks;
using tile::stores_complete;

// run(desc, m, t, k) executes template task k (descriptor desc) of matrix m
// (tile count t) with the whole workgroup.
template <class Run>
__device__ __forceinline__ void bsched_loop(const BSchedArgs& g, Run run) {
  __shared__ int s_v, s_m, s_t, s_skip;
  __shared__ __attribute__((aligned(16))) DevTask s_desc;
  static_assert(sizeof(DevTask) == 32, "the descriptor moves as two 16-byte vectors");
  int prev = -1;   // thread 0
  int claim = -1;  // thread 0: ticket claimed during the previous task (or -1)
  for (;;) {
    if (threadIdx.x == 0) {
      if (prev >= 0)
        __hip_atomic_fetch_add(&g.ctrl[CTRL_DONE], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (claim < 0)
        claim = __hip_atomic_fetch_add(&g.ctrl[CTRL_TICKET], 1, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
      int v = claim < g.ntotal ? claim : -1;
      claim = -1;
      int m = 0, t = 0;
      if (v >= 0) {
        const int e = g.disp[v];
        m = e >> BT_SHIFT;
        const int k = e & BT_MASK;
        const int4 mi = g.mat[m];
        t = mi.x & BM_T;
        typedef int i4v __attribute__((ext_vector_type(4)));
        const i4v* src = reinterpret_cast<const i4v*>(g.tmpl[t] + k);
        const i4v d0 = src[0], d1 = src[1];
        int32_t* cnt = g.indeg + mi.y + k;
        int deg = __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        reinterpret_cast<i4v*>(&s_desc)[0] = d0;
        reinterpret_cast<i4v*>(&s_desc)[1] = d1;
        // bounded wait: gives up after spin_limit ticks of the 100 MHz clock
        const long long t0 = now_ticks();
        long long spins = 0;
        while (deg > 0) {
          __builtin_amdgcn_s_sleep(1);
          if ((++spins & 63) == 0) {
            if (__hip_atomic_load(&g.ctrl[CTRL_ABORT], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
              v = -1;
              break;
            }
            if (now_ticks() - t0 > g.spin_limit) {
              __hip_atomic_store(&g.ctrl[CTRL_ABORT], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              v = -1;
              break;
            }
          }
          deg = __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (v >= 0) {
          // the copy-out task runs after a failure too: it reports INFO
          const int kind = d0.x & 0xff;
          s_skip = kind == K_BCOPYOUT ? 0
                                      : __hip_atomic_load(&g.mctrl[CTRL_WORDS * m + CTRL_FAILED],
                                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      s_v = v;
      s_m = m;
      s_t = t;
      prev = v;
    }
    __syncthreads();
    const int v = __builtin_amdgcn_readfirstlane(s_v);
    if (v < 0) break;
    const int m = __builtin_amdgcn_readfirstlane(s_m);
    const int t = __builtin_amdgcn_readfirstlane(s_t);
    const DevTask d = s_desc;
    const int base = __builtin_amdgcn_readfirstlane(g.mat[m].y);
    const int nsucc = d.succ_end - d.succ_begin;
    const int32_t* succ = g.tsucc[t];
    const int my_succ = (int)threadIdx.x < nsucc ? base + succ[d.succ_begin + threadIdx.x] : -1;
    if (!__builtin_amdgcn_readfirstlane(s_skip)) run(d, m, t);
    if (threadIdx.x == 0)
      claim = __hip_atomic_fetch_add(&g.ctrl[CTRL_TICKET], 1, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
    stores_complete();
    __syncthreads();
    // every store of the task has completed: release its successors
    if (my_succ >= 0)
      __hip_atomic_fetch_sub(&g.indeg[my_succ], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int e = threadIdx.x + NTHREADS; e < nsucc; e += NTHREADS)
      __hip_atomic_fetch_sub(&g.indeg[base + succ[d.succ_begin + e]], 1, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    // the copy-out task frees the matrix's pool slot for its next occupant
    if (threadIdx.x == 0 && (d.kind & 0xff) == K_BCOPYOUT) {
      const int nxt = g.mat[m].w;
      if (nxt >= 0)
        __hip_atomic_fetch_sub(&g.indeg[nxt], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
  }
}

// One workgroup per matrix: claims a matrix, runs its template's tasks in
// template order (a topological order, so every task is ready when it runs:
// the previous task's stores have completed before the barrier), skipping
// to the copy-out task once the matrix's factorization broke down.
// As in sched_loop, the thread-0 region (the count of the previous matrix
// and the next claim) is the only divergent region and sits between
// barriers, with a barrier closing the loop body: a thread-0 region at the
// end of the body, adjacent to the claim across the back edge, lets the
// compiler nest loops around a barrier.
template <class Run>
__device__ __forceinline__ void bseq_loop(const BSchedArgs& g, Run run) {
  __shared__ int s_m;
  bool counted = true;  // thread 0: the previous matrix is counted
  for (;;) {
    if (threadIdx.x == 0) {
      if (!counted)
        __hip_atomic_fetch_add(&g.ctrl[CTRL_DONE], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int v = __hip_atomic_fetch_add(&g.ctrl[CTRL_TICKET], 1, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
      s_m = v < g.ntotal ? (g.disp[v] >> BT_SHIFT) : -1;
      counted = s_m < 0;
    }
    __syncthreads();
    const int m = __builtin_amdgcn_readfirstlane(s_m);
    if (m < 0) break;
    const int t = __builtin_amdgcn_readfirstlane(g.mat[m].x) & BM_T;
    const int nt = g.tntask[t];
    int32_t* failed = &g.mctrl[CTRL_WORDS * m + CTRL_FAILED];
    for (int k = 0; k < nt; ++k) {
      const DevTask d = g.tmpl[t][k];
      const bool last = k == nt - 1;
      if (!last && __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                       failed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)))
        continue;
      run(d, m, t);
      stores_complete();
      __syncthreads();
    }
    __syncthreads();  // convergence point before the next claim
  }
}

}  // namespace
}  // namespace spdinv
