// The persistent worker loop of the dependency-tracked scheduler, shared by
// the FP64 scheduler (device.hip) and the FP32 one of the mixed-precision
// form (mixed.hip); run(task) executes one tile task with the whole
// workgroup.
#pragma once
#include "device.hpp"
#include "mfma_tile.hpp"

namespace spdinv {
namespace {

using tile::now_ticks;
using tile::stores_complete;

// Persistent worker loop.  On the device the tasks are numbered in dispatch
// order (the planner's list-scheduling order, a topological order), so a
// dispatch ticket is the task id itself.  Thread 0 claims tickets and waits
// until a claimed task's in-degree is zero; since tickets are topological,
// every claimed task's predecessors hold earlier tickets, which makes the
// loop deadlock-free for any number of resident workgroups.
// Latency hiding at the task boundary:
//  - the ticket for the next task is claimed while the current task's
//    stores drain (its readiness is tested only after the current task has
//    released its successors, so a claimed task that depends on the current
//    one cannot block it);
//  - thread 0 fetches the task descriptor together with the first
//    in-degree poll and hands it to the workgroup through LDS;
//  - the successor ids are loaded when the task starts, one per thread, so
//    that at its end (once every thread's stores have completed) the threads
//    release the successors with parallel in-degree decrements.
// Every divergent region (the thread-0 claim and poll, the release) sits
// between workgroup barriers, which keeps the loop body, and every barrier
// in it, one level deep.  Counters and tiles are accessed with agent-scope
// coherence, so no cache maintenance is needed.
template <class Run>
__device__ __forceinline__ void sched_loop(const SchedArgs& g, Run run) {
  __shared__ int s_task;
  __shared__ int s_skip;
  __shared__ __attribute__((aligned(16))) DevTask s_desc;
  static_assert(sizeof(DevTask) == 32, "the descriptor moves as two 16-byte vectors");
  int prev = -1;   // meaningful in thread 0 only
  int claim = -1;  // thread 0: ticket claimed during the previous task (or -1)
  long long t_claim = 0;
  for (;;) {
    if (threadIdx.x == 0) {
      if (prev >= 0) {
        if (g.trace) g.trace[4 * (size_t)prev + 3] = now_ticks();
        __hip_atomic_fetch_add(&g.ctrl[CTRL_DONE], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (claim < 0) {
        if (g.trace) t_claim = now_ticks();
        claim = __hip_atomic_fetch_add(&g.ctrl[CTRL_TICKET], 1, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
      }
      int v = claim < g.ntask ? claim : -1;
      claim = -1;
      if (v >= 0) {
        // the descriptor and the first in-degree poll are in flight
        // together; the descriptor goes to LDS as soon as it arrives (every
        // thread copied the previous one two barriers ago), so that it is
        // not held in registers across the wait
        // (moved as two 16-byte vectors: a struct copy would go through
        // private memory)
        typedef int i4v __attribute__((ext_vector_type(4)));
        const i4v* src = reinterpret_cast<const i4v*>(g.tasks + v);
        const i4v d0 = src[0], d1 = src[1];
        int deg = __hip_atomic_load(&g.indeg[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
          deg = __hip_atomic_load(&g.indeg[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      if (v >= 0) {
        if (g.trace) {
          g.trace[4 * (size_t)v + 0] = blockIdx.x;
          g.trace[4 * (size_t)v + 1] = t_claim;
          g.trace[4 * (size_t)v + 2] = now_ticks();
        }
        s_skip = __hip_atomic_load(&g.ctrl[CTRL_FAILED], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      s_task = v;
      prev = v;
    }
    __syncthreads();
    // s_task and s_skip hold one value for the whole workgroup; reading them
    // through readfirstlane makes the loop exit and the task dispatch
    // wave-uniform
    const int v = __builtin_amdgcn_readfirstlane(s_task);
    if (v < 0) break;
    const DevTask t = s_desc;
    const int nsucc = t.succ_end - t.succ_begin;
    const int my_succ = (int)threadIdx.x < nsucc ? g.succ[t.succ_begin + threadIdx.x] : -1;
    if (!__builtin_amdgcn_readfirstlane(s_skip)) run(t);
    // claim the next ticket while the stores drain
    if (threadIdx.x == 0) {
      if (g.trace) t_claim = now_ticks();
      claim = __hip_atomic_fetch_add(&g.ctrl[CTRL_TICKET], 1, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
    }
    stores_complete();
    __syncthreads();
    // every store of the task has completed: release its successors
    if (my_succ >= 0)
      __hip_atomic_fetch_sub(&g.indeg[my_succ], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int e = threadIdx.x + NTHREADS; e < nsucc; e += NTHREADS)
      __hip_atomic_fetch_sub(&g.indeg[g.succ[t.succ_begin + e]], 1, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    // convergence point: the divergent release and the thread-0 region at
    // the loop head must not be merged across the back edge (the loop body,
    // with its barriers, has to stay one level deep)
    __syncthreads();
  }
}

}  // namespace
}  // namespace spdinv
