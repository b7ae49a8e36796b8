// Batched form of the SPD inverse on gfx950 (MI355X): many independent
// matrices of uneven order as one dependency-tracked DAG, run by one
// persistent launch (own translation unit, so that its kernel does not share
// out-of-line code with the single-matrix scheduler).
//
// Every matrix runs the task template of its tile count t = ceil(n / NB):
// its own copy-in, the tile tasks of Algorithm 1 (renamed, UDU, pipelined,
// the scheduler's own tile kernels) on its own tile pool, its copy-out; a
// matrix with n <= NB is one task that inverts it in LDS.  The host
// interleaves the templates (bsched_loop.hpp), so the workers run the tasks
// of many matrices side by side and no worker idles while one matrix waits
// on its diagonal-tile chain.
#include "bsched_loop.hpp"
#include "device.hpp"
#include "small_inverse.hpp"
#include "tile_tasks.hpp"

namespace spdinv {
namespace {

__device__ __forceinline__ void tri_decode_b(int x, int& ti, int& tj) {
  int i = 0;
  while ((i + 1) * (i + 2) / 2 <= x) ++i;
  ti = i;
  tj = x - i * (i + 1) / 2;
}

// Lower triangle of A (column-major, lda, order n, t = ceil(n/NB) tiles per
// side) -> the A tiles of the matrix's pool, identity padding beyond n
// (agent-coherent stores: other workgroups read the tiles).
__device__ void bcopy_in(const double* A, int lda, int n, int t, double* pool) {
  const int T = t * (t + 1) / 2;
  const int tid = threadIdx.x;
  for (int x = 0; x < T; ++x) {
    int ti, tj;
    tri_decode_b(x, ti, tj);
    const rsrc_t rd = tile_rsrc(tile_ptr(pool, x));
#pragma unroll 4
    for (int q = 0; q < NB * NB / 2 / NTHREADS; ++q) {
      const int e = 2 * (tid + NTHREADS * q), rr = e & (NB - 1), cc = e >> 7;
      const int gr = ti * NB + rr, gc = tj * NB + cc;
      double v[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = gr + h;
        if (r < n && gc < n)
          v[h] = (r >= gc) ? A[r + (size_t)lda * gc] : 0.0;
        else
          v[h] = (r == gc) ? 1.0 : 0.0;
      }
      st2(rd, e, d2{v[0], v[1]});
    }
  }
}

// A tiles of the pool -> lower triangle of A (and its mirror if fill_upper).
__device__ void bcopy_out(double* pool, int t, double* A, int lda, int n, int fill_upper) {
  const int T = t * (t + 1) / 2;
  const int tid = threadIdx.x;
  for (int x = 0; x < T; ++x) {
    int ti, tj;
    tri_decode_b(x, ti, tj);
    const rsrc_t rs = tile_rsrc(tile_ptr(pool, x));
#pragma unroll 4
    for (int q = 0; q < NB * NB / 2 / NTHREADS; ++q) {
      const int e = 2 * (tid + NTHREADS * q), rr = e & (NB - 1), cc = e >> 7;
      const int gc = tj * NB + cc;
      const d2 v = ld2(rs, e);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = ti * NB + rr + h;
        if (r < n && gc < n && r >= gc) {
          const double val = h ? v.y : v.x;
          A[r + (size_t)lda * gc] = val;
          if (fill_upper && r > gc) A[gc + (size_t)lda * r] = val;
        }
      }
    }
  }
}

__device__ __forceinline__ int load_uniform(int32_t* p) {
  return __builtin_amdgcn_readfirstlane(
      __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Two workgroups per CU: every task needs at most TASK_SMEM doubles of LDS
// and 256 registers per lane.
__global__ __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(2, 2)))
void bsched_kernel(BSchedArgs g) {
  __shared__ double smem[TASK_SMEM];
  auto run = [&](const DevTask& d, int m, int t) __attribute__((always_inline)) {
    const int kind = d.kind & 0xff;
    int32_t* mc = g.mctrl + CTRL_WORDS * m;
    int n, lda;
    double* A;
    if (kind == K_BSMALL) {
      int info = -1;
      if (batch_entry(g, m, 1, &n, &lda, &A))
        info = n ? small_inverse<double>(A, lda, n, g.fill_upper, smem) : 0;
      batch_info(g, m, info);
      return;
    }
    // one workgroup per matrix: the workgroup's own pool, else the matrix's slot
    const size_t first = g.seq ? (size_t)blockIdx.x * (size_t)g.wg_pool_tiles
                               : (size_t)__builtin_amdgcn_readfirstlane(g.mat[m].z);
    double* pool = static_cast<double*>(g.pool) + first * TILE;
    if (kind == K_BCOPYIN) {
      if (batch_entry(g, m, t, &n, &lda, &A)) {
        bcopy_in(A, lda, n, t, pool);
      } else if (threadIdx.x == 0) {  // every later task of the matrix is skipped
        __hip_atomic_store(&mc[CTRL_INFO], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&mc[CTRL_FAILED], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      return;
    }
    if (kind == K_BCOPYOUT) {
      if (load_uniform(&mc[CTRL_FAILED])) {
        batch_info(g, m, load_uniform(&mc[CTRL_INFO]));
        return;
      }
      batch_entry(g, m, t, &n, &lda, &A);  // checked by the copy-in task
      bcopy_out(pool, t, A, lda, n, g.fill_upper);
      batch_info(g, m, 0);
      return;
    }
    SchedArgs s{};
    s.pool = pool;
    s.ctrl = mc;
    s.links = g.tlinks[t];
    // the write-once read marks hold in a pool slot's first occupant only:
    // a later occupant's reads could meet lines of the earlier one in an L2
    // (a workgroup's own pool is reused by each of its matrices)
    s.coherent_only =
        (g.seq || (__builtin_amdgcn_readfirstlane(g.mat[m].x) & BM_PREV)) ? 1 : 0;
    s.last_valid = __builtin_amdgcn_readfirstlane(g.n[m]) - (t - 1) * NB;
    s.info_base = 0;
    s.d_base = g.tdbase[t];
    run_task<true>(d, s, smem, t * (t + 1) / 2, t);
  };
  if (g.seq)
    bseq_loop(g, run);
  else
    bsched_loop(g, run);
}

__global__ void breset_kernel(BSchedArgs g, int batch) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x < g.ntotal && !g.seq) {
    const int e = g.disp[x];
    const int m = e >> BT_SHIFT, k = e & BT_MASK;
    const int4 mi = g.mat[m];
    g.indeg[mi.y + k] = g.tindeg0[mi.x & BM_T][k] + ((k == 0 && (mi.x & BM_PREV)) ? 1 : 0);
  }
  if (x < batch) {
    g.mctrl[CTRL_WORDS * x + CTRL_INFO] = INT_MAX;
    g.mctrl[CTRL_WORDS * x + CTRL_FAILED] = 0;
  }
  if (x < CTRL_WORDS) g.ctrl[x] = 0;
}

}  // namespace

hipError_t launch_breset(const BSchedArgs& b, int batch, hipStream_t s) {
  int total = b.ntotal > batch ? b.ntotal : batch;
  if (total < CTRL_WORDS) total = CTRL_WORDS;
  hipLaunchKernelGGL(breset_kernel, dim3((total + 255) / 256), dim3(256), 0, s, b, batch);
  return hipGetLastError();
}

hipError_t launch_bsched(const BSchedArgs& b, int grid, hipStream_t s) {
  hipLaunchKernelGGL(bsched_kernel, dim3(grid), dim3(NTHREADS), 0, s, b);
  return hipGetLastError();
}

int bsched_blocks_per_cu() {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, bsched_kernel, NTHREADS, 0) != hipSuccess)
    return 1;
  return blocks > 0 ? blocks : 1;
}

}  // namespace spdinv
