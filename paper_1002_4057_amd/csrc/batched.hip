// Batched form of the SPD inverse on gfx950 (MI355X): many independent
// matrices of uneven order in one persistent launch (own translation unit, so
// that its kernel does not share out-of-line code with the scheduler).
#include "device.hpp"
#include "tile_tasks.hpp"

namespace spdinv {
namespace {

// ---------------------------------------------------------------------------
// Batched form: many independent matrices of uneven order in one persistent
// launch.  A device-side counting sort orders the matrices by decreasing
// order (largest first, so that the tail of the launch holds the small
// ones); each workgroup then claims one matrix at a time and inverts it on
// its own, with no synchronization between workgroups:
//   n <= NB: the whole matrix in LDS -- the packed blocked factorization and
//            in-place inverse of the diagonal-tile task over ceil(n/16)
//            blocks only, then Y = X^T X from 16 x 16 MFMA blocks;
//   n >  NB: the tile plan for t = ceil(n/NB) tiles executed in program order
//            (the sequential task stream of Algorithm 1, renamed by default)
//            by the scheduler's own tile tasks, on the workgroup's private
//            tile pool.
// ---------------------------------------------------------------------------

// acc (16x16 block) += op(A)_blk op(B)_blk over K = 16; op(A)_blk[m][k] is
// A[m + lda*k] (or A[k + lda*m] when ta), op(B)_blk[k][n] is B[n + ldb*k]
// when tb (or B[k + ldb*n]).
__device__ __forceinline__ d4 blk_mma16x(d4 acc, const double* A, int lda, bool ta, const double* B,
                                         int ldb, bool tb) {
  const int lane = opaque_tid() & 63, lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int k = 4 * kk + lk;
    const double a = ta ? A[k + lda * lr] : A[lr + lda * k];
    const double b = tb ? B[lr + ldb * k] : B[k + ldb * lr];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, acc, 0, 0, 0);
  }
  return acc;
}

// Lower triangle of A (column-major, lda, 1 <= n <= NB) <- lower triangle of
// A^{-1} (and the strictly upper triangle <- its mirror when fill_upper).
// Returns 0 or INFO (1-based index of the first non-positive pivot; A is then
// left unchanged).  The matrix, padded to 16 * ceil(n/16) with the identity,
// is held as the packed lower 16 x 16 blocks of the diagonal-tile task
// (factor_packed, then inverse_packed leave X = L^{-1} in place); then
// Y = X^T X, Y_IJ = sum_{K >= I} X_KI^T X_KJ for I >= J, is formed in
// registers (at most 9 blocks per wave) and written to A from there.
__device__ int small_inverse(double* A, int lda, int n, int fill_upper, double* smem) {
  double* T = smem;
  double* rd = smem + PK_BLOCKS * PK_STRIDE;
  int* flag = reinterpret_cast<int*>(rd + NB);
  const int tid = opaque_tid(), w = tid >> 6;
  const int P = (n + 15) >> 4;
  const int nblk = P * (P + 1) / 2;
  for (int e = tid; e < nblk * 256; e += NTHREADS) {
    const int b = e >> 8, lr = e & 15, lc = (e >> 4) & 15;
    int I = 0;
    while ((I + 1) * (I + 2) / 2 <= b) ++I;
    const int J = b - I * (I + 1) / 2;
    const int r = 16 * I + lr, c = 16 * J + lc;
    double v;
    if (r < n && c < n)
      v = (r >= c) ? A[r + (size_t)lda * c] : 0.0;
    else
      v = (r == c) ? 1.0 : 0.0;
    T[PK_STRIDE * b + lr + PK_LD * lc] = v;
  }
  __syncthreads();
  const int f = factor_packed(T, rd, rd + NB + 8, flag, P);
  if (f) return f;
  inverse_packed(T, rd, P);
  constexpr int PER_WAVE = (PK_BLOCKS + 3) / 4;
  d4 y[PER_WAVE];
#pragma unroll
  for (int s2 = 0; s2 < PER_WAVE; ++s2) {
    const int q = w + 4 * s2;
    y[s2] = d4{0.0, 0.0, 0.0, 0.0};
    if (q < nblk) {
      int I = 0;
      while ((I + 1) * (I + 2) / 2 <= q) ++I;
      const int J = q - I * (I + 1) / 2;
      for (int K = I; K < P; ++K)  // X_KI^T X_KJ
        y[s2] = blk_mma16x(y[s2], pk_blk(T, K, I), PK_LD, true, pk_blk(T, K, J), PK_LD, false);
    }
  }
  // lane l, register q of block (I, J) holds Y(16 I + l % 16, 16 J + l / 16 + 4 q)
  const int lane = tid & 63, lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int s2 = 0; s2 < PER_WAVE; ++s2) {
    const int q = w + 4 * s2;
    if (q >= nblk) continue;
    int I = 0;
    while ((I + 1) * (I + 2) / 2 <= q) ++I;
    const int J = q - I * (I + 1) / 2;
    const int r = 16 * I + lr;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = 16 * J + lk + 4 * u;
      if (r < n && c <= r) {
        A[r + (size_t)lda * c] = y[s2][u];
        if (fill_upper && r > c) A[c + (size_t)lda * r] = y[s2][u];
      }
    }
  }
  return 0;
}

// One matrix of order n > NB through its tile plan, in program order, on the
// private pool `pool` (pool_tiles(t) tiles) with the control words `ctrl`.
// Returns 0 or INFO.
__device__ int tile_sequential(double* A, int lda, int n, int fill_upper, const DevTask* tasks,
                               const int32_t* links, int ntask, double* pool, int32_t* ctrl,
                               double* smem) {
  const int t = (n + NB - 1) / NB, T = t * (t + 1) / 2;
  const int tid = threadIdx.x;
  // copy-in with identity padding (agent-coherent stores, like every access
  // of the tile tasks)
  for (int x = 0; x < T; ++x) {
    int ti = 0;
    while ((ti + 1) * (ti + 2) / 2 <= x) ++ti;
    const int tj = x - ti * (ti + 1) / 2;
    const rsrc_t rd = tile_rsrc(tile_ptr(pool, x));
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
  if (tid == 0) {
    __hip_atomic_store(&ctrl[CTRL_INFO], INT_MAX, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ctrl[CTRL_FAILED], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  stores_complete();
  __syncthreads();
  SchedArgs g{};
  g.pool = pool;
  g.ctrl = ctrl;
  g.info_base = 0;
  g.links = links;
  // the pool is reused by the next matrix: keep every read device-coherent
  g.coherent_only = 1;
  g.last_valid = n - (t - 1) * NB;
  __shared__ int s_info;
  for (int k = 0; k < ntask; ++k) {
    const DevTask task = tasks[k];
    run_task<true>(task, g, smem, T, t);
    stores_complete();
    __syncthreads();
    if ((task.kind & 0xff) == K_POTRF) {
      // a failed diagonal factorization left INFO in the control words
      if (tid == 0)
        s_info = __hip_atomic_load(&ctrl[CTRL_FAILED], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                     ? __hip_atomic_load(&ctrl[CTRL_INFO], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                     : 0;
      __syncthreads();
      const int info = __builtin_amdgcn_readfirstlane(s_info);
      __syncthreads();
      if (info) return info;
    }
  }
  // copy-out of the lower triangle (and its mirror)
  for (int x = 0; x < T; ++x) {
    int ti = 0;
    while ((ti + 1) * (ti + 2) / 2 <= x) ++ti;
    const int tj = x - ti * (ti + 1) / 2;
    const rsrc_t rs = tile_rsrc(tile_ptr(pool, x));
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
  return 0;
}

__device__ __forceinline__ double* read_ptr_uniform(double* const* p) {
  const unsigned long long u = (unsigned long long)(*p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
  return (double*)(((unsigned long long)hi << 32) | lo);
}

// Two workgroups per CU: every path needs at most TASK_SMEM doubles of LDS
// and 256 registers per lane, and the matrices of a batch are independent.
__global__ __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(2, 2)))
void batched_kernel(BatchArgs b) {
  __shared__ double smem[TASK_SMEM];
  __shared__ int s_m;
  double* pool = b.pool + (size_t)blockIdx.x * (size_t)b.pool_tiles * TILE;
  int32_t* ctrl = b.ctrl + blockIdx.x * CTRL_WORDS;
  for (;;) {
    if (threadIdx.x == 0) {
      const int tk = __hip_atomic_fetch_add(b.ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_m = tk < b.batch ? b.order[tk] : -1;
    }
    __syncthreads();
    const int m = __builtin_amdgcn_readfirstlane(s_m);
    if (m < 0) break;
    const int n = __builtin_amdgcn_readfirstlane(b.n[m]);
    const int lda = __builtin_amdgcn_readfirstlane(b.lda[m]);
    double* A = read_ptr_uniform(b.A + m);
    const int t = (n + NB - 1) / NB;
    int info = 0;
    if (n < 0 || lda < (n > 1 ? n : 1) || (n > 0 && !A) || t > b.tmax) {
      info = -1;
    } else if (n == 0) {
      info = 0;
    } else if (n <= NB) {
      info = small_inverse(A, lda, n, b.fill_upper, smem);
    } else {
      info = tile_sequential(A, lda, n, b.fill_upper, b.plan[t], b.plan_links[t], b.plan_ntask[t],
                             pool, ctrl, smem);
    }
    if (threadIdx.x == 0 && b.info) b.info[m] = info;
    __syncthreads();  // LDS (and s_m) are reused by the next matrix
  }
}

// order <- matrix indices by decreasing order n (counting sort over the
// clamped keys 0..maxn+1; ties in any order), and the dispatch ticket <- 0.
__global__ __launch_bounds__(1024) void batch_sort_kernel(const int* __restrict__ n, int batch,
                                                          int maxn, int32_t* __restrict__ order,
                                                          int32_t* __restrict__ ticket) {
  extern __shared__ int hist[];  // maxn + 2 bins
  auto key = [&](int v) { return v < 0 ? 0 : (v > maxn ? maxn + 1 : v); };
  for (int v = threadIdx.x; v <= maxn + 1; v += blockDim.x) hist[v] = 0;
  __syncthreads();
  for (int m = threadIdx.x; m < batch; m += blockDim.x) atomicAdd(&hist[key(n[m])], 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int v = maxn + 1; v >= 0; --v) {
      const int c = hist[v];
      hist[v] = run;
      run += c;
    }
    *ticket = 0;
  }
  __syncthreads();
  for (int m = threadIdx.x; m < batch; m += blockDim.x) order[atomicAdd(&hist[key(n[m])], 1)] = m;
}

}  // namespace

hipError_t launch_batched(const BatchArgs& b, int grid, int maxn, hipStream_t s) {
  const size_t lds = (size_t)(maxn + 2) * sizeof(int);
  hipLaunchKernelGGL(batch_sort_kernel, dim3(1), dim3(1024), lds, s, b.n, b.batch, maxn,
                     const_cast<int32_t*>(b.order), b.ticket);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(batched_kernel, dim3(grid), dim3(NTHREADS), 0, s, b);
  return hipGetLastError();
}

int batched_blocks_per_cu() {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batched_kernel, NTHREADS, 0) != hipSuccess)
    return 1;
  return blocks > 0 ? blocks : 1;
}

}  // namespace spdinv
