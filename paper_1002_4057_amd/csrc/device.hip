// HIP kernels for gfx950 (MI355X): the persistent, dependency-tracked
// scheduler that runs the tile tasks of one SPD inverse (tile_tasks.hpp), and
// the copies between the caller's column-major matrix and the tile pool.
#include "device.hpp"
#include "sched_loop.hpp"
#include "tile_tasks.hpp"

#include <climits>
#include <map>
#include <mutex>

namespace spdinv {
namespace {

// Two workgroups per CU: a task needs at most TASK_SMEM doubles of LDS (half
// the CU's) and 256 registers per lane, so that while one workgroup waits
// (loads, barriers, dependencies) the other keeps the matrix cores busy.
__global__ __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(2, 2)))
void sched_kernel(SchedArgs g, int T, int tiles) {
  __shared__ double smem[TASK_SMEM];
  sched_loop(g, [&](const DevTask& t) { run_task(t, g, smem, T, tiles); });
}

__global__ void reset_kernel(const int32_t* __restrict__ indeg0, int32_t* __restrict__ indeg,
                             int ntask, int32_t* ctrl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ntask) indeg[i] = indeg0[i];
  if (i < CTRL_WORDS) ctrl[i] = (i == CTRL_INFO) ? INT_MAX : 0;
}

__device__ __forceinline__ void tri_decode(int x, int& ti, int& tj) {
  int i = (int)((sqrtf(8.0f * (float)x + 1.0f) - 1.0f) * 0.5f);
  while (i * (i + 1) / 2 > x) --i;
  while ((i + 1) * (i + 2) / 2 <= x) ++i;
  ti = i;
  tj = x - i * (i + 1) / 2;
}

// What step 1 leaves for step 2 when the Cholesky factor is given (the
// inverse from a factor, Algorithm 1 steps 2 and 3): the transposed renaming
// copies B_ij = L_ij^T (i > j) and the inverted diagonal tiles D_j, D_j^T.
// One workgroup per lower tile of the pool (tile tri(i, j) holds L_ij).  A
// zero diagonal entry of L sets INFO and the failure flag, so that the
// scheduler skips every task.
__global__ __launch_bounds__(NTHREADS) void factor_prologue_kernel(double* pool, int t,
                                                                   int32_t* ctrl) {
  __shared__ double smem[TASK_SMEM];
  int ti, tj;
  tri_decode(blockIdx.x, ti, tj);
  const int T = t * (t + 1) / 2;
  const double* L = pool + (size_t)blockIdx.x * TILE;
  if (ti == tj) {
    const int f = trtri_inv_tile(L, pool + (size_t)(3 * T + tj) * TILE,
                                 pool + (size_t)(3 * T + t + tj) * TILE, smem);
    if (f && threadIdx.x == 0) {
      atomicMin(&ctrl[CTRL_INFO], tj * NB + f);
      __hip_atomic_store(&ctrl[CTRL_FAILED], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  // B_ij = L_ij^T through LDS, 64 rows of L at a time: R[c + RLD * r]
  double* B = pool + (size_t)(T + blockIdx.x) * TILE;
  double* R = smem;
  for (int h = 0; h < 2; ++h) {
    for (int e = threadIdx.x; e < 64 * NB; e += NTHREADS) {
      const int r = e & 63, c = e >> 6;  // L(64h + r, c), read down the columns
      R[c + RLD * r] = L[(64 * h + r) + NB * c];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * NB; e += NTHREADS) {
      const int rr = e & (NB - 1), cl = e >> 7;  // B(rr, 64h + cl) = L(64h + cl, rr)
      B[rr + NB * (64 * h + cl)] = R[rr + RLD * cl];
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(NTHREADS) void copy_in_kernel(const double* __restrict__ A, int lda,
                                                           int n, double* __restrict__ pool) {
  int ti, tj;
  tri_decode(blockIdx.x, ti, tj);
  double* dst = pool + (size_t)blockIdx.x * TILE;
  for (int e = threadIdx.x; e < (int)TILE; e += NTHREADS) {
    const int r = e & (NB - 1), c = e >> 7;
    const int gr = ti * NB + r, gc = tj * NB + c;
    double v;
    if (gr < n && gc < n)
      v = (gr >= gc) ? A[gr + (size_t)lda * gc] : 0.0;
    else
      v = (gr == gc) ? 1.0 : 0.0;
    dst[e] = v;
  }
}

__global__ __launch_bounds__(NTHREADS) void copy_out_kernel(const double* __restrict__ pool,
                                                            double* __restrict__ A, int lda, int n,
                                                            int fill_upper) {
  int ti, tj;
  tri_decode(blockIdx.x, ti, tj);
  const double* src = pool + (size_t)blockIdx.x * TILE;
  for (int e = threadIdx.x; e < (int)TILE; e += NTHREADS) {
    const int r = e & (NB - 1), c = e >> 7;
    const int gr = ti * NB + r, gc = tj * NB + c;
    if (gr < n && gc < n && gr >= gc) {
      const double v = src[e];
      A[gr + (size_t)lda * gc] = v;
      if (fill_upper && gr > gc) A[gc + (size_t)lda * gr] = v;
    }
  }
}

__global__ void info_zero_kernel(int* d_info) { d_info[0] = 0; }

// A synthetic SPD matrix for timing runs (the autotuner): a_ij = 1/(1+|i-j|)
// off the diagonal, a_ii = n (strictly diagonally dominant), column-major
// with ld = n; in FP64 or FP32, for every matrix of a pointer array.
template <class E>
__global__ void fill_spd_kernel(E* const* mats, const int* orders, int count) {
  for (int m = blockIdx.y; m < count; m += gridDim.y) {
    const int n = orders[m];
    E* A = mats[m];
    const long long total = (long long)n * n;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
      const int r = (int)(e % n), c = (int)(e / n);
      A[e] = r == c ? (E)n : (E)(1.0 / (1.0 + (r > c ? r - c : c - r)));
    }
  }
}

__global__ void info_out_kernel(const int32_t* ctrl, int* d_info) {
  const int v = ctrl[CTRL_INFO];
  d_info[0] = (v == INT_MAX) ? 0 : v;
}

// Right-hand sides (column-major n x nrhs, ldb) <-> the transposed tiles
// R_ic^T (tile i + t c of the block R: element (r, q) is B(128 i + q,
// 128 c + r)), zero outside B.  Global accesses run down the columns of B.
__global__ __launch_bounds__(NTHREADS) void rhs_in_kernel(const double* __restrict__ B, int ldb,
                                                          int n, int nrhs, int t,
                                                          double* __restrict__ R) {
  const int i = blockIdx.x % t, c = blockIdx.x / t;
  double* dst = R + (size_t)blockIdx.x * TILE;
  for (int e = threadIdx.x; e < (int)TILE; e += NTHREADS) {
    const int q = e & (NB - 1), r = e >> 7;  // matrix row 128 i + q, right-hand side 128 c + r
    const int gr = i * NB + q, gc = c * NB + r;
    dst[r + NB * q] = (gr < n && gc < nrhs) ? B[gr + (size_t)ldb * gc] : 0.0;
  }
}

__global__ __launch_bounds__(NTHREADS) void rhs_out_kernel(const double* __restrict__ R, int t,
                                                           int n, int nrhs, double* __restrict__ B,
                                                           int ldb) {
  const int i = blockIdx.x % t, c = blockIdx.x / t;
  const double* src = R + (size_t)blockIdx.x * TILE;
  for (int e = threadIdx.x; e < (int)TILE; e += NTHREADS) {
    const int q = e & (NB - 1), r = e >> 7;
    const int gr = i * NB + q, gc = c * NB + r;
    if (gr < n && gc < nrhs) B[gr + (size_t)ldb * gc] = src[r + NB * q];
  }
}

}  // namespace

hipError_t launch_reset(const int32_t* indeg0, int32_t* indeg, int ntask, int32_t* ctrl,
                        hipStream_t s) {
  const int total = ntask > CTRL_WORDS ? ntask : CTRL_WORDS;
  const int blocks = (total + 255) / 256;
  hipLaunchKernelGGL(reset_kernel, dim3(blocks), dim3(256), 0, s, indeg0, indeg, ntask, ctrl);
  return hipGetLastError();
}

hipError_t launch_rhs_in(const double* B, int ldb, int n, int nrhs, int t, double* R,
                         hipStream_t s) {
  const int tiles = t * ((nrhs + NB - 1) / NB);
  hipLaunchKernelGGL(rhs_in_kernel, dim3(tiles), dim3(NTHREADS), 0, s, B, ldb, n, nrhs, t, R);
  return hipGetLastError();
}

hipError_t launch_rhs_out(const double* R, int t, int n, int nrhs, double* B, int ldb,
                          hipStream_t s) {
  const int tiles = t * ((nrhs + NB - 1) / NB);
  hipLaunchKernelGGL(rhs_out_kernel, dim3(tiles), dim3(NTHREADS), 0, s, R, t, n, nrhs, B, ldb);
  return hipGetLastError();
}

hipError_t launch_factor_prologue(double* pool, int t, int32_t* ctrl, hipStream_t s) {
  const int T = t * (t + 1) / 2;
  hipLaunchKernelGGL(factor_prologue_kernel, dim3(T), dim3(NTHREADS), 0, s, pool, t, ctrl);
  return hipGetLastError();
}

hipError_t launch_copy_in(const double* A, int lda, int n, int t, double* pool, hipStream_t s) {
  const int T = t * (t + 1) / 2;
  hipLaunchKernelGGL(copy_in_kernel, dim3(T), dim3(NTHREADS), 0, s, A, lda, n, pool);
  return hipGetLastError();
}

hipError_t launch_copy_out(const double* pool, int t, double* A, int lda, int n, int fill_upper,
                           hipStream_t s) {
  const int T = t * (t + 1) / 2;
  hipLaunchKernelGGL(copy_out_kernel, dim3(T), dim3(NTHREADS), 0, s, pool, A, lda, n, fill_upper);
  return hipGetLastError();
}

hipError_t launch_fill_spd(void* const* mats, const int* orders, int count, bool fp32,
                           hipStream_t s) {
  const dim3 grid(64, count < 4096 ? count : 4096);
  if (fp32)
    hipLaunchKernelGGL(fill_spd_kernel<float>, grid, dim3(256), 0, s, (float* const*)mats, orders,
                       count);
  else
    hipLaunchKernelGGL(fill_spd_kernel<double>, grid, dim3(256), 0, s, (double* const*)mats,
                       orders, count);
  return hipGetLastError();
}

hipError_t launch_info_zero(int* d_info, hipStream_t s) {
  if (!d_info) return hipSuccess;
  hipLaunchKernelGGL(info_zero_kernel, dim3(1), dim3(1), 0, s, d_info);
  return hipGetLastError();
}

hipError_t launch_info_out(const int32_t* ctrl, int* d_info, hipStream_t s) {
  if (!d_info) return hipSuccess;
  hipLaunchKernelGGL(info_out_kernel, dim3(1), dim3(1), 0, s, ctrl, d_info);
  return hipGetLastError();
}

// One workgroup per CU is enforced by asking for unused dynamic LDS, so that
// a second one no longer fits (the hardware would otherwise be free to pair
// two of the grid's workgroups on one CU and leave another CU idle).
constexpr unsigned kSoloLdsPad = 8192;
static_assert(TASK_SMEM * 8 + kSoloLdsPad > 80 * 1024, "the pad must exclude a second workgroup");

hipError_t launch_sched(const SchedArgs& a, int grid, int per_cu, hipStream_t s) {
  hipLaunchKernelGGL(sched_kernel, dim3(grid), dim3(NTHREADS), per_cu == 1 ? kSoloLdsPad : 0, s, a,
                     a.tiles_T, a.tiles);
  return hipGetLastError();
}

int sched_blocks_per_cu() {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, sched_kernel, NTHREADS, 0) != hipSuccess)
    return 1;
  return blocks > 0 ? blocks : 1;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free entry point.  Host code never uses the
// array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device with that device current.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch(void** ptr, size_t* bytes) {
  static std::mutex mu;
  static std::map<int, void*> addr;  // device -> address of its scratch
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  auto it = addr.find(device);
  if (it == addr.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    it = addr.emplace(device, p).first;
  }
  *ptr = it->second;
  *bytes = NOALLOC_SCRATCH_BYTES;
  return hipSuccess;
}

}  // namespace spdinv
