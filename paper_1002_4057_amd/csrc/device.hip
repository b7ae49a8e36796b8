// HIP kernels for gfx950 (MI355X): the tile tasks of the SPD inverse and the
// persistent, dependency-tracked scheduler that runs them.
//
// Tiles are NB x NB (NB = 128) binary64, column-major, each contiguous
// (128 KiB).  One workgroup of 256 threads (4 wave64) executes one task at a
// time; every task kind of the paper's Algorithm 1 maps to one of
//   * a tile product on the FP64 matrix cores (v_mfma_f64_16x16x4),
//     C = beta*C + alpha*op(A)*op(B) with optional triangular masking of an
//     operand and a lower-only output, staged through LDS in k-panels, and
//     an optional second destination (the renaming copy of Section 3);
//   * the diagonal-tile factorization POTRF, which also produces the inverse
//     of the factor tile, computed with the tile resident in registers
//     (2D cyclic over a 16 x 16 thread grid), pivot columns and rows broadcast
//     through LDS and the finished factor kept in LDS for the inverse;
//   * a tile copy (TRTRI reuses the inverse made by POTRF, bit for bit).
#include "device.hpp"

#include <climits>

namespace spdinv {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int KC = 16;                    // k-panel depth
constexpr int NCH = NB / KC;              // k-panels per tile
constexpr int LDS_STRIDE = NB + 16;       // padded row of a [k][m] panel (doubles)
constexpr int PANEL = KC * LDS_STRIDE;    // doubles per operand panel
constexpr int GEMM_SMEM = 4 * PANEL;      // 2 buffers x 2 operands
constexpr int POTRF_SMEM = 8 * NB + NB * NB;  // broadcast rows + the factor tile
constexpr int SMEM_DOUBLES = GEMM_SMEM > POTRF_SMEM ? GEMM_SMEM : POTRF_SMEM;
constexpr size_t TILE = (size_t)NB * NB;

__device__ __forceinline__ double* tile_ptr(double* pool, int idx) {
  return pool + (size_t)idx * TILE;
}

// ---------------------------------------------------------------------------
// k-panel staging.  A panel holds op(X)[r][k] for r = 0..127 (the output row
// for the left operand, the output column for the right one) and k in one
// KC-deep slice, stored in LDS as S[k * LDS_STRIDE + r].
//   CONTIG: element (r, k) is X[r + NB*k] (r runs down a stored column)
//  !CONTIG: element (r, k) is X[k + NB*r] (k runs down a stored column)
// MASK treats X as lower triangular (entries above its diagonal read as 0);
// NEG negates the panel.  Each thread moves 4 pairs of doubles per panel with
// 16-byte global loads.
// ---------------------------------------------------------------------------
template <bool CONTIG>
__device__ __forceinline__ void panel_load(const double* __restrict__ X, int k0, d2 (&r)[4]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int p = tid + NTHREADS * q;
    if (CONTIG) {
      r[q] = reinterpret_cast<const d2*>(X + (size_t)NB * k0)[p];
    } else {
      const int rr = p >> 3, kk = (p & 7) * 2;
      r[q] = *reinterpret_cast<const d2*>(X + k0 + kk + (size_t)NB * rr);
    }
  }
}

template <bool CONTIG, bool MASK, bool NEG>
__device__ __forceinline__ void panel_store(double* __restrict__ S, int k0, const d2 (&r)[4]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int p = tid + NTHREADS * q;
    double v0 = r[q].x, v1 = r[q].y;
    if (NEG) { v0 = -v0; v1 = -v1; }
    if (CONTIG) {
      const int e = 2 * p, rr = e & (NB - 1), kk = e >> 7;
      // stored element (row rr+s, col k0+kk); lower triangle keeps row >= col
      if (MASK) {
        if (rr < k0 + kk) v0 = 0.0;
        if (rr + 1 < k0 + kk) v1 = 0.0;
      }
      d2 v;
      v.x = v0;
      v.y = v1;
      *reinterpret_cast<d2*>(S + kk * LDS_STRIDE + rr) = v;
    } else {
      const int rr = p >> 3, kk = (p & 7) * 2;
      // stored element (row k0+kk+s, col rr)
      if (MASK) {
        if (k0 + kk < rr) v0 = 0.0;
        if (k0 + kk + 1 < rr) v1 = 0.0;
      }
      S[kk * LDS_STRIDE + rr] = v0;
      S[(kk + 1) * LDS_STRIDE + rr] = v1;
    }
  }
}

// ---------------------------------------------------------------------------
// Tile product on the FP64 matrix cores.
//   C (+)= (NEG ? -1 : 1) * op(A) * op(B),   op(A) = TA ? A^T : A,
//                                            op(B) = TB ? B^T : B
// ACC: accumulate into C (else overwrite).  MA/MB: the operand tile is lower
// triangular.  LOWER: only the output blocks on or below the diagonal are
// stored (the wave owning rows 0-63 x columns 64-127 computes but does not
// store: it runs alone on its SIMD, so skipping its work would save no time
// and would cost registers).  C may alias A
// or B: every operand read precedes the first store.  copy (may be null)
// receives the same result.
// Waves form a 2 x 2 grid of 64 x 64 output blocks, each a 4 x 4 array of
// 16 x 16 MFMA accumulators.
// ---------------------------------------------------------------------------
template <bool TA, bool TB, bool MA, bool MB, bool LOWER, bool NEG, bool ACC>
__device__ __forceinline__ void tile_mma(double* C, const double* A, const double* B, double* copy,
                         double* smem) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int wm = w & 1, wn = w >> 1;
  const int lr = lane & 15, lk = lane >> 4;
  const bool active = !(LOWER && wm == 0 && wn == 1);

  // v_mfma_f64_16x16x4(x, y, d): d[i][j] += sum_k x[i][k] y[k][j] with x[i][k]
  // from lane i+16k, y[k][j] from lane j+16k, and d[i][j] in register r = i/4
  // of lane j + 16*(i%4).  The operands are passed as (op(B) block, op(A)
  // block), so that d is the transposed 16x16 output block: lane l, register
  // r holds output row (l%16) of column (l/16) + 4r, and a group of 16 lanes
  // covers 16 consecutive rows of one column (one 128-byte segment).
  d4 acc[4][4];
  if (ACC) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double* p = C + (wm * 64 + i * 16 + lr) + (size_t)NB * (wn * 64 + j * 16 + lk);
        acc[i][j] = d4{p[0], p[4 * NB], p[8 * NB], p[12 * NB]};
      }
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  }

  d2 ra[4], rb[4];
  panel_load<!TA>(A, 0, ra);
  panel_load<TB>(B, 0, rb);
  panel_store<!TA, MA, NEG>(smem, 0, ra);
  panel_store<TB, MB, false>(smem + PANEL, 0, rb);
  __syncthreads();

  for (int c = 0; c < NCH; ++c) {
    double* As = smem + (c & 1) * 2 * PANEL;
    double* Bs = As + PANEL;
    if (c + 1 < NCH) {
      panel_load<!TA>(A, (c + 1) * KC, ra);
      panel_load<TB>(B, (c + 1) * KC, rb);
    }
    {
#pragma unroll
      for (int ks = 0; ks < KC / 4; ++ks) {
        const double* Ar = As + (4 * ks + lk) * LDS_STRIDE + wm * 64 + lr;
        const double* Br = Bs + (4 * ks + lk) * LDS_STRIDE + wn * 64 + lr;
        double a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          a[i] = Ar[16 * i];
          b[i] = Br[16 * i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[j], a[i], acc[i][j], 0, 0, 0);
      }
    }
    if (c + 1 < NCH) {
      double* An = smem + ((c + 1) & 1) * 2 * PANEL;
      panel_store<!TA, MA, NEG>(An, (c + 1) * KC, ra);
      panel_store<TB, MB, false>(An + PANEL, (c + 1) * KC, rb);
    }
    __syncthreads();
  }

  if (!active) return;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const size_t off = (wm * 64 + i * 16 + lr) + (size_t)NB * (wn * 64 + j * 16 + lk);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        C[off + (size_t)NB * 4 * r] = acc[i][j][r];
        if (copy) copy[off + (size_t)NB * 4 * r] = acc[i][j][r];
      }
    }
}

// ---------------------------------------------------------------------------
// Diagonal tile: Cholesky factor L of the lower triangle of A (right-looking,
// one column per step) and its inverse X = L^{-1} (forward substitution of
// L X = I, one row per step).  Thread (tr, tc) = (tid % 16, tid / 16) owns the
// entries (tr + 16a, tc + 16b), a, b = 0..7, in registers; the pivot column
// (factorization) or the pivot row and column (inverse) are broadcast through
// LDS, double-buffered so that one barrier per step suffices.
// Returns 0, or the 1-based local index of the first pivot that is not
// positive (or NaN).  On failure nothing is stored.
// ---------------------------------------------------------------------------
// Register slot of the owned entry (tr+16a, tc+16b), b <= a: only blocks on
// or below the diagonal are held (36 doubles per thread).
#define PK(a, b) ((a) * ((a) + 1) / 2 + (b))

__device__ __attribute__((noinline)) int potrf_inv_tile(const double* Ain, double* Lout, double* Lcopy,
                                              double* Xout, double* smem) {
  const int tid = threadIdx.x;
  const int tr = tid & 15, tc = tid >> 4;
  double* colbuf = smem;               // [2][NB]
  double* rdiag = smem + 2 * NB;       // [NB]
  double* xrow = smem + 4 * NB;        // [2][NB]
  double* Ls = smem + 8 * NB;          // [NB * NB], the finished factor

  // entry (tr+16a, tc+16b) is on or below the diagonal iff b < a, or b == a
  // and tr >= tc
  const bool own_lower_diag = tr >= tc;
  double L[36];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      const double v = Ain[(tr + 16 * a) + (size_t)NB * (tc + 16 * b)];
      L[PK(a, b)] = (b < a || own_lower_diag) ? v : 0.0;
    }

  int fail = 0;
  for (int j = 0; j < NB; ++j) {
    double* cb = colbuf + (j & 1) * NB;
    const int q = j >> 4, jl = j & 15;
    if (tc == jl) {
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        double v = 0.0;
#pragma unroll
        for (int b = 0; b <= a; ++b)
          if (b == q) v = L[PK(a, b)];
        cb[tr + 16 * a] = v;
      }
    }
    __syncthreads();
    const double d = cb[j];
    // every thread reads the same pivot; readfirstlane makes the exit visibly
    // wave-uniform, so that the compiler keeps this loop (and its barriers)
    // uniform instead of splitting lanes across iterations
    if (__builtin_amdgcn_readfirstlane(!(d > 0.0) ? 1 : 0)) {
      fail = j + 1;
      break;
    }
    const double ljj = sqrt(d);
    const double rinv = 1.0 / ljj;
    double lk[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) lk[b] = cb[tc + 16 * b] * rinv;
    // trailing update of entries (i, k) with i >= k > j: row block a >= q,
    // column block q <= b <= a; at the block edges the thread's offset decides
    const bool row_past = tr > jl;   // row tr+16q is below the pivot
    const bool col_past = tc > jl;   // column tc+16q is right of the pivot
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      if (a >= q) {
        const double li = cb[tr + 16 * a] * rinv;
#pragma unroll
        for (int b = 0; b <= a; ++b) {
          if (b >= q) {
            const bool ok = (b > q || col_past) && (b < a || own_lower_diag) && (a > q || row_past);
            if (ok) L[PK(a, b)] = fma(-li, lk[b], L[PK(a, b)]);
          }
        }
        // the pivot column itself becomes column j of the factor
        if (tc == jl) {
#pragma unroll
          for (int b = 0; b <= a; ++b)
            if (b == q) {
              if (a > q || row_past) L[PK(a, b)] = li;
              else if (tr == jl) L[PK(a, b)] = ljj;
            }
        }
      }
    }
  }
  if (fail) return fail;

  // the factor goes to LDS (column-major, zeros above the diagonal) and to
  // its global destinations; registers are reused for the inverse
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const size_t off = (tr + 16 * a) + (size_t)NB * (tc + 16 * b);
      const double v = (b <= a) ? L[PK(a, b < a ? b : a)] : 0.0;
      Ls[off] = v;
      Lout[off] = v;
      if (Lcopy) Lcopy[off] = v;
    }
  if (tr == tc) {
#pragma unroll
    for (int a = 0; a < 8; ++a) rdiag[tr + 16 * a] = 1.0 / L[PK(a, a)];
  }
  // inverse of the factor: row r of X is final at step r, then the rows
  // below it are updated with column r of L
  const bool own_diag = tr == tc;
  double X[36];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b <= a; ++b) X[PK(a, b)] = (a == b && own_diag) ? 1.0 : 0.0;
  __syncthreads();

  for (int r = 0; r < NB; ++r) {
    double* xr = xrow + (r & 1) * NB;
    const int q = r >> 4;
    const int rl = r & 15;
    const bool col_le = tc <= rl;    // column tc+16q is at or left of r
    if (tr == rl) {
      const double s = rdiag[r];
#pragma unroll
      for (int a = 0; a < 8; ++a)
        if (a == q) {
#pragma unroll
          for (int b = 0; b <= a; ++b) {
            if (b < q || col_le) X[PK(a, b)] *= s;
            xr[tc + 16 * b] = X[PK(a, b)];
          }
        }
    }
    __syncthreads();
    const double* lc = Ls + (size_t)NB * r;
    const bool row_gt = tr > rl;     // row tr+16q is below r
    double xk[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) xk[b] = xr[tc + 16 * b];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      if (a >= q) {
        const double l = lc[tr + 16 * a];
#pragma unroll
        for (int b = 0; b <= a; ++b) {
          if (b <= q) {
            const bool ok = (a > q || row_gt) && (b < q || col_le);
            if (ok) X[PK(a, b)] = fma(-l, xk[b], X[PK(a, b)]);
          }
        }
      }
    }
  }

#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b)
      Xout[(tr + 16 * a) + (size_t)NB * (tc + 16 * b)] = (b <= a) ? X[PK(a, b < a ? b : a)] : 0.0;
  return 0;
}
#undef PK

__device__ __forceinline__ void tile_copy2(const double* __restrict__ src, double* dst0, double* dst1) {
  const d2* s = reinterpret_cast<const d2*>(src);
  for (int p = threadIdx.x; p < (int)(TILE / 2); p += NTHREADS) {
    const d2 v = s[p];
    reinterpret_cast<d2*>(dst0)[p] = v;
    if (dst1) reinterpret_cast<d2*>(dst1)[p] = v;
  }
}

__device__ __forceinline__ void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

__device__ __forceinline__ long long now_ticks() {
  return (long long)__builtin_amdgcn_s_memrealtime();
}

__device__ __forceinline__ void run_task(const DevTask& t, const SchedArgs& g, double* smem, int T) {
  double* P = g.pool;
  double* out = t.out >= 0 ? tile_ptr(P, t.out) : nullptr;
  const double* a = t.a >= 0 ? tile_ptr(P, t.a) : nullptr;
  const double* b = t.b >= 0 ? tile_ptr(P, t.b) : nullptr;
  double* cp = t.copy >= 0 ? tile_ptr(P, t.copy) : nullptr;
  switch (t.kind) {
    case K_SYRK1:   // A_jj -= A_jk A_jk^T
      tile_mma<false, true, false, false, true, true, true>(out, a, a, nullptr, smem);
      break;
    case K_GEMM1:   // A_ij -= A_ik A_jk^T
      tile_mma<false, true, false, false, false, true, true>(out, a, b, nullptr, smem);
      break;
    case K_TRSM1:   // A_ij <- A_ij D_j^T, D_j = L_jj^{-1}
      tile_mma<false, true, false, true, false, false, false>(out, out, b, cp, smem);
      break;
    case K_TRMM2L:  // A_ij <- X_ii A_ij
      tile_mma<false, false, true, false, false, false, false>(out, a, out, nullptr, smem);
      break;
    case K_GEMM2:   // A_ij += X_ik L_kj
      tile_mma<false, false, false, false, false, false, true>(out, a, b, nullptr, smem);
      break;
    case K_TRSM2R:  // A_ij <- -A_ij D_j
      tile_mma<false, false, false, true, false, true, false>(out, out, b, cp, smem);
      break;
    case K_TRMM3:   // A_ij <- X_ii^T A_ij
      tile_mma<true, false, true, false, false, false, false>(out, a, out, nullptr, smem);
      break;
    case K_LAUUM:   // A_ii <- A_ii^T A_ii (lower)
      tile_mma<true, false, true, true, true, false, false>(out, out, out, nullptr, smem);
      break;
    case K_GEMM3:   // A_ij += X_ki^T X_kj
      tile_mma<true, false, false, false, false, false, true>(out, a, b, nullptr, smem);
      break;
    case K_SYRK3:   // A_ii += X_ki^T X_ki (lower)
      tile_mma<true, false, false, false, true, false, true>(out, a, a, nullptr, smem);
      break;
    case K_POTRF: {
      double* X = tile_ptr(P, t.aux);
      const int f = potrf_inv_tile(out, out, cp, X, smem);
      if (f && threadIdx.x == 0) {
        const int jt = t.aux - 3 * T;  // diagonal tile index
        atomicMin(&g.ctrl[CTRL_INFO], g.info_base + jt * NB + f);
        __hip_atomic_store(&g.ctrl[CTRL_FAILED], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      break;
    }
    case K_TRTRI:   // A_jj <- D_j (inverse made by POTRF(j))
      tile_copy2(b, out, cp);
      break;
    default:
      break;
  }
}

// Persistent worker loop.  Thread 0 of each workgroup is the only one that
// talks to the scheduler state: at the head of every iteration it first
// releases the successors of the task the workgroup just finished (one
// decrement of each successor's in-degree, after the release fence that all
// threads executed), then claims the next dispatch ticket and waits until
// that task's in-degree is zero.  Keeping both in one thread-0 region at the
// loop head leaves the loop body (and every barrier in it) in uniform control
// flow.
__global__ __launch_bounds__(NTHREADS) void sched_kernel(SchedArgs g, int T) {
  __shared__ double smem[SMEM_DOUBLES];
  __shared__ int s_task;
  __shared__ int s_skip;
  int prev = -1;  // meaningful in thread 0 only
  for (;;) {
    if (threadIdx.x == 0) {
      if (prev >= 0) {
        if (g.trace) g.trace[4 * (size_t)prev + 3] = now_ticks();
        const DevTask& pt = g.tasks[prev];
        for (int e = pt.succ_begin; e < pt.succ_end; ++e)
          __hip_atomic_fetch_sub(&g.indeg[g.succ[e]], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&g.ctrl[CTRL_DONE], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      long long t_claim = 0;
      if (g.trace) t_claim = now_ticks();
      const int tk = __hip_atomic_fetch_add(&g.ctrl[CTRL_TICKET], 1, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
      int v = tk < g.ntask ? g.order[tk] : -1;
      if (v >= 0) {
        // bounded wait: gives up after spin_limit ticks of the 100 MHz clock
        const long long t0 = now_ticks();
        long long spins = 0;
        while (__hip_atomic_load(&g.indeg[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > 0) {
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
        }
      }
      if (v >= 0) {
        fence_acquire();
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
    fence_acquire();
    const DevTask t = g.tasks[v];
    if (!__builtin_amdgcn_readfirstlane(s_skip)) run_task(t, g, smem, T);
    fence_release();
    __syncthreads();
  }
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

__global__ void info_out_kernel(const int32_t* ctrl, int* d_info) {
  const int v = ctrl[CTRL_INFO];
  d_info[0] = (v == INT_MAX) ? 0 : v;
}

}  // namespace

hipError_t launch_reset(const int32_t* indeg0, int32_t* indeg, int ntask, int32_t* ctrl,
                        hipStream_t s) {
  const int total = ntask > CTRL_WORDS ? ntask : CTRL_WORDS;
  const int blocks = (total + 255) / 256;
  hipLaunchKernelGGL(reset_kernel, dim3(blocks), dim3(256), 0, s, indeg0, indeg, ntask, ctrl);
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

hipError_t launch_info_out(const int32_t* ctrl, int* d_info, hipStream_t s) {
  if (!d_info) return hipSuccess;
  hipLaunchKernelGGL(info_out_kernel, dim3(1), dim3(1), 0, s, ctrl, d_info);
  return hipGetLastError();
}

hipError_t launch_sched(const SchedArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(sched_kernel, dim3(grid), dim3(NTHREADS), 0, s, a, a.tiles_T);
  return hipGetLastError();
}

int sched_blocks_per_cu() {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, sched_kernel, NTHREADS, 0) != hipSuccess)
    return 1;
  return blocks > 0 ? blocks : 1;
}

}  // namespace spdinv
