// Dense kernels on tile-major square matrices: symmetric packing, the chained
// FP64 MFMA product C = +-A B^T over whole tile rows, and unpacking with a
// mirror.  They serve the backward of the inverse,
//   grad_A = -X sym(G) X,  X = A^{-1} (symmetric),  sym(G) = (G + G^T) / 2,
// computed as W = X S (S = sym(G)), then the lower tiles of -W X, mirrored.
//
// Square tile-major layout: t x t tiles of NB x NB, tile (i, j) at index
// i + t*j, each tile column-major and contiguous.  Entries beyond the order n
// are zero, so the padding adds nothing to any product.
#include <algorithm>

#include "dense.hpp"
#include "mfma_tile.hpp"

namespace spdinv {
namespace {

using namespace tile;

constexpr int SB = 32;  // sub-block of the transposing copies

// dst tile (bi, bj) of the square tile-major matrix, from a column-major
// source (ld) of order n:
//   mode PACK_SYM_LOWER: the symmetric matrix whose lower triangle is src's
//                        (entry (r, c) = src(max, min))
//   mode PACK_SYM_AVG:   (src + src^T) / 2
// The transposed reads go through LDS in 32 x 32 sub-blocks so that every
// global access is a run of 32 consecutive doubles.
__global__ __launch_bounds__(NTHREADS) void pack_kernel(const double* __restrict__ src, int ld,
                                                        int n, int t, int mode,
                                                        double* __restrict__ dst) {
  __shared__ double L[SB][SB + 1];
  const int bi = blockIdx.x % t, bj = blockIdx.x / t;
  double* out = dst + (size_t)blockIdx.x * TILE;
  const int tx = threadIdx.x & (SB - 1), ty = threadIdx.x / SB;  // ty in 0..7
  for (int sb = 0; sb < (NB / SB) * (NB / SB); ++sb) {
    const int lr0 = (sb % (NB / SB)) * SB, lc0 = (sb / (NB / SB)) * SB;  // within the tile
    const int r0 = bi * NB + lr0, c0 = bj * NB + lc0;                      // global
    // transposed source block: element (c0 + tx, r0 + j) into L[tx][j]
#pragma unroll
    for (int q = 0; q < SB / 8; ++q) {
      const int j = ty + 8 * q;
      const int sr = c0 + tx, sc = r0 + j;
      L[tx][j] = (sr < n && sc < n) ? src[sr + (size_t)ld * sc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < SB / 8; ++q) {
      const int j = ty + 8 * q;
      const int gr = r0 + tx, gc = c0 + j;
      const double tv = L[j][tx];  // src(gc, gr)
      const double dv = (gr < n && gc < n) ? src[gr + (size_t)ld * gc] : 0.0;
      double v;
      if (mode == PACK_SYM_LOWER)
        v = (gr >= gc) ? dv : tv;
      else
        v = 0.5 * (dv + tv);
      out[(lr0 + tx) + NB * (lc0 + j)] = v;
    }
    __syncthreads();
  }
}

// Output tile list: all t*t tiles (lower = 0) or the t(t+1)/2 lower tiles
// (lower = 1), consecutive blocks spread over the XCDs in contiguous runs so
// that the workgroups of one XCD share operand tiles in its L2.
__device__ __forceinline__ void out_tile(int b, int nblk, int t, bool lower, int& i, int& j) {
  // blocks are handed to the 8 XCDs round-robin (block b to XCD b % 8): XCD
  // x receives the contiguous run of logical ids starting at
  // x * (nblk / 8) + min(x, nblk % 8)
  const int x = b % 8, y = b / 8, q = nblk / 8, r = nblk % 8;
  const int id = x * q + min(x, r) + y;
  if (!lower) {
    // groups of 4 tile rows, column-major inside a group
    const int G = 4;
    const int grp = id / (G * t), rem = id % (G * t);
    const int rows = min(G, t - grp * G);
    i = grp * G + rem % rows;
    j = rem / rows;
  } else {
    int r = (int)((sqrtf(8.0f * (float)id + 1.0f) - 1.0f) * 0.5f);
    while (r * (r + 1) / 2 > id) --r;
    while ((r + 1) * (r + 2) / 2 <= id) ++r;
    i = r;
    j = id - r * (r + 1) / 2;
  }
}

// C(i, j) = Cin(i, j) + s * sum_k A(i, k) B(j, k)^T (+ the identity on the
// first diag_n diagonal entries), one output tile per workgroup; s = -1 when
// neg, Cin may be null (zero).  With lower = 1 only tiles i >= j are formed.
// 16-deep k-panels (66.6 KB of LDS) and 256 registers per lane: two
// workgroups share a CU, one's MFMAs covering the other's loads and barriers.
constexpr int DKD = 16;

__global__ __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(2, 2)))
void gemm_nt_kernel(const double* __restrict__ A, const double* __restrict__ B,
                    double* __restrict__ C, int t, int lower, int neg,
                    const double* __restrict__ Cin, int diag_n) {
  __shared__ double smem[4 * DKD * LDS_STRIDE];
  const int nblk = lower ? t * (t + 1) / 2 : t * t;
  int i, j;
  out_tile(blockIdx.x, nblk, t, lower != 0, i, j);
  Acc acc;
  const size_t ct = (size_t)(i + t * j) * TILE;
  if (Cin) {
    // start from -Cin when negating: Cin - P is rounded as -(-Cin + P)
    acc_load<0>(tile_rsrc(Cin + ct), acc, neg != 0);
  } else {
    acc_zero(acc);
  }
  auto pair = [&](int k, const double*& pa, const double*& pb) {
    pa = A + (size_t)(i + t * k) * TILE;
    pb = B + (size_t)(j + t * k) * TILE;
  };
  mma_chain<0, DKD>(acc, t, pair, smem);
  if (diag_n > 0 && i == j) {
    // lane l, register r of accumulator (a, b) holds tile element
    // (row, col) = acc_offset(a, b) + 4 NB r, i.e. column (off / NB) + 4 r
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int off = acc_offset(a, b);
        const int row = off & (NB - 1), col0 = off >> 7;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (row == col0 + 4 * r && i * NB + row < diag_n) acc[a][b][r] += neg ? -1.0 : 1.0;
      }
  }
  acc_store_tile<0>(tile_rsrc(C + ct), acc, neg != 0);
}

// Thin chained product: C(i) = Cin(i) +- sum_k P(k) Q(i, k)^T for i < t,
// where P and C are tile columns (t tiles of NB x NB, tile k at k) and Q is
// square tile-major (tile (i, k) at i + t k).  One output tile per
// workgroup, the k-panels of the t links streamed as in gemm_nt_kernel.
// (With symmetric Q, P the transposed tiles of a thin matrix V, the result
// holds the transposed tiles of Q V.)
__global__ __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(2, 2)))
void gemm_thin_kernel(const double* __restrict__ P, const double* __restrict__ Q,
                      double* __restrict__ C, int t, int neg, const double* __restrict__ Cin) {
  __shared__ double smem[4 * DKD * LDS_STRIDE];
  const int i = blockIdx.x;
  Acc acc;
  const size_t ct = (size_t)i * TILE;
  if (Cin)
    acc_load<0>(tile_rsrc(Cin + ct), acc, neg != 0);
  else
    acc_zero(acc);
  auto pair = [&](int k, const double*& pa, const double*& pb) {
    pa = P + (size_t)k * TILE;
    pb = Q + (size_t)(i + t * k) * TILE;
  };
  mma_chain<0, DKD>(acc, t, pair, smem);
  acc_store_tile<0>(tile_rsrc(C + ct), acc, neg != 0);
}

// Random sign probes: the transposed tiles of V (n rows padded to t tiles,
// NB columns), V(r, c) = +-1 from a hash of (r, c) for r < n, 0 beyond n:
// tile k holds V^T's columns 128 k .. 128 k + 127, element (c, rr) at
// c + NB rr for matrix row 128 k + rr.
__global__ __launch_bounds__(NTHREADS) void fill_probe_kernel(double* __restrict__ Vt, int t,
                                                              int n) {
  const size_t total = (size_t)t * TILE;
  for (size_t e = (size_t)blockIdx.x * NTHREADS + threadIdx.x; e < total;
       e += (size_t)gridDim.x * NTHREADS) {
    const int k = (int)(e / TILE), w = (int)(e % TILE), c = w & (NB - 1), rr = w >> 7;
    const int r = NB * k + rr;
    // splitmix64 of (r, c): a fixed, platform-independent sign pattern
    unsigned long long z = ((unsigned long long)r << 32 | (unsigned)c) + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    Vt[e] = r < n ? ((z & 1) ? 1.0 : -1.0) : 0.0;
  }
}

// partial[b] = sum of squares of the entries of tile b (fixed summation
// order, so the result does not depend on the launch)
__global__ __launch_bounds__(NTHREADS) void sumsq_tiles_kernel(const double* __restrict__ M,
                                                               double* __restrict__ partial) {
  __shared__ double red[NTHREADS];
  const double* tile = M + (size_t)blockIdx.x * TILE;
  double s = 0.0;
  for (int e = threadIdx.x; e < (int)TILE; e += NTHREADS) s = fma(tile[e], tile[e], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = NTHREADS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// out[0] = sum of partial[0..count) (one block, fixed order)
__global__ __launch_bounds__(NTHREADS) void sum_kernel(const double* __restrict__ partial, int count,
                                                       double* __restrict__ out) {
  __shared__ double red[NTHREADS];
  double s = 0.0;
  for (int e = threadIdx.x; e < count; e += NTHREADS) s += partial[e];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = NTHREADS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// Makes the square tile-major M symmetric from its lower tiles: tile (i, j),
// i < j, <- tile (j, i)^T, and the upper part of each diagonal tile <- the
// mirror of its lower part.  One block per tile (i, j) with i <= j.
__global__ __launch_bounds__(NTHREADS) void mirror_lower_kernel(double* __restrict__ M, int t) {
  constexpr int SBm = 32;
  __shared__ double L[SBm][SBm + 1];
  const int bi = blockIdx.x % t, bj = blockIdx.x / t;
  if (bi > bj) return;  // uniform per block
  double* dst = M + (size_t)(bi + t * bj) * TILE;
  const double* src = M + (size_t)(bj + t * bi) * TILE;  // tile (bj, bi)
  const int tx = threadIdx.x & (SBm - 1), ty = threadIdx.x / SBm;
  for (int sb = 0; sb < (NB / SBm) * (NB / SBm); ++sb) {
    const int lr0 = (sb % (NB / SBm)) * SBm, lc0 = (sb / (NB / SBm)) * SBm;
    // dst element (lr, lc) <- src element (lc, lr)
#pragma unroll
    for (int q = 0; q < SBm / 8; ++q) {
      const int j = ty + 8 * q;
      L[tx][j] = src[(lc0 + tx) + NB * (lr0 + j)];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < SBm / 8; ++q) {
      const int j = ty + 8 * q;
      const int lr = lr0 + tx, lc = lc0 + j;
      if (bi < bj || lr < lc) dst[lr + NB * lc] = L[j][tx];
    }
    __syncthreads();
  }
}

// out (column-major, ld, order n) <- the symmetric matrix whose lower tiles
// (i >= j) are in the square tile-major src; both triangles are written, or
// only the lower one with lower_only.
__global__ __launch_bounds__(NTHREADS) void unpack_sym_kernel(const double* __restrict__ src,
                                                              int t, int n,
                                                              double* __restrict__ out, int ld,
                                                              int lower_only) {
  __shared__ double L[SB][SB + 1];
  const int bi = blockIdx.x % t, bj = blockIdx.x / t;
  const int tx = threadIdx.x & (SB - 1), ty = threadIdx.x / SB;
  // output tile (bi, bj): lower tiles are copied, upper ones are the
  // transpose of tile (bj, bi); a diagonal tile mirrors its own lower part
  const int si = bi >= bj ? bi : bj, sj = bi >= bj ? bj : bi;
  const double* s = src + (size_t)(si + t * sj) * TILE;
  for (int sb = 0; sb < (NB / SB) * (NB / SB); ++sb) {
    const int lr0 = (sb % (NB / SB)) * SB, lc0 = (sb / (NB / SB)) * SB;
    // transposed: element (lc0 + tx, lr0 + j) of the source tile into L[tx][j]
#pragma unroll
    for (int q = 0; q < SB / 8; ++q) {
      const int j = ty + 8 * q;
      L[tx][j] = s[(lc0 + tx) + NB * (lr0 + j)];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < SB / 8; ++q) {
      const int j = ty + 8 * q;
      const int lr = lr0 + tx, lc = lc0 + j;
      const int gr = bi * NB + lr, gc = bj * NB + lc;
      if (gr < n && gc < n && (!lower_only || gr >= gc)) {
        double v;
        if (bi > bj || (bi == bj && lr >= lc))
          v = s[lr + NB * lc];
        else
          v = L[j][tx];  // source element (lc, lr)
        out[gr + (size_t)ld * gc] = v;
      }
    }
    __syncthreads();
  }
}

// ---- batched backward (see BBackArgs) ------------------------------------
// Counters and control words <- 0 (a fill kernel: the sequence stays
// capturable in a graph).
__global__ void zero_kernel(int32_t* __restrict__ cnt, int ncnt, int32_t* __restrict__ ctrl) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x < ncnt) cnt[x] = 0;
  if (x < CTRL_WORDS) ctrl[x] = 0;
}

// Tile (bi, bj) of the square tile-major form of a column-major source of
// order n (mode as pack_kernel), written with agent-coherent stores (other
// workgroups read it in the same launch).
__device__ void bb_pack_tile(const double* __restrict__ src, int ld, int n, int mode, int bi,
                             int bj, double* out, double (*L)[SB + 1]) {
  const rsrc_t ro = tile_rsrc(out);
  const int tx = threadIdx.x & (SB - 1), ty = threadIdx.x / SB;
  for (int sb = 0; sb < (NB / SB) * (NB / SB); ++sb) {
    const int lr0 = (sb % (NB / SB)) * SB, lc0 = (sb / (NB / SB)) * SB;
    const int r0 = bi * NB + lr0, c0 = bj * NB + lc0;
#pragma unroll
    for (int q = 0; q < SB / 8; ++q) {
      const int j = ty + 8 * q;
      const int sr = c0 + tx, sc = r0 + j;
      L[tx][j] = (sr < n && sc < n) ? src[sr + (size_t)ld * sc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < SB / 8; ++q) {
      const int j = ty + 8 * q;
      const int gr = r0 + tx, gc = c0 + j;
      const double tv = L[j][tx];
      const double dv = (gr < n && gc < n) ? src[gr + (size_t)ld * gc] : 0.0;
      const double v = mode == PACK_SYM_LOWER ? ((gr >= gc) ? dv : tv) : 0.5 * (dv + tv);
      st1(ro, (lr0 + tx) + NB * (lc0 + j), v);
    }
    __syncthreads();
  }
}

// Output tile (bi, bj) of the column-major symmetric matrix whose lower tiles
// are in the square tile-major src (as unpack_sym_kernel, both triangles).
__device__ void bb_unpack_tile(const double* src, int t, int n, double* out, int ld, int bi,
                               int bj, double (*L)[SB + 1]) {
  const int tx = threadIdx.x & (SB - 1), ty = threadIdx.x / SB;
  const int si = bi >= bj ? bi : bj, sj = bi >= bj ? bj : bi;
  const rsrc_t rs = tile_rsrc(src + (size_t)(si + t * sj) * TILE);
  for (int sb = 0; sb < (NB / SB) * (NB / SB); ++sb) {
    const int lr0 = (sb % (NB / SB)) * SB, lc0 = (sb / (NB / SB)) * SB;
#pragma unroll
    for (int q = 0; q < SB / 8; ++q) {
      const int j = ty + 8 * q;
      L[tx][j] = ld1(rs, (lc0 + tx) + NB * (lr0 + j));
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < SB / 8; ++q) {
      const int j = ty + 8 * q;
      const int lr = lr0 + tx, lc = lc0 + j;
      const int gr = bi * NB + lr, gc = bj * NB + lc;
      if (gr < n && gc < n) {
        const double v = (bi > bj || (bi == bj && lr >= lc)) ? ld1(rs, lr + NB * lc) : L[j][tx];
        out[gr + (size_t)ld * gc] = v;
      }
    }
    __syncthreads();
  }
}

// C tile <- s sum_k A(i, k) B(j, k)^T over t links (s = -1 when neg), stored
// agent-coherent.  The operand tiles are written once in the launch and read
// only after that write, so they are read through the L2.
__device__ void bb_gemm_tile(const double* A, const double* B, double* C, int t, int i, int j,
                             bool neg, double* smem) {
  Acc acc;
  acc_zero(acc);
  auto pair = [&](int k, const double*& pa, const double*& pb) {
    pa = A + (size_t)(i + t * k) * TILE;
    pb = B + (size_t)(j + t * k) * TILE;
  };
  mma_chain<0, DKD>(acc, t, pair, smem);
  acc_store_tile<CPOL_AGENT>(tile_rsrc(C), acc, neg);
}

__device__ __forceinline__ int bb_ready(int32_t* c, int target, const BBackArgs& g) {
  const long long t0 = now_ticks();
  long long spins = 0;
  while (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    __builtin_amdgcn_s_sleep(1);
    if ((++spins & 63) == 0) {
      if (__hip_atomic_load(&g.ctrl[CTRL_ABORT], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        return 0;
      if (now_ticks() - t0 > g.spin_limit) {
        __hip_atomic_store(&g.ctrl[CTRL_ABORT], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return 0;
      }
    }
  }
  return 1;
}

// The persistent loop: thread 0 claims a ticket and waits for the task's
// inputs (counters of earlier phases, which hold earlier tickets: the loop is
// deadlock-free for any grid); the workgroup runs the task; once its stores
// have completed, thread 0 counts it.  Divergent regions sit between
// barriers, and a barrier closes the loop body.
__global__ __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(2, 2)))
void bback_kernel(BBackArgs g) {
  __shared__ double smem[4 * DKD * LDS_STRIDE];
  __shared__ int s_v;
  double(*L)[SB + 1] = reinterpret_cast<double(*)[SB + 1]>(smem);
  int32_t* done = nullptr;  // thread 0: counter of the previous task (or null)
  for (;;) {
    if (threadIdx.x == 0) {
      if (done) __hip_atomic_fetch_add(done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      done = nullptr;
      int v = __hip_atomic_fetch_add(&g.ctrl[CTRL_TICKET], 1, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
      if (v >= g.ntask) v = -1;
      if (v >= 0) {
        const int2 tk = g.task[v];
        const int4 mi = g.mat[tk.x];
        const int t = mi.x, phase = tk.y >> BB_PHASE_SHIFT, i = (tk.y >> 8) & 0xff,
                  j = tk.y & 0xff;
        int32_t* c = g.cnt + mi.z;
        int ok = 1;
        if (phase == 1) ok = bb_ready(c, t * t, g);
        else if (phase == 2) ok = bb_ready(c + 1 + i, t, g);
        else if (phase == 3) ok = bb_ready(c + 1 + t + (i >= j ? i + t * j : j + t * i), 1, g);
        if (!ok) v = -1;
        if (phase == 0) done = c;
        else if (phase == 1) done = c + 1 + i;
        else if (phase == 2) done = c + 1 + t + i + t * j;
      }
      s_v = v;
    }
    __syncthreads();
    const int v = __builtin_amdgcn_readfirstlane(s_v);
    if (v < 0) break;
    const int2 tk = g.task[v];
    const int m = __builtin_amdgcn_readfirstlane(tk.x);
    const int code = __builtin_amdgcn_readfirstlane(tk.y);
    const int4 mi = g.mat[m];
    const int t = __builtin_amdgcn_readfirstlane(mi.x);
    const long long tb = (long long)__builtin_amdgcn_readfirstlane(mi.y);
    const int phase = code >> BB_PHASE_SHIFT, i = (code >> 8) & 0xff, j = code & 0xff;
    double* Xt = g.tiles + (size_t)tb * TILE;
    double* St = Xt + (size_t)t * t * TILE;
    double* Wt = St + (size_t)t * t * TILE;
    double* Gt = Wt + (size_t)t * t * TILE;
    // an order or leading dimension that does not fit the matrix's tile
    // count is taken as order 0: its tasks run on zero tiles and write nothing
    const int n0 = __builtin_amdgcn_readfirstlane(g.n[m]);
    const int n = ((n0 + NB - 1) / NB == t) ? n0 : 0;
    if (phase == 0) {
      const int lx = __builtin_amdgcn_readfirstlane(g.ldx[m]);
      const int lg = __builtin_amdgcn_readfirstlane(g.ldg[m]);
      const int nn = (lx >= n && lg >= n) ? n : 0;
      bb_pack_tile(uniform_ptr(g.X[m]), lx, nn, PACK_SYM_LOWER, i, j, Xt + (size_t)(i + t * j) * TILE, L);
      bb_pack_tile(uniform_ptr(g.G[m]), lg, nn, PACK_SYM_AVG, i, j, St + (size_t)(i + t * j) * TILE, L);
    } else if (phase == 1) {
      // W = X S: W(i, j) = sum_k X(i, k) S(j, k)^T (S symmetric)
      bb_gemm_tile(Xt, St, Wt + (size_t)(i + t * j) * TILE, t, i, j, false, smem);
    } else if (phase == 2) {
      // lower tile of -W X: -sum_k W(i, k) X(j, k)^T (X symmetric)
      bb_gemm_tile(Wt, Xt, Gt + (size_t)(i + t * j) * TILE, t, i, j, true, smem);
    } else {
      const int lo = __builtin_amdgcn_readfirstlane(g.ldga[m]);
      bb_unpack_tile(Gt, t, lo >= n ? n : 0, uniform_ptr(g.gradA[m]), lo, i, j, L);
    }
    stores_complete();
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_bback(const BBackArgs& b, int ncnt, int grid, hipStream_t s) {
  const int total = ncnt > CTRL_WORDS ? ncnt : CTRL_WORDS;
  hipLaunchKernelGGL(zero_kernel, dim3((total + 255) / 256), dim3(256), 0, s, b.cnt, ncnt, b.ctrl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(bback_kernel, dim3(grid), dim3(NTHREADS), 0, s, b);
  return hipGetLastError();
}

int bback_blocks_per_cu() {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, bback_kernel, NTHREADS, 0) != hipSuccess)
    return 1;
  return blocks > 0 ? blocks : 1;
}

hipError_t launch_pack(const double* src, int ld, int n, int t, int mode, double* dst,
                       hipStream_t s) {
  hipLaunchKernelGGL(pack_kernel, dim3(t * t), dim3(NTHREADS), 0, s, src, ld, n, t, mode, dst);
  return hipGetLastError();
}

hipError_t launch_gemm_thin(const double* P, const double* Q, double* C, int t, int neg,
                            hipStream_t s, const double* Cin) {
  if (t < 1) return hipErrorInvalidValue;  // the chain takes at least one link
  hipLaunchKernelGGL(gemm_thin_kernel, dim3(t), dim3(NTHREADS), 0, s, P, Q, C, t, neg, Cin);
  return hipGetLastError();
}

hipError_t launch_fill_probe(double* Vt, int t, int n, hipStream_t s) {
  const size_t total = (size_t)t * TILE;
  const size_t blocks = std::min<size_t>((total + NTHREADS - 1) / NTHREADS, 4096);
  hipLaunchKernelGGL(fill_probe_kernel, dim3((unsigned)blocks), dim3(NTHREADS), 0, s, Vt, t, n);
  return hipGetLastError();
}

hipError_t launch_gemm_nt(const double* A, const double* B, double* C, int t, int lower, int neg,
                          hipStream_t s, const double* Cin, int diag_n) {
  if (t < 1) return hipErrorInvalidValue;  // the kernel's chain takes at least one link
  const int nblk = lower ? t * (t + 1) / 2 : t * t;
  hipLaunchKernelGGL(gemm_nt_kernel, dim3(nblk), dim3(NTHREADS), 0, s, A, B, C, t, lower, neg, Cin,
                     diag_n);
  return hipGetLastError();
}

hipError_t launch_unpack_sym(const double* src, int t, int n, double* out, int ld, hipStream_t s,
                             int lower_only) {
  hipLaunchKernelGGL(unpack_sym_kernel, dim3(t * t), dim3(NTHREADS), 0, s, src, t, n, out, ld,
                     lower_only);
  return hipGetLastError();
}

hipError_t launch_sumsq(const double* M, int ntiles, double* partial, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sumsq_tiles_kernel, dim3(ntiles), dim3(NTHREADS), 0, s, M, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(NTHREADS), 0, s, partial, ntiles, out);
  return hipGetLastError();
}

hipError_t launch_mirror_lower(double* M, int t, hipStream_t s) {
  hipLaunchKernelGGL(mirror_lower_kernel, dim3(t * t), dim3(NTHREADS), 0, s, M, t);
  return hipGetLastError();
}

}  // namespace spdinv
