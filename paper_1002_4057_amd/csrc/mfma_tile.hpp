// Building blocks of the FP64 tile products on the gfx950 matrix cores, shared
// by the scheduler's tile tasks and the dense kernels (backward, refinement).
//
// A tile is NB x NB (NB = 128) binary64, column-major and contiguous
// (128 KiB).  One workgroup of 256 threads (4 wave64) computes one 128 x 128
// output: the waves form a 2 x 2 grid of 64 x 64 blocks, each a 4 x 4 array
// of 16 x 16 accumulators of v_mfma_f64_16x16x4f64.
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace spdinv {
namespace tile {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int KC = 32;                    // k-panel depth
constexpr int NCH = NB / KC;              // k-panels per tile
// Row stride of a [k][r] panel in LDS (doubles).  With 130, element (k, r)
// falls in dword bank (4k + 2r) mod 64: the transposing stores (4
// consecutive r x 16 even k per wave) cover all 64 banks, contiguous stores
// of a k-row are conflict-free, and operand reads (16 consecutive r of 4
// consecutive k) conflict at most 2-way.
constexpr int LDS_STRIDE = NB + 2;
constexpr size_t TILE = (size_t)NB * NB;
constexpr int PAIRS = NB * KC / 2 / NTHREADS;  // 16-byte loads per thread per panel

__device__ __forceinline__ double* tile_ptr(double* pool, int idx) {
  return pool + (size_t)idx * TILE;
}

// ---------------------------------------------------------------------------
// Tile access through buffer resources (bounds-checked against the 128 KiB
// tile).  The cache policy is a template parameter: CPOL_AGENT (sc1, the
// policy of agent-scope atomics) makes each access coherent across the whole
// device by itself, which the scheduler needs because a tile written by one
// task is read by workgroups on other XCDs, whose L2 caches are not kept
// coherent with the writer's.  Kernels whose operands were written by an
// earlier launch use the default policy (0) and keep L2 reuse.
// ---------------------------------------------------------------------------
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
typedef unsigned int u2v __attribute__((ext_vector_type(2)));
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int CPOL_AGENT = 16;                 // sc1
constexpr int RSRC_WORD3 = 0x00020000;         // raw dword access (gfx9 family)

__device__ __forceinline__ rsrc_t tile_rsrc(const double* tile) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(tile), 0, (int)(TILE * 8),
                                           RSRC_WORD3);
}
template <int CP = CPOL_AGENT>
__device__ __forceinline__ d2 ld2(rsrc_t r, int elem) {
  return __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, elem * 8, 0, CP));
}
template <int CP = CPOL_AGENT>
__device__ __forceinline__ double ld1(rsrc_t r, int elem) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, elem * 8, 0, CP));
}
template <int CP = CPOL_AGENT>
__device__ __forceinline__ void st2(rsrc_t r, int elem, d2 v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4v, v), r, elem * 8, 0, CP);
}
template <int CP = CPOL_AGENT>
__device__ __forceinline__ void st1(rsrc_t r, int elem, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2v, v), r, elem * 8, 0, CP);
}

// ---------------------------------------------------------------------------
// k-panel staging.  A panel holds op(X)[r][k] for r = 0..127 (the output row
// for the left operand, the output column for the right one) and k in one
// KC-deep slice, stored in LDS as S[k * LDS_STRIDE + r].
//   contig: element (r, k) is X[r + NB*k] (r runs down a stored column)
//  !contig: element (r, k) is X[k + NB*r] (k runs down a stored column)
// mask treats X as lower triangular (entries above its diagonal read as 0).
// Each thread moves PAIRS pairs of doubles per panel with 16-byte loads.
// ---------------------------------------------------------------------------
// KD is the panel depth (KC unless a caller stages shallower panels).
template <int KD>
constexpr int panel_pairs() { return NB * KD / 2 / NTHREADS; }

template <int CP = CPOL_AGENT, int KD = KC>
__device__ __forceinline__ void panel_load(rsrc_t X, int k0, bool contig,
                                           d2 (&r)[panel_pairs<KD>()], int skip = 0) {
  const int tid = threadIdx.x;
  if (contig) {  // (skip: added to this lane's offsets; past the tile, a load reads zero)
#pragma unroll
    for (int q = 0; q < panel_pairs<KD>(); ++q)
      r[q] = ld2<CP>(X, NB * k0 + 2 * (tid + NTHREADS * q) + skip);
  } else {
#pragma unroll
    for (int q = 0; q < panel_pairs<KD>(); ++q) {
      const int p = tid + NTHREADS * q;
      const int rr = p / (KD / 2), kk = (p % (KD / 2)) * 2;
      r[q] = ld2<CP>(X, k0 + kk + NB * rr);
    }
  }
}

template <int KD = KC>
__device__ __forceinline__ void panel_store(double* __restrict__ S, int k0, bool contig, bool mask,
                                            const d2 (&r)[panel_pairs<KD>()]) {
  const int tid = threadIdx.x;
  if (contig) {
#pragma unroll
    for (int q = 0; q < panel_pairs<KD>(); ++q) {
      const int e = 2 * (tid + NTHREADS * q), rr = e & (NB - 1), kk = e >> 7;
      d2 v = r[q];
      // stored element (row rr+s, col k0+kk); lower triangle keeps row >= col
      if (mask) {
        if (rr < k0 + kk) v.x = 0.0;
        if (rr + 1 < k0 + kk) v.y = 0.0;
      }
      *reinterpret_cast<d2*>(S + kk * LDS_STRIDE + rr) = v;
    }
  } else {
#pragma unroll
    for (int q = 0; q < panel_pairs<KD>(); ++q) {
      const int p = tid + NTHREADS * q;
      const int rr = p / (KD / 2), kk = (p % (KD / 2)) * 2;
      double v0 = r[q].x, v1 = r[q].y;
      // stored element (row k0+kk+s, col rr)
      if (mask) {
        if (k0 + kk < rr) v0 = 0.0;
        if (k0 + kk + 1 < rr) v1 = 0.0;
      }
      S[kk * LDS_STRIDE + rr] = v0;
      S[(kk + 1) * LDS_STRIDE + rr] = v1;
    }
  }
}


// ---------------------------------------------------------------------------
// MFMA register layout.  v_mfma_f64_16x16x4(x, y, d): d[i][j] += sum_k
// x[i][k] y[k][j] with x[i][k] from lane i+16k, y[k][j] from lane j+16k, and
// d[i][j] in register r = i/4 of lane j + 16*(i%4).  The products below pass
// (op(B) block, op(A) block), so that d is the transposed 16x16 output block:
// lane l, register r holds output row (l%16) of column (l/16) + 4r, and a
// group of 16 lanes covers 16 consecutive rows of one column (one 128-byte
// segment).  Wave w owns rows 64*(w%2) .. +63 and columns 64*(w/2) .. +63.
// ---------------------------------------------------------------------------
typedef d4 Acc[4][4];

__device__ __forceinline__ void acc_zero(Acc& acc) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
}

// Offset in a tile of element (row, col) held by register 0 of accumulator
// (i, j) in this lane; register r adds 4*NB*r.
__device__ __forceinline__ int acc_offset(int i, int j) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  return ((w & 1) * 64 + i * 16 + (lane & 15)) + NB * ((w >> 1) * 64 + j * 16 + (lane >> 4));
}

// One KD-deep panel step: acc += op(A)[:, k-panel] op(B)[k-panel, :] from the
// LDS panels As, Bs (layout of panel_store).
template <int KD = KC>
__device__ __forceinline__ void panel_mma(Acc& acc, const double* As, const double* Bs) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w & 1, wn = w >> 1, lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int ks = 0; ks < KD / 4; ++ks) {
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

// Chained product: acc += sum_{p < count} A_p B_p^T, where pair(p, a, b)
// names the two contiguous tiles of link p.  Both operands are read along
// stored columns.  The k-panels of all links form one double-buffered
// stream through LDS (smem: 4 * KD * LDS_STRIDE doubles for KD-deep
// panels), so the first panel of link p+1 is loaded while the last panel of
// link p is multiplied.  Each panel's body is one branch-free scheduling
// region in which the next panel's loads (first quarter of the k-steps) and
// their staging into LDS (last quarter) are interleaved with the MFMAs;
// past the last panel the loads read a zero-size buffer
// (zeros, no memory access).  The pair function must give the same pointers
// in every thread, and count must be at least 1.  The accumulator is never
// written to memory here.
template <int CP, int KD = KC, class PairFn>
__device__ __forceinline__ void mma_chain(Acc& acc, int count, PairFn pair, double* smem) {
  // count >= 1 (a bypass path for count = 0 would keep a second copy of the
  // accumulator alive across the loop)
  __builtin_assume(count >= 1);
  const double *pa, *pb;
  pair(0, pa, pb);
  const rsrc_t none = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(pa), 0, 0, RSRC_WORD3);
  d2 ra[panel_pairs<KD>()], rb[panel_pairs<KD>()];
  panel_load<CP, KD>(tile_rsrc(pa), 0, true, ra);
  panel_load<CP, KD>(tile_rsrc(pb), 0, true, rb);
  panel_store<KD>(smem, 0, true, false, ra);
  panel_store<KD>(smem + (KD * LDS_STRIDE), 0, true, false, rb);
  __syncthreads();
  // two rolled loops (links, then the k-panels of a link) with the next
  // link's tiles resolved once per link: this keeps the accumulator in the
  // matrix-core registers for the whole chain (other loop shapes made the
  // compiler copy it out and back every iteration)
#pragma unroll 1
  for (int p = 0; p < count; ++p) {
    const double *qa, *qb;
    pair(p + 1 < count ? p + 1 : p, qa, qb);
    const bool last = p + 1 >= count;
    const rsrc_t rA = tile_rsrc(pa), rB = tile_rsrc(pb);
    const rsrc_t nA = last ? none : tile_rsrc(qa), nB = last ? none : tile_rsrc(qb);
#pragma unroll 1
    for (int c = 0; c < (NB / KD); ++c) {
      const double* As = smem + (c & 1) * 2 * (KD * LDS_STRIDE);
      const double* Bs = As + (KD * LDS_STRIDE);
      double* An = smem + ((c + 1) & 1) * 2 * (KD * LDS_STRIDE);
      const bool wrap = c + 1 == (NB / KD);
      panel_load<CP, KD>(wrap ? nA : rA, ((c + 1) % (NB / KD)) * KD, true, ra);
      panel_load<CP, KD>(wrap ? nB : rB, ((c + 1) % (NB / KD)) * KD, true, rb);
      panel_mma<KD>(acc, As, Bs);
      // the next panel's buffer was released by the previous barrier
      panel_store<KD>(An, 0, true, false, ra);
      panel_store<KD>(An + (KD * LDS_STRIDE), 0, true, false, rb);
      __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
#pragma unroll
      for (int ks = 0; ks < KD / 4; ++ks) {
        __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
        // the loads over the first quarter of the k-steps, their LDS
        // stores over the last quarter
        if (ks < KD / 16) __builtin_amdgcn_sched_group_barrier(0x020, 8, 0);
        if (ks >= 3 * KD / 16) __builtin_amdgcn_sched_group_barrier(0x200, 8, 0);
        if (ks + 1 < KD / 4) __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
      }
      __syncthreads();
    }
    pa = qa;
    pb = qb;
  }
}

// Accumulator (i, j), register r of this lane holds tile element
// acc_lane_base() + 16 i + NB (16 j + 4 r).  The loads and stores below keep
// only the per-lane part in a register (made opaque at every call, so that
// the compiler recomputes it instead of keeping 64 addresses live across a
// persistent loop) and pass the rest as the instruction's immediate and
// scalar offsets.
__device__ __forceinline__ int opaque_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

__device__ __forceinline__ int acc_lane_bytes() {
  const int t = opaque_tid(), lane = t & 63, w = t >> 6;
  return 8 * (((w & 1) * 64 + (lane & 15)) + NB * ((w >> 1) * 64 + (lane >> 4)));
}

template <int CP = CPOL_AGENT>
__device__ __forceinline__ void acc_load(rsrc_t r, d4 (&acc)[4][4], bool neg) {
  const int vb = acc_lane_bytes();
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double x = __builtin_bit_cast(
            double, __builtin_amdgcn_raw_buffer_load_b64(r, vb + 128 * i, 8 * NB * (16 * j + 4 * q), CP));
        acc[i][j][q] = neg ? -x : x;
      }
}

template <int CP = CPOL_AGENT>
__device__ __forceinline__ void acc_store_tile(rsrc_t r, const d4 (&acc)[4][4], bool neg) {
  const int vb = acc_lane_bytes();
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double x = neg ? -acc[i][j][q] : acc[i][j][q];
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2v, x), r, vb + 128 * i,
                                              8 * NB * (16 * j + 4 * q), CP);
      }
}

// The same for 16 IN rows of a tile from row row0 (IN = 4: a half, 2: a
// quarter), the four waves side by side: wave w holds the rows
// (accumulators i < IN) of columns 32 w .. 32 w + 31 (accumulators
// j = 0..1); register r of accumulator (i, j) of this lane holds tile element
// row0 + 16 i + lane % 16 + NB (32 w + 16 j + lane / 16 + 4 r).
__device__ __forceinline__ int acc_lane_bytes_r64(int row0) {
  const int t = opaque_tid(), lane = t & 63, w = t >> 6;
  return 8 * ((lane & 15) + NB * (32 * w + (lane >> 4))) + 8 * row0;
}

template <int IN = 4, int CP = CPOL_AGENT>
__device__ __forceinline__ void acc_load_r64(rsrc_t r, d4 (&acc)[4][4], bool neg, int row0 = 0) {
  const int vb = acc_lane_bytes_r64(row0);
#pragma unroll
  for (int i = 0; i < IN; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double x = __builtin_bit_cast(
            double, __builtin_amdgcn_raw_buffer_load_b64(r, vb + 128 * i, 8 * NB * (16 * j + 4 * q), CP));
        acc[i][j][q] = neg ? -x : x;
      }
}

template <int IN = 4, int CP = CPOL_AGENT>
__device__ __forceinline__ void acc_store_r64(rsrc_t r, const d4 (&acc)[4][4], bool neg,
                                              int row0 = 0) {
  const int vb = acc_lane_bytes_r64(row0);
#pragma unroll
  for (int i = 0; i < IN; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double x = neg ? -acc[i][j][q] : acc[i][j][q];
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2v, x), r, vb + 128 * i,
                                              8 * NB * (16 * j + 4 * q), CP);
      }
}

// C <- s * acc for one output tile (s = +1 or -1, exact); `lower` skips the
// block that lies strictly above the diagonal (rows 0-63 x columns 64-127).
template <int CP>
__device__ __forceinline__ void acc_store(double* C, const Acc& acc, bool neg, bool lower) {
  const int w = threadIdx.x >> 6;
  if (lower && w == 2) return;
  const rsrc_t rC = tile_rsrc(C);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int off = acc_offset(i, j);
#pragma unroll
      for (int r = 0; r < 4; ++r) st1<CP>(rC, off + NB * 4 * r, neg ? -acc[i][j][r] : acc[i][j][r]);
    }
}

// Arguments of an out-of-line device function arrive in vector registers,
// where the compiler has to assume that they differ between lanes: a buffer
// access through such a pointer becomes a loop over its distinct values.
// The callers pass wave-uniform values, so re-reading them from the first
// lane is exact and gives scalar addressing back.  (LDS pointers are left
// alone: the compiler has already resolved their address space.)
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return reinterpret_cast<T*>(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

// A task's results are published when its agent-coherent stores have
// completed: every thread waits for its outstanding memory operations before
// the workgroup barrier that precedes the successors' counter decrements.
__device__ __forceinline__ void stores_complete() { __builtin_amdgcn_s_waitcnt(0); }

__device__ __forceinline__ long long now_ticks() {
  return (long long)__builtin_amdgcn_s_memrealtime();
}

}  // namespace tile
}  // namespace spdinv
