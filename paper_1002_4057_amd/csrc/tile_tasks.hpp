// The tile tasks of the SPD inverse on gfx950 (MI355X), as device functions
// shared by the persistent scheduler (device.hip) and the batched kernel
// (batched.hip).  Everything is in an anonymous namespace on purpose: each
// kernel's translation unit gets its own copy of the out-of-line functions,
// whose register allocation would otherwise be shared by both kernels.
//
// Tiles are NB x NB (NB = 128) binary64, column-major, each contiguous
// (128 KiB).  One workgroup of 256 threads (4 wave64) executes one task at a
// time; every task kind of the paper's Algorithm 1 maps to one of
//   * a tile product on the FP64 matrix cores (v_mfma_f64_16x16x4),
//     C = beta*C + alpha*op(A)*op(B) with optional triangular masking of an
//     operand and a lower-only output, staged through LDS in k-panels, and
//     an optional second destination (the renaming copy of Section 3);
//   * the diagonal-tile factorization POTRF, which also produces the inverse
//     of the factor tile, blocked by 16 with the lower blocks of the tile
//     resident in LDS (factor_packed and inverse_packed);
//   * a tile copy (TRTRI reuses the inverse made by POTRF, bit for bit).
#pragma once
#include <climits>

#include "device.hpp"
#include "mfma_tile.hpp"

namespace spdinv {
namespace {

using namespace tile;

// The scheduler's tile products stage 16-deep k-panels (8 per tile): the
// two double-buffered operand panels take 66.6 KB of LDS, the renaming copy
// is staged half a tile at a time (66 KB) and the diagonal-tile task keeps
// only the lower 16 x 16 blocks (78.1 KB), so that a task needs at most
// TASK_SMEM doubles (under 80 KB: two workgroups per CU).
constexpr int SKC = 16;
constexpr int SNCH = NB / SKC;
constexpr int SPAIRS = panel_pairs<SKC>();
constexpr int SPANEL = SKC * LDS_STRIDE;
constexpr int SGEMM_SMEM = 4 * SPANEL;
constexpr int RLD = NB + 1;            // row stride of a staged copy
constexpr int COPY_SMEM = 64 * RLD;    // half a tile
constexpr int PK_LD = 17;              // packed diagonal tile, see pk_blk
constexpr int PK_STRIDE = 16 * PK_LD;
constexpr int PK_BLOCKS = 8 * 9 / 2;
// blocks + reciprocal pivots + flag + the column broadcast of chol16
constexpr int PK_SMEM = PK_BLOCKS * PK_STRIDE + NB + 8 + 64;
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int TASK_SMEM = cmax(cmax(SGEMM_SMEM, COPY_SMEM), PK_SMEM);
static_assert(TASK_SMEM * 8 <= 80 * 1024, "a task must fit half of the CU's LDS");


// Renaming copy of a product's result (as is, or transposed with copy_t):
// the result is staged in LDS one half of its rows at a time, as
// R[col + RLD * row] (odd stride RLD, conflict-free for these writes), and
// leaves as contiguous 16-byte stores.  The caller's k-loop has ended with a
// barrier, so smem is free.
__device__ __forceinline__ void copy_epilogue(double* copy, const d4 (&acc)[4][4], bool neg,
                                              bool copy_t, double* smem) {
  const int tid = opaque_tid(), lane = tid & 63, w = tid >> 6;
  const int wm = w & 1, wn = w >> 1, lr = lane & 15, lk = lane >> 4;
  const rsrc_t rD = tile_rsrc(copy);
  double* R = smem;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (wm == h) {  // the waves holding result rows 64h .. 64h+63
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = i * 16 + lr, col0 = wn * 64 + j * 16 + lk;
#pragma unroll
          for (int r = 0; r < 4; ++r)
            R[(col0 + 4 * r) + RLD * row] = neg ? -acc[i][j][r] : acc[i][j][r];
        }
    }
    __syncthreads();
#pragma unroll 4
    for (int q = 0; q < NB * 64 / 2 / NTHREADS; ++q) {
      const int e2 = 2 * (tid + NTHREADS * q);
      d2 v;
      int e;
      if (copy_t) {  // copy(rr, 64h + cl) = result(64h + cl, rr): copy columns of this half
        const int rr = e2 & (NB - 1), cl = e2 >> 7;
        v.x = R[rr + RLD * cl];
        v.y = R[rr + 1 + RLD * cl];
        e = rr + NB * (64 * h + cl);
      } else {       // copy(64h + rl, cc) = result(64h + rl, cc): copy rows of this half
        const int rl = e2 & 63, cc = e2 >> 6;
        v.x = R[cc + RLD * rl];
        v.y = R[cc + RLD * (rl + 1)];
        e = 64 * h + rl + NB * cc;
      }
      st2(rD, e, v);
    }
    if (h == 0) __syncthreads();  // half 1 overwrites R
  }
}

// The renaming copy of a row-part product (RN rows from row0, the waves side
// by side as in acc_load_r64): the part is staged in LDS as in copy_epilogue
// and leaves as contiguous 16-byte stores, columns row0 .. row0+RN-1 of the
// copy (copy_t) or its rows row0 .. row0+RN-1.
template <int RN>
__device__ __forceinline__ void copy_epilogue_r64(double* copy, const d4 (&acc)[4][4], bool neg,
                                                  bool copy_t, double* smem, int row0) {
  const int tid = opaque_tid(), lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const rsrc_t rD = tile_rsrc(copy);
  double* R = smem;
#pragma unroll
  for (int i = 0; i < RN / 16; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int row = i * 16 + lr, col0 = w * 32 + j * 16 + lk;
#pragma unroll
      for (int r = 0; r < 4; ++r) R[(col0 + 4 * r) + RLD * row] = neg ? -acc[i][j][r] : acc[i][j][r];
    }
  __syncthreads();
#pragma unroll 4
  for (int q = 0; q < NB * RN / 2 / NTHREADS; ++q) {
    const int e2 = 2 * (tid + NTHREADS * q);
    d2 v;
    int e;
    if (copy_t) {  // copy(rr, row0 + cl) = result(row0 + cl, rr)
      const int rr = e2 & (NB - 1), cl = e2 >> 7;
      v.x = R[rr + RLD * cl];
      v.y = R[rr + 1 + RLD * cl];
      e = rr + NB * (row0 + cl);
    } else {       // copy(row0 + rl, cc) = result(row0 + rl, cc)
      const int rl = e2 & (RN - 1), cc = e2 / RN;
      v.x = R[cc + RLD * rl];
      v.y = R[cc + RLD * (rl + 1)];
      e = row0 + rl + NB * cc;
    }
    st2(rD, e, v);
  }
}

// ---------------------------------------------------------------------------
// Tile product on the FP64 matrix cores.
//   C (+)= (F_NEG ? -1 : 1) * op(A) * op(B),   op(A) = F_TA ? A^T : A,
//                                              op(B) = F_TB ? B^T : B
// (FAST: the renamed plan's case op(A) = A, op(B) = B^T without masks)
// F_ACC: accumulate into C (else overwrite).  F_MA/F_MB: the operand tile is
// lower triangular.  F_LOWER: only the output blocks on or below the diagonal
// are stored (the wave owning rows 0-63 x columns 64-127 computes but does
// not store: it runs alone on its SIMD, so skipping its work would save no
// time).  C may alias A or B: every operand read precedes the first store.
// copy (may be null) receives the same result, transposed with F_COPYT.
// npan: k-panels to run (fewer than SNCH skips the padded tail of a ragged
// last tile block, see K_KLAST).  R64: only the RN output rows from row0
// are formed and stored (with their part of the copy); per output element
// the MFMA sequence is that of the whole-tile product.
// Waves form a 2 x 2 grid of 64 x 64 output blocks, each a 4 x 4 array of
// 16 x 16 MFMA accumulators.  The sign is handled without touching the
// operands: the accumulator starts from -C and the result is negated on the
// way out (both exact), so that C - P is rounded exactly like -(-C + P).
// The panels are double-buffered in LDS; the next panel's global loads are
// issued before the current panel's MFMAs and consumed after them
// (scheduling barriers keep the compiler from pulling their consumers into
// the MFMA sequence).
// ---------------------------------------------------------------------------
template <bool FAST, bool R64 = false, int RN = 64>
__device__ __forceinline__ void tile_mma(int f, double* C, const double* A, const double* B,
                                         double* copy, double* smem, bool nca = false,
                                         bool ncb = false, int npan = SNCH, int prow = 0) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int wm = w & 1, wn = w >> 1;
  const int lr = lane & 15, lk = lane >> 4;
  // FAST: op(A) = A, op(B) = B^T, no triangular masks (both operands read
  // along contiguous columns); otherwise every flag is honoured
  const bool a_contig = FAST || !(f & F_TA), b_contig = FAST || (f & F_TB) != 0;
  const bool ma = !FAST && (f & F_MA) != 0, mb = !FAST && (f & F_MB) != 0;
  const bool neg = (f & F_NEG) != 0, copy_t = (f & F_COPYT) != 0;
  const rsrc_t rA = tile_rsrc(A), rB = tile_rsrc(B), rC = tile_rsrc(C);
  const bool accum = (f & F_ACC) != 0;
  // (F_LOWER: the blocks skipped are those of the whole-tile product)
  const bool active = R64 ? !((f & F_LOWER) && prow < 64 && w >= 2)
                          : !((f & F_LOWER) && wm == 0 && wn == 1);
  // R64: RN rows only, the waves side by side (32 columns each)
  const int row0 = R64 ? prow : wm * 64, col0 = R64 ? w * 32 : wn * 64;
  constexpr int JN = R64 ? 2 : 4, IN = R64 ? RN / 16 : 4;

  // v_mfma_f64_16x16x4(x, y, d): d[i][j] += sum_k x[i][k] y[k][j] with x[i][k]
  // from lane i+16k, y[k][j] from lane j+16k, and d[i][j] in register r = i/4
  // of lane j + 16*(i%4).  The operands are passed as (op(B) block, op(A)
  // block), so that d is the transposed 16x16 output block: lane l, register
  // r holds output row (l%16) of column (l/16) + 4r, and a group of 16 lanes
  // covers 16 consecutive rows of one column (one 128-byte segment).
  d4 acc[4][4];
  if (accum) {
    if constexpr (R64) acc_load_r64<IN>(rC, acc, neg, prow);
    else acc_load(rC, acc, neg);
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  }

  d2 ra[SPAIRS], rb[SPAIRS];
  // R64: a lane holds rows 2 (lane % 64) and 2 (lane % 64) + 1 of the A
  // panel; lanes whose rows lie outside this part skip their loads (an
  // offset past the tile reads zero without touching memory), so a row part
  // reads only its own rows of A
  const int lrow = 2 * (threadIdx.x & 63);
  const int a_skip = (R64 && (lrow < prow || lrow >= prow + RN)) ? (1 << 26) : 0;
  // operand panels: through the L2 when the planner allows it for this read
  // (nca / ncb), device-coherent otherwise
  auto load_a = [&](int k0) {
    if (nca) panel_load<0, SKC>(rA, k0, a_contig, ra, a_skip);
    else panel_load<CPOL_AGENT, SKC>(rA, k0, a_contig, ra, a_skip);
  };
  auto load_b = [&](int k0) {
    if (ncb) panel_load<0, SKC>(rB, k0, b_contig, rb);
    else panel_load<CPOL_AGENT, SKC>(rB, k0, b_contig, rb);
  };
  load_a(0);
  load_b(0);
  panel_store<SKC>(smem, 0, a_contig, ma, ra);
  panel_store<SKC>(smem + SPANEL, 0, b_contig, mb, rb);
  __syncthreads();

#pragma unroll 1
  for (int c = 0; c < npan; ++c) {
    const double* As = smem + (c & 1) * 2 * SPANEL;
    const double* Bs = As + SPANEL;
    const bool more = c + 1 < npan;
    if (more) {
      load_a((c + 1) * SKC);
      load_b((c + 1) * SKC);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int ks = 0; ks < SKC / 4; ++ks) {
      const double* Ar = As + (4 * ks + lk) * LDS_STRIDE + row0 + lr;
      const double* Br = Bs + (4 * ks + lk) * LDS_STRIDE + col0 + lr;
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (i < IN) a[i] = Ar[16 * i];
        if (i < JN) b[i] = Br[16 * i];
      }
#pragma unroll
      for (int i = 0; i < IN; ++i)
#pragma unroll
        for (int j = 0; j < JN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[j], a[i], acc[i][j], 0, 0, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (more) {
      double* An = smem + ((c + 1) & 1) * 2 * SPANEL;
      panel_store<SKC>(An, (c + 1) * SKC, a_contig, ma, ra);
      panel_store<SKC>(An + SPANEL, (c + 1) * SKC, b_contig, mb, rb);
    }
    __syncthreads();
  }

  if constexpr (R64) {
    if (active) acc_store_r64<IN>(rC, acc, neg, prow);
    if (!copy) return;  // uniform: the copy pointer is the same in every thread
    copy_epilogue_r64<RN>(copy, acc, neg, copy_t, smem, prow);
  } else {
    if (active) acc_store_tile(rC, acc, neg);
    if (!copy) return;  // uniform: the copy pointer is the same in every thread
    copy_epilogue(copy, acc, neg, copy_t, smem);
  }
}

// ---------------------------------------------------------------------------
// Chained tile product: C (+)= +-(A_0 B_0^T + A_1 B_1^T + ... + A_L B_L^T),
// the consecutive products of one output tile's update chain run as one task
// (op(A) = A, op(B) = B^T for every link; flags as in tile_mma).  Link 0 is
// (A, B); link p >= 1 reads the tiles named by links[2(p-1)] and
// links[2(p-1)+1].  Link 0 runs npan0 k-panels, a link marked LINK_KLAST
// npan_last, any other SNCH (see K_KLAST).  The accumulator starts from +-C
// and takes the links' products in order, k-panel by k-panel, so every rounding is that of the
// separate tasks (whose stores and reloads of the intermediate tile are
// exact); C is read and written once.  The k-panels of all links form one
// double-buffered stream through LDS, and each panel's body is a single
// scheduling region in which the next panel's global loads (first k-step)
// and their staging into LDS (last k-step) are interleaved with the MFMAs: a
// wave issues in order, and issuing all loads of a panel at once kept the
// matrix cores idle for about half a microsecond per panel.  For that the
// body has no branch: past the last panel the loads read a zero-size buffer
// (they return zeros without touching memory), and every operand read is
// device-coherent (the cache policy is an immediate of the instruction, so
// L2-cacheable marks would need a branch; the planner sets none on chained
// tasks).  Two rolled
// loops (links, then panels) keep the accumulator in registers for the whole
// chain.  Inlined into the scheduler: as an out-of-line call it saved and
// restored 77 callee-saved registers through scratch memory on every task.
// ---------------------------------------------------------------------------
template <bool R64 = false>
__device__ __forceinline__ void tile_mma_chain(int f, double* C, const double* A,
                                                         const double* B, double* copy,
                                                         double* smem, const int32_t* links,
                                                         int nlink, double* pool, int npan0,
                                                         int npan_last) {
  f = uniform_int(f);
  C = uniform_ptr(C);
  A = uniform_ptr(A);
  B = uniform_ptr(B);
  copy = uniform_ptr(copy);
  links = uniform_ptr(links);
  nlink = uniform_int(nlink);
  pool = uniform_ptr(pool);
  npan0 = uniform_int(npan0);
  npan_last = uniform_int(npan_last);
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int wm = w & 1, wn = w >> 1;
  const int lr = lane & 15, lk = lane >> 4;
  const bool neg = (f & F_NEG) != 0, copy_t = (f & F_COPYT) != 0;
  const bool accum = (f & F_ACC) != 0;
  const bool active = R64 ? !((f & F_LOWER) && w >= 2) : !((f & F_LOWER) && wm == 0 && wn == 1);
  const int row0 = R64 ? 0 : wm * 64, col0 = R64 ? w * 32 : wn * 64;
  constexpr int JN = R64 ? 2 : 4;
  const rsrc_t rC = tile_rsrc(C);

  d4 acc[4][4];
  if (accum) {
    if constexpr (R64) acc_load_r64(rC, acc, neg);
    else acc_load(rC, acc, neg);
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  }

  d2 ra[SPAIRS], rb[SPAIRS];
  // The link table is read one link ahead: the entries of link p+1 are
  // loaded at the head of link p-1, so that turning them into scalars at
  // the head of link p waits for nothing (a load issued there and used at
  // once stalls the wave for a memory round trip on every link).
  // (global, not flat, loads: a flat load also counts as an LDS access, so
  // the k-loop's LDS waits would wait for it too)
  typedef const __attribute__((address_space(1))) int32_t* gint_ptr;
  const gint_ptr LT = (gint_ptr)links;
  int qa = 0, qb = 0;
  if (nlink >= 1) {
    qa = LT[0];
    qb = LT[1];
  }
  const rsrc_t none = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(A), 0, 0, RSRC_WORD3);
  rsrc_t cA = tile_rsrc(A), cB = tile_rsrc(B);
  panel_load<CPOL_AGENT, SKC>(cA, 0, true, ra);
  panel_load<CPOL_AGENT, SKC>(cB, 0, true, rb);
  panel_store<SKC>(smem, 0, true, false, ra);
  panel_store<SKC>(smem + SPANEL, 0, true, false, rb);
  __syncthreads();

  // panels run by link p (npan) and by link p+1 (nnext); gp counts panels
  // over the whole chain for the LDS double buffer
  int npan = npan0, gp = 0;
#pragma unroll 1
  for (int p = 0; p <= nlink; ++p) {
    const bool last = p == nlink;
    rsrc_t nA = none, nB = none;
    int nnext = SNCH;
    if (!last) {  // operands of link p+1, then the table entries of link p+2
      const int va = __builtin_amdgcn_readfirstlane(qa);
      const int vb = __builtin_amdgcn_readfirstlane(qb);
      nA = tile_rsrc(tile_ptr(pool, va & ~LINK_KLAST));
      nB = tile_rsrc(tile_ptr(pool, vb));
      nnext = (va & LINK_KLAST) ? npan_last : SNCH;
      if (p + 2 <= nlink) {
        qa = LT[2 * (p + 1)];
        qb = LT[2 * (p + 1) + 1];
      }
    }
#pragma unroll 1
    for (int c = 0; c < npan; ++c, ++gp) {
      const double* As = smem + (gp & 1) * 2 * SPANEL;
      const double* Bs = As + SPANEL;
      double* An = smem + ((gp + 1) & 1) * 2 * SPANEL;
      const bool wrap = c + 1 == npan;
      const rsrc_t sA = wrap ? nA : cA, sB = wrap ? nB : cB;
      const int k0 = wrap ? 0 : (c + 1) * SKC;
      panel_load<CPOL_AGENT, SKC>(sA, k0, true, ra);
      panel_load<CPOL_AGENT, SKC>(sB, k0, true, rb);
#pragma unroll
      for (int ks = 0; ks < SKC / 4; ++ks) {
        const double* Ar = As + (4 * ks + lk) * LDS_STRIDE + row0 + lr;
        const double* Br = Bs + (4 * ks + lk) * LDS_STRIDE + col0 + lr;
        double a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          a[i] = Ar[16 * i];
          if (i < JN) b[i] = Br[16 * i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < JN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[j], a[i], acc[i][j], 0, 0, 0);
      }
      // the next panel's buffer was released by the previous barrier
      panel_store<SKC>(An, 0, true, false, ra);
      panel_store<SKC>(An + SPANEL, 0, true, false, rb);
      // order of the region: the operands of k-step 0, then per k-step half
      // of its MFMAs, the next panel's loads (k-step 0) or their LDS stores
      // (last k-step), the next k-step's operands, the other half
      constexpr int MF = 4 * JN / 2, DR = R64 ? 3 : 4;  // MFMAs per half k-step, LDS reads
      __builtin_amdgcn_sched_group_barrier(0x100, DR, 0);
#pragma unroll
      for (int ks = 0; ks < SKC / 4; ++ks) {
        __builtin_amdgcn_sched_group_barrier(0x008, MF, 0);
        if (ks == 0) __builtin_amdgcn_sched_group_barrier(0x020, 8, 0);
        if (ks == SKC / 4 - 1) __builtin_amdgcn_sched_group_barrier(0x200, 8, 0);
        if (ks + 1 < SKC / 4) __builtin_amdgcn_sched_group_barrier(0x100, DR, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, MF, 0);
      }
      __syncthreads();
    }
    cA = nA;
    cB = nB;
    npan = nnext;
  }

  if constexpr (R64) {
    if (active) acc_store_r64(rC, acc, neg);  // no renaming copy (the caller's rule)
  } else {
    if (active) acc_store_tile(rC, acc, neg);
    if (!copy) return;  // uniform
    copy_epilogue(copy, acc, neg, copy_t, smem);
  }
}

// The general product (transposed or triangular operands) serves only the
// in-place plan; it is kept out of line so that its registers do not weigh
// on the inlined fast product.
__device__ __attribute__((noinline)) void tile_mma_general(int f, double* C, const double* A,
                                                           const double* B, double* copy,
                                                           double* smem) {
  tile_mma<false>(uniform_int(f), uniform_ptr(C), uniform_ptr(A), uniform_ptr(B),
                  uniform_ptr(copy), smem);
}

// ---------------------------------------------------------------------------
// Diagonal tile: Cholesky factor L of the lower triangle of A and its inverse
// X = L^{-1}, blocked by 16 with the lower blocks of the tile held in LDS
// (factor_packed, then inverse_packed, below).
// MFMA 16x16 blocks use the same lane layout as tile_mma: lane l, register r
// holds row l%16, column l/16 + 4r of the block.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const unsigned long long u = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)u, lane);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Orders the LDS stores of some lanes of a wave before later LDS loads of
// other lanes of the same wave.  The LDS executes one wave's operations in
// order, so no wait is needed; the fences keep the compiler from moving the
// accesses across each other.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cholesky factor of the 16 x 16 block at S (column-major, ld), executed by
// one whole wave.  Lane 16 q + r holds row r, columns 4 j + q (j = 0..3).
// Step k:
//   - the pivot d = a_kk gives 1/L_kk (hardware rsq plus one Newton step,
//     y <- y + y (1 - d y^2) / 2) and L_kk = d / sqrt(d);
//   - the lanes of column k scale it into the multipliers m_r = a_rk / L_kk
//     (zero for r <= k) and broadcast them through col (64 doubles of LDS,
//     one 16-double slice per lane group, so that no lane is masked off);
//   - every lane applies a_rc <- a_rc - m_r m_c to its four entries.  Entries
//     that are already final, or lie above the diagonal, see a zero
//     multiplier (a no-op up to the sign of a zero) or are discarded.
// The next pivot a_{k+1,k+1} - m_{k+1}^2 is formed from a_{k+1,k} and
// a_{k+1,k+1} in uniform registers, with the operations of the lane that
// holds it, so the chain of pivots does not wait for the broadcast.
// Writes L (zeros above the diagonal) back to S and the reciprocal pivots
// 1/L_kk to rd[0..15].  Returns 0, or the 1-based index of the first pivot
// that is not positive (or NaN), uniform; S is then left unchanged.
__device__ __forceinline__ int chol16(double* S, int ld, double* rd, double* col) {
  const int tid = opaque_tid(), r = tid & 15, q = (tid >> 4) & 3;
  double a[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = 4 * j + q;
    a[j] = (c <= r) ? S[r + ld * c] : 0.0;
  }
  int fail = 0;
  double d = readlane_d(a[0], 0);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int qk = k & 3, jk = k >> 2;  // column k: lane group qk, slot jk
    if (fail == 0 && !(d > 0.0)) fail = k + 1;
    double rinv = __builtin_amdgcn_rsq(d);
    const double h = d * rinv;
    rinv = fma(rinv * 0.5, fma(-h, rinv, 1.0), rinv);
    const double lkk = d * rinv;
    if ((tid & 63) == 0) rd[k] = rinv;
    if (k == 15) {
      if (q == qk && r == k) a[jk] = lkk;
      break;
    }
    const int k1 = k + 1, q1 = k1 & 3, j1 = k1 >> 2;
    const double u1 = readlane_d(a[jk], 16 * qk + k1);  // a_{k+1,k}
    const double u2 = readlane_d(a[j1], 16 * q1 + k1);  // a_{k+1,k+1}
    const double m = (r > k) ? a[jk] * rinv : 0.0;
    col[16 * q + r] = m;
    const double mn = u1 * rinv;
    d = fma(-mn, mn, u2);
    wave_lds_sync();
    const double mr = col[16 * qk + r];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (4 * j + 3 > k) a[j] = fma(-mr, col[16 * qk + 4 * j + q], a[j]);
    wave_lds_sync();
    if (q == qk) a[jk] = (r == k) ? lkk : m;
  }
  if (fail) return fail;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = 4 * j + q;
    S[r + ld * c] = (c <= r) ? a[j] : 0.0;
  }
  return 0;
}

// acc (one 16x16 block, MFMA layout) += A_blk * op(B)_blk over K = 16, with
// A_blk[m][k] = A[m + lda*k] and op(B)_blk[k][n] = B[n + ldb*k] (tb, i.e. the
// block B^T of a column-major B) or B[k + ldb*n] (!tb).
__device__ __forceinline__ d4 blk_mma16(d4 acc, const double* A, int lda, const double* B, int ldb,
                                        bool tb) {
  const int lane = opaque_tid() & 63, lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int k = 4 * kk + lk;
    const double a = A[lr + lda * k];
    const double b = tb ? B[lr + ldb * k] : B[k + ldb * lr];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, acc, 0, 0, 0);
  }
  return acc;
}

__device__ __forceinline__ d4 blk_load(const double* S, int ld) {
  const int lane = opaque_tid() & 63, lr = lane & 15, lk = lane >> 4;
  return d4{S[lr + ld * lk], S[lr + ld * (lk + 4)], S[lr + ld * (lk + 8)], S[lr + ld * (lk + 12)]};
}

__device__ __forceinline__ void blk_store(double* S, int ld, d4 v) {
  const int lane = opaque_tid() & 63, lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) S[lr + ld * (lk + 4 * q)] = v[q];
}

// ---------------------------------------------------------------------------
// Diagonal tile in packed form: only the 36 lower 16 x 16 blocks of the tile
// are held in LDS, block (i, p) (i >= p) at PK_STRIDE * (i(i+1)/2 + p),
// column-major with the odd leading dimension PK_LD (transposed reads spread
// over the banks).  78.1 KB with the pivots and chol16's broadcast buffer,
// so that the scheduler's workgroups fit two per CU.
// ---------------------------------------------------------------------------
static_assert(PK_BLOCKS * 128 % NTHREADS == 0, "packed load assumes whole passes");

__device__ __forceinline__ double* pk_blk(double* T, int i, int p) {
  return T + PK_STRIDE * (i * (i + 1) / 2 + p);
}

// Block row i of the packed index b = i(i+1)/2 + j (0 <= b < 36), without a
// loop: a loop of taken branches per block cost half the tile load's time.
__device__ __forceinline__ int pk_row(int b) {
  return (b >= 1) + (b >= 3) + (b >= 6) + (b >= 10) + (b >= 15) + (b >= 21) + (b >= 28);
}

// Blocked Cholesky factorization of the leading 16P x 16P block of the
// packed tile, in place, with one block of lookahead: wave 0 factors the
// 16 x 16 diagonal block (chol16); the panel below it solves
// L_ip = A_ip L_pp^{-T} by forward substitution, one row per thread; of the
// updates A_ij -= L_im L_jm^T (16x16x16 MFMA blocks), wave 0 applies the
// last one to the next diagonal block and factors it, while waves 1-3 bring
// the rest of the next block column up to date and apply panel p to the
// later diagonal blocks.  Every block sums its updates in the order
// m = 0, 1, ... as a right-looking update would (the LDS round trips and
// sign changes between them are exact); deferring the off-diagonal ones
// keeps each step's work near the diagonal block's.  rd receives the 16P
// reciprocal pivots; col is chol16's broadcast buffer.  Returns 0 or the
// 1-based index of the first pivot that is not positive (or NaN), uniform
// over the workgroup.
__device__ __forceinline__ int factor_packed(double* T, double* rd, double* col, int* flag, int P) {
  const int tid = opaque_tid(), w = tid >> 6;
  if (w == 0) {
    const int f = chol16(pk_blk(T, 0, 0), PK_LD, rd, col);
    if (tid == 0) *flag = f;
  }
  __syncthreads();
  int fail = __builtin_amdgcn_readfirstlane(*flag);
  if (fail) return fail;
  for (int p = 0; p < P; ++p) {
    // panel: row R of the blocks below the diagonal block solves x L_pp^T = a
    const int rows = 16 * (P - 1 - p);
    if (tid < rows) {
      const int R = 16 * (p + 1) + tid;
      const double* Lpp = pk_blk(T, p, p);
      double* a = pk_blk(T, R >> 4, p) + (R & 15);
      double x[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        double s = a[PK_LD * c];
#pragma unroll
        for (int m = 0; m < c; ++m) s = fma(-x[m], Lpp[c + PK_LD * m], s);
        x[c] = s * rd[16 * p + c];
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) a[PK_LD * c] = x[c];
    }
    __syncthreads();
    if (p + 1 == P) break;
    const int nb = P - 1 - p;
    if (w == 0) {
      double* Cnn = pk_blk(T, p + 1, p + 1);
      const double* Lnp = pk_blk(T, p + 1, p);
      d4 acc = -blk_load(Cnn, PK_LD);
      acc = blk_mma16(acc, Lnp, PK_LD, Lnp, PK_LD, true);
      blk_store(Cnn, PK_LD, -acc);
      const int f = chol16(Cnn, PK_LD, rd + 16 * (p + 1), col);
      if (tid == 0) *flag = f ? 16 * (p + 1) + f : 0;
    } else {
      // waves 1-3: the blocks below the diagonal in column p+1 (the next
      // panel) take all their updates m = 0..p now, as one chain, and the
      // later diagonal blocks take the update of panel p
      for (int u = w - 1; u < nb - 1; u += 3) {
        const int bi = p + 2 + u;
        double* Cij = pk_blk(T, bi, p + 1);
        d4 acc = -blk_load(Cij, PK_LD);
        for (int m = 0; m <= p; ++m)
          acc = blk_mma16(acc, pk_blk(T, bi, m), PK_LD, pk_blk(T, p + 1, m), PK_LD, true);
        blk_store(Cij, PK_LD, -acc);
        double* Cjj = pk_blk(T, bi, bi);
        d4 acd = -blk_load(Cjj, PK_LD);
        acd = blk_mma16(acd, pk_blk(T, bi, p), PK_LD, pk_blk(T, bi, p), PK_LD, true);
        blk_store(Cjj, PK_LD, -acd);
      }
    }
    __syncthreads();
    fail = __builtin_amdgcn_readfirstlane(*flag);
    if (fail) return fail;
  }
  return 0;
}

// acc += A_blk * op(B)_blk as blk_mma16, with A_blk held in registers in
// the accumulator layout (lane l, register r: row l%16, column l/16 + 4r),
// which is the layout in which each MFMA step takes its A operand: the
// result of one block product feeds the next without a trip through LDS.
__device__ __forceinline__ d4 blk_mma16_areg(d4 acc, const d4& A, const double* B, int ldb,
                                             bool tb) {
  const int lane = opaque_tid() & 63, lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int k = 4 * kk + lk;
    const double b = tb ? B[lr + ldb * k] : B[k + ldb * lr];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(b, A[kk], acc, 0, 0, 0);
  }
  return acc;
}

// One level of the recursive inverse: the groups of S diagonal blocks
// starting at 2 S g are joined pairwise.  With L = [L11 0; L21 L22] over a
// pair and X11 = L11^{-1}, X22 = L22^{-1} already formed, the off-diagonal
// part of the inverse is X21 = -(X22 L21) X11.  Phase A forms
// W = X22 L21 in place of L21, wave w taking one block column of one pair
// (every column costs S(S+1)/2 block products); phase B forms -W X11 in
// place of W, wave w taking one block row (the same count).  A pair whose
// second group starts at or past P is skipped: its L21 is zero (padding),
// so is its X21.
template <int S>
__device__ __forceinline__ void inverse_level(double* T, int P) {
  const int w = opaque_tid() >> 6, g = w / S, u = w % S;
  const int b1 = 2 * S * g, b2 = b1 + S;   // first blocks of the two groups
  const bool live = b2 < P;
  d4 acc[S];
  if (live) {                              // column u of W
#pragma unroll
    for (int i = 0; i < S; ++i) {
      acc[i] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k = 0; k <= i; ++k)
        acc[i] = blk_mma16(acc[i], pk_blk(T, b2 + i, b2 + k), PK_LD, pk_blk(T, b2 + k, b1 + u),
                           PK_LD, false);
    }
#pragma unroll
    for (int i = 0; i < S; ++i) blk_store(pk_blk(T, b2 + i, b1 + u), PK_LD, acc[i]);
  }
  __syncthreads();
  if (live) {                              // row u of X21
#pragma unroll
    for (int j = 0; j < S; ++j) {
      acc[j] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k = j; k < S; ++k)
        acc[j] = blk_mma16(acc[j], pk_blk(T, b2 + u, b1 + k), PK_LD, pk_blk(T, b1 + k, b1 + j),
                           PK_LD, false);
    }
#pragma unroll
    for (int j = 0; j < S; ++j) blk_store(pk_blk(T, b2 + u, b1 + j), PK_LD, -acc[j]);
  }
  __syncthreads();
}

// X = L^{-1} in place on the packed factor (its first P blocks of 16).
// First X_pp = L_pp^{-1} for every diagonal block (16 lanes per block, one
// column per lane, by forward substitution with the reciprocal pivots rd).
// Then recursive doubling: pairs of single blocks (wave w joins blocks 2w
// and 2w + 1, the product X22 L21 passed to the second product in
// registers), then pairs of 2-block groups and the pair of 4-block groups
// (inverse_level).  Blocks past P are the identity with zero cross blocks
// and stay so.
__device__ __forceinline__ void inverse_packed(double* T, const double* rd, int P) {
  const int tid = opaque_tid(), w = tid >> 6;
  {
    const int g = tid >> 4, c = tid & 15;
    double x[16];
    if (g < P) {
      const double* Lb = pk_blk(T, g, g);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        double s = (r == c) ? 1.0 : 0.0;
#pragma unroll
        for (int m = 0; m < r; ++m) s = fma(-Lb[r + PK_LD * m], x[m], s);
        x[r] = s * rd[16 * g + r];
      }
    }
    __syncthreads();
    if (g < P) {
      double* Xb = pk_blk(T, g, g);
#pragma unroll
      for (int r = 0; r < 16; ++r) Xb[r + PK_LD * c] = x[r];
    }
    __syncthreads();
  }
  {
    const int a = 2 * w;
    if (a + 1 < P) {
      d4 y = blk_mma16(d4{0.0, 0.0, 0.0, 0.0}, pk_blk(T, a + 1, a + 1), PK_LD,
                       pk_blk(T, a + 1, a), PK_LD, false);
      d4 x = blk_mma16_areg(d4{0.0, 0.0, 0.0, 0.0}, y, pk_blk(T, a, a), PK_LD, false);
      blk_store(pk_blk(T, a + 1, a), PK_LD, -x);
    }
    __syncthreads();
  }
  inverse_level<2>(T, P);
  inverse_level<4>(T, P);
}

// The lower 16 x 16 blocks of a tile (rIn) into the packed layout T; entries
// above the diagonal of the diagonal blocks read as zero.  16 x 16 blocks as
// 128 pairs of rows: all 18 pairs of a thread are issued before the first
// LDS write, so that their latencies overlap (a wave stays inside one block).
__device__ __forceinline__ void load_packed_tile(rsrc_t rIn, double* T) {
  const int tid = opaque_tid();
  constexpr int NLD = PK_BLOCKS * 128 / NTHREADS;
  d2 v[NLD];
#pragma unroll
  for (int u = 0; u < NLD; ++u) {
    const int b = (NTHREADS * u + tid) >> 7;  // per lane: keeps the caller's scalar registers free
    const int bi = pk_row(b);
    const int bj = b - bi * (bi + 1) / 2;
    const int e = 2 * (tid & 127);
    v[u] = ld2(rIn, (16 * bi + (e & 15)) + NB * (16 * bj + (e >> 4)));
  }
#pragma unroll
  for (int u = 0; u < NLD; ++u) {
    const int b = (NTHREADS * u + tid) >> 7;  // per lane: keeps the caller's scalar registers free
    const int bi = pk_row(b);
    const bool diag = b == bi * (bi + 1) / 2 + bi;
    const int e = 2 * (tid & 127), lr = e & 15, lc = e >> 4;
    double* dst = T + PK_STRIDE * b + lr + PK_LD * lc;
    dst[0] = (diag && lr < lc) ? 0.0 : v[u].x;
    dst[1] = (diag && lr + 1 < lc) ? 0.0 : v[u].y;
  }
}

// The packed lower triangle T as a full tile X (explicit zeros above the
// diagonal) and, with both, as X^T too, in contiguous 16-byte stores.  Lane
// l of wave w stores rows 2(l%64), 2(l%64) + 1 of columns w, w + 4, ...:
// the row's block and offset are fixed per lane and the column's per wave,
// so each element costs one LDS read and a select.
__device__ __forceinline__ void store_packed(const double* T, rsrc_t rX, rsrc_t rXT, bool both) {
  const int tid = opaque_tid(), w = tid >> 6;
  const int rr = 2 * (tid & 63), rb = rr >> 4, rl = rr & 15, rtri = rb * (rb + 1) / 2;
#pragma unroll 4
  for (int q = 0; q < NB * NB / 2 / NTHREADS; ++q) {
    const int cc = w + 4 * q, cb = cc >> 4, cl = cc & 15, e = rr + NB * cc;
    const double* x = T + PK_STRIDE * (rtri + cb) + rl + PK_LD * cl;  // X(rr, cc)
    st2(rX, e, d2{rr >= cc ? x[0] : 0.0, rr + 1 >= cc ? x[1] : 0.0});
    if (both) {
      // X(cc, rr): block (cb, rb), in bounds even above the diagonal
      const double* y = T + PK_STRIDE * (cb * (cb + 1) / 2 + rb) + cl + PK_LD * rl;
      st2(rXT, e, d2{cc >= rr ? y[0] : 0.0, cc >= rr + 1 ? y[PK_LD] : 0.0});
    }
  }
}

// Outputs: the factor (Lout, may be null: not stored), its transpose (LcopyT,
// may be null), the inverse of the factor (Xout) and its transpose (XoutT,
// may be null), each with explicit zeros in the other triangle.  Only the first P blocks of
// 16 are factored and inverted: past them the tile must be an identity block
// with zero cross blocks (the padding of a ragged order), whose factor and
// inverse are the identity.  Returns 0, or the 1-based local index of the
// first pivot that is not positive (or NaN); on failure nothing is stored.
__device__ __attribute__((noinline)) int potrf_inv_tile(const double* Ain, double* Lout,
                                                         double* LcopyT, double* Xout,
                                                         double* XoutT, double* smem, int P) {
  P = uniform_int(P);
  Ain = uniform_ptr(Ain);
  Lout = uniform_ptr(Lout);
  LcopyT = uniform_ptr(LcopyT);
  Xout = uniform_ptr(Xout);
  XoutT = uniform_ptr(XoutT);
  double* T = smem;                          // the 36 packed blocks
  double* rd = smem + PK_BLOCKS * PK_STRIDE;  // reciprocal pivots
  int* flag = reinterpret_cast<int*>(rd + NB);
  const rsrc_t rIn = tile_rsrc(Ain), rL = tile_rsrc(Lout ? Lout : Xout), rX = tile_rsrc(Xout),
               rXT = tile_rsrc(XoutT);

  load_packed_tile(rIn, T);
  __syncthreads();

  const int ff = factor_packed(T, rd, rd + NB + 8, flag, P);
  if (ff) return ff;

  // the factor and its transpose; skipped when nothing reads them
  if (Lout) store_packed(T, rL, tile_rsrc(LcopyT ? LcopyT : Xout), LcopyT != nullptr);
  __syncthreads();  // the inverse overwrites the factor

  inverse_packed(T, rd, P);
  // the blocks past P (padding) still hold the identity block loaded with
  // the tile
  store_packed(T, rX, rXT, XoutT != nullptr);
  return 0;
}

// Diagonal tile of a given Cholesky factor (the inverse from a factor): X =
// L^{-1} and X^T from the lower triangle of Lin, by the steps of
// potrf_inv_tile without the factorization; the reciprocal pivots are 1/L_kk
// (a division).  Returns 0, or the 1-based local index of the first zero
// diagonal entry (the factor is singular; nothing is stored).
__device__ __attribute__((noinline)) int trtri_inv_tile(const double* Lin, double* Xout,
                                                        double* XoutT, double* smem) {
  Lin = uniform_ptr(Lin);
  Xout = uniform_ptr(Xout);
  XoutT = uniform_ptr(XoutT);
  double* T = smem;
  double* rd = smem + PK_BLOCKS * PK_STRIDE;
  int* flag = reinterpret_cast<int*>(rd + NB);
  const int tid = opaque_tid();
  if (tid == 0) *flag = INT_MAX;
  load_packed_tile(tile_rsrc(Lin), T);
  __syncthreads();
  if (tid < NB) {
    const double d = pk_blk(T, tid >> 4, tid >> 4)[(tid & 15) * (PK_LD + 1)];
    rd[tid] = 1.0 / d;
    if (d == 0.0) atomicMin(flag, tid + 1);
  }
  __syncthreads();
  const int f = __builtin_amdgcn_readfirstlane(*flag);
  if (f != INT_MAX) return f;
  inverse_packed(T, rd, NB / 16);
  store_packed(T, tile_rsrc(Xout), tile_rsrc(XoutT), true);
  return 0;
}

// dst <- src for one tile; loads are issued in batches of 16 independent
// 16-byte loads per thread so that their latencies overlap.
// dst += src (dst -= src with neg), elementwise over the tile, with
// agent-coherent accesses like every pool access of the scheduler.
__device__ __forceinline__ void tile_add(const double* src, double* dst, bool neg) {
  const rsrc_t rs = tile_rsrc(src), rd = tile_rsrc(dst);
#pragma unroll 4
  for (int q = 0; q < NB * NB / 2 / NTHREADS; ++q) {
    const int e = 2 * (threadIdx.x + NTHREADS * q);
    const d2 x = ld2(rs, e), y = ld2(rd, e);
    st2(rd, e, neg ? y - x : y + x);
  }
}

__device__ __forceinline__ void tile_copy(const double* src, double* dst) {
  const rsrc_t rs = tile_rsrc(src), rd = tile_rsrc(dst);
#pragma unroll
  for (int h = 0; h < (int)(TILE / 2) / (NTHREADS * 16); ++h) {
    d2 v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = ld2(rs, 2 * (h * NTHREADS * 16 + threadIdx.x + NTHREADS * u));
#pragma unroll
    for (int u = 0; u < 16; ++u) st2(rd, 2 * (h * NTHREADS * 16 + threadIdx.x + NTHREADS * u), v[u]);
  }
}


// ALLOW_R64 (the batched kernel): a product without a renaming copy whose
// output tile lies in the last tile row of a matrix with at most 64 valid
// rows there computes only rows 0-63, the four waves side by side.  The
// padded rows of such an output keep their values (zero, or the identity
// padding of the last diagonal tile): every operand row that reaches them
// is padding too.  Per output element the MFMA sequence is the same, so the
// result is bit-identical.
template <bool ALLOW_R64 = false>
__device__ __forceinline__ void run_task(const DevTask& t, const SchedArgs& g, double* smem, int T,
                                         int tiles) {
  double* P = g.pool;
  const int kind = t.kind & 0xff, f = (t.kind >> 8) & 0xff;  // see DevTask::kind
  double* out = t.out >= 0 ? tile_ptr(P, t.out) : nullptr;
  const double* a = t.a >= 0 ? tile_ptr(P, t.a) : nullptr;
  const double* b = t.b >= 0 ? tile_ptr(P, t.b) : nullptr;
  double* cp = t.copy >= 0 ? tile_ptr(P, t.copy) : nullptr;
  // a near-critical task issues ahead of the co-resident workgroup's waves
  // (one workgroup per matrix in the batched form: nothing to overtake)
  const bool urgent = !ALLOW_R64 && (t.kind & K_URGENT) != 0;
  if (urgent) __builtin_amdgcn_s_setprio(2);
  switch (kind) {
    case K_SYRK1: case K_GEMM1: case K_TRSM1: case K_TRMM2L: case K_GEMM2: case K_TRSM2R:
    case K_TRMM3: case K_LAUUM: case K_GEMM3: case K_SYRK3: case K_GEMMS: case K_TRSMS:
      // tile products; the planner chose operands and flags (Algorithm 1's
      // operation on the renamed or in-place tiles)
      if ((f & (F_TA | F_MA | F_MB)) == 0 && (f & F_TB)) {
        const int nl = (t.kind & K_LINKS_MASK) >> K_LINKS_SHIFT;
        const bool nca = !g.coherent_only && (t.kind & K_NC_A) != 0;
        const bool ncb = !g.coherent_only && (t.kind & K_NC_B) != 0;
        // k-panels of a product over the (possibly ragged) last tile block
        const int npan_last = (g.last_valid + SKC - 1) / SKC;
        const int npan = (t.kind & K_KLAST) ? npan_last : SNCH;
        const bool r64 = ALLOW_R64 && !cp && g.last_valid <= 64 && t.out >= T - tiles &&
                         t.out < T;
        if (nl) {
          if (r64)
            tile_mma_chain<true>(f, out, a, b, cp, smem, g.links + 2 * t.aux, nl, P, npan,
                                 npan_last);
          else
            tile_mma_chain(f, out, a, b, cp, smem, g.links + 2 * t.aux, nl, P, npan, npan_last);
        } else if (t.kind & K_PART) {  // one row part of a split product
          const int idx = (t.kind >> K_PART_SHIFT) & 3;
          if (t.kind & K_PARTS4)
            tile_mma<true, true, 32>(f, out, a, b, cp, smem, nca, ncb, npan, 32 * idx);
          else
            tile_mma<true, true>(f, out, a, b, cp, smem, nca, ncb, npan, 64 * idx);
        } else {
          if (r64) tile_mma<true, true>(f, out, a, b, cp, smem, nca, ncb, npan);
          else tile_mma<true>(f, out, a, b, cp, smem, nca, ncb, npan);
        }
      }
      else
        tile_mma_general(f, out, a, b, cp, smem);
      break;
    case K_POTRF: {
      double* X = tile_ptr(P, t.aux);
      double* Xt = tile_ptr(P, t.aux + tiles);
      const bool live = !(t.kind & K_POTRF_FACTOR_DEAD);
      // the last diagonal tile of a ragged order: its padded part is an exact
      // identity block (zero cross blocks), so only its first
      // ceil(last_valid / 16) blocks of 16 are factored and inverted
      const bool ragged = t.aux - g.d_base == tiles - 1;
      const int P16 = ragged ? (g.last_valid + 15) / 16 : NB / 16;
      // POTRF heads the step-1 critical path and is bound by the latency of
      // its dependent chains: its waves issue ahead of the co-resident
      // workgroup's product waves while it runs
      __builtin_amdgcn_s_setprio(3);
      const int fl = potrf_inv_tile(out, live ? out : nullptr, cp, X,
                                    (t.kind & K_POTRF_INVT_DEAD) ? nullptr : Xt, smem, P16);
      if (urgent) __builtin_amdgcn_s_setprio(2);
      else __builtin_amdgcn_s_setprio(0);
      if (fl && threadIdx.x == 0) {
        const int jt = t.aux - g.d_base;  // diagonal tile index
        atomicMin(&g.ctrl[CTRL_INFO], g.info_base + jt * NB + fl);
        __hip_atomic_store(&g.ctrl[CTRL_FAILED], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      break;
    }
    case K_TADD:    // tree reduction: A_ij (or a partial sum) += the partial sum a
      tile_add(a, out, (f & F_NEG) != 0);
      break;
    case K_TRTRI:   // A_jj <- D_j, and C_jj <- D_j^T (inverse made by POTRF(j))
      tile_copy(a, out);
      if (cp) tile_copy(b, cp);
      break;
    default:
      break;
  }
  if (urgent) __builtin_amdgcn_s_setprio(0);
}

}  // namespace
}  // namespace spdinv
