// FP32 and mixed-precision forms of the SPD inverse on gfx950 (MI355X): the
// renamed, pipelined tile DAG of Section 3 executed with FP32 tiles, chained
// tasks included.  Tile products run on the FP32 matrix cores
// (v_mfma_f32_16x16x4f32, FP32 accumulation) or, in the BF16 variant, on
// bfloat16 operands rounded from the FP32 tiles (v_mfma_f32_16x16x16_bf16,
// FP32 accumulation); the diagonal tiles are factored and inverted in
// binary64 (the packed LDS code of the FP64 path) and rounded back.  The FP32
// form stops there; in the mixed forms the result is the starting inverse X0
// that the Newton-Schulz refinement corrects (binary64 residuals in
// dense.hip; the corrections that another residual follows on the FP32
// matrix cores, gemm_nt32_lower_kernel below).  The batched FP32 form runs
// the same tasks per matrix (bsched_kernel32).
//
// FP32 tiles are NB x NB floats, column-major, contiguous (64 KiB), in the
// same pool layout as the FP64 path: A tiles, the transposed renaming copies
// B and C, the inverted diagonal factor tiles D_j and D_j^T.
#include <algorithm>

#include "bsched_loop.hpp"
#include "device.hpp"
#include "mfma_tile.hpp"
#include "mixed.hpp"
#include "sched_loop.hpp"
#include "small_inverse.hpp"
#include "tile_tasks.hpp"

namespace spdinv {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, rounded to nearest even (finite inputs)
__device__ __forceinline__ short bf16_rne(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// Panel row stride in floats.  Operand reads take 16 consecutive rows r of
// 4 consecutive k per wave: with a stride of 144 floats (144 mod 64 = 16
// banks) the four k rows fall on disjoint bank groups.
constexpr int LDS32 = NB + 16;
constexpr int PANEL32 = KC * LDS32;               // floats per operand panel
constexpr int Q32 = NB * KC / 4 / NTHREADS;       // 16-byte loads per thread per panel
constexpr size_t TILE_BYTES32 = TILE * sizeof(float);

__device__ __forceinline__ float* tile32(float* pool, int idx) { return pool + (size_t)idx * TILE; }

__device__ __forceinline__ rsrc_t rsrc32(const float* t) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(t), 0, (int)TILE_BYTES32, RSRC_WORD3);
}
__device__ __forceinline__ f4 ld4f(rsrc_t r, int elem) {
  return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, elem * 4, 0, CPOL_AGENT));
}
__device__ __forceinline__ float ld1f(rsrc_t r, int elem) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, elem * 4, 0, CPOL_AGENT));
}
__device__ __forceinline__ void st4f(rsrc_t r, int elem, f4 v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4v, v), r, elem * 4, 0, CPOL_AGENT);
}
__device__ __forceinline__ void st1f(rsrc_t r, int elem, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, elem * 4, 0, CPOL_AGENT);
}

// k-panel k0..k0+KC-1 of a tile read along stored columns (element (r, k) is
// X[r + NB*k]), staged in LDS as S[k * LDS32 + r].
__device__ __forceinline__ void panel_load32(rsrc_t X, int k0, f4 (&v)[Q32]) {
#pragma unroll
  for (int q = 0; q < Q32; ++q) v[q] = ld4f(X, NB * k0 + 4 * (threadIdx.x + NTHREADS * q));
}
__device__ __forceinline__ void panel_store32(float* S, const f4 (&v)[Q32]) {
#pragma unroll
  for (int q = 0; q < Q32; ++q) {
    const int e = 4 * (threadIdx.x + NTHREADS * q), rr = e & (NB - 1), kk = e >> 7;
    *reinterpret_cast<f4*>(S + kk * LDS32 + rr) = v[q];
  }
}

// Tile product C (+)= +-A B^T on the FP32 matrix cores (the renamed plan's
// only form: both operands read along stored columns), with the flags of the
// FP64 product: F_NEG, F_ACC, F_LOWER (the block above the diagonal is not
// stored), and the renaming copy (transposed with F_COPYT).  A chained task
// (nl further links) adds the products of the link pairs links[2(p-1)],
// links[2(p-1)+1] (tile indices into pool; the last-block mark is ignored:
// the FP32 forms run every k-panel) in order, the k-panels of all links
// forming one double-buffered stream; the accumulator stays in registers,
// and as a separate task's FP32 store and reload of C would be exact, every
// rounding is that of the separate tasks.
// v_mfma_f32_16x16x4f32(x, y, d): x[i][k] from lane i+16k, y[k][j] from lane
// j+16k, d[i][j] in register i%4 of lane j + 16*(i/4).  The operands are
// passed as (B block, A block), so lane l, register r holds output row l%16
// of column 4*(l/16) + r.
template <bool BF16>
__device__ __forceinline__ void tile_mma32(int f, float* C, const float* A, const float* B,
                                           float* copy, double* smem_d,
                                           const int32_t* links = nullptr, int nl = 0,
                                           float* pool = nullptr) {
  float* smem = reinterpret_cast<float*>(smem_d);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w & 1, wn = w >> 1, lr = lane & 15, lk = lane >> 4;
  const bool neg = (f & F_NEG) != 0, accum = (f & F_ACC) != 0, copy_t = (f & F_COPYT) != 0;
  const bool active = !((f & F_LOWER) && wm == 0 && wn == 1);
  const rsrc_t rA = rsrc32(A), rB = rsrc32(B), rC = rsrc32(C);
  auto off = [&](int i, int j, int r) {
    return (wm * 64 + i * 16 + lr) + NB * (wn * 64 + j * 16 + 4 * lk + r);
  };
  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float c = accum ? ld1f(rC, off(i, j, r)) : 0.0f;
        acc[i][j][r] = neg ? -c : c;  // start from -C: C - P is rounded as -(-C + P)
      }
  f4 va[Q32], vb[Q32];
  panel_load32(rA, 0, va);
  panel_load32(rB, 0, vb);
  panel_store32(smem, va);
  panel_store32(smem + PANEL32, vb);
  __syncthreads();
  // operand tiles of link l (0: A and B)
  auto link_rsrc = [&](int l, rsrc_t& ra, rsrc_t& rb) {
    if (l == 0) {
      ra = rA;
      rb = rB;
    } else {
      const int ia = __builtin_amdgcn_readfirstlane(links[2 * (l - 1)]) & ~LINK_KLAST;
      const int ib = __builtin_amdgcn_readfirstlane(links[2 * (l - 1) + 1]);
      ra = rsrc32(tile32(pool, ia));
      rb = rsrc32(tile32(pool, ib));
    }
  };
  const int npan = (1 + nl) * NCH;
#pragma unroll 1
  for (int c = 0; c < npan; ++c) {
    const float* As = smem + (c & 1) * 2 * PANEL32;
    const float* Bs = As + PANEL32;
    const bool more = c + 1 < npan;
    if (more) {
      const int l = (c + 1) / NCH, k0 = ((c + 1) - NCH * l) * KC;
      rsrc_t ra, rb;
      link_rsrc(l, ra, rb);
      panel_load32(ra, k0, va);
      panel_load32(rb, k0, vb);
    }
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (!BF16) {
#pragma unroll
      for (int ks = 0; ks < KC / 4; ++ks) {
        const float* Ar = As + (4 * ks + lk) * LDS32 + wm * 64 + lr;
        const float* Br = Bs + (4 * ks + lk) * LDS32 + wn * 64 + lr;
        float a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          a[i] = Ar[16 * i];
          b[i] = Br[16 * i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[j], a[i], acc[i][j], 0, 0, 0);
      }
    } else {
      // v_mfma_f32_16x16x16_bf16: x[i][k] and y[k][j] from lane i (or j) +
      // 16*(k/4), element k%4, accumulator layout as the FP32 instruction;
      // the operands are rounded to bfloat16 as they leave LDS
#pragma unroll
      for (int kq = 0; kq < KC / 16; ++kq) {
        s4 a[4], b[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float* Ar = As + (16 * kq + 4 * lk + e) * LDS32 + wm * 64 + lr;
          const float* Br = Bs + (16 * kq + 4 * lk + e) * LDS32 + wn * 64 + lr;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            a[i][e] = bf16_rne(Ar[16 * i]);
            b[i][e] = bf16_rne(Br[16 * i]);
          }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(b[j], a[i], acc[i][j], 0, 0, 0);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    if (more) {
      float* An = smem + ((c + 1) & 1) * 2 * PANEL32;
      panel_store32(An, va);
      panel_store32(An + PANEL32, vb);
    }
    __syncthreads();
  }
  if (active) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) st1f(rC, off(i, j, r), neg ? -acc[i][j][r] : acc[i][j][r]);
  }
  if (!copy) return;  // uniform
  // renaming copy, staged in LDS as R[col + RLD * row] and written with
  // contiguous 16-byte stores
  constexpr int RLD = NB + 1;
  float* R = smem;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wm * 64 + i * 16 + lr, col = wn * 64 + j * 16 + 4 * lk + r;
        R[col + RLD * row] = neg ? -acc[i][j][r] : acc[i][j][r];
      }
  __syncthreads();
  const rsrc_t rD = rsrc32(copy);
#pragma unroll 4
  for (int q = 0; q < NB * NB / 4 / NTHREADS; ++q) {
    const int e = 4 * (threadIdx.x + NTHREADS * q), rr = e & (NB - 1), cc = e >> 7;
    f4 v;  // copy element (rr + s, cc) is result(cc, rr + s) or result(rr + s, cc)
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = copy_t ? R[(rr + s) + RLD * cc] : R[cc + RLD * (rr + s)];
    st4f(rD, e, v);
  }
}

// Diagonal tile in binary64, in the packed layout of the FP64 path (only
// the 36 lower 16 x 16 blocks in LDS, 78 KB, so that two workgroups share a
// CU): the FP32 tile is widened (exactly) into LDS, factored and inverted
// by the FP64 path's packed code, and L, L^T, X = L^{-1} and X^T are rounded
// to FP32.  Returns 0 or the 1-based local index of the first non-positive
// pivot (nothing is stored then).
// The packed lower triangle T, rounded to FP32, as a full tile X (explicit
// zeros above the diagonal) and, with both, as X^T too, in 16-byte stores:
// lane l stores rows 4(l%32) .. 4(l%32) + 3 of columns l/32, l/32 + 8, ...,
// with its rows' block offsets computed once.
__device__ __forceinline__ void store_packed32(const double* T, rsrc_t rX, rsrc_t rXT, bool both) {
  const int tid = opaque_tid();
  const int rr = 4 * (tid & 31), rb = rr >> 4, rl = rr & 15, rtri = rb * (rb + 1) / 2;
#pragma unroll 2
  for (int q = 0; q < NB * NB / 4 / NTHREADS; ++q) {
    const int cc = (tid >> 5) + 8 * q, cb = cc >> 4, cl = cc & 15, e = rr + NB * cc;
    const double* x = T + PK_STRIDE * (rtri + cb) + rl + PK_LD * cl;  // X(rr + s, cc)
    f4 vx;
#pragma unroll
    for (int s = 0; s < 4; ++s) vx[s] = (float)(rr + s >= cc ? x[s] : 0.0);
    st4f(rX, e, vx);
    if (both) {
      // X(cc, rr + s): block (cb, rb), in bounds even above the diagonal
      const double* y = T + PK_STRIDE * (cb * (cb + 1) / 2 + rb) + cl + PK_LD * rl;
      f4 vy;
#pragma unroll
      for (int s = 0; s < 4; ++s) vy[s] = (float)(cc >= rr + s ? y[PK_LD * s] : 0.0);
      st4f(rXT, e, vy);
    }
  }
}

__device__ __attribute__((noinline)) int potrf_inv_tile32(const float* Ain, float* Lout,
                                                           float* LcopyT, float* Xout,
                                                           float* XoutT, double* smem) {
  Ain = uniform_ptr(Ain);
  Lout = uniform_ptr(Lout);
  LcopyT = uniform_ptr(LcopyT);
  Xout = uniform_ptr(Xout);
  XoutT = uniform_ptr(XoutT);
  double* T = smem;                          // the 36 packed blocks
  double* rd = smem + PK_BLOCKS * PK_STRIDE;  // reciprocal pivots
  int* flag = reinterpret_cast<int*>(rd + NB);
  const int tid = opaque_tid();
  const rsrc_t rIn = rsrc32(Ain), rL = rsrc32(Lout ? Lout : Xout), rX = rsrc32(Xout),
               rXT = rsrc32(XoutT);
  // the lower blocks: 64 16-byte loads per block (4 rows of one column
  // each), every wave inside one block; all loads of a thread are issued
  // before the first LDS write
  constexpr int NLD = PK_BLOCKS * 64 / NTHREADS;
  static_assert(PK_BLOCKS * 64 % NTHREADS == 0, "whole passes");
  f4 v[NLD];
#pragma unroll
  for (int u = 0; u < NLD; ++u) {
    const int b = (NTHREADS * u + tid) >> 6;  // per lane: keeps the caller's scalar registers free
    const int bi = pk_row(b);
    const int bj = b - bi * (bi + 1) / 2;
    const int e = tid & 63, lr = 4 * (e & 3), lc = e >> 2;
    v[u] = ld4f(rIn, (16 * bi + lr) + NB * (16 * bj + lc));
  }
#pragma unroll
  for (int u = 0; u < NLD; ++u) {
    const int b = (NTHREADS * u + tid) >> 6;  // per lane: keeps the caller's scalar registers free
    const int bi = pk_row(b);
    const bool diag = b == bi * (bi + 1) / 2 + bi;
    const int e = tid & 63, lr = 4 * (e & 3), lc = e >> 2;
    double* dst = T + PK_STRIDE * b + lr + PK_LD * lc;
#pragma unroll
    for (int s = 0; s < 4; ++s) dst[s] = (diag && lr + s < lc) ? 0.0 : (double)v[u][s];
  }
  __syncthreads();
  const int ff = factor_packed(T, rd, rd + NB + 8, flag, NB / 16);
  if (ff) return ff;
  // the factor and its transpose; skipped when nothing reads them
  if (Lout) store_packed32(T, rL, rsrc32(LcopyT ? LcopyT : Xout), LcopyT != nullptr);
  __syncthreads();  // the inverse overwrites the factor
  inverse_packed(T, rd, NB / 16);
  store_packed32(T, rX, rXT, true);
  return 0;
}

__device__ __forceinline__ void tile_copy32(const float* src, float* dst) {
  const rsrc_t rs = rsrc32(src), rd = rsrc32(dst);
#pragma unroll
  for (int h = 0; h < (int)(TILE / 4) / (NTHREADS * 16); ++h) {
    f4 v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = ld4f(rs, 4 * (h * NTHREADS * 16 + threadIdx.x + NTHREADS * u));
#pragma unroll
    for (int u = 0; u < 16; ++u) st4f(rd, 4 * (h * NTHREADS * 16 + threadIdx.x + NTHREADS * u), v[u]);
  }
}

template <bool BF16>
__device__ __forceinline__ void run_task32(const DevTask& t, const SchedArgs& g, double* smem,
                                           int T, int tiles) {
  float* P = reinterpret_cast<float*>(g.pool);
  const int kind = t.kind & 0xff, f = (t.kind >> 8) & 0xff;
  float* out = t.out >= 0 ? tile32(P, t.out) : nullptr;
  const float* a = t.a >= 0 ? tile32(P, t.a) : nullptr;
  const float* b = t.b >= 0 ? tile32(P, t.b) : nullptr;
  float* cp = t.copy >= 0 ? tile32(P, t.copy) : nullptr;
  switch (kind) {
    case K_SYRK1: case K_GEMM1: case K_TRSM1: case K_TRMM2L: case K_GEMM2: case K_TRSM2R:
    case K_TRMM3: case K_LAUUM: case K_GEMM3: case K_SYRK3:
      // renamed plan: A B^T products only, single or chained
      {
        const int nl = (t.kind & K_LINKS_MASK) >> K_LINKS_SHIFT;
        tile_mma32<BF16>(f, out, a, b, cp, smem, nl ? g.links + 2 * t.aux : nullptr, nl, P);
      }
      break;
    case K_POTRF: {
      float* X = tile32(P, t.aux);
      float* Xt = tile32(P, t.aux + tiles);
      const bool live = !(t.kind & K_POTRF_FACTOR_DEAD);
      const int fl = potrf_inv_tile32(out, live ? out : nullptr, cp, X, Xt, smem);
      if (fl && threadIdx.x == 0) {
        const int jt = t.aux - 3 * T;
        atomicMin(&g.ctrl[CTRL_INFO], g.info_base + jt * NB + fl);
        __hip_atomic_store(&g.ctrl[CTRL_FAILED], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      break;
    }
    case K_TRTRI:
      tile_copy32(a, out);
      if (cp) tile_copy32(b, cp);
      break;
    default:
      break;
  }
}

constexpr unsigned kSoloLdsPad32 = 8192;
static_assert(TASK_SMEM * 8 + kSoloLdsPad32 > 80 * 1024, "the pad must exclude a second workgroup");

// Two workgroups per CU: every task fits TASK_SMEM doubles of LDS and 256
// registers per lane.
template <bool BF16>
__global__ __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(2, 2)))
void sched_kernel32(SchedArgs g, int T, int tiles) {
  __shared__ double smem[TASK_SMEM];
  sched_loop(g, [&](const DevTask& t) { run_task32<BF16>(t, g, smem, T, tiles); });
}

__device__ __forceinline__ void tri_decode32(int x, int& ti, int& tj) {
  int i = (int)((sqrtf(8.0f * (float)x + 1.0f) - 1.0f) * 0.5f);
  while (i * (i + 1) / 2 > x) --i;
  while ((i + 1) * (i + 2) / 2 <= x) ++i;
  ti = i;
  tj = x - i * (i + 1) / 2;
}

// dst = src rounded to FP32 (round to nearest), 4 elements per thread and
// step; count4 = elements / 4.
__global__ __launch_bounds__(NTHREADS) void round32_kernel(const double* __restrict__ src,
                                                         float* __restrict__ dst, size_t count4) {
  const size_t stride = (size_t)gridDim.x * NTHREADS;
  for (size_t q = (size_t)blockIdx.x * NTHREADS + threadIdx.x; q < count4; q += stride) {
    const double2 a = reinterpret_cast<const double2*>(src)[2 * q];
    const double2 b = reinterpret_cast<const double2*>(src)[2 * q + 1];
    const f4 v = {(float)a.x, (float)a.y, (float)b.x, (float)b.y};
    reinterpret_cast<f4*>(dst)[q] = v;
  }
}

// C(i, j) = Cin(i, j) + sum_k A(i, k) B(j, k)^T for the lower tiles i >= j
// of square tile-major matrices (t x t tiles of NB x NB, tile (i, j) at
// i + t j, column-major): the products on the FP32 matrix cores from FP32
// operands with FP32 accumulation over the whole sum, added to Cin in
// binary64.  One output tile per workgroup (blockIdx.x = i (i + 1) / 2 + j);
// the k-panels of the t tile pairs stream through LDS double-buffered as in
// tile_mma32.  Cin and C are distinct.
__global__ __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(2, 2)))
void gemm_nt32_lower_kernel(const float* __restrict__ A, const float* __restrict__ B,
                            const double* __restrict__ Cin, double* __restrict__ C, int t) {
  __shared__ float smem[4 * PANEL32];
  int ti, tj;
  tri_decode32(blockIdx.x, ti, tj);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w & 1, wn = w >> 1, lr = lane & 15, lk = lane >> 4;
  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  f4 va[Q32], vb[Q32];
  auto load = [&](int p) {
    const int k = p / NCH, c = p - NCH * k;
    panel_load32(rsrc32(A + (size_t)(ti + t * k) * TILE), c * KC, va);
    panel_load32(rsrc32(B + (size_t)(tj + t * k) * TILE), c * KC, vb);
  };
  const int np = t * NCH;
  load(0);
  panel_store32(smem, va);
  panel_store32(smem + PANEL32, vb);
  __syncthreads();
#pragma unroll 1
  for (int p = 0; p < np; ++p) {
    const float* As = smem + (p & 1) * 2 * PANEL32;
    const float* Bs = As + PANEL32;
    const bool more = p + 1 < np;
    if (more) load(p + 1);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const float* Ar = As + (4 * ks + lk) * LDS32 + wm * 64 + lr;
      const float* Br = Bs + (4 * ks + lk) * LDS32 + wn * 64 + lr;
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = Ar[16 * i];
        b[i] = Br[16 * i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[j], a[i], acc[i][j], 0, 0, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (more) {
      float* Sn = smem + ((p + 1) & 1) * 2 * PANEL32;
      panel_store32(Sn, va);
      panel_store32(Sn + PANEL32, vb);
    }
    __syncthreads();
  }
  // lane l, register r of accumulator (i, j): row wm*64 + 16 i + l%16,
  // column wn*64 + 16 j + 4 (l/16) + r
  const size_t ct = (size_t)(ti + t * tj) * TILE;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const size_t e = ct + (wm * 64 + i * 16 + lr) + (size_t)NB * (wn * 64 + j * 16 + 4 * lk + r);
        C[e] = Cin[e] + (double)acc[i][j][r];
      }
}

// Lower triangle of the FP64 column-major A -> FP32 lower tiles (rounded to
// nearest), identity padding beyond n.
__global__ __launch_bounds__(NTHREADS) void copy_in32_kernel(const double* __restrict__ A, int lda,
                                                             int n, float* __restrict__ pool) {
  int ti, tj;
  tri_decode32(blockIdx.x, ti, tj);
  float* dst = pool + (size_t)blockIdx.x * TILE;
  for (int e = threadIdx.x; e < (int)TILE; e += NTHREADS) {
    const int r = e & (NB - 1), c = e >> 7;
    const int gr = ti * NB + r, gc = tj * NB + c;
    double v;
    if (gr < n && gc < n)
      v = (gr >= gc) ? A[gr + (size_t)lda * gc] : 0.0;
    else
      v = (gr == gc) ? 1.0 : 0.0;
    dst[e] = (float)v;
  }
}

// X0 (FP32 lower tiles of the pool) -> square tile-major FP64 symmetric X of
// t x t tiles (tile (i, j) at i + t*j), zero beyond n.
__global__ __launch_bounds__(NTHREADS) void x0_to_sym64_kernel(const float* __restrict__ pool, int t,
                                                               int n, double* __restrict__ X) {
  constexpr int SB = 32;
  __shared__ float L[SB][SB + 1];
  const int bi = blockIdx.x % t, bj = blockIdx.x / t;
  const int si = bi >= bj ? bi : bj, sj = bi >= bj ? bj : bi;
  const float* s = pool + (size_t)(si * (si + 1) / 2 + sj) * TILE;
  double* out = X + (size_t)blockIdx.x * TILE;
  const int tx = threadIdx.x & (SB - 1), ty = threadIdx.x / SB;
  for (int sb = 0; sb < (NB / SB) * (NB / SB); ++sb) {
    const int lr0 = (sb % (NB / SB)) * SB, lc0 = (sb / (NB / SB)) * SB;
#pragma unroll
    for (int q = 0; q < SB / 8; ++q) {
      const int j = ty + 8 * q;
      L[tx][j] = s[(lc0 + tx) + NB * (lr0 + j)];  // source element (lc0 + tx, lr0 + j)
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < SB / 8; ++q) {
      const int j = ty + 8 * q;
      const int lr = lr0 + tx, lc = lc0 + j;
      const int gr = bi * NB + lr, gc = bj * NB + lc;
      float v;
      if (bi > bj || (bi == bj && lr >= lc))
        v = s[lr + NB * lc];
      else
        v = L[j][tx];  // source element (lc, lr)
      out[lr + NB * lc] = (gr < n && gc < n) ? (double)v : 0.0;
    }
    __syncthreads();
  }
}

// FP32 storage (the SPDINV_FP32 mode): lower triangle of the FP32
// column-major A -> FP32 lower tiles, identity padding beyond n; and back.
__global__ __launch_bounds__(NTHREADS) void copy_in32f_kernel(const float* __restrict__ A, int lda,
                                                              int n, float* __restrict__ pool) {
  int ti, tj;
  tri_decode32(blockIdx.x, ti, tj);
  float* dst = pool + (size_t)blockIdx.x * TILE;
  for (int e = threadIdx.x; e < (int)TILE; e += NTHREADS) {
    const int r = e & (NB - 1), c = e >> 7;
    const int gr = ti * NB + r, gc = tj * NB + c;
    float v;
    if (gr < n && gc < n)
      v = (gr >= gc) ? A[gr + (size_t)lda * gc] : 0.0f;
    else
      v = (gr == gc) ? 1.0f : 0.0f;
    dst[e] = v;
  }
}

__global__ __launch_bounds__(NTHREADS) void copy_out32f_kernel(const float* __restrict__ pool,
                                                               float* __restrict__ A, int lda, int n,
                                                               int fill_upper) {
  int ti, tj;
  tri_decode32(blockIdx.x, ti, tj);
  const float* src = pool + (size_t)blockIdx.x * TILE;
  for (int e = threadIdx.x; e < (int)TILE; e += NTHREADS) {
    const int r = e & (NB - 1), c = e >> 7;
    const int gr = ti * NB + r, gc = tj * NB + c;
    if (gr < n && gc < n && gr >= gc) {
      const float v = src[e];
      A[gr + (size_t)lda * gc] = v;
      if (fill_upper && gr > gc) A[gc + (size_t)lda * gr] = v;
    }
  }
}

// ---- batched form in FP32 (bsched_loop.hpp): the FP32 tile tasks --------
// Copy-in of one matrix of the batch into its FP32 tiles (agent-coherent
// stores), and the copy-out.
__device__ void bcopy_in32(const float* A, int lda, int n, int t, float* pool) {
  const int T = t * (t + 1) / 2;
  for (int x = 0; x < T; ++x) {
    int ti = 0;
    while ((ti + 1) * (ti + 2) / 2 <= x) ++ti;
    const int tj = x - ti * (ti + 1) / 2;
    const rsrc_t rd = rsrc32(tile32(pool, x));
#pragma unroll 4
    for (int q = 0; q < NB * NB / 4 / NTHREADS; ++q) {
      const int e = 4 * (threadIdx.x + NTHREADS * q), rr = e & (NB - 1), cc = e >> 7;
      const int gc = tj * NB + cc;
      f4 v;
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const int r = ti * NB + rr + h;
        if (r < n && gc < n)
          v[h] = (r >= gc) ? A[r + (size_t)lda * gc] : 0.0f;
        else
          v[h] = (r == gc) ? 1.0f : 0.0f;
      }
      st4f(rd, e, v);
    }
  }
}

__device__ void bcopy_out32(float* pool, int t, float* A, int lda, int n, int fill_upper) {
  const int T = t * (t + 1) / 2;
  for (int x = 0; x < T; ++x) {
    int ti = 0;
    while ((ti + 1) * (ti + 2) / 2 <= x) ++ti;
    const int tj = x - ti * (ti + 1) / 2;
    const rsrc_t rs = rsrc32(tile32(pool, x));
#pragma unroll 4
    for (int q = 0; q < NB * NB / 4 / NTHREADS; ++q) {
      const int e = 4 * (threadIdx.x + NTHREADS * q), rr = e & (NB - 1), cc = e >> 7;
      const int gc = tj * NB + cc;
      const f4 v = ld4f(rs, e);
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const int r = ti * NB + rr + h;
        if (r < n && gc < n && r >= gc) {
          A[r + (size_t)lda * gc] = v[h];
          if (fill_upper && r > gc) A[gc + (size_t)lda * r] = v[h];
        }
      }
    }
  }
}

__device__ __forceinline__ int load_uniform32(int32_t* p) {
  return __builtin_amdgcn_readfirstlane(
      __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Two workgroups per CU, as the FP32 scheduler.
__global__ __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(2, 2)))
void bsched_kernel32(BSchedArgs g) {
  __shared__ double smem[TASK_SMEM];
  auto run = [&](const DevTask& d, int m, int t) __attribute__((always_inline)) {
    const int kind = d.kind & 0xff;
    int32_t* mc = g.mctrl + CTRL_WORDS * m;
    int n, lda;
    float* A;
    if (kind == K_BSMALL) {
      int info = -1;
      if (batch_entry(g, m, 1, &n, &lda, &A))
        info = n ? small_inverse<float>(A, lda, n, g.fill_upper, smem) : 0;
      batch_info(g, m, info);
      return;
    }
    // one workgroup per matrix: the workgroup's own pool, else the matrix's slot
    const size_t first = g.seq ? (size_t)blockIdx.x * (size_t)g.wg_pool_tiles
                               : (size_t)__builtin_amdgcn_readfirstlane(g.mat[m].z);
    float* pool = static_cast<float*>(g.pool) + first * TILE;
    if (kind == K_BCOPYIN) {
      if (batch_entry(g, m, t, &n, &lda, &A)) {
        bcopy_in32(A, lda, n, t, pool);
      } else if (threadIdx.x == 0) {
        __hip_atomic_store(&mc[CTRL_INFO], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&mc[CTRL_FAILED], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      return;
    }
    if (kind == K_BCOPYOUT) {
      if (load_uniform32(&mc[CTRL_FAILED])) {
        batch_info(g, m, load_uniform32(&mc[CTRL_INFO]));
        return;
      }
      batch_entry(g, m, t, &n, &lda, &A);
      bcopy_out32(pool, t, A, lda, n, g.fill_upper);
      batch_info(g, m, 0);
      return;
    }
    SchedArgs s{};
    s.pool = reinterpret_cast<double*>(pool);
    s.ctrl = mc;
    s.links = g.tlinks[t];  // the template's chained-product links
    s.info_base = 0;
    run_task32<false>(d, s, smem, t * (t + 1) / 2, t);
  };
  if (g.seq)
    bseq_loop(g, run);
  else
    bsched_loop(g, run);
}

}  // namespace

hipError_t launch_copy_in32f(const float* A, int lda, int n, int t, float* pool, hipStream_t s) {
  const int T = t * (t + 1) / 2;
  hipLaunchKernelGGL(copy_in32f_kernel, dim3(T), dim3(NTHREADS), 0, s, A, lda, n, pool);
  return hipGetLastError();
}

hipError_t launch_copy_out32f(const float* pool, int t, float* A, int lda, int n, int fill_upper,
                              hipStream_t s) {
  const int T = t * (t + 1) / 2;
  hipLaunchKernelGGL(copy_out32f_kernel, dim3(T), dim3(NTHREADS), 0, s, pool, A, lda, n,
                     fill_upper);
  return hipGetLastError();
}

hipError_t launch_bsched32(const BSchedArgs& b, int grid, hipStream_t s) {
  hipLaunchKernelGGL(bsched_kernel32, dim3(grid), dim3(NTHREADS), 0, s, b);
  return hipGetLastError();
}

int bsched32_blocks_per_cu() {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, bsched_kernel32, NTHREADS, 0) !=
      hipSuccess)
    return 1;
  return blocks > 0 ? blocks : 1;
}

size_t pool_bytes32(int t) { return (size_t)pool_tiles(t) * TILE_BYTES32; }

hipError_t launch_copy_in32(const double* A, int lda, int n, int t, float* pool, hipStream_t s) {
  const int T = t * (t + 1) / 2;
  hipLaunchKernelGGL(copy_in32_kernel, dim3(T), dim3(NTHREADS), 0, s, A, lda, n, pool);
  return hipGetLastError();
}

hipError_t launch_sched32(const SchedArgs& a, int grid, int per_cu, bool bf16, hipStream_t s) {
  // one workgroup per CU: unused dynamic LDS keeps a second one off the CU
  const unsigned pad = per_cu == 1 ? kSoloLdsPad32 : 0;
  if (bf16)
    hipLaunchKernelGGL(sched_kernel32<true>, dim3(grid), dim3(NTHREADS), pad, s, a, a.tiles_T,
                       a.tiles);
  else
    hipLaunchKernelGGL(sched_kernel32<false>, dim3(grid), dim3(NTHREADS), pad, s, a, a.tiles_T,
                       a.tiles);
  return hipGetLastError();
}

hipError_t launch_round32(const double* src, float* dst, size_t count, hipStream_t s) {
  if (count % 4) return hipErrorInvalidValue;
  const size_t q = count / 4;
  const size_t blocks = std::min<size_t>((q + NTHREADS - 1) / NTHREADS, 8192);
  if (!blocks) return hipSuccess;
  hipLaunchKernelGGL(round32_kernel, dim3((unsigned)blocks), dim3(NTHREADS), 0, s, src, dst, q);
  return hipGetLastError();
}

hipError_t launch_gemm_nt32_lower(const float* A, const float* B, const double* Cin, double* C,
                                  int t, hipStream_t s) {
  if (t < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gemm_nt32_lower_kernel, dim3(t * (t + 1) / 2), dim3(NTHREADS), 0, s, A, B,
                     Cin, C, t);
  return hipGetLastError();
}

hipError_t launch_x0_to_sym64(const float* pool, int t, int n, double* X, hipStream_t s) {
  hipLaunchKernelGGL(x0_to_sym64_kernel, dim3(t * t), dim3(NTHREADS), 0, s, pool, t, n, X);
  return hipGetLastError();
}

int sched32_blocks_per_cu() {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, sched_kernel32<false>, NTHREADS, 0) !=
      hipSuccess)
    return 1;
  return blocks > 0 ? blocks : 1;
}

}  // namespace spdinv
