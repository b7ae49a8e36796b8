// A matrix of order n <= NB inverted by one workgroup entirely in LDS, in
// binary64: the batched form's task for its small matrices (FP64 and FP32
// storage).  Included after tile_tasks.hpp, whose packed diagonal-tile
// factorization and in-place inverse it runs.
#pragma once
#include "tile_tasks.hpp"

namespace spdinv {
namespace {

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

// Lower triangle of A (column-major, lda, 1 <= n <= NB, elements of type E:
// double or float) <- lower triangle of A^{-1} (and the strictly upper
// triangle <- its mirror when fill_upper).  Returns 0 or INFO (1-based index
// of the first non-positive pivot; A is then left unchanged).  The matrix,
// widened to binary64 and padded to 16 * ceil(n/16) with the identity, is
// held as the packed lower 16 x 16 blocks of the diagonal-tile task
// (factor_packed, then inverse_packed leave X = L^{-1} in place); then
// Y = X^T X, Y_IJ = sum_{K >= I} X_KI^T X_KJ for I >= J, is formed in
// registers (at most 9 blocks per wave) and written to A from there, rounded
// to E.
template <class E>
__device__ int small_inverse(E* A, int lda, int n, int fill_upper, double* smem) {
  double* T = smem;
  double* rd = smem + PK_BLOCKS * PK_STRIDE;
  int* flag = reinterpret_cast<int*>(rd + NB);
  const int tid = opaque_tid(), w = tid >> 6;
  const int P = (n + 15) >> 4;
  const int nblk = P * (P + 1) / 2;
  for (int e = tid; e < nblk * 256; e += NTHREADS) {
    const int b = e >> 8, lr = e & 15, lc = (e >> 4) & 15;
    const int I = pk_row(b);
    const int J = b - I * (I + 1) / 2;
    const int r = 16 * I + lr, c = 16 * J + lc;
    double v;
    if (r < n && c < n)
      v = (r >= c) ? (double)A[r + (size_t)lda * c] : 0.0;
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
      const int I = pk_row(q);
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
    const int I = pk_row(q);
    const int J = q - I * (I + 1) / 2;
    const int r = 16 * I + lr;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = 16 * J + lk + 4 * u;
      if (r < n && c <= r) {
        const E v = (E)y[s2][u];
        A[r + (size_t)lda * c] = v;
        if (fill_upper && r > c) A[c + (size_t)lda * r] = v;
      }
    }
  }
  return 0;
}

__device__ __forceinline__ void* read_ptr_uniform(void* const* p) {
  const unsigned long long u = (unsigned long long)(*p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
  return (void*)(((unsigned long long)hi << 32) | lo);
}

// The order, leading dimension and pointer of matrix m, as wave-uniform
// values, and whether they are valid for a matrix of the template of tile
// count t (t = 1: 0 <= n <= NB; t >= 2: ceil(n / NB) = t).
template <class E>
__device__ __forceinline__ bool batch_entry(const BSchedArgs& g, int m, int t, int* n, int* lda,
                                            E** A) {
  *n = __builtin_amdgcn_readfirstlane(g.n[m]);
  *lda = __builtin_amdgcn_readfirstlane(g.lda[m]);
  *A = static_cast<E*>(read_ptr_uniform(g.A + m));
  const bool order_ok = t <= 1 ? (*n >= 0 && *n <= NB) : ((*n + NB - 1) / NB == t);
  return order_ok && *lda >= (*n > 1 ? *n : 1) && (*n == 0 || *A != nullptr);
}

// Writes the INFO word of matrix m (thread 0).
__device__ __forceinline__ void batch_info(const BSchedArgs& g, int m, int info) {
  if (threadIdx.x == 0 && g.info) g.info[m] = info;
}

}  // namespace
}  // namespace spdinv
