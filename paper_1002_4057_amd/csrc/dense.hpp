// Internal interface of the dense kernels (dense.hip): packing of column-major
// matrices into square tile-major form, the chained tile product and
// unpacking.  Not part of the public header.
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace spdinv {

enum PackMode : int {
  PACK_SYM_LOWER = 0,  // symmetric matrix from the lower triangle
  PACK_SYM_AVG = 1     // (M + M^T) / 2 of a full matrix
};

// Square tile-major t x t tiles (tile (i, j) at i + t*j) from a column-major
// matrix of order n (zero beyond n).
hipError_t launch_pack(const double* src, int ld, int n, int t, int mode, double* dst,
                       hipStream_t s);

// C(i, j) = Cin(i, j) -+ sum_k A(i, k) B(j, k)^T (+- the identity on the
// first diag_n diagonal entries) for every tile (lower = 0) or the lower
// tiles (lower = 1); Cin may be null.
hipError_t launch_gemm_nt(const double* A, const double* B, double* C, int t, int lower, int neg,
                          hipStream_t s, const double* Cin = nullptr, int diag_n = 0);

// C(i) = Cin(i) -+ sum_k P(k) Q(i, k)^T for the t tiles of a tile column:
// P and C tile columns, Q square tile-major (the residual probes of the
// mixed form); Cin may be null.
hipError_t launch_gemm_thin(const double* P, const double* Q, double* C, int t, int neg,
                            hipStream_t s, const double* Cin = nullptr);

// The transposed tiles of an n x NB matrix of random signs (zero rows past n).
hipError_t launch_fill_probe(double* Vt, int t, int n, hipStream_t s);

// Column-major symmetric matrix (both triangles, or the lower one) from the
// lower tiles of src.
hipError_t launch_unpack_sym(const double* src, int t, int n, double* out, int ld, hipStream_t s,
                             int lower_only = 0);

// out[0] = sum of squares of the ntiles tiles of M (partial: ntiles doubles).
hipError_t launch_sumsq(const double* M, int ntiles, double* partial, double* out, hipStream_t s);

// Upper tiles (and the upper part of diagonal tiles) <- mirror of the lower.
hipError_t launch_mirror_lower(double* M, int t, hipStream_t s);

// Batched backward: grad_i = -X_i sym(G_i) X_i for every matrix of a batch in
// one persistent launch.  Tasks (m, code) with code = phase << 16 | i << 8 | j
// run in ticket order, phases in order: 0 packs tile (i, j) of X_m (from its
// lower triangle) and of S_m = sym(G_m); 1 forms W_m(i, j) = sum_k X(i, k)
// S(j, k)^T once every tile of m is packed; 2 forms the lower tile (i, j) of
// -W X once tile row i of W is complete; 3 writes output tile (i, j) of
// grad_m (column-major, both triangles) once its lower source tile is done.
// Per matrix (mat[m]: t, first workspace tile, first counter, 0): 4 t^2
// tiles (X, S, W, the gradient) and 1 + t + t^2 counters.
constexpr int BB_PHASE_SHIFT = 16;
struct BBackArgs {
  const int2* task;
  int ntask;
  const int4* mat;
  const int* n;
  const double* const* X;
  const int* ldx;
  const double* const* G;
  const int* ldg;
  double* const* gradA;
  const int* ldga;
  double* tiles;
  int32_t* cnt;    // counters of every matrix
  int32_t* ctrl;   // CTRL_WORDS: ticket, abort
  long long spin_limit;
};
hipError_t launch_bback(const BBackArgs& b, int ncnt, int grid, hipStream_t s);
int bback_blocks_per_cu();

}  // namespace spdinv
