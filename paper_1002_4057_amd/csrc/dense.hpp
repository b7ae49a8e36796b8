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

// Column-major symmetric matrix (both triangles, or the lower one) from the
// lower tiles of src.
hipError_t launch_unpack_sym(const double* src, int t, int n, double* out, int ld, hipStream_t s,
                             int lower_only = 0);

// out[0] = sum of squares of the ntiles tiles of M (partial: ntiles doubles).
hipError_t launch_sumsq(const double* M, int ntiles, double* partial, double* out, hipStream_t s);

// Upper tiles (and the upper part of diagonal tiles) <- mirror of the lower.
hipError_t launch_mirror_lower(double* M, int t, hipStream_t s);

}  // namespace spdinv
