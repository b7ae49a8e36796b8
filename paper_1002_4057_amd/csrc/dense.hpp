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

// C(i, j) = -+ sum_k A(i, k) B(j, k)^T for every tile (lower = 0) or the
// lower tiles (lower = 1).
hipError_t launch_gemm_nt(const double* A, const double* B, double* C, int t, int lower, int neg,
                          hipStream_t s);

// Column-major full symmetric matrix from the lower tiles of src.
hipError_t launch_unpack_sym(const double* src, int t, int n, double* out, int ld, hipStream_t s);

}  // namespace spdinv
