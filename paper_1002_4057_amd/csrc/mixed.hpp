// Internal interface of the FP32 tile path of the mixed-precision form
// (mixed.hip).  Not part of the public header.
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace spdinv {

// Bytes of the FP32 tile pool for t tiles per side (pool layout as FP64).
size_t pool_bytes32(int t);

// Lower triangle of the FP64 column-major A -> FP32 lower tiles, identity
// padding beyond n.
hipError_t launch_copy_in32(const double* A, int lda, int n, int t, float* pool, hipStream_t s);

// Persistent scheduler over the renamed plan with FP32 tile tasks (bf16: the
// products take bfloat16 operands).
hipError_t launch_sched32(const SchedArgs& a, int grid, int per_cu, bool bf16, hipStream_t s);

// FP32 lower tiles -> square tile-major FP64 symmetric matrix (zero beyond n).
hipError_t launch_x0_to_sym64(const float* pool, int t, int n, double* X, hipStream_t s);

int sched32_blocks_per_cu();

// dst = src rounded to FP32 (count a multiple of 4).
hipError_t launch_round32(const double* src, float* dst, size_t count, hipStream_t s);

// C = Cin + A B^T on the lower tiles of square tile-major matrices (t x t
// tiles): FP32 operands and FP32 accumulation on the matrix cores, the sum
// with Cin in binary64 (the refinement's low-precision correction X R).
hipError_t launch_gemm_nt32_lower(const float* A, const float* B, const double* Cin, double* C,
                                  int t, hipStream_t s);

// FP32 storage (SPDINV_FP32): FP32 column-major lower triangle <-> FP32 tiles.
hipError_t launch_copy_in32f(const float* A, int lda, int n, int t, float* pool, hipStream_t s);
hipError_t launch_copy_out32f(const float* pool, int t, float* A, int lda, int n, int fill_upper,
                              hipStream_t s);

// The FP32 batched scheduler (bsched_loop.hpp with the FP32 tile tasks).
hipError_t launch_bsched32(const BSchedArgs& b, int grid, hipStream_t s);
int bsched32_blocks_per_cu();

}  // namespace spdinv
