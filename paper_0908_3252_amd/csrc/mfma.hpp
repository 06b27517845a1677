// Matrix-core (MFMA) helpers for gfx950.
//
// The 16x16x4 forms compute C[16][16] += A[16][4] * B[4][16] per wavefront.
// Operand layout (lane l of 64):  A operand = A[l % 16][l / 16],
// B operand = B[l / 16][l % 16].  Accumulators (measured on gfx950):
//   FP32: register r of lane l holds C[4 * (l / 16) + r][l % 16]
//   FP64: register r of lane l holds C[(l / 16) + 4 * r][l % 16]
#pragma once
#include <hip/hip_runtime.h>

namespace recon {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mfma_f32_16x16x4(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4d mfma_f64_16x16x4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Row (within the 16x16 block) of accumulator register r of this lane.
__device__ __forceinline__ int mfma16_row(int lane, int r) { return 4 * (lane >> 4) + r; }
__device__ __forceinline__ int mfma16_row_f64(int lane, int r) { return (lane >> 4) + 4 * r; }
__device__ __forceinline__ int mfma16_col(int lane) { return lane & 15; }

}  // namespace recon
