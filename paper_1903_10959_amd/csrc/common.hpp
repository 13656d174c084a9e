// Shared device helpers for the gfx950 kernels (MFMA wrappers, vector types).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace chfsi {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// 16x16x4 MFMA tiles.  Lane l supplies A[i = l%16][k = l/16] and
// B[k = l/16][j = l%16].  Accumulator element r (0..3) of lane l holds
// D[acc_row(l/16, r)][l%16]: rows l/16 + 4r for FP64 (strided), rows
// 4(l/16) + r for FP32 and BF16 (contiguous) -- measured on gfx950.
__device__ __forceinline__ v4d mfma16x4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma16x4(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// 16x16x32 BF16 tile, FP32 accumulation.  Lane l supplies
// A[i = l%16][k = 8*(l/16) + t] and B[k = 8*(l/16) + t][j = l%16], t = 0..7.
__device__ __forceinline__ v4f mfma16x32bf(v8bf a, v8bf b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <typename T> __device__ __forceinline__ int acc_row(int kq, int r);
template <> __device__ __forceinline__ int acc_row<double>(int kq, int r) { return kq + 4 * r; }
template <> __device__ __forceinline__ int acc_row<float>(int kq, int r) { return 4 * kq + r; }

// Re-express an FP32 16x16 accumulator in the FP64 row layout: FP64 lane
// (g, j) element q holds row g + 4q, which the FP32 layout keeps in lane
// (q, j) element g -- a 4x4 transpose across the four 16-lane groups.
__device__ __forceinline__ v4d f32acc_to_f64_layout(v4f a, int lane) {
  const int g = lane >> 4, j = lane & 15;
  v4d out = {0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float v = __shfl(a[s], q * 16 + j, 64);
      if (g == s) out[q] = (double)v;
    }
  return out;
}

template <typename T> struct acc4;
template <> struct acc4<double> { typedef v4d type; };
template <> struct acc4<float> { typedef v4f type; };

}  // namespace chfsi
