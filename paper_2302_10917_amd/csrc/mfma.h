// MFMA tile wrappers shared by the factorisation kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace mhdg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// 16x16x4 MFMA tiles: lane l holds A[l%16][l/16] and B[l/16][l%16]; the
// accumulator element v of lane l is D[drow(l/16, v)][l%16] (row order
// measured on gfx950 for each instruction).
template <> struct Mfma<double> {
  typedef d4 acc;
  static __device__ __forceinline__ acc run(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int g, int v) { return g + 4 * v; }
};
template <> struct Mfma<float> {
  typedef f4 acc;
  static __device__ __forceinline__ acc run(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int g, int v) { return 4 * g + v; }
};

}  // namespace mhdg
