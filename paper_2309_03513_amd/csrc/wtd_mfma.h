// Matrix-core (MFMA) helpers shared by the GEMM and the exchange contraction.
//
// v_mfma_{f32,f64}_16x16x4 (wave64): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16].  Accumulator register i of lane l holds
// D[4 (l / 16) + i][l % 16] for the f32 instruction and D[l / 16 + 4 i][l % 16]
// for the f64 one (checked against numpy by the GEMM unit test).
#pragma once
#include <hip/hip_runtime.h>

namespace wtd {

typedef double mfma_d4_t __attribute__((ext_vector_type(4)));
typedef float mfma_f4_t __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef mfma_d4_t acc_t;
  static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int i) { return (lane >> 4) + 4 * i; }
};
template <>
struct Mfma<float> {
  typedef mfma_f4_t acc_t;
  static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

}  // namespace wtd
