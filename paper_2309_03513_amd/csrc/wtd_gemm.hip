// Dense GEMMs on the matrix cores (MFMA) for the projector onto the
// unoccupied manifold (P_c, defined after the paper's Eq. k2dterm) and the
// D term in the transition basis.
//
// C[m][n] = sum_k A[m*lda + k] * B(k, n), with B(k, n) = B[n*ldb + k]
// (B_KMAJOR) or B[k*ldb + n].  64x64 output tile per 256-thread workgroup,
// 16-deep K slices staged in LDS; each wave owns a 32x32 quadrant computed as
// 2x2 blocks of v_mfma_{f64,f32}_16x16x4.
//
// MFMA 16x16x4 operand layout (wave64): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16].  Accumulator register i of lane l holds
// D[4 (l / 16) + i][l % 16] for the f32 instruction and D[l / 16 + 4 i][l % 16]
// for the f64 one (checked against numpy by the GEMM unit test).
#include "wtd_internal.h"

namespace wtd {

namespace {

constexpr int BM = 64, BN = 64, BK = 16;

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename T>
struct Acc;
template <>
struct Acc<double> {
  typedef d4_t type;
  static __device__ __forceinline__ type mfma(double a, double b, type c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int i) { return (lane >> 4) + 4 * i; }
};
template <>
struct Acc<float> {
  typedef f4_t type;
  static __device__ __forceinline__ type mfma(float a, float b, type c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

template <typename T, bool B_KMAJOR>
__global__ void __launch_bounds__(256)
k_gemm(int M, int N, int K, const T* __restrict__ A, int lda, const T* __restrict__ B, int ldb,
       T* __restrict__ C, int ldc) {
  __shared__ T As[BK][BM + 1];
  __shared__ T Bs[BK][BN + 1];
  typedef typename Acc<T>::type acc_t;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  acc_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  for (int k0 = 0; k0 < K; k0 += BK) {
    {  // A tile: row = tid / 4, four consecutive k
      const int row = tid >> 2, kq = (tid & 3) * 4;
      const int gm = m0 + row;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gk = k0 + kq + i;
        As[kq + i][row] = (gm < M && gk < K) ? A[(int64_t)gm * lda + gk] : T(0);
      }
    }
    if (B_KMAJOR) {
      const int col = tid >> 2, kq = (tid & 3) * 4;
      const int gn = n0 + col;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gk = k0 + kq + i;
        Bs[kq + i][col] = (gn < N && gk < K) ? B[(int64_t)gn * ldb + gk] : T(0);
      }
    } else {
      const int kk = tid >> 4, nq = (tid & 15) * 4;
      const int gk = k0 + kk;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gn = n0 + nq + i;
        Bs[kk][nq + i] = (gn < N && gk < K) ? B[(int64_t)gk * ldb + gn] : T(0);
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kk + (lane >> 4)][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk + (lane >> 4)][wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = Acc<T>::mfma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int gn = n0 + wn * 32 + j * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gm = m0 + wm * 32 + i * 16 + Acc<T>::row(lane, e);
        if (gm < M && gn < N) C[(int64_t)gm * ldc + gn] = acc[i][j][e];
      }
    }
}

}  // namespace

template <typename T, bool B_KMAJOR>
void launch_gemm(int M, int N, int K, const T* A, int lda, const T* B, int ldb, T* C, int ldc,
                 hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM);
  WTD_REQUIRE(grid.y < 65536, WTD_ERR_SHAPE, "GEMM M too large");
  hipLaunchKernelGGL((k_gemm<T, B_KMAJOR>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C,
                     ldc);
  WTD_HIP(hipGetLastError());
}

template void launch_gemm<double, true>(int, int, int, const double*, int, const double*, int,
                                        double*, int, hipStream_t);
template void launch_gemm<double, false>(int, int, int, const double*, int, const double*, int,
                                         double*, int, hipStream_t);
template void launch_gemm<float, true>(int, int, int, const float*, int, const float*, int,
                                       float*, int, hipStream_t);
template void launch_gemm<float, false>(int, int, int, const float*, int, const float*, int,
                                        float*, int, hipStream_t);

}  // namespace wtd
