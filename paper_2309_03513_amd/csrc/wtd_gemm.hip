// Dense GEMMs on the matrix cores (MFMA) for the projector onto the
// unoccupied manifold (P_c, defined after the paper's Eq. k2dterm) and the
// D term in the transition basis.
//
// C[m][n] = sum_k A[m*lda + k] * B(k, n), with B(k, n) = B[n*ldb + k]
// (B_KMAJOR) or B[k*ldb + n].  64x64 output tile per 256-thread workgroup,
// 16-deep K slices staged in LDS; each wave owns a 32x32 quadrant computed as
// 2x2 blocks of v_mfma_{f64,f32}_16x16x4.
//
// Operand layouts: see wtd_mfma.h.
#include "wtd_internal.h"
#include "wtd_mfma.h"

#include <algorithm>

namespace wtd {

namespace {

constexpr int BM = 64, BN = 64, BK = 16;

template <typename T, bool B_KMAJOR>
__global__ void __launch_bounds__(256)
k_gemm(int M, int N, int K, int kchunk, const T* __restrict__ A, int lda,
       const T* __restrict__ B, int ldb, T* __restrict__ C, int ldc, int64_t zstride) {
  __shared__ T As[BK][BM + 1];
  __shared__ T Bs[BK][BN + 1];
  typedef typename Mfma<T>::acc_t acc_t;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  acc_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  // split-K: slice z covers [kbeg, kend) and writes its own partial result
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);
  C += (int64_t)blockIdx.z * zstride;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    {  // A tile: row = tid / 4, four consecutive k
      const int row = tid >> 2, kq = (tid & 3) * 4;
      const int gm = m0 + row;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gk = k0 + kq + i;
        As[kq + i][row] = (gm < M && gk < kend) ? A[(int64_t)gm * lda + gk] : T(0);
      }
    }
    if (B_KMAJOR) {
      const int col = tid >> 2, kq = (tid & 3) * 4;
      const int gn = n0 + col;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gk = k0 + kq + i;
        Bs[kq + i][col] = (gn < N && gk < kend) ? B[(int64_t)gn * ldb + gk] : T(0);
      }
    } else {
      const int kk = tid >> 4, nq = (tid & 15) * 4;
      const int gk = k0 + kk;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gn = n0 + nq + i;
        Bs[kk][nq + i] = (gn < N && gk < kend) ? B[(int64_t)gk * ldb + gn] : T(0);
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
        for (int j = 0; j < 2; ++j) acc[i][j] = Mfma<T>::run(a[i], b[j], acc[i][j]);
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
        const int gm = m0 + wm * 32 + i * 16 + Mfma<T>::row(lane, e);
        if (gm < M && gn < N) C[(int64_t)gm * ldc + gn] = acc[i][j][e];
      }
    }
}

// C[m][n] = sum_z P[z][m][n] (fixed order: deterministic)
template <typename T>
__global__ void k_sum_splits(const T* __restrict__ P, int nz, int M, int N, T* __restrict__ C,
                             int ldc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * N) return;
  const int m = (int)(i / N), n = (int)(i % N);
  T acc = T(0);
  for (int z = 0; z < nz; ++z) acc += P[(int64_t)z * M * N + i];
  C[(int64_t)m * ldc + n] = acc;
}

}  // namespace

template <typename T, bool B_KMAJOR>
void launch_gemm(int M, int N, int K, const T* A, int lda, const T* B, int ldb, T* C, int ldc,
                 hipStream_t s, T* scratch, size_t scratch_elems) {
  if (M <= 0 || N <= 0) return;
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, 1);
  WTD_REQUIRE(grid.y < 65536, WTD_ERR_SHAPE, "GEMM M too large");
  // few output tiles and a long K: split K over up to 16 slices into scratch
  int nz = 1;
  const int tiles = (int)(grid.x * grid.y);
  if (scratch && tiles < 512 && K >= 8 * BK) {
    nz = std::min(16, std::max(1, 1024 / tiles));
    nz = std::min(nz, (K + 4 * BK - 1) / (4 * BK));
    while (nz > 1 && (size_t)nz * M * N > scratch_elems) --nz;
  }
  if (nz == 1) {
    hipLaunchKernelGGL((k_gemm<T, B_KMAJOR>), grid, dim3(256), 0, s, M, N, K, K, A, lda, B, ldb,
                       C, ldc, (int64_t)0);
  } else {
    const int kchunk = ((K + nz - 1) / nz + BK - 1) / BK * BK;
    nz = (K + kchunk - 1) / kchunk;
    grid.z = nz;
    hipLaunchKernelGGL((k_gemm<T, B_KMAJOR>), grid, dim3(256), 0, s, M, N, K, kchunk, A, lda, B,
                       ldb, scratch, N, (int64_t)M * N);
    const int64_t tot = (int64_t)M * N;
    hipLaunchKernelGGL(k_sum_splits<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                       scratch, nz, M, N, C, ldc);
  }
  WTD_HIP(hipGetLastError());
}

template void launch_gemm<double, true>(int, int, int, const double*, int, const double*, int,
                                        double*, int, hipStream_t, double*, size_t);
template void launch_gemm<double, false>(int, int, int, const double*, int, const double*, int,
                                         double*, int, hipStream_t, double*, size_t);
template void launch_gemm<float, true>(int, int, int, const float*, int, const float*, int,
                                       float*, int, hipStream_t, float*, size_t);
template void launch_gemm<float, false>(int, int, int, const float*, int, const float*, int,
                                        float*, int, hipStream_t, float*, size_t);

}  // namespace wtd
