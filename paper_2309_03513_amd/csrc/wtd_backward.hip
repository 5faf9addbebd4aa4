// Kernels of the adjoint (backward) Liouville apply.
//
// E = Re sum conj(g) (L a).  Through the real-space occupied orbitals phi_w
// (the derivative of A^T (D + K1e - K1d) A with respect to the occupied
// orbitals in the paper's Eq. z-v-eq / SI Eq. Zvectoreq is this map with g = a):
//   gamma_w = c_K sum_b [ g~_bw F(drho_b) + a~_bw F(drho^g_b) ]
//             - alpha sum_v' phi_v' v_c * (M_wv' + M_v'w),   M_vv' = sum_b g~_bv a~_bv'
// with F = v_c * + f_xc.  The pair densities P_wv' = M_wv' + M_v'w are of the
// "orbital times trial" kind; they are formed per grid point on the matrix
// cores, Poisson-solved by the pair pipeline of the forward apply and never
// kept beyond one backward call.
#include "wtd_internal.h"
#include "wtd_mfma.h"

namespace wtd {

namespace {

template <typename T>
struct PTile {
  static constexpr int THREADS = 512;
  static constexpr int TP = sizeof(T) == 4 ? 16 : 8;  // points per workgroup
  static constexpr int PPW = TP / 8;                  // points per wave
  static constexpr int NE = 256 * TP;
  static __device__ __forceinline__ int at(int q, int p) {
    const int h = (q >> 4) + 17 * (q & 15);
    return q * TP + ((p + h) & (TP - 1));
  }
};

// X[b][K*16 + w] tile at q = 16 b_loc + w_loc (fields [b][nocc][nr])
template <typename T>
__device__ __forceinline__ void load_bw(T* s, const T* __restrict__ X, int K, int nb, int nocc,
                                        int64_t nr, int64_t r0) {
  typedef PTile<T> C;
  const int p = threadIdx.x % C::TP;
  const int g = threadIdx.x / C::TP;
  constexpr int G = C::THREADS / C::TP;
  const int64_t r = r0 + p;
  const bool rin = r < nr;
#pragma unroll
  for (int it = 0; it < 256 / G; ++it) {
    const int c = g + it * G;
    const int b = c >> 4, w = K * 16 + (c & 15);
    T val = T(0);
    if (rin && b < nb && w < nocc) val = X[((int64_t)b * nocc + w) * nr + r];
    s[C::at(c, p)] = val;
  }
}

// P[pair(w, v')] = sum_b (X[b][w] Y[b][v'] + Y[b][w] X[b][v']) for w in rows
// [A0, A0 + nA) and v' in [B0, B0 + nB) (diag: A0 == B0 and w <= v'), nb <= 16.
// Pair (w, v') is stored at local index i nA - i (i + 1) / 2 + j on the
// diagonal (i = w - A0 <= j = v' - B0) and i nB + j off it.
template <typename T>
__global__ void __launch_bounds__(512)
k_pair_density(int nb, int nocc, int64_t nr, int ntile, const T* __restrict__ X,
               const T* __restrict__ Y, int A0, int nA, int B0, int nB, int diag,
               T* __restrict__ P) {
  typedef PTile<T> C;
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T sXI[C::NE], sYI[C::NE], sXJ[C::NE], sYJ[C::NE];
  const int per = (ntile + 7) / 8;
  const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (tile >= ntile) return;
  const int64_t r0 = (int64_t)tile * C::TP;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lx = lane & 15, ly = lane >> 4;
  const int ntA = (nA + 15) / 16, ntB = (nB + 15) / 16;
  const int tA = A0 / 16, tB = B0 / 16;
  for (int I = 0; I < ntA; ++I) {
    __syncthreads();
    load_bw(sXI, X, tA + I, nb, nocc, nr, r0);
    load_bw(sYI, Y, tA + I, nb, nocc, nr, r0);
    for (int J = diag ? I : 0; J < ntB; ++J) {
      const bool same = diag && J == I;
      __syncthreads();
      if (!same) {
        load_bw(sXJ, X, tB + J, nb, nocc, nr, r0);
        load_bw(sYJ, Y, tB + J, nb, nocc, nr, r0);
      }
      __syncthreads();
      const T* xj = same ? sXI : sXJ;
      const T* yj = same ? sYI : sYJ;
      acc_t acc[C::PPW];
#pragma unroll
      for (int pp = 0; pp < C::PPW; ++pp) {
        const int p = wave * C::PPW + pp;
        acc[pp] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          // A[w][b] = X_I[b][w], B[b][v'] = Y_J[b][v']  (and Y_I, X_J)
          const int q = (4 * k + ly) * 16 + lx;
          acc[pp] = Mfma<T>::run(sXI[C::at(q, p)], yj[C::at(q, p)], acc[pp]);
          acc[pp] = Mfma<T>::run(sYI[C::at(q, p)], xj[C::at(q, p)], acc[pp]);
        }
      }
      // stage the 16x16 tile through LDS (sXJ is free now) and write rows of points
      __syncthreads();
#pragma unroll
      for (int pp = 0; pp < C::PPW; ++pp)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          sXJ[C::at(Mfma<T>::row(lane, e) * 16 + lx, wave * C::PPW + pp)] = acc[pp][e];
      __syncthreads();
      const int p = threadIdx.x % C::TP;
      const int g = threadIdx.x / C::TP;
      constexpr int G = C::THREADS / C::TP;
      const int64_t r = r0 + p;
      if (r < nr) {
#pragma unroll
        for (int it = 0; it < 256 / G; ++it) {
          const int c = g + it * G;
          const int i = I * 16 + (c >> 4), j = J * 16 + (c & 15);
          if (i >= nA || j >= nB || (diag && i > j)) continue;
          const int64_t idx = diag ? (int64_t)i * nA - (int64_t)i * (i + 1) / 2 + j
                                   : (int64_t)i * nB + j;
          P[idx * nr + r] = sXJ[C::at(c, p)];
        }
      }
    }
  }
}

// gamma[w] += c_K sum_b [ gt[b][w] (vh[b] + f drho[b]) + at[b][w] (vhg[b] + f drhog[b]) ]
template <typename T>
__global__ void k_gamma_k1e(int nb, int nocc, int64_t nr, T ck, const T* __restrict__ gt,
                            const T* __restrict__ at, const T* __restrict__ vh,
                            const T* __restrict__ drho, const T* __restrict__ vhg,
                            const T* __restrict__ drhog, const T* __restrict__ fxc,
                            T* __restrict__ gamma) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int w = blockIdx.y;
  if (r >= nr) return;
  const T f = fxc[r];
  T s = T(0);
  for (int b = 0; b < nb; ++b) {
    const int64_t o = ((int64_t)b * nocc + w) * nr + r;
    const T F = vh[(int64_t)b * nr + r] + f * drho[(int64_t)b * nr + r];
    const T Fg = vhg[(int64_t)b * nr + r] + f * drhog[(int64_t)b * nr + r];
    s += gt[o] * F + at[o] * Fg;
  }
  gamma[(int64_t)w * nr + r] += ck * s;
}

// Per plane-wave weights on [nf][npw][2]: mode 0: x /= w_m; mode 1: x *= w_m.
// The imaginary part at m = 0 is set to zero in both modes.
template <typename T>
__global__ void k_gamma_weights(T* __restrict__ x, int64_t nf, int npw, int mode) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf * npw) return;
  const int h = (int)(i % npw);
  T* e = x + 2 * i;
  if (h == 0) {
    e[1] = T(0);
    return;
  }
  const T w = mode ? T(2) : T(0.5);
  e[0] *= w;
  e[1] *= w;
}

}  // namespace

template <typename T>
void launch_pair_density(const Geometry& g, int nb, int nocc, const T* X, const T* Y, int A0,
                         int nA, int B0, int nB, bool diag, T* P, hipStream_t s) {
  WTD_REQUIRE(nb <= 16, WTD_ERR_SHAPE, "pair densities support at most 16 trials per call");
  WTD_REQUIRE(A0 % 16 == 0 && B0 % 16 == 0 && A0 + nA <= nocc && B0 + nB <= nocc &&
                  (!diag || (A0 == B0 && nA == nB)),
              WTD_ERR_SHAPE, "pair-density row blocks out of range");
  typedef PTile<T> C;
  const int64_t ntile64 = (g.nr + C::TP - 1) / C::TP;
  WTD_REQUIRE(ntile64 < (1ll << 30), WTD_ERR_SHAPE, "pair-density grid too large");
  const int ntile = (int)ntile64;
  const int per = (ntile + 7) / 8;
  hipLaunchKernelGGL(k_pair_density<T>, dim3(8 * per), dim3(C::THREADS), 0, s, nb, nocc, g.nr,
                     ntile, X, Y, A0, nA, B0, nB, diag ? 1 : 0, P);
  WTD_HIP(hipGetLastError());
}

template <typename T>
void launch_gamma_k1e(const Geometry& g, int nb, int nocc, T ck, const T* gt, const T* at,
                      const T* vh, const T* drho, const T* vhg, const T* drhog, const T* fxc,
                      T* gamma, hipStream_t s) {
  dim3 grid((unsigned)((g.nr + 255) / 256), nocc);
  hipLaunchKernelGGL(k_gamma_k1e<T>, grid, dim3(256), 0, s, nb, nocc, g.nr, ck, gt, at, vh, drho,
                     vhg, drhog, fxc, gamma);
  WTD_HIP(hipGetLastError());
}

template <typename T>
void launch_weights(T* x, int64_t nf, int npw, int mode, hipStream_t s) {
  const int64_t tot = nf * npw;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_gamma_weights<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, x,
                     nf, npw, mode);
  WTD_HIP(hipGetLastError());
}

#define WTD_BWD_INST(T)                                                                        \
  template void launch_pair_density<T>(const Geometry&, int, int, const T*, const T*, int, int, \
                                       int, int, bool, T*, hipStream_t);                       \
  template void launch_gamma_k1e<T>(const Geometry&, int, int, T, const T*, const T*, const T*, \
                                    const T*, const T*, const T*, const T*, T*, hipStream_t);  \
  template void launch_weights<T>(T*, int64_t, int, int, hipStream_t);

WTD_BWD_INST(float)
WTD_BWD_INST(double)

}  // namespace wtd
