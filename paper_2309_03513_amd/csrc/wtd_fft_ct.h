// Compile-time-planned batched line FFTs in LDS (same Stockham scheme as
// lds_fft in wtd_fft.h, with every size known to the compiler).
//
// The radix plan of N is the greedy factorisation with radices 9, 8, 5, 4, 3, 2,
// applied odd radices first, then even ones, each group ascending: the first
// pass (p = 1) writes with a stride equal to its radix, and an odd stride keeps
// LDS bank conflicts low.
// Twiddles come from an LDS copy of the FP64-generated table
// tw[j] = exp(-2 pi i j / N), j < N: w and w^2 of each butterfly are read, the
// higher powers formed by complex products.
#pragma once
#include "wtd_fft.h"

namespace wtd {

constexpr int ct_pick(int n) {
  return (n % 9 == 0) ? 9 : (n % 8 == 0) ? 8 : (n % 5 == 0) ? 5 : (n % 4 == 0) ? 4
         : (n % 3 == 0) ? 3 : 2;
}

constexpr int ct_greedy_count(int n) {
  int np = 0;
  while (n > 1) {
    n /= ct_pick(n);
    ++np;
  }
  return np;
}

// radix of pass `pass`
constexpr int ct_radix(int n, int pass) {
  int r[16] = {};
  int np = 0;
  while (n > 1) {
    const int f = ct_pick(n);
    r[np++] = f;
    n /= f;
  }
  // order: odd radices before even ones, ascending within each group
  for (int i = 1; i < np; ++i)
    for (int j = i; j > 0; --j) {
      const int a = r[j - 1], b = r[j];
      const bool swap = ((a % 2 == 0) && (b % 2 == 1)) || ((a % 2 == b % 2) && a > b);
      if (!swap) break;
      r[j] = a;
      r[j - 1] = b;
    }
  return r[pass];
}

constexpr int ct_prod(int n, int pass) {
  int p = 1;
  for (int i = 0; i < pass; ++i) p *= ct_radix(n, i);
  return p;
}

constexpr bool ct_supported(int n) {
  int m = n;
  while (m % 2 == 0) m /= 2;
  while (m % 3 == 0) m /= 3;
  while (m % 5 == 0) m /= 5;
  return m == 1 && n >= 2;
}

template <int R, int S, typename T>
__device__ __forceinline__ void ct_dft(cplx<T>* v) {
  if constexpr (R == 2) dft2<S>(v);
  else if constexpr (R == 3) dft3<S>(v);
  else if constexpr (R == 4) dft4<S>(v);
  else if constexpr (R == 5) dft5<S>(v);
  else if constexpr (R == 9) dft9<S>(v);
  else dft8<S>(v);
}

// One Stockham pass and the rest of the plan.  NL lines of length N; element j
// of line l at buf[l * LS + j * ES]; NTHR threads; LF: consecutive threads take
// consecutive lines (use when LS == 1), otherwise consecutive butterflies.
template <int S, int N, int NL, int ES, int LS, int NTHR, bool LF, int PASS, typename T>
__device__ __forceinline__ void ct_pass(cplx<T>* buf, const cplx<T>* tw) {
  if constexpr (PASS < ct_greedy_count(N)) {
    constexpr int R = ct_radix(N, PASS);
    constexpr int P = ct_prod(N, PASS);
    constexpr int M = N / R;
    constexpr int TWS = N / (P * R);
    constexpr int B = NL * M;
    constexpr int UB = (B + NTHR - 1) / NTHR;
    const int tid = threadIdx.x;
    cplx<T> v[UB][R];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int b = tid + u * NTHR;
      if (B % NTHR == 0 || b < B) {
        const int line = LF ? b % NL : b / M;
        const int i = LF ? b / NL : b % M;
        const int k = i % P;
        cplx<T>* base = buf + line * LS;
        // twiddle powers w^t: w and w^2 from the table, the rest as products of
        // two lower powers (at most two roundings deep for radices up to 9),
        // which saves LDS reads in the passes after the first
        cplx<T> wp[R];
        if constexpr (P > 1) {
          wp[1] = tw[k * TWS];
          if constexpr (R > 2) wp[2] = tw[2 * k * TWS];
#pragma unroll
          for (int t = 3; t < R; ++t) wp[t] = cmul(wp[t / 2], wp[t - t / 2]);
        }
#pragma unroll
        for (int t = 0; t < R; ++t) {
          cplx<T> x = base[(i + t * M) * ES];
          if (P > 1 && t > 0) x = (S < 0) ? cmul(x, wp[t]) : cmulc(x, wp[t]);
          v[u][t] = x;
        }
        ct_dft<R, S>(v[u]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int b = tid + u * NTHR;
      if (B % NTHR == 0 || b < B) {
        const int line = LF ? b % NL : b / M;
        const int i = LF ? b / NL : b % M;
        const int k = i % P;
        const int j0 = (i - k) * R + k;
        cplx<T>* base = buf + line * LS;
#pragma unroll
        for (int q = 0; q < R; ++q) base[(j0 + q * P) * ES] = v[u][q];
      }
    }
    __syncthreads();
    ct_pass<S, N, NL, ES, LS, NTHR, LF, PASS + 1>(buf, tw);
  }
}

template <int S, int N, int NL, int ES, int LS, int NTHR, bool LF, typename T>
__device__ __forceinline__ void ct_fft(cplx<T>* buf, const cplx<T>* tw) {
  ct_pass<S, N, NL, ES, LS, NTHR, LF, 0>(buf, tw);
}

// The column passes of an N x N plane [k1][k2] restricted to the nl = 2 cut + 1
// columns k2 = 0..cut and N - cut..N - 1: consecutive threads take consecutive
// columns of that set; butterfly b is (column slot b mod nl, index b / nl),
// with the quotient from a float product that is exact here (b < 2^13,
// nl < 128: the fraction of (b + 1/2) / nl stays at least 1 / (2 nl) away
// from an integer, far beyond the product's rounding).
template <int S, int N, int NTHR, int PASS, typename T>
__device__ __forceinline__ void ct_pass_cols(cplx<T>* buf, const cplx<T>* tw, int nl, int cut,
                                             float inv_nl) {
  if constexpr (PASS < ct_greedy_count(N)) {
    constexpr int R = ct_radix(N, PASS);
    constexpr int P = ct_prod(N, PASS);
    constexpr int M = N / R;
    constexpr int TWS = N / (P * R);
    constexpr int UB = (N * M + NTHR - 1) / NTHR;
    static_assert(N * M < (1 << 13) && N < 128, "exact quotient by a float product");
    const int B = nl * M;
    const int tid = threadIdx.x;
    cplx<T> v[UB][R];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int b = tid + u * NTHR;
      if (b < B) {
        const int i = (int)(((float)b + 0.5f) * inv_nl);
        const int slot = b - i * nl;
        const int col = slot <= cut ? slot : slot + (N - nl);
        const int k = i % P;
        cplx<T>* base = buf + col;
        cplx<T> wp[R];
        if constexpr (P > 1) {
          wp[1] = tw[k * TWS];
          if constexpr (R > 2) wp[2] = tw[2 * k * TWS];
#pragma unroll
          for (int t = 3; t < R; ++t) wp[t] = cmul(wp[t / 2], wp[t - t / 2]);
        }
#pragma unroll
        for (int t = 0; t < R; ++t) {
          cplx<T> x = base[(i + t * M) * N];
          if (P > 1 && t > 0) x = (S < 0) ? cmul(x, wp[t]) : cmulc(x, wp[t]);
          v[u][t] = x;
        }
        ct_dft<R, S>(v[u]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int b = tid + u * NTHR;
      if (b < B) {
        const int i = (int)(((float)b + 0.5f) * inv_nl);
        const int slot = b - i * nl;
        const int col = slot <= cut ? slot : slot + (N - nl);
        const int k = i % P;
        const int j0 = (i - k) * R + k;
        cplx<T>* base = buf + col;
#pragma unroll
        for (int q = 0; q < R; ++q) base[(j0 + q * P) * N] = v[u][q];
      }
    }
    __syncthreads();
    ct_pass_cols<S, N, NTHR, PASS + 1>(buf, tw, nl, cut, inv_nl);
  }
}

// Column passes of an N x N plane: every column (cut < 0) or the 2 cut + 1 a
// stick set reaches.
template <int S, int N, int NTHR, typename T>
__device__ __forceinline__ void ct_fft_cols(cplx<T>* buf, const cplx<T>* tw, int cut) {
  if (cut < 0) {
    ct_fft<S, N, N, N, 1, NTHR, true>(buf, tw);
  } else {
    const int nl = 2 * cut + 1;
    ct_pass_cols<S, N, NTHR, 0>(buf, tw, nl, cut, 1.0f / (float)nl);
  }
}

}  // namespace wtd
