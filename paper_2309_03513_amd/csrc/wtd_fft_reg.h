// In-register FFTs: the values of one line are held by one thread (fft_reg)
// or by a quad of lanes that exchange values by DPP (fft_quad_*), and every
// index, permutation and twiddle factor is fixed at compile time, so the values
// never leave registers.  Used by the plane kernels of grids whose complex
// plane does not fit in LDS (FP64 108 x 108).
//
// fft_reg<N, S> is a recursive mixed-radix Cooley-Tukey transform (decimation
// in time): N = R M, the R sub-sequences x[r + R m] are transformed
// recursively, multiplied by w^(r k) with w = exp(S 2 pi i / N), and combined
// by R-point DFTs: X[k + M q] = sum_r w_R^(r q) w^(r k) Y_r[k].  S = -1 is the
// forward, S = +1 the inverse (unnormalised) transform; input and output are in
// natural order.  Twiddles are cos and sin of 2 pi j / N evaluated in double
// at compile time (below) and rounded to the working precision.
#pragma once
#include <type_traits>
#include <utility>

#include "wtd_fft.h"

namespace wtd {

namespace regfft {

constexpr double kTwoPi = 6.28318530717958647692528676655900577;

// sin and cos of x in [0, pi/4] by their Taylor series (terms below 1e-22)
constexpr double taylor_sin(double x) {
  double t = x, s = x;
  for (int k = 1; k < 14; ++k) {
    t *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    s += t;
  }
  return s;
}
constexpr double taylor_cos(double x) {
  double t = 1.0, s = 1.0;
  for (int k = 1; k < 14; ++k) {
    t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    s += t;
  }
  return s;
}

// cos(2 pi j / n) and sin(2 pi j / n): the turn fraction is reduced to
// [0, 1/8] by the half-, quarter- and eighth-turn symmetries
struct CS {
  double c, s;
};
constexpr CS turn(int j, int n) {
  j = ((j % n) + n) % n;
  double f = (double)j / (double)n;
  double sc = 1.0, ss = 1.0;
  if (f >= 0.5) {  // rotation by pi
    f -= 0.5;
    sc = -1.0;
    ss = -1.0;
  }
  // now angle a = 2 pi f in [0, pi)
  if (f >= 0.25) {  // a = pi/2 + b: cos a = -sin b, sin a = cos b
    const double g = f - 0.25;
    const double cb = (g <= 0.125) ? taylor_cos(kTwoPi * g) : taylor_sin(kTwoPi * (0.25 - g));
    const double sb = (g <= 0.125) ? taylor_sin(kTwoPi * g) : taylor_cos(kTwoPi * (0.25 - g));
    return {-sb * sc, cb * ss};
  }
  const double c = (f <= 0.125) ? taylor_cos(kTwoPi * f) : taylor_sin(kTwoPi * (0.25 - f));
  const double s = (f <= 0.125) ? taylor_sin(kTwoPi * f) : taylor_cos(kTwoPi * (0.25 - f));
  return {c * sc, s * ss};
}

// radix taken first for a line of length n (the sub-lines are n / radix)
constexpr int first_radix(int n) {
  return (n % 8 == 0 && n != 16) ? 8 : (n % 9 == 0) ? 9 : (n % 4 == 0) ? 4 : (n % 5 == 0) ? 5
         : (n % 3 == 0) ? 3 : 2;
}
constexpr bool is_codelet(int n) {
  return n == 2 || n == 3 || n == 4 || n == 5 || n == 8 || n == 9;
}

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

template <int R, int S, typename T>
__device__ __forceinline__ void codelet(cplx<T>* v) {
  if constexpr (R == 2) dft2<S>(v);
  else if constexpr (R == 3) dft3<S>(v);
  else if constexpr (R == 4) dft4<S>(v);
  else if constexpr (R == 5) dft5<S>(v);
  else if constexpr (R == 8) dft8<S>(v);
  else dft9<S>(v);
}

// z * exp(S 2 pi i j / n), with the multiples of a quarter turn done exactly
template <int J, int N, int S, typename T>
__device__ __forceinline__ cplx<T> twiddle(cplx<T> z) {
  constexpr int j = ((J % N) + N) % N;
  if constexpr (j == 0) {
    return z;
  } else if constexpr (2 * j == N) {
    return {-z.x, -z.y};
  } else if constexpr (4 * j == N) {
    return mul_si<S>(z);
  } else if constexpr (4 * j == 3 * N) {
    return mul_si<-S>(z);
  } else {
    constexpr CS w = turn(j, N);
    const T c = T(w.c), s = T(S * w.s);
    return {z.x * c - z.y * s, z.x * s + z.y * c};
  }
}

// z * w^(e K), w = exp(S 2 pi i / N), for a lane-dependent e < L: the factor is
// selected among compile-time constants (e = 0: exactly 1), then one product
template <int K, int N, int S, int L, typename T>
__device__ __forceinline__ cplx<T> twiddle_lane(cplx<T> z, int e) {
  constexpr CS w1 = turn(K, N);
  constexpr CS w2 = turn(2 * K, N);
  constexpr CS w3 = turn(3 * K, N);
  T c = T(1), s = T(0);
  if (e == 1) c = T(w1.c), s = T(S * w1.s);
  if (L > 2 && e == 2) c = T(w2.c), s = T(S * w2.s);
  if (L > 3 && e == 3) c = T(w3.c), s = T(S * w3.s);
  return {z.x * c - z.y * s, z.x * s + z.y * c};
}

}  // namespace regfft

template <int N, int S, typename T>
__device__ __forceinline__ void fft_reg(cplx<T> (&x)[N]) {
  using namespace regfft;
  if constexpr (N == 1) {
    return;
  } else if constexpr (is_codelet(N)) {
    codelet<N, S>(x);
  } else {
    constexpr int R = first_radix(N);
    constexpr int M = N / R;
    cplx<T> sub[R][M];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int m = 0; m < M; ++m) sub[r][m] = x[r + R * m];
#pragma unroll
    for (int r = 0; r < R; ++r) fft_reg<M, S>(sub[r]);
    static_for<0, M>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      cplx<T> y[R];
      static_for<0, R>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        y[r] = twiddle<r * k, N, S>(sub[r][k]);
      });
      codelet<R, S>(y);
#pragma unroll
      for (int q = 0; q < R; ++q) x[k + M * q] = y[q];
    });
  }
}

// ---------------------------------------------------------------------------
// A line of N = 4 M points held by a quad of lanes e = e0 + 2 e1 (the low two
// bits of the lane index); q(e) = 2 e0 + e1 is the block of the transformed
// line a lane holds.  The 4-point DFT across the quad is two radix-2 steps
// (lanes differing in e1, then in e0, for the forward; the reverse order for
// the inverse) with a quarter-turn twiddle on lane 3 between them.  All four
// lanes of a quad must be active.
__device__ __forceinline__ int quad_block(int e) { return ((e & 1) << 1) | (e >> 1); }

namespace regfft {

// value of the lane whose index differs in the bits of X (1 or 2), by DPP
// quad_perm [1, 0, 3, 2] or [2, 3, 0, 1]
template <int X>
__device__ __forceinline__ float lane_xor(float v) {
  constexpr int ctrl = X == 1 ? 0xB1 : 0x4E;
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), ctrl, 0xF, 0xF, false));
}
template <int X>
__device__ __forceinline__ double lane_xor(double v) {
  constexpr int ctrl = X == 1 ? 0xB1 : 0x4E;
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), ctrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), ctrl, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int X, typename T>
__device__ __forceinline__ cplx<T> lane_xor(cplx<T> z) {
  return {lane_xor<X>(z.x), lane_xor<X>(z.y)};
}

// radix-2 step between lanes differing in bit X: the lane with the bit clear
// keeps mine + other, the other lane other - mine (one fused multiply-add with
// a lane sign, exact for +-1)
template <int X, int M, typename T>
__device__ __forceinline__ void lane_butterfly(cplx<T> (&x)[M], bool hi) {
  const T sg = hi ? T(-1) : T(1);
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const cplx<T> o = lane_xor<X>(x[k]);
    x[k] = {fma(sg, x[k].x, o.x), fma(sg, x[k].y, o.y)};
  }
}

}  // namespace regfft


// The same quad, with the real-space side in contiguous blocks.  Forward:
// lane e holds x[e M + m] on entry and X[4 k + q(e)] on return (the 4-point
// DFT across the quad first, then the twiddles w^(m q), then the M-point
// transform).  Inverse: lane e holds X[4 k + q(e)] on entry and x[e M + m] on
// return (the same steps in reverse order).
template <int N, typename T>
__device__ __forceinline__ void fft_quad_fwd_contig(cplx<T> (&x)[N / 4], int e) {
  using namespace regfft;
  constexpr int M = N / 4;
  lane_butterfly<2>(x, (e & 2) != 0);
  if (e == 3) {
#pragma unroll
    for (int m = 0; m < M; ++m) x[m] = mul_si<-1>(x[m]);
  }
  lane_butterfly<1>(x, (e & 1) != 0);
  const int q = quad_block(e);
  static_for<0, M>([&](auto mc) {
    constexpr int m = decltype(mc)::value;
    x[m] = twiddle_lane<m, N, -1, 4>(x[m], q);
  });
  fft_reg<M, -1>(x);
}

template <int N, typename T>
__device__ __forceinline__ void fft_quad_inv_contig(cplx<T> (&x)[N / 4], int e) {
  using namespace regfft;
  constexpr int M = N / 4;
  fft_reg<M, +1>(x);
  const int q = quad_block(e);
  static_for<0, M>([&](auto mc) {
    constexpr int m = decltype(mc)::value;
    x[m] = twiddle_lane<m, N, +1, 4>(x[m], q);
  });
  lane_butterfly<1>(x, (e & 1) != 0);
  if (e == 3) {
#pragma unroll
    for (int m = 0; m < M; ++m) x[m] = mul_si<+1>(x[m]);
  }
  lane_butterfly<2>(x, (e & 2) != 0);
}

}  // namespace wtd
