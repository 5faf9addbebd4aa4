// Device-side building blocks: complex arithmetic and batched 1D FFTs of
// lines held in LDS.
//
// The 3D transforms between reciprocal and direct space (the FFTs of the
// paper's Sec. 4) are split into a "stick" pass along i0 and a "plane" pass
// over (i1, i2); both stage their lines in LDS and call lds_fft below.
//
// lds_fft is a mixed-radix Stockham autosort transform (radices 2, 3, 4, 5, 8),
// done in place: in every pass each thread loads the inputs of its butterflies
// into registers, the workgroup synchronises, and the outputs are written back.
// For a pass of radix r after radices whose product is p (N = line length,
// M = N / r), butterfly i (k = i mod p) reads x_t = buf[i + t M] (t < r),
// multiplies x_t by w^(t k) with w = exp(s 2 pi i / (p r)), forms the r-point
// DFT y_q and writes y_q to buf[(i - k) r + k + q p].  s = -1 forward, +1
// inverse (unnormalised).  Twiddles come from an FP64-generated table of
// exp(-2 pi i j / N), j < N, stored in the working precision.
#pragma once
#include <hip/hip_runtime.h>

namespace wtd {

template <typename T>
struct cplx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by conj(b)
template <typename T>
__device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by s*i, s = +-1
template <int S, typename T>
__device__ __forceinline__ cplx<T> mul_si(cplx<T> a) {
  return S > 0 ? cplx<T>{-a.y, a.x} : cplx<T>{a.y, -a.x};
}

constexpr int kMaxPasses = 8;
constexpr int kMaxRadix = 8;

// Radix plan of one line length: passes in order, p = product of earlier radices.
struct FFTPlan {
  int n;
  int np;
  int rad[kMaxPasses];
  int p[kMaxPasses];
  // compile-time plane passes along this axis: transform only the lines
  // (columns k2) 0..cut and n2 - cut..n2 - 1, the ones a stick set reaches
  // (-1: every line)
  int cut;
};

// r-point DFTs with sign S on v[0..r-1] (in place).
template <int S, typename T>
__device__ __forceinline__ void dft2(cplx<T>* v) {
  cplx<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <int S, typename T>
__device__ __forceinline__ void dft3(cplx<T>* v) {
  // c = cos(2 pi/3) = -1/2, s = sin(2 pi/3) = sqrt(3)/2
  const T h = T(0.86602540378443864676372317075294);
  cplx<T> a = v[0], b = v[1], c = v[2];
  cplx<T> t = cadd(b, c);
  cplx<T> d = csub(b, c);
  cplx<T> m = {a.x - T(0.5) * t.x, a.y - T(0.5) * t.y};
  cplx<T> r = mul_si<S>(cscale(d, h));
  v[0] = cadd(a, t);
  v[1] = cadd(m, r);
  v[2] = csub(m, r);
}

template <int S, typename T>
__device__ __forceinline__ void dft4(cplx<T>* v) {
  cplx<T> a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
  cplx<T> b0 = cadd(v[1], v[3]), b1 = mul_si<S>(csub(v[1], v[3]));
  v[0] = cadd(a0, b0);
  v[2] = csub(a0, b0);
  v[1] = cadd(a1, b1);
  v[3] = csub(a1, b1);
}

template <int S, typename T>
__device__ __forceinline__ void dft5(cplx<T>* v) {
  // cos(2pi/5), cos(4pi/5), sin(2pi/5), sin(4pi/5)
  const T c1 = T(0.30901699437494742410229341718282);
  const T c2 = T(-0.80901699437494742410229341718282);
  const T s1 = T(0.95105651629515357211643933337938);
  const T s2 = T(0.58778525229247312916870595463907);
  cplx<T> x0 = v[0];
  cplx<T> p1 = cadd(v[1], v[4]), m1 = csub(v[1], v[4]);
  cplx<T> p2 = cadd(v[2], v[3]), m2 = csub(v[2], v[3]);
  cplx<T> a1 = {x0.x + c1 * p1.x + c2 * p2.x, x0.y + c1 * p1.y + c2 * p2.y};
  cplx<T> a2 = {x0.x + c2 * p1.x + c1 * p2.x, x0.y + c2 * p1.y + c1 * p2.y};
  cplx<T> b1 = mul_si<S>(cplx<T>{s1 * m1.x + s2 * m2.x, s1 * m1.y + s2 * m2.y});
  cplx<T> b2 = mul_si<S>(cplx<T>{s2 * m1.x - s1 * m2.x, s2 * m1.y - s1 * m2.y});
  v[0] = cadd(x0, cadd(p1, p2));
  v[1] = cadd(a1, b1);
  v[4] = csub(a1, b1);
  v[2] = cadd(a2, b2);
  v[3] = csub(a2, b2);
}

template <int S, typename T>
__device__ __forceinline__ void dft8(cplx<T>* v) {
  const T h = T(0.70710678118654752440084436210485);
  // radix-2 over stride 4, then twiddles w8^k on the odd half, then radix-4
  cplx<T> e[4], o[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    e[k] = v[2 * k];
    o[k] = v[2 * k + 1];
  }
  dft4<S>(e);
  dft4<S>(o);
  // o[k] *= exp(S 2 pi i k / 8)
  cplx<T> o1 = o[1], o2 = o[2], o3 = o[3];
  o[1] = {h * (o1.x - S * o1.y), h * (o1.y + S * o1.x)};
  o[2] = mul_si<S>(o2);
  o[3] = {h * (-o3.x - S * o3.y), h * (-o3.y + S * o3.x)};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = cadd(e[k], o[k]);
    v[k + 4] = csub(e[k], o[k]);
  }
}

// 9-point DFT as 3 x 3: DFT3 over n1 of x[3 n1 + n2], twiddles w9^(n2 k1),
// DFT3 over n2; output index k1 + 3 k2.
template <int S, typename T>
__device__ __forceinline__ void dft9(cplx<T>* v) {
  const T c1 = T(0.76604444311897803520239265055542);   // cos(2 pi/9)
  const T s1 = T(0.64278760968653932632264340990726);   // sin(2 pi/9)
  const T c2 = T(0.17364817766693034885171662676931);   // cos(4 pi/9)
  const T s2 = T(0.98480775301220805936674302458952);   // sin(4 pi/9)
  const T c4 = T(-0.93969262078590838405410927732473);  // cos(8 pi/9)
  const T s4 = T(0.34202014332566873304409961468226);   // sin(8 pi/9)
  cplx<T> y0[3] = {v[0], v[3], v[6]};
  cplx<T> y1[3] = {v[1], v[4], v[7]};
  cplx<T> y2[3] = {v[2], v[5], v[8]};
  dft3<S>(y0);
  dft3<S>(y1);
  dft3<S>(y2);
  auto rot = [](cplx<T> z, T c, T s) -> cplx<T> {
    return {z.x * c - T(S) * z.y * s, z.y * c + T(S) * z.x * s};
  };
  y1[1] = rot(y1[1], c1, s1);
  y1[2] = rot(y1[2], c2, s2);
  y2[1] = rot(y2[1], c2, s2);
  y2[2] = rot(y2[2], c4, s4);
#pragma unroll
  for (int k1 = 0; k1 < 3; ++k1) {
    cplx<T> z[3] = {y0[k1], y1[k1], y2[k1]};
    dft3<S>(z);
    v[k1] = z[0];
    v[k1 + 3] = z[1];
    v[k1 + 6] = z[2];
  }
}

template <int S, typename T>
__device__ __forceinline__ void dft_r(int r, cplx<T>* v) {
  switch (r) {
    case 2: dft2<S>(v); break;
    case 3: dft3<S>(v); break;
    case 4: dft4<S>(v); break;
    case 5: dft5<S>(v); break;
    case 8: dft8<S>(v); break;
    default: break;
  }
}

// Batched in-place FFT of `nlines` lines of length P.n held in LDS.
// Element j of line l lives at buf[l * ls + j * es].
// LINE_FAST selects the thread mapping: consecutive threads take consecutive
// lines (use when ls == 1) or consecutive butterflies of one line (es == 1).
// MAXB bounds the butterflies per thread per pass: nlines * n / min radix
// must not exceed MAXB * blockDim.x (checked on the host at launch).
template <int S, int MAXB, bool LINE_FAST, typename T>
__device__ void lds_fft(cplx<T>* buf, const FFTPlan& P, int nlines, int es, int ls,
                        const cplx<T>* __restrict__ tw) {
  const int n = P.n;
  const int nthr = blockDim.x;
  const int tid = threadIdx.x;
  for (int pass = 0; pass < P.np; ++pass) {
    const int r = P.rad[pass];
    const int p = P.p[pass];
    const int M = n / r;
    const int tws = n / (p * r);
    const int total = nlines * M;
    cplx<T> v[MAXB][kMaxRadix];
#pragma unroll
    for (int u = 0; u < MAXB; ++u) {
      const int b = tid + u * nthr;
      if (b < total) {
        int line, i;
        if (LINE_FAST) {
          line = b % nlines;
          i = b / nlines;
        } else {
          line = b / M;
          i = b - line * M;
        }
        const int k = i % p;
        cplx<T>* base = buf + line * ls;
#pragma unroll
        for (int t = 0; t < kMaxRadix; ++t) {
          if (t < r) {
            cplx<T> x = base[(i + t * M) * es];
            if (t > 0 && k > 0) {
              cplx<T> w = tw[t * k * tws];
              x = (S < 0) ? cmul(x, w) : cmulc(x, w);
            }
            v[u][t] = x;
          }
        }
        dft_r<S>(r, v[u]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MAXB; ++u) {
      const int b = tid + u * nthr;
      if (b < total) {
        int line, i;
        if (LINE_FAST) {
          line = b % nlines;
          i = b / nlines;
        } else {
          line = b / M;
          i = b - line * M;
        }
        const int k = i % p;
        const int j0 = (i - k) * r + k;
        cplx<T>* base = buf + line * ls;
#pragma unroll
        for (int q = 0; q < kMaxRadix; ++q)
          if (q < r) base[(j0 + q * p) * es] = v[u][q];
      }
    }
    __syncthreads();
  }
}

}  // namespace wtd
