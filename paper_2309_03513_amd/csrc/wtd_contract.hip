// Exchange + density-response contraction on the matrix cores.
//
// For every grid point r and trial b (the integrands of the paper's Eqs.
// k1eterm and k1d, with the pair potentials tau_vv' of Eq. trunc):
//   R[b][v](r) = c_K phi_v(r) (v_H,b(r) + f_xc(r) drho_b(r))
//                - alpha sum_v' tau_vv'(r) a~[b][v'](r)
// At a fixed point the exchange sum is a dense (Nocc x Nocc) . (Nocc x Nb)
// product, done as 16x16x4 MFMAs (M = v, N = b, K = v').
//
// Work split: one workgroup owns TP consecutive points (16 FP32 / 8 FP64), all
// Nocc <= 16 NT rows and 16 trials; each wave owns TP/8 points and keeps R for
// all rows in accumulators.  The
// workgroup walks the upper triangle of 16x16 (v, v') tiles: each unique tau
// value is read from HBM once and used twice (R[I] += tau[I][J] a[J] and
// R[J] += tau[I][J]^T a[I]).
//
// LDS tiles are [q][point] with q = 16 x + y (x the slow index) and a rotation
// of the point index by h(q) = x + 17 y: global loads are 64-byte rows, and
// the MFMA operand reads (lanes varying x, or lanes varying y) hit distinct
// banks up to one 2-way collision.
#include "wtd_internal.h"
#include "wtd_mfma.h"

namespace wtd {

namespace {

template <typename T>
struct CTile {
  // 8 waves x 16 points (FP32, two per wave) or 8 points (FP64, one per wave):
  // 64-byte rows, and the accumulators of all row tiles stay in registers
  static constexpr int THREADS = 512;
  static constexpr int TP = sizeof(T) == 4 ? 16 : 8;
  static constexpr int PPW = TP / (THREADS / 64);  // points per wave
  static constexpr int NE = 256 * TP;              // elements per LDS tile
  static __device__ __forceinline__ int at(int q, int p) {
    const int h = (q >> 4) + 17 * (q & 15);
    return q * TP + ((p + h) & (TP - 1));
  }
};

__device__ __forceinline__ int64_t pair_of(int v, int w, int nocc) {
  if (v > w) {
    const int t = v;
    v = w;
    w = t;
  }
  return (int64_t)v * nocc - (int64_t)v * (v - 1) / 2 + (w - v);
}

// tau[I][J] tile: element (v_loc, w_loc) at q = 16 v_loc + w_loc
template <typename T>
__device__ __forceinline__ void load_tau(T* s, const T* __restrict__ tau, int I, int J, int nocc,
                                         int64_t nr, int64_t r0) {
  typedef CTile<T> C;
  const int p = threadIdx.x % C::TP;
  const int g = threadIdx.x / C::TP;
  constexpr int G = C::THREADS / C::TP;
  const int64_t r = r0 + p;
  const bool rin = r < nr;
#pragma unroll
  for (int it = 0; it < 256 / G; ++it) {
    const int c = g + it * G;
    const int v = I * 16 + (c >> 4), w = J * 16 + (c & 15);
    T val = T(0);
    if (rin && v < nocc && w < nocc) val = tau[pair_of(v, w, nocc) * nr + r];
    s[C::at(c, p)] = val;
  }
}

// a~[b0 + b][K*16 + v'] tile: element (v'_loc, b_loc) at q = 16 v'_loc + b_loc
template <typename T>
__device__ __forceinline__ void load_at(T* s, const T* __restrict__ at, int K, int b0, int nb,
                                        int nocc, int64_t nr, int64_t r0) {
  typedef CTile<T> C;
  const int p = threadIdx.x % C::TP;
  const int g = threadIdx.x / C::TP;
  constexpr int G = C::THREADS / C::TP;
  const int64_t r = r0 + p;
  const bool rin = r < nr;
#pragma unroll
  for (int it = 0; it < 256 / G; ++it) {
    const int c = g + it * G;
    const int v = K * 16 + (c >> 4), b = b0 + (c & 15);
    T val = T(0);
    if (rin && v < nocc && b < nb) val = at[((int64_t)b * nocc + v) * nr + r];
    s[C::at(c, p)] = val;
  }
}

struct CArgs {
  int nb, nocc, b0;
  int64_t nr, r0;
  int lane, wave;
  // full-tile fast path: per-thread bases and the LDS table of row offsets
  const int64_t* rbnr;  // rbnr[v] = (v Nocc - v (v + 1) / 2) N_r: tau pair (v, w >= v) starts at rbnr[v] + w N_r
  int64_t wl_off;       // (w_loc) N_r + r of this thread's tau column
  int64_t a_off;        // ((b0 + b_loc) Nocc + v_loc0) N_r + r of this thread's trial element
};

// Guard-free tile loads for full tiles (Nocc % 16 == 0, Nb % 16 == 0, N_r % TP == 0).
// Thread t handles point p = t % TP and combos c = g + it G (g = t / TP): row
// v_loc = (g >> 4) + it (G >> 4), column w_loc = g & 15.
template <typename T>
__device__ __forceinline__ void load_tau_full(T* s, const T* __restrict__ tau, int I, int J,
                                              const CArgs& a) {
  typedef CTile<T> C;
  const int p = threadIdx.x % C::TP;
  const int g = threadIdx.x / C::TP;
  constexpr int G = C::THREADS / C::TP;
  const int wl = g & 15;
  if (I != J) {
    const int64_t col = a.wl_off + (int64_t)J * 16 * a.nr;
#pragma unroll
    for (int it = 0; it < 256 / G; ++it) {
      const int vl = (g >> 4) + it * (G >> 4);
      s[C::at(vl * 16 + wl, p)] = tau[a.rbnr[I * 16 + vl] + col];
    }
  } else {
    const int64_t r = a.r0 + p;
#pragma unroll
    for (int it = 0; it < 256 / G; ++it) {
      const int vl = (g >> 4) + it * (G >> 4);
      const int lo = I * 16 + min(vl, wl), hi = I * 16 + max(vl, wl);
      s[C::at(vl * 16 + wl, p)] = tau[a.rbnr[lo] + (int64_t)hi * a.nr + r];
    }
  }
}

// Register-staged variants used for prefetching: fetch_* issue the global
// loads of a tile into registers, put_* store them into the LDS tile.
template <typename T>
constexpr int kPer = 256 / (CTile<T>::THREADS / CTile<T>::TP);

template <typename T>
__device__ __forceinline__ void fetch_tau(T (&v)[kPer<T>], const T* __restrict__ tau, int I, int J,
                                          const CArgs& a) {
  typedef CTile<T> C;
  const int g = threadIdx.x / C::TP;
  constexpr int G = C::THREADS / C::TP;
  const int wl = g & 15;
  if (I != J) {
    const int64_t col = a.wl_off + (int64_t)J * 16 * a.nr;
#pragma unroll
    for (int it = 0; it < kPer<T>; ++it)
      v[it] = tau[a.rbnr[I * 16 + (g >> 4) + it * (G >> 4)] + col];
  } else {
    const int64_t r = a.r0 + threadIdx.x % C::TP;
#pragma unroll
    for (int it = 0; it < kPer<T>; ++it) {
      const int vl = (g >> 4) + it * (G >> 4);
      const int lo = I * 16 + min(vl, wl), hi = I * 16 + max(vl, wl);
      v[it] = tau[a.rbnr[lo] + (int64_t)hi * a.nr + r];
    }
  }
}

template <typename T>
__device__ __forceinline__ void fetch_at(T (&v)[kPer<T>], const T* __restrict__ at, int K,
                                         const CArgs& a) {
  typedef CTile<T> C;
  constexpr int G = C::THREADS / C::TP;
  const T* base = at + a.a_off + (int64_t)K * 16 * a.nr;
#pragma unroll
  for (int it = 0; it < kPer<T>; ++it) v[it] = base[(int64_t)it * (G >> 4) * a.nr];
}

template <typename T>
__device__ __forceinline__ void put_tile(T* s, const T (&v)[kPer<T>]) {
  typedef CTile<T> C;
  const int p = threadIdx.x % C::TP;
  const int g = threadIdx.x / C::TP;
  constexpr int G = C::THREADS / C::TP;
#pragma unroll
  for (int it = 0; it < kPer<T>; ++it)
    s[C::at(((g >> 4) + it * (G >> 4)) * 16 + (g & 15), p)] = v[it];
}

template <typename T>
__device__ __forceinline__ void load_at_full(T* s, const T* __restrict__ at, int K,
                                             const CArgs& a) {
  typedef CTile<T> C;
  const int p = threadIdx.x % C::TP;
  const int g = threadIdx.x / C::TP;
  constexpr int G = C::THREADS / C::TP;
  const T* base = at + a.a_off + (int64_t)K * 16 * a.nr;
#pragma unroll
  for (int it = 0; it < 256 / G; ++it) {
    const int vl = (g >> 4) + it * (G >> 4);
    s[C::at(vl * 16 + (g & 15), p)] = base[(int64_t)it * (G >> 4) * a.nr];
  }
}

// Walk of the upper triangle of (I, J) tiles with runtime loops over the row
// tile I and the column tile J >= I.  The accumulators acc[..][I] and
// acc[..][J] are selected through uniform branch chains, so every register
// index is a compile-time constant while no loads are hoisted out of the walk.
template <int NT, typename T>
__device__ __forceinline__ void mfma_into(typename Mfma<T>::acc_t (&acc)[NT], int tile,
                                          const T (&x)[4], const T (&y)[4]) {
#pragma unroll
  for (int t = 0; t < NT; ++t)
    if (tile == t) {
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[t] = Mfma<T>::run(x[k], y[k], acc[t]);
    }
}

template <typename T, int NT, bool FULL>
__device__ __forceinline__ void tri_walk(typename Mfma<T>::acc_t (&acc)[CTile<T>::PPW][NT],
                                         T* s_tau, T* s_a, const T* __restrict__ at,
                                         const T* __restrict__ tau, const CArgs& a) {
  typedef CTile<T> C;
  const int lx = a.lane & 15, ly = a.lane >> 4;
  T pt[kPer<T>], pa[kPer<T>];  // prefetched tiles of the next step (full tiles only)
#pragma unroll 1
  for (int I = 0; I < NT; ++I) {
    // a[I] in LDS; its B' operands (v = 4k + ly, b = lx) kept in registers
    __syncthreads();
    if constexpr (FULL) {
      fetch_at(pa, at, I, a);
      fetch_tau(pt, tau, I, I, a);
      put_tile(s_a, pa);
    } else {
      load_at(s_a, at, I, a.b0, a.nb, a.nocc, a.nr, a.r0);
    }
    __syncthreads();
    T bI[C::PPW][4];
#pragma unroll
    for (int pp = 0; pp < C::PPW; ++pp)
#pragma unroll
      for (int k = 0; k < 4; ++k)
        bI[pp][k] = s_a[C::at((4 * k + ly) * 16 + lx, a.wave * C::PPW + pp)];
#pragma unroll 1
    for (int J = I; J < NT; ++J) {
      __syncthreads();
      if constexpr (FULL) {
        put_tile(s_tau, pt);
        if (J != I) put_tile(s_a, pa);
      } else {
        load_tau(s_tau, tau, I, J, a.nocc, a.nr, a.r0);
        if (J != I) load_at(s_a, at, J, a.b0, a.nb, a.nocc, a.nr, a.r0);
      }
      __syncthreads();
      if constexpr (FULL) {
        // the next step's loads are in flight while this step's MFMAs run
        if (J + 1 < NT) {
          fetch_tau(pt, tau, I, J + 1, a);
          fetch_at(pa, at, J + 1, a);
        }
      }
#pragma unroll
      for (int pp = 0; pp < C::PPW; ++pp) {
        const int p = a.wave * C::PPW + pp;
        // R[I] += tau[I][J] a[J]:  A[v][v'] = tau[v = lx][v' = 4k + ly], B = a[J][v' = 4k + ly][b = lx]
        T x[4], y[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          x[k] = s_tau[C::at(lx * 16 + 4 * k + ly, p)];
          y[k] = s_a[C::at((4 * k + ly) * 16 + lx, p)];
        }
        mfma_into<NT, T>(acc[pp], I, x, y);
        if (J != I) {
          // R[J] += tau[I][J]^T a[I]:  A'[v'][v] = tau[v = 4k + ly][v' = lx], B' = bI
#pragma unroll
          for (int k = 0; k < 4; ++k) x[k] = s_tau[C::at((4 * k + ly) * 16 + lx, p)];
          mfma_into<NT, T>(acc[pp], J, x, bI[pp]);
        }
      }
    }
  }
}

// R = c_K phi (v_H + f_xc drho) - alpha acc for row tile I, staged through LDS.
template <typename T, int NT, int I>
__device__ __forceinline__ void write_rows(const typename Mfma<T>::acc_t (&acc)[CTile<T>::PPW][NT],
                                           T* s_o, const T* __restrict__ phi,
                                           const T* __restrict__ vh, const T* __restrict__ drho,
                                           T fx, T ck, T alpha, int k1e, T* __restrict__ R,
                                           const CArgs& a) {
  typedef CTile<T> C;
  if constexpr (I < NT) {
    asm volatile("" ::: "memory");
    const int lx = a.lane & 15;
    __syncthreads();
#pragma unroll
    for (int pp = 0; pp < C::PPW; ++pp)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int vl = Mfma<T>::row(a.lane, e);
        s_o[C::at(vl * 16 + lx, a.wave * C::PPW + pp)] = acc[pp][I][e];
      }
    __syncthreads();
    const int p = threadIdx.x % C::TP;
    const int g = threadIdx.x / C::TP;
    constexpr int G = C::THREADS / C::TP;
    const int64_t r = a.r0 + p;
    if (r < a.nr) {
#pragma unroll
      for (int it = 0; it < 256 / G; ++it) {
        const int c = g + it * G;
        const int v = I * 16 + (c >> 4), b = a.b0 + (c & 15);
        if (v >= a.nocc || b >= a.nb) continue;
        T val = -alpha * s_o[C::at(c, p)];
        if (k1e) {
          const T d = drho[(int64_t)b * a.nr + r];
          val += ck * phi[(int64_t)v * a.nr + r] * (vh[(int64_t)b * a.nr + r] + fx * d);
        }
        R[((int64_t)b * a.nocc + v) * a.nr + r] = val;
      }
    }
    write_rows<T, NT, I + 1>(acc, s_o, phi, vh, drho, fx, ck, alpha, k1e, R, a);
  }
}

template <typename T, int NT, bool FULL>
__global__ void __launch_bounds__(CTile<T>::THREADS)
k_contract_mfma(int nb, int nocc, int64_t nr, int ntile, const T* __restrict__ phi,
                const T* __restrict__ at, const T* __restrict__ tau, const T* __restrict__ vh,
                const T* __restrict__ drho, const T* __restrict__ fxc, T ck, T alpha, int k1e,
                int k1d, T* __restrict__ R) {
  typedef CTile<T> C;
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T s_tau[C::NE];
  __shared__ T s_a[C::NE];
  __shared__ int64_t s_rbnr[16 * NT];
  // XCD-aware order: each XCD takes a contiguous range of point tiles, so the
  // rows of neighbouring tiles are fetched through one L2.
  const int per = (ntile + 7) / 8;
  const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (tile >= ntile) return;
  CArgs a;
  a.nb = nb;
  a.nocc = nocc;
  a.b0 = blockIdx.y * 16;
  a.nr = nr;
  a.r0 = (int64_t)tile * C::TP;
  a.lane = threadIdx.x & 63;
  a.wave = threadIdx.x >> 6;
  if constexpr (FULL) {
    for (int v = threadIdx.x; v < 16 * NT; v += blockDim.x)
      s_rbnr[v] = ((int64_t)v * nocc - (int64_t)v * (v + 1) / 2) * nr;
    const int g = threadIdx.x / C::TP;
    const int64_t r = a.r0 + threadIdx.x % C::TP;
    a.rbnr = s_rbnr;
    a.wl_off = (int64_t)(g & 15) * nr + r;
    a.a_off = ((int64_t)(a.b0 + (g & 15)) * nocc + (g >> 4)) * nr + r;
  }

  acc_t acc[C::PPW][NT];
#pragma unroll
  for (int pp = 0; pp < C::PPW; ++pp)
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[pp][i] = acc_t{0, 0, 0, 0};
  if (k1d) tri_walk<T, NT, FULL>(acc, s_tau, s_a, at, tau, a);
  const int64_t r = a.r0 + threadIdx.x % C::TP;
  const T fx = (r < nr && k1e) ? fxc[r] : T(0);
  write_rows<T, NT, 0>(acc, s_tau, phi, vh, drho, fx, ck, alpha, k1e, R, a);
}

// ---------------------------------------------------------------------------
// Block form for large Nocc: the pair triangle is processed in blocks of rows
// (A, B), A <= B, of at most 4 row tiles each.  tau holds the block's pairs:
// a rectangle (v in A, w in B) stored row-major, or, for A == B, the upper
// triangle (w >= v) stored row-major.  The kernel adds
//   R[A] -= alpha tau[A][B] a[B]   and, for A != B,   R[B] -= alpha tau[A][B]^T a[A]
// to R (read-modify-write).  Accumulator slots 0..3 hold R[A] tiles, 4..7 R[B].
struct BArgs {
  int A0, nA, B0, nB, diag;
};

template <typename T>
__device__ __forceinline__ int64_t block_pair(const BArgs& bk, int i, int j) {
  // i, j local row / column indices inside the block
  if (bk.diag) {
    if (i > j) {
      const int t = i;
      i = j;
      j = t;
    }
    return (int64_t)i * bk.nA - (int64_t)i * (i + 1) / 2 + j;
  }
  return (int64_t)i * bk.nB + j;
}

template <typename T>
__device__ __forceinline__ void load_tau_block(T* s, const T* __restrict__ tau, int I, int J,
                                               const BArgs& bk, int64_t nr, int64_t r0) {
  typedef CTile<T> C;
  const int p = threadIdx.x % C::TP;
  const int g = threadIdx.x / C::TP;
  constexpr int G = C::THREADS / C::TP;
  const int64_t r = r0 + p;
  const bool rin = r < nr;
#pragma unroll
  for (int it = 0; it < 256 / G; ++it) {
    const int c = g + it * G;
    const int i = I * 16 + (c >> 4), j = J * 16 + (c & 15);
    T val = T(0);
    if (rin && i < bk.nA && j < (bk.diag ? bk.nA : bk.nB))
      val = tau[block_pair<T>(bk, i, j) * nr + r];
    s[C::at(c, p)] = val;
  }
}

template <typename T>
__global__ void __launch_bounds__(CTile<T>::THREADS)
k_contract_block(int nb, int nocc, int64_t nr, int ntile, const T* __restrict__ at,
                 const T* __restrict__ tau, BArgs bk, T alpha, T* __restrict__ R) {
  typedef CTile<T> C;
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T s_tau[C::NE];
  __shared__ T s_a[C::NE];
  const int per = (ntile + 7) / 8;
  const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (tile >= ntile) return;
  const int b0 = blockIdx.y * 16;
  const int64_t r0 = (int64_t)tile * C::TP;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lx = lane & 15, ly = lane >> 4;
  const int ntA = (bk.nA + 15) / 16, ntB = bk.diag ? ntA : (bk.nB + 15) / 16;
  acc_t acc[C::PPW][8];
#pragma unroll
  for (int pp = 0; pp < C::PPW; ++pp)
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[pp][i] = acc_t{0, 0, 0, 0};
#pragma unroll 1
  for (int I = 0; I < ntA; ++I) {
    // a at the rows of tile I of block A (B' operands of the transposed term)
    __syncthreads();
    load_at(s_a, at, bk.A0 / 16 + I, b0, nb, nocc, nr, r0);
    __syncthreads();
    T bI[C::PPW][4];
#pragma unroll
    for (int pp = 0; pp < C::PPW; ++pp)
#pragma unroll
      for (int k = 0; k < 4; ++k)
        bI[pp][k] = s_a[C::at((4 * k + ly) * 16 + lx, wave * C::PPW + pp)];
#pragma unroll 1
    for (int J = bk.diag ? I : 0; J < ntB; ++J) {
      const bool dtile = bk.diag && J == I;
      __syncthreads();
      load_tau_block(s_tau, tau, I, J, bk, nr, r0);
      if (!dtile) load_at(s_a, at, (bk.diag ? bk.A0 : bk.B0) / 16 + J, b0, nb, nocc, nr, r0);
      __syncthreads();
      const int slotI = I;
      const int slotJ = bk.diag ? J : 4 + J;
#pragma unroll
      for (int pp = 0; pp < C::PPW; ++pp) {
        const int p = wave * C::PPW + pp;
        T x[4], y[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          x[k] = s_tau[C::at(lx * 16 + 4 * k + ly, p)];
          y[k] = s_a[C::at((4 * k + ly) * 16 + lx, p)];
        }
        mfma_into<8, T>(acc[pp], slotI, x, y);
        if (!dtile) {
#pragma unroll
          for (int k = 0; k < 4; ++k) x[k] = s_tau[C::at((4 * k + ly) * 16 + lx, p)];
          mfma_into<8, T>(acc[pp], slotJ, x, bI[pp]);
        }
      }
    }
  }
  // R += -alpha acc for the rows of A (slots 0..3) and, off the diagonal, of B (4..7)
  const int p = threadIdx.x % C::TP;
  const int g = threadIdx.x / C::TP;
  constexpr int G = C::THREADS / C::TP;
  const int64_t r = r0 + p;
#pragma unroll
  for (int slot = 0; slot < 8; ++slot) {
    const bool isA = slot < 4;
    const int tl = isA ? slot : slot - 4;
    if (!isA && bk.diag) break;
    const int base = isA ? bk.A0 : bk.B0;
    const int nrows = isA ? bk.nA : bk.nB;
    if (tl * 16 >= nrows) continue;
    __syncthreads();
#pragma unroll
    for (int pp = 0; pp < C::PPW; ++pp)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        s_tau[C::at(Mfma<T>::row(lane, e) * 16 + lx, wave * C::PPW + pp)] = acc[pp][slot][e];
    __syncthreads();
    if (r < nr) {
#pragma unroll
      for (int it = 0; it < 256 / G; ++it) {
        const int c = g + it * G;
        const int vl = tl * 16 + (c >> 4), b = b0 + (c & 15);
        if (vl >= nrows || b >= nb) continue;
        T* o = R + ((int64_t)b * nocc + base + vl) * nr + r;
        *o += -alpha * s_tau[C::at(c, p)];
      }
    }
  }
}

// R[b][v] = c_K phi_v (v_H,b + f_xc drho_b), or 0 without the response term
template <typename T>
__global__ void k_response_rows(int nb, int nocc, int64_t nr, const T* __restrict__ phi,
                                const T* __restrict__ vh, const T* __restrict__ drho,
                                const T* __restrict__ fxc, T ck, int k1e, T* __restrict__ R) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int bv = blockIdx.y;
  if (r >= nr) return;
  const int b = bv / nocc, v = bv - b * nocc;
  T val = T(0);
  if (k1e) val = ck * phi[(int64_t)v * nr + r] * (vh[(int64_t)b * nr + r] + fxc[r] * drho[(int64_t)b * nr + r]);
  R[(int64_t)bv * nr + r] = val;
}

}  // namespace

template <typename T>
bool launch_contract_mfma(const Geometry& g, int nb, int nocc, const T* phi, const T* at,
                          const T* tau, const T* vh, const T* drho, const T* fxc, T ck, T alpha,
                          bool k1e, bool k1d, T* R, hipStream_t s) {
  const int nt = (nocc + 15) / 16;
  if (nt > 8) return false;
  typedef CTile<T> C;
  const int64_t ntile64 = (g.nr + C::TP - 1) / C::TP;
  WTD_REQUIRE(ntile64 < (1ll << 30), WTD_ERR_SHAPE, "contraction grid too large");
  const int ntile = (int)ntile64;
  const int per = (ntile + 7) / 8;
  dim3 grid(8 * per, (nb + 15) / 16);
  const bool full = nocc % 16 == 0 && nb % 16 == 0 && g.nr % C::TP == 0;
#define WTD_CT(NTV)                                                                          \
  case NTV:                                                                                  \
    if (full)                                                                                \
      hipLaunchKernelGGL((k_contract_mfma<T, NTV, true>), grid, dim3(C::THREADS), 0, s, nb,  \
                         nocc, g.nr, ntile, phi, at, tau, vh, drho, fxc, ck, alpha, (int)k1e, \
                         (int)k1d, R);                                                       \
    else                                                                                     \
      hipLaunchKernelGGL((k_contract_mfma<T, NTV, false>), grid, dim3(C::THREADS), 0, s, nb, \
                         nocc, g.nr, ntile, phi, at, tau, vh, drho, fxc, ck, alpha, (int)k1e, \
                         (int)k1d, R);                                                       \
    break;
  switch (nt) {
    WTD_CT(1)
    WTD_CT(2)
    WTD_CT(3)
    WTD_CT(4)
    WTD_CT(5)
    WTD_CT(6)
    WTD_CT(7)
    WTD_CT(8)
    default:
      return false;
  }
#undef WTD_CT
  WTD_HIP(hipGetLastError());
  return true;
}

template bool launch_contract_mfma<float>(const Geometry&, int, int, const float*, const float*,
                                          const float*, const float*, const float*, const float*,
                                          float, float, bool, bool, float*, hipStream_t);
template bool launch_contract_mfma<double>(const Geometry&, int, int, const double*,
                                           const double*, const double*, const double*,
                                           const double*, const double*, double, double, bool,
                                           bool, double*, hipStream_t);

}  // namespace wtd

namespace wtd {

template <typename T>
void launch_response_rows(const Geometry& g, int nb, int nocc, const T* phi, const T* vh,
                          const T* drho, const T* fxc, T ck, bool k1e, T* R, hipStream_t s) {
  dim3 grid((unsigned)((g.nr + 255) / 256), (unsigned)(nb * nocc));
  hipLaunchKernelGGL(k_response_rows<T>, grid, dim3(256), 0, s, nb, nocc, g.nr, phi, vh, drho, fxc,
                     ck, (int)k1e, R);
  WTD_HIP(hipGetLastError());
}

template <typename T>
void launch_contract_block(const Geometry& g, int nb, int nocc, const T* at, const T* tau, int A0,
                           int nA, int B0, int nB, bool diag, T alpha, T* R, hipStream_t s) {
  WTD_REQUIRE(nA <= 64 && nB <= 64 && A0 % 16 == 0 && B0 % 16 == 0, WTD_ERR_SHAPE,
              "row blocks of the exchange contraction must be <= 64 rows, 16-aligned");
  typedef CTile<T> C;
  const int64_t ntile64 = (g.nr + C::TP - 1) / C::TP;
  WTD_REQUIRE(ntile64 < (1ll << 30), WTD_ERR_SHAPE, "contraction grid too large");
  const int ntile = (int)ntile64;
  const int per = (ntile + 7) / 8;
  dim3 grid(8 * per, (nb + 15) / 16);
  BArgs bk{A0, nA, B0, nB, diag ? 1 : 0};
  hipLaunchKernelGGL(k_contract_block<T>, grid, dim3(C::THREADS), 0, s, nb, nocc, g.nr, ntile, at,
                     tau, bk, alpha, R);
  WTD_HIP(hipGetLastError());
}

template void launch_response_rows<float>(const Geometry&, int, int, const float*, const float*,
                                          const float*, const float*, float, bool, float*,
                                          hipStream_t);
template void launch_response_rows<double>(const Geometry&, int, int, const double*,
                                           const double*, const double*, const double*, double,
                                           bool, double*, hipStream_t);
template void launch_contract_block<float>(const Geometry&, int, int, const float*, const float*,
                                           int, int, int, int, bool, float, float*, hipStream_t);
template void launch_contract_block<double>(const Geometry&, int, int, const double*,
                                            const double*, int, int, int, int, bool, double,
                                            double*, hipStream_t);

}  // namespace wtd
