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

// Grouped walk for full tiles: the column tiles J = I..NT-1 of row tile I are
// taken G at a time.  A group's G tau tiles and G trial tiles are staged in LDS
// together, and the next group's global loads are issued (into registers)
// before the current group's MFMAs, so one memory latency is paid per group
// rather than per tile.  The B' operands of a[I] come from slot 0 of the
// first group of row I (J = I).
template <int G>
__device__ __forceinline__ bool next_group(int NT, int& I, int& J0) {
  if (J0 + G < NT) {
    J0 += G;
    return true;
  }
  ++I;
  J0 = I;
  return I < NT;
}

template <typename T, int NT, int G>
__device__ __forceinline__ void tri_walk_grouped(
    typename Mfma<T>::acc_t (&acc)[CTile<T>::PPW][NT], T* s_tau, T* s_a,
    const T* __restrict__ at, const T* __restrict__ tau, const CArgs& a) {
  typedef CTile<T> C;
  const int lx = a.lane & 15, ly = a.lane >> 4;
  T pt[G][kPer<T>], pa[G][kPer<T>];
  // loads of group (0, 0)
#pragma unroll
  for (int k = 0; k < G; ++k)
    if (k < NT) {
      fetch_tau(pt[k], tau, 0, k, a);
      fetch_at(pa[k], at, k, a);
    }
  T bI[C::PPW][4];
  int I = 0, J0 = 0;
#pragma unroll 1
  while (true) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < G; ++k)
      if (J0 + k < NT) {
        put_tile(s_tau + k * C::NE, pt[k]);
        put_tile(s_a + k * C::NE, pa[k]);
      }
    __syncthreads();
    const int Ic = I, J0c = J0;
    const bool more = next_group<G>(NT, I, J0);
    if (more) {
#pragma unroll
      for (int k = 0; k < G; ++k)
        if (J0 + k < NT) {
          fetch_tau(pt[k], tau, I, J0 + k, a);
          fetch_at(pa[k], at, J0 + k, a);
        }
    }
    if (J0c == Ic) {
#pragma unroll
      for (int pp = 0; pp < C::PPW; ++pp)
#pragma unroll
        for (int k = 0; k < 4; ++k)
          bI[pp][k] = s_a[C::at((4 * k + ly) * 16 + lx, a.wave * C::PPW + pp)];
    }
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int J = J0c + k;
      if (J < NT) {
        const T* st = s_tau + k * C::NE;
        const T* sa = s_a + k * C::NE;
#pragma unroll
        for (int pp = 0; pp < C::PPW; ++pp) {
          const int p = a.wave * C::PPW + pp;
          T x[4], y[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            x[q] = st[C::at(lx * 16 + 4 * q + ly, p)];
            y[q] = sa[C::at((4 * q + ly) * 16 + lx, p)];
          }
          mfma_into<NT, T>(acc[pp], Ic, x, y);
          if (J != Ic) {
#pragma unroll
            for (int q = 0; q < 4; ++q) x[q] = st[C::at((4 * q + ly) * 16 + lx, p)];
            mfma_into<NT, T>(acc[pp], J, x, bI[pp]);
          }
        }
      }
    }
    if (!more) break;
  }
}

// tiles staged together by the grouped walk
template <typename T>
constexpr int kGroup = 2;

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
  constexpr int NG = FULL ? kGroup<T> : 1;
  __shared__ T s_tau[NG * C::NE];
  __shared__ T s_a[NG * C::NE];
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
  if (k1d) {
    if constexpr (FULL)
      tri_walk_grouped<T, NT, NG>(acc, s_tau, s_a, at, tau, a);
    else
      tri_walk<T, NT, FULL>(acc, s_tau, s_a, at, tau, a);
  }
  const int64_t r = a.r0 + threadIdx.x % C::TP;
  const T fx = (r < nr && k1e) ? fxc[r] : T(0);
  write_rows<T, NT, 0>(acc, s_tau, phi, vh, drho, fx, ck, alpha, k1e, R, a);
}

// ---------------------------------------------------------------------------
// Round-robin form for Nocc = 128 (eight row tiles of 16), FP32 and FP64.
//
// Wave w owns row tile w: its accumulators hold R[w] (16 rows x 16 trials) for
// all TP points of the workgroup (8 in FP32, 4 in FP64), indexed at compile
// time, so the MFMA chains of the points are independent.  The 36 tau tiles of
// the upper triangle are visited in 8 rounds of a round-robin tournament: in
// round r < 7 the row tiles pair up as {r, 7} and {(r + k) mod 7, (r - k) mod 7},
// k = 1..3 (four off-diagonal tiles, each used by both of its waves, once
// directly and once transposed); round 7 holds the eight diagonal tiles.
// All eight trial tiles stay in LDS for the whole walk; the tau tiles of the
// next rounds are in flight in registers while the current round computes.
//
// tau holds the pairs tile by tile (rr_tile_base) in the 4-pair interleaved
// layout, so the 16-byte loads of one group at the TP points of a workgroup
// read one whole 128-byte line.  An off-diagonal tile is one 16-byte load per
// thread; a diagonal round (eight packed triangles of 34 groups) at most five.
// Few, wide loads keep several rounds in flight within the per-wave limit on
// outstanding loads, and they carry the streaming hint (tau is read once; at
// 72^3 the contraction took 4.43 -> 4.39 ms with it, while the same hint on the
// trial-field loads, 32-byte pieces of rows, or on the R stores made it slower).
// The response-term inputs (phi, v_H, drho, f_xc) are read after the walk.
//
// LDS tile layout: element (q, p) of a square tile, q = 16 row + column, at
// p * 264 + perm(q), perm(q) = q ^ (((q >> 6) & 3) << 2): the point stride and
// the permutation spread the MFMA operand reads (fixed point, lanes over
// (lx, ly)) over the banks, and the permutation keeps aligned runs of four q
// together, so a staged load is one 16-byte store.  A diagonal tile is kept as
// its packed triangle: element (k, p) at p * 264 + k.
template <typename T>
struct RRTile {
  static constexpr int TP = 32 / sizeof(T);       // points per workgroup
  static constexpr int THREADS = 512;
  static constexpr int PS = 264;                  // point stride (elements)
  static constexpr int NE = PS * TP;              // elements per tile
  static constexpr int EPL = 16 / sizeof(T);      // elements per 16-byte load
  static constexpr int LPG = 4 / EPL;             // loads per 4-pair group and point
  static constexpr int DIAG = 8 * 34 * TP * LPG;  // 16-byte loads of a diagonal round
  static constexpr int DIAG_LOADS = (DIAG + THREADS - 1) / THREADS;
  static __device__ __forceinline__ int perm(int q) { return q ^ (((q >> 6) & 3) << 2); }
  static __device__ __forceinline__ int at(int q, int p) { return p * PS + perm(q); }
};
static_assert(kTauIl == 4, "the round-robin staging reads 4-pair groups");
static_assert(rr_tile_base(7, 7) + 136 == 128 * 129 / 2, "the tile order covers the pair triangle");
static_assert(64 * RRTile<float>::TP * RRTile<float>::LPG == RRTile<float>::THREADS &&
                  64 * RRTile<double>::TP * RRTile<double>::LPG == RRTile<double>::THREADS,
              "one 16-byte load per thread per tile");

template <typename T>
using rr_vec = T __attribute__((ext_vector_type(16 / sizeof(T))));

// partner of row tile w in round r (r < 7), and the slot of the pair's tile
__device__ __forceinline__ void rr_pair(int r, int w, int& partner, int& slot) {
  if (w == 7 || w == r) {
    partner = (w == 7) ? r : 7;
    slot = 0;
    return;
  }
  const int d = (w - r + 7) % 7;
  partner = (2 * r - w + 14) % 7;
  slot = d <= 3 ? d : 7 - d;
}

// (I, J), I < J, of slot `slot` in an off-diagonal round r < 7
__device__ __forceinline__ void rr_tile(int r, int slot, int& I, int& J) {
  int a, b;
  if (slot == 0) {
    a = r;
    b = 7;
  } else {
    a = (r + slot) % 7;
    b = (r - slot + 7) % 7;
  }
  I = min(a, b);
  J = max(a, b);
}

// rounds of tau loads in flight (FP32 with 16-byte loads: 2, 3, 4 and 6 rounds
// at 72^3 took 4.32, 4.40, 4.54 and 4.96 ms)
constexpr int kRRDepth = 2;

template <typename T>
__global__ void __launch_bounds__(RRTile<T>::THREADS)
k_contract_rr(int nb, int nocc, int64_t nr, int ntile, const T* __restrict__ phi,
              const T* __restrict__ at, const T* __restrict__ tau, const T* __restrict__ vh,
              const T* __restrict__ drho, const T* __restrict__ fxc, T ck, T alpha, int k1e,
              int k1d, T* __restrict__ R) {
  typedef RRTile<T> C;
  typedef rr_vec<T> V;
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int TP = C::TP, EPL = C::EPL, LPG = C::LPG;
  __shared__ T s_a[8 * C::NE];   // trial tiles a~[b0 + b][16 K + v'], K = 0..7
  __shared__ T s_t[8 * C::NE];   // tau tiles of one round; reused to stage R
  const int per = (ntile + 7) / 8;
  const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (tile >= ntile) return;
  const int b0 = blockIdx.y * 16;
  const int64_t r0 = (int64_t)tile * TP;
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int lx = lane & 15, ly = lane >> 4;
  // tau as 16-byte vectors: the load `sub` of group G at point r is vector
  // (G N_r + r) LPG + sub
  const V* __restrict__ tauv = reinterpret_cast<const V*>(tau);

  // off-diagonal tiles: thread t loads part sub = t % LPG of group
  // g = t / (LPG TP) of the tile (row g / 4, columns 4 (g % 4) .. + 3) at
  // point (t / LPG) % TP
  const int tsub = t % LPG, tp = (t / LPG) % TP, tg = t / (LPG * TP);
  const int64_t toff = ((int64_t)tg * nr + r0 + tp) * LPG + tsub;
  const int tput = tp * C::PS + C::perm(4 * tg) + EPL * tsub;
  // diagonal round: load j of thread t is element t + 512 j of the eight
  // triangles x 34 groups x TP points x LPG parts
  int64_t doff[C::DIAG_LOADS];
  int dput[C::DIAG_LOADS];
#pragma unroll
  for (int j = 0; j < C::DIAG_LOADS; ++j) {
    const int idx = min(t + C::THREADS * j, C::DIAG - 1);
    const int dt = idx / (34 * TP * LPG), m = idx - dt * 34 * TP * LPG;
    const int sub = m % LPG, p = (m / LPG) % TP, k4 = m / (LPG * TP);
    doff[j] = ((int64_t)(rr_tile_base(dt, dt) / kTauIl + k4) * nr + r0 + p) * LPG + sub;
    dput[j] = dt * C::NE + p * C::PS + 4 * k4 + EPL * sub;
  }
  const bool dlast = t + C::THREADS * (C::DIAG_LOADS - 1) < C::DIAG;
  auto fetch = [&](V (&v)[C::DIAG_LOADS], int r) {
    if (r < 7) {
#pragma unroll
      for (int sl = 0; sl < 4; ++sl) {
        int I, J;
        rr_tile(r, sl, I, J);
        v[sl] = __builtin_nontemporal_load(
            &tauv[(int64_t)(rr_tile_base(I, J) / kTauIl) * nr * LPG + toff]);
      }
    } else {
#pragma unroll
      for (int j = 0; j < C::DIAG_LOADS; ++j)
        if (j < C::DIAG_LOADS - 1 || dlast) v[j] = __builtin_nontemporal_load(&tauv[doff[j]]);
    }
  };
  auto put = [&](const V (&v)[C::DIAG_LOADS], int r) {
    if (r < 7) {
#pragma unroll
      for (int sl = 0; sl < 4; ++sl) *reinterpret_cast<V*>(s_t + sl * C::NE + tput) = v[sl];
    } else {
#pragma unroll
      for (int j = 0; j < C::DIAG_LOADS; ++j)
        if (j < C::DIAG_LOADS - 1 || dlast) *reinterpret_cast<V*>(s_t + dput[j]) = v[j];
    }
  };

  acc_t acc[TP];
#pragma unroll
  for (int p = 0; p < TP; ++p) acc[p] = acc_t{0, 0, 0, 0};

  // trial and output rows of thread t: trial b = b0 + (t / 2) % 16, orbital
  // v_j = t / 32 + 16 j (j = 0..7), points EPL (t % 2) .. + EPL - 1
  const int h = t & 1, bl = (t >> 1) & 15;
  const bool bin = b0 + bl < nb;
  const int64_t rq = r0 + EPL * h;
  const V zero = V(T(0));
  // response-term inputs of these outputs
  V ph[8], vhb = zero, drb = zero, fx = zero;
#pragma unroll
  for (int j = 0; j < 8; ++j) ph[j] = zero;
  auto load_response = [&]() {
    if (k1e && bin) {
#pragma unroll
      for (int j = 0; j < 8; ++j)
        ph[j] = *reinterpret_cast<const V*>(phi + (int64_t)((t >> 5) + 16 * j) * nr + rq);
      vhb = *reinterpret_cast<const V*>(vh + (int64_t)(b0 + bl) * nr + rq);
      drb = *reinterpret_cast<const V*>(drho + (int64_t)(b0 + bl) * nr + rq);
      fx = *reinterpret_cast<const V*>(fxc + rq);
    }
  };

  if (k1d) {
    V vb[kRRDepth][C::DIAG_LOADS];
    {
      V ta[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        // trials past nb (a ragged last trial tile) enter as zeros
        const int v = (t >> 5) + 16 * j;
        ta[j] = bin ? *reinterpret_cast<const V*>(at + ((int64_t)(b0 + bl) * nocc + v) * nr + rq)
                    : zero;
      }
#pragma unroll
      for (int r = 0; r < kRRDepth; ++r) fetch(vb[r], r);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int v = (t >> 5) + 16 * j;
        T* d = s_a + (v >> 4) * C::NE + C::at((v & 15) * 16 + bl, EPL * h);
#pragma unroll
        for (int e = 0; e < EPL; ++e) d[e * C::PS] = ta[j][e];
      }
    }
    // lane-constant LDS offsets of the MFMA operands for K-step s4:
    // direct A[m = lx][k = 4 s4 + ly] = tau[v = lx][w = 4 s4 + ly];
    // transposed A = tau[v = 4 s4 + ly][w = lx]; diagonal A = the triangle
    // element of (min, max); B[k = v'][n = b] = a~[4 s4 + ly][lx]
    int oa_d[4], oa_t[4], oa_r[4];
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int k = 4 * s4 + ly;
      oa_d[s4] = C::perm(lx * 16 + k);
      oa_t[s4] = C::perm(k * 16 + lx);
      oa_r[s4] = rr_tri_index(min(lx, k), max(lx, k));
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      __syncthreads();
      put(vb[r % kRRDepth], r);
      __syncthreads();
      if (r + kRRDepth < 8) fetch(vb[r % kRRDepth], r + kRRDepth);
      int partner, slot;
      if (r < 7) {
        rr_pair(r, w, partner, slot);
      } else {
        partner = w;
        slot = w;
      }
      const T* st = s_t + slot * C::NE;
      const T* sa = s_a + partner * C::NE;
      const bool direct = w <= partner;
      // operands of K-step s4 for the TP points, loaded one step ahead
      T xa[2][TP], xb[2][TP];
#pragma unroll
      for (int s4 = 0; s4 < 5; ++s4) {
        if (s4 < 4) {
          const T* pa = st + (r == 7 ? oa_r[s4] : direct ? oa_d[s4] : oa_t[s4]);
          const T* pb = sa + oa_t[s4];
#pragma unroll
          for (int p = 0; p < TP; ++p) {
            xa[s4 & 1][p] = pa[p * C::PS];
            xb[s4 & 1][p] = pb[p * C::PS];
          }
        }
        if (s4 > 0) {
#pragma unroll
          for (int p = 0; p < TP; ++p)
            acc[p] = Mfma<T>::run(xa[(s4 - 1) & 1][p], xb[(s4 - 1) & 1][p], acc[p]);
        }
      }
    }
  }
  // (after the walk: loaded during round 5 they measured 3 % slower, holding
  // 44 more registers through the last rounds)
  load_response();

  // R[b][16 w + row] = -alpha acc (+ c_K phi (v_H + f_xc drho)), staged through LDS
  __syncthreads();
  T* so = s_t + w * C::NE;
#pragma unroll
  for (int p = 0; p < TP; ++p)
#pragma unroll
    for (int e = 0; e < 4; ++e) so[C::at(Mfma<T>::row(lane, e) * 16 + lx, p)] = acc[p][e];
  __syncthreads();
  if (!bin) return;
  const V vb_resp = vhb + fx * drb;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int v = (t >> 5) + 16 * j;
    const T* src = s_t + (v >> 4) * C::NE + C::at((v & 15) * 16 + bl, EPL * h);
    V val;
#pragma unroll
    for (int e = 0; e < EPL; ++e) val[e] = -alpha * src[e * C::PS];
    if (k1e) val += ck * ph[j] * vb_resp;
    *reinterpret_cast<V*>(R + ((int64_t)(b0 + bl) * nocc + v) * nr + rq) = val;
  }
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
// One thread per grid point and group of kRespRows rows v: the rows' phi values
// are read once and reused for every trial, whose potential c_K (v_H + f_xc drho)
// is formed once per trial.
constexpr int kRespRows = 8;
template <typename T>
__global__ void k_response_rows(int nb, int nocc, int64_t nr, const T* __restrict__ phi,
                                const T* __restrict__ vh, const T* __restrict__ drho,
                                const T* __restrict__ fxc, T ck, int k1e, T* __restrict__ R) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int v0 = blockIdx.y * kRespRows;
  if (r >= nr) return;
  T ph[kRespRows];
#pragma unroll
  for (int j = 0; j < kRespRows; ++j)
    ph[j] = (k1e && v0 + j < nocc) ? phi[(int64_t)(v0 + j) * nr + r] : T(0);
  const T fx = k1e ? fxc[r] : T(0);
  for (int b = 0; b < nb; ++b) {
    const T u = k1e ? ck * (vh[(int64_t)b * nr + r] + fx * drho[(int64_t)b * nr + r]) : T(0);
    T* o = R + ((int64_t)b * nocc + v0) * nr + r;
#pragma unroll
    for (int j = 0; j < kRespRows; ++j)
      if (v0 + j < nocc) o[(int64_t)j * nr] = ph[j] * u;
  }
}

}  // namespace

template <typename T>
bool contract_rr_applies(const Geometry& g, int nb, int nocc) {
  // any trial count: a ragged last tile of trials is zero-padded in the kernel,
  // so the pair-potential layout of a context does not depend on nb
  // 16-byte loads of whole point runs: N_r a multiple of 8 (FP32 reads 8
  // points per workgroup, FP64 4, both in 16-byte vectors)
  return nocc == 128 && nb >= 1 && g.nr % 8 == 0;
}

template <typename T>
bool launch_contract_mfma(const Geometry& g, int nb, int nocc, const T* phi, const T* at,
                          const T* tau, const T* vh, const T* drho, const T* fxc, T ck, T alpha,
                          bool k1e, bool k1d, T* R, hipStream_t s, bool tau_il) {
  const int nt = (nocc + 15) / 16;
  if (nt > 8) return false;
  WTD_REQUIRE(!tau_il || contract_rr_applies<T>(g, nb, nocc), WTD_ERR_SHAPE,
              "tile-ordered pair potentials need the round-robin contraction");
  if (tau_il) {
    const int64_t nt64 = g.nr / RRTile<T>::TP;
    WTD_REQUIRE(nt64 < (1ll << 30), WTD_ERR_SHAPE, "contraction grid too large");
    const int ntile = (int)nt64;
    dim3 grid(8 * ((ntile + 7) / 8), (nb + 15) / 16);
    hipLaunchKernelGGL(k_contract_rr<T>, grid, dim3(RRTile<T>::THREADS), 0, s, nb, nocc, g.nr,
                       ntile, phi, at, tau, vh, drho, fxc, ck, alpha, (int)k1e, (int)k1d, R);
    WTD_HIP(hipGetLastError());
    return true;
  }
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

template bool contract_rr_applies<float>(const Geometry&, int, int);
template bool contract_rr_applies<double>(const Geometry&, int, int);
template bool launch_contract_mfma<float>(const Geometry&, int, int, const float*, const float*,
                                          const float*, const float*, const float*, const float*,
                                          float, float, bool, bool, float*, hipStream_t, bool);
template bool launch_contract_mfma<double>(const Geometry&, int, int, const double*,
                                           const double*, const double*, const double*,
                                           const double*, const double*, double, double, bool,
                                           bool, double*, hipStream_t, bool);

}  // namespace wtd

namespace wtd {

template <typename T>
void launch_response_rows(const Geometry& g, int nb, int nocc, const T* phi, const T* vh,
                          const T* drho, const T* fxc, T ck, bool k1e, T* R, hipStream_t s) {
  dim3 grid((unsigned)((g.nr + 255) / 256), (unsigned)((nocc + kRespRows - 1) / kRespRows));
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

namespace {
// ---------------------------------------------------------------------------
// Row-blocked contraction, FP32, trial fields in registers.  A workgroup owns 8
// grid points (one per wave) and 16 NT trials of one block pair (A, B): every
// wave first takes the MFMA operand fragments of a[A] and a[B] (16 x 16 tiles,
// NT trial tiles) for its point into registers, then walks the block's tau
// tiles once, staged through LDS with the next tiles' loads in flight, and adds
// R[A] += tau a[B] and R[B] += tau^T a[A] (upper-triangle tiles and
// R[A] += tau a[A] on the diagonal block) into accumulators that are written
// back once: tau is read once per 16 NT trials and a once per block pair.
// Launched with NT = 1: with half the registers of NT = 2, two workgroups
// share a CU, which outweighs reading tau once per 16 trials instead of 32.
// tau is in the 4-pair interleaved layout: block-local pair P at point r is
// element ((P / 4) N_r + r) 4 + P % 4.
struct BRTile {
  static constexpr int TP = 8;
  static constexpr int THREADS = 512;
  static constexpr int NE = 256 * TP;  // one 16 x 16 tile for TP points
  static __device__ __forceinline__ int at(int q, int p) {
    const int h = (q >> 4) + 17 * (q & 15);
    return q * TP + ((p + h) & (TP - 1));
  }
};

template <bool DIAG>
__device__ __forceinline__ void br_load_tau(float (&pf)[4], const float* __restrict__ tau,
                                            int I, int J, const BArgs& bk, int64_t nr,
                                            int64_t r0) {
  const int nJ = DIAG ? bk.nA : bk.nB;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = threadIdx.x + u * BRTile::THREADS;
    const int p = (e >> 2) & 7, quad = e >> 5;
    const int i = I * 16 + (quad >> 2), j = J * 16 + (quad & 3) * 4 + (e & 3);
    const int64_t r = r0 + p;
    float v = 0.f;
    if (r < nr && i < bk.nA && j < nJ) {
      const int64_t P = block_pair<float>(bk, i, j);
      v = tau[(((P >> 2) * nr + r) << 2) + (P & 3)];
    }
    pf[u] = v;
  }
}

__device__ __forceinline__ void br_store_tau(float* s, const float (&pf)[4]) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = threadIdx.x + u * BRTile::THREADS;
    const int p = (e >> 2) & 7, quad = e >> 5;
    const int q = (quad >> 2) * 16 + (quad & 3) * 4 + (e & 3);
    s[BRTile::at(q, p)] = pf[u];
  }
}

// tile n of the walk -> (I, J): the 4 x 4 rectangle row by row, or the upper
// triangle I <= J row by row on the diagonal block
template <bool DIAG>
__device__ __forceinline__ constexpr int br_tile_i(int n) {
  if (!DIAG) return n >> 2;
  int i = 0;
  while (n >= 4 - i) n -= 4 - i, ++i;
  return i;
}
template <bool DIAG>
__device__ __forceinline__ constexpr int br_tile_j(int n) {
  if (!DIAG) return n & 3;
  int i = 0;
  while (n >= 4 - i) n -= 4 - i, ++i;
  return i + n;
}

// tau tiles in flight ahead of the current one; the 16-trial workgroup is held
// to 128 VGPRs (two workgroups per CU), where four tiles spill 12 bytes per lane
// and still measured fastest (contraction per 108^3 / Nb = 32 apply: 3, 4, 5 and
// 6 tiles 697, 646, 648 and 662 ms)
constexpr int kBRDepth = 4;

template <bool DIAG, int PD, int NT>
__global__ void __launch_bounds__(BRTile::THREADS)
__attribute__((amdgpu_waves_per_eu(NT == 1 ? 4 : 1)))
k_contract_block_rr(int nb, int nocc, int64_t nr, int ntile, const float* __restrict__ at,
                    const float* __restrict__ tau, BArgs bk, float alpha,
                    float* __restrict__ R) {
  typedef Mfma<float>::acc_t acc_t;
  constexpr int NS = DIAG ? 1 : 2;  // row blocks with accumulators: A (and B)
  constexpr int NRT = 4 * NS;       // row tiles of a and R the workgroup touches
  constexpr int NTILE = DIAG ? 10 : 16;
  __shared__ float s_a[NT * BRTile::NE];
  __shared__ float s_t[2][BRTile::NE];
  const int per = (ntile + 7) / 8;
  const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (tile >= ntile) return;
  const int b0 = blockIdx.y * 16 * NT;
  const int64_t r0 = (int64_t)tile * BRTile::TP;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lx = lane & 15, ly = lane >> 4;
  const int base[2] = {bk.A0, DIAG ? bk.A0 : bk.B0};
  const int nrow[2] = {bk.nA, DIAG ? bk.nA : bk.nB};
  // element u of this thread in a 16-row x 16 NT-trial x 8-point slab of a or R
  constexpr int NBT = 16 * NT;               // trials per workgroup
  constexpr int SU = 16 * NBT * 8 / BRTile::THREADS;  // slab elements per thread
  constexpr int RS = NT == 2 ? 8 : 7;        // log2(trials x points) of one slab row
  auto slab_ok = [&](int rt, int u) {
    const int e = threadIdx.x + u * BRTile::THREADS;
    const int sd = rt >> 2, v = (rt & 3) * 16 + (e >> RS);
    return v < nrow[sd] && b0 + ((e >> 3) & (NBT - 1)) < nb && r0 + (e & 7) < nr;
  };
  auto slab_off = [&](int rt, int u) {
    const int e = threadIdx.x + u * BRTile::THREADS;
    const int sd = rt >> 2, v = (rt & 3) * 16 + (e >> RS);
    return ((int64_t)(b0 + ((e >> 3) & (NBT - 1))) * nocc + base[sd] + v) * nr + r0 + (e & 7);
  };
  auto slab_lds = [&](int u) {
    const int e = threadIdx.x + u * BRTile::THREADS;
    const int b = (e >> 3) & (NBT - 1);
    return (b >> 4) * BRTile::NE + BRTile::at((e >> RS) * 16 + (b & 15), e & 7);
  };

  // 1. every a load of the workgroup in flight at once, then the operand
  // fragments y[row tile][trial tile][k] = a[row 4k + ly][trial lx] per wave
  float la[NRT][SU];
#pragma unroll
  for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
    for (int u = 0; u < SU; ++u) la[rt][u] = slab_ok(rt, u) ? at[slab_off(rt, u)] : 0.f;
  float y[NRT][NT][4];
#pragma unroll
  for (int rt = 0; rt < NRT; ++rt) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < SU; ++u) s_a[slab_lds(u)] = la[rt][u];
    __syncthreads();
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
      for (int k = 0; k < 4; ++k)
        y[rt][tt][k] = s_a[tt * BRTile::NE + BRTile::at((4 * k + ly) * 16 + lx, wave)];
  }

  acc_t acc[NRT][NT];
#pragma unroll
  for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) acc[rt][tt] = acc_t{0.f, 0.f, 0.f, 0.f};

  // 2. tau tiles, PD tiles of loads in flight, staged through two LDS buffers
  float pf[PD][4];
#pragma unroll
  for (int d = 0; d < PD; ++d)
    if (d < NTILE)
      br_load_tau<DIAG>(pf[d], tau, br_tile_i<DIAG>(d), br_tile_j<DIAG>(d), bk, nr, r0);
#pragma unroll
  for (int n = 0; n < NTILE; ++n) {
    constexpr int SB = DIAG ? 0 : 4;  // row-tile offset of block B
    const int I = br_tile_i<DIAG>(n), J = br_tile_j<DIAG>(n);
    float* st = s_t[n & 1];
    br_store_tau(st, pf[n % PD]);
    __syncthreads();
    if (n + PD < NTILE)
      br_load_tau<DIAG>(pf[n % PD], tau, br_tile_i<DIAG>(n + PD), br_tile_j<DIAG>(n + PD), bk,
                        nr, r0);
    float x[4], xt[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      x[k] = st[BRTile::at(lx * 16 + 4 * k + ly, wave)];
      xt[k] = st[BRTile::at((4 * k + ly) * 16 + lx, wave)];
    }
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
      // R[A]_I += tau_IJ a[B]_J  (a[A]_J on the diagonal block)
#pragma unroll
      for (int k = 0; k < 4; ++k)
        acc[I][tt] = Mfma<float>::run(x[k], y[SB + J][tt][k], acc[I][tt]);
      // R[B]_J += tau_IJ^T a[A]_I  (R[A]_J off the diagonal tiles of the diagonal block)
      if (!DIAG || I != J) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
          acc[SB + J][tt] = Mfma<float>::run(xt[k], y[I][tt][k], acc[SB + J][tt]);
      }
    }
  }

  // 3. R -= alpha acc: every R load in flight at once, then per row tile the
  // accumulators are staged through LDS so that the stores are coalesced
#pragma unroll
  for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
    for (int u = 0; u < SU; ++u) la[rt][u] = slab_ok(rt, u) ? R[slab_off(rt, u)] : 0.f;
#pragma unroll
  for (int rt = 0; rt < NRT; ++rt) {
    if ((rt & 3) * 16 >= nrow[rt >> 2]) continue;
    __syncthreads();
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        s_a[tt * BRTile::NE + BRTile::at(Mfma<float>::row(lane, e) * 16 + lx, wave)] =
            acc[rt][tt][e];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < SU; ++u)
      if (slab_ok(rt, u)) R[slab_off(rt, u)] = la[rt][u] - alpha * s_a[slab_lds(u)];
  }
}

// One thread per (grid point, row v): the point's sum over the chunk's rows v'
// reads W once, coalesced along the grid; phi_v'(r) is shared by the nocc
// workgroups of one point range and comes from L2.  Memory-bound: no reuse of
// W across points, so no matrix-core tiling.
template <typename T>
__global__ void __launch_bounds__(256)
k_k2d_rows(int64_t nr, int nocc, int nrows, int r0, const T* __restrict__ phi,
           const T* __restrict__ W, T alpha, T* __restrict__ R) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (r >= nr) return;
  T acc = T(0);
  const T* w = W + (int64_t)v * nr + r;
  const T* f = phi + (int64_t)r0 * nr + r;
  for (int j = 0; j < nrows; ++j) acc += f[(int64_t)j * nr] * w[(int64_t)j * nocc * nr];
  R[(int64_t)v * nr + r] -= alpha * acc;
}
}  // namespace

template <typename T>
bool contract_block_rr_applies(int nb) {
  return sizeof(T) == 4 && nb >= 1;
}

template <typename T>
void launch_contract_block_rr(const Geometry& g, int nb, int nocc, const T* at, const T* tau,
                              int A0, int nA, int B0, int nB, bool diag, T alpha, T* R,
                              hipStream_t s) {
  if constexpr (sizeof(T) != 4) {
    throw StatusError{WTD_ERR_SHAPE, "interleaved block contraction is FP32 only"};
  } else {
    WTD_REQUIRE(nA <= 64 && nB <= 64 && nA >= 1 && nB >= 1 && A0 >= 0 && B0 >= 0 &&
                    A0 + nA <= nocc && B0 + nB <= nocc,
                WTD_ERR_SHAPE, "row blocks of the exchange contraction must be <= 64 rows");
    const int64_t ntile64 = (g.nr + BRTile::TP - 1) / BRTile::TP;
    WTD_REQUIRE(ntile64 < (1ll << 30), WTD_ERR_SHAPE, "contraction grid too large");
    const int ntile = (int)ntile64;
    const int per = (ntile + 7) / 8;
    BArgs bk{A0, nA, B0, nB, diag ? 1 : 0};
    // 16 trials per workgroup: half the registers of a 32-trial workgroup, so
    // two workgroups share a CU and one's loads overlap the other's MFMA work
    // (faster even where tau is then read once per 16 trials: 108^3 / Nb = 32
    // 1,748 -> 1,612 ms per apply; 96^3 / Nb = 10 272 -> 209 ms)
    dim3 grid(8 * per, (nb + 15) / 16);
    if (diag)
      hipLaunchKernelGGL((k_contract_block_rr<true, kBRDepth, 1>), grid, dim3(BRTile::THREADS), 0,
                         s, nb, nocc, g.nr, ntile, at, tau, bk, alpha, R);
    else
      hipLaunchKernelGGL((k_contract_block_rr<false, kBRDepth, 1>), grid, dim3(BRTile::THREADS), 0,
                         s, nb, nocc, g.nr, ntile, at, tau, bk, alpha, R);
    WTD_HIP(hipGetLastError());
  }
}

template bool contract_block_rr_applies<float>(int);
template bool contract_block_rr_applies<double>(int);
template void launch_contract_block_rr<float>(const Geometry&, int, int, const float*,
                                              const float*, int, int, int, int, bool, float,
                                              float*, hipStream_t);
template void launch_contract_block_rr<double>(const Geometry&, int, int, const double*,
                                               const double*, int, int, int, int, bool, double,
                                               double*, hipStream_t);

template <typename T>
void launch_k2d_rows(const Geometry& g, int nocc, int nrows, int r0, const T* phi, const T* W,
                     T alpha, T* R, hipStream_t s) {
  WTD_REQUIRE(nocc >= 1 && nocc <= 65535 && nrows >= 1 && r0 >= 0 && r0 + nrows <= nocc,
              WTD_ERR_SHAPE, "K2d row chunk out of range");
  dim3 grid((unsigned)((g.nr + 255) / 256), (unsigned)nocc);
  hipLaunchKernelGGL(k_k2d_rows<T>, grid, dim3(256), 0, s, g.nr, nocc, nrows, r0, phi, W, alpha,
                     R);
  WTD_HIP(hipGetLastError());
}

template void launch_k2d_rows<float>(const Geometry&, int, int, int, const float*, const float*,
                                     float, float*, hipStream_t);
template void launch_k2d_rows<double>(const Geometry&, int, int, int, const double*,
                                      const double*, double, double*, hipStream_t);

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
